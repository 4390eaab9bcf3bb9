// newell.h -- the demag kernel of Sec. 4.4 in double-double arithmetic.
//
// Near field: the cell-averaged tensor of Newell, Williams & Dunlop (1993),
// built from the auxiliary functions f (for the diagonal) and g (for the off
// diagonal) through a 27-point second-difference stencil with weights
// 2 (zero shift) / -1 (+-1 shift) per axis, divided by 4 pi dx dy dz.  The
// stencil cancels ~R^6-fold at distance R cells, so f and g are evaluated in
// double-double and only the final entry is rounded to double.
// Far field: the point dipole of Eq. (dipole) with moment V Ms m.
// The demag kernel K (h = K M) is -N in the near field.
#pragma once
#include "dd.h"

#pragma clang fp contract(off)

namespace mmx {

// Newell f, even in every argument; x, y, z >= 0.
__host__ __device__ inline dd newell_f(dd x, dd y, dd z)
{
    dd x2 = dd_mul(x, x), y2 = dd_mul(y, y), z2 = dd_mul(z, z);
    dd R2 = dd_add(dd_add(x2, y2), z2);
    if (R2.hi == 0.0) return dd_from(0.0);
    dd R = dd_sqrt(R2);
    // (2x^2 - y^2 - z^2) R / 6
    dd s = dd_div_d(dd_mul(dd_sub(dd_sub(dd_mul_d(x2, 2.0), y2), z2), R), 6.0);
    dd xz2 = dd_add(x2, z2);
    if (xz2.hi > 0.0) {  // y/2 (z^2 - x^2) asinh(y / sqrt(x^2 + z^2))
        dd a = dd_asinh_pos(dd_div(y, dd_sqrt(xz2)));
        s = dd_add(s, dd_mul(dd_mul_d(dd_mul(y, dd_sub(z2, x2)), 0.5), a));
    }
    dd xy2 = dd_add(x2, y2);
    if (xy2.hi > 0.0) {  // z/2 (y^2 - x^2) asinh(z / sqrt(x^2 + y^2))
        dd a = dd_asinh_pos(dd_div(z, dd_sqrt(xy2)));
        s = dd_add(s, dd_mul(dd_mul_d(dd_mul(z, dd_sub(y2, x2)), 0.5), a));
    }
    if (x.hi > 0.0) {  // - x y z atan(y z / (x R))
        dd xyz = dd_mul(dd_mul(x, y), z);
        dd a = dd_atan(dd_div(dd_mul(y, z), dd_mul(x, R)));
        s = dd_sub(s, dd_mul(xyz, a));
    }
    return s;
}

// Newell g for x, y, z >= 0 (the caller applies the odd parity in x and y).
__host__ __device__ inline dd newell_g(dd x, dd y, dd z)
{
    dd x2 = dd_mul(x, x), y2 = dd_mul(y, y), z2 = dd_mul(z, z);
    dd R2 = dd_add(dd_add(x2, y2), z2);
    if (R2.hi == 0.0) return dd_from(0.0);
    dd R = dd_sqrt(R2);
    dd s = dd_neg(dd_div_d(dd_mul(dd_mul(x, y), R), 3.0));  // - x y R / 3
    dd xy2 = dd_add(x2, y2);
    if (xy2.hi > 0.0)  // x y z asinh(z / sqrt(x^2 + y^2))
        s = dd_add(s, dd_mul(dd_mul(dd_mul(x, y), z), dd_asinh_pos(dd_div(z, dd_sqrt(xy2)))));
    dd yz2 = dd_add(y2, z2);
    if (yz2.hi > 0.0) {  // y/6 (3 z^2 - y^2) asinh(x / sqrt(y^2 + z^2))
        dd c = dd_div_d(dd_mul(y, dd_sub(dd_mul_d(z2, 3.0), y2)), 6.0);
        s = dd_add(s, dd_mul(c, dd_asinh_pos(dd_div(x, dd_sqrt(yz2)))));
    }
    dd xz2 = dd_add(x2, z2);
    if (xz2.hi > 0.0) {  // x/6 (3 z^2 - x^2) asinh(y / sqrt(x^2 + z^2))
        dd c = dd_div_d(dd_mul(x, dd_sub(dd_mul_d(z2, 3.0), x2)), 6.0);
        s = dd_add(s, dd_mul(c, dd_asinh_pos(dd_div(y, dd_sqrt(xz2)))));
    }
    if (z.hi > 0.0) {  // - z^3/6 atan(x y / (z R))
        dd c = dd_div_d(dd_mul(z, z2), 6.0);
        s = dd_sub(s, dd_mul(c, dd_atan(dd_div(dd_mul(x, y), dd_mul(z, R)))));
    }
    if (y.hi > 0.0) {  // - z y^2/2 atan(x z / (y R))
        dd c = dd_mul_d(dd_mul(z, y2), 0.5);
        s = dd_sub(s, dd_mul(c, dd_atan(dd_div(dd_mul(x, z), dd_mul(y, R)))));
    }
    if (x.hi > 0.0) {  // - z x^2/2 atan(y z / (x R))
        dd c = dd_mul_d(dd_mul(z, x2), 0.5);
        s = dd_sub(s, dd_mul(c, dd_atan(dd_div(dd_mul(y, z), dd_mul(x, R)))));
    }
    return s;
}

// Stencil sum for one tensor component.  (I, J, K) is the cell offset along
// the component's own axis order, (a, b, c) the matching cell sizes; which = 0
// uses f, 1 uses g.  Returns N (positive self term).
__host__ __device__ inline double newell_component(int which, int I, int J, int K, double a,
                                                   double b, double c)
{
    dd acc = dd_from(0.0);
    for (int e1 = -1; e1 <= 1; ++e1)
        for (int e2 = -1; e2 <= 1; ++e2)
            for (int e3 = -1; e3 <= 1; ++e3) {
                const double w = (e1 == 0 ? 2.0 : -1.0) * (e2 == 0 ? 2.0 : -1.0) *
                                 (e3 == 0 ? 2.0 : -1.0);
                int u = I + e1, v = J + e2, q = K + e3;
                double sg = 1.0;
                if (which == 1) {  // g is odd in its first two arguments
                    if (u < 0) { u = -u; sg = -sg; }
                    if (v < 0) { v = -v; sg = -sg; }
                } else {
                    u = u < 0 ? -u : u;
                    v = v < 0 ? -v : v;
                }
                q = q < 0 ? -q : q;
                // the coordinates (integer) * (cell size) are exact in double-double
                dd X = two_prod((double)u, a), Y = two_prod((double)v, b), Z = two_prod((double)q, c);
                dd val = which == 0 ? newell_f(X, Y, Z) : newell_g(X, Y, Z);
                acc = dd_add(acc, dd_mul_d(val, w * sg));
            }
    dd den = dd_mul_d(dd_mul_d(dd_mul_d(dd_mul_d(dd_pi(), 4.0), a), b), c);
    dd r = dd_div(acc, den);
    return r.hi + r.lo;
}

// Demag kernel entry K_s (h = K M) for offset (I, J, K) >= 0 in cells, near
// field: -N.  s = 0..5 -> xx, yy, zz, xy, xz, yz.
__host__ __device__ inline double kernel_near(int s, int I, int J, int K, double dx, double dy,
                                              double dz)
{
    switch (s) {
    case 0: return -newell_component(0, I, J, K, dx, dy, dz);
    case 1: return -newell_component(0, J, I, K, dy, dx, dz);
    case 2: return -newell_component(0, K, J, I, dz, dy, dx);
    case 3: return -newell_component(1, I, J, K, dx, dy, dz);
    case 4: return -newell_component(1, I, K, J, dx, dz, dy);
    default: return -newell_component(1, J, K, I, dy, dz, dx);
    }
}

// Far field: point dipole (Eq. dipole), h = V/(4 pi) (3 r (M.r) - r^2 M) / r^5.
__host__ __device__ inline double kernel_dipole(int s, int I, int J, int K, double dx, double dy,
                                                double dz)
{
    const double rx = I * dx, ry = J * dy, rz = K * dz;
    const double r2 = rx * rx + ry * ry + rz * rz;
    const double pre = dx * dy * dz / (4.0 * M_PI) / (r2 * r2 * sqrt(r2));
    switch (s) {
    case 0: return pre * (3.0 * rx * rx - r2);
    case 1: return pre * (3.0 * ry * ry - r2);
    case 2: return pre * (3.0 * rz * rz - r2);
    case 3: return pre * 3.0 * rx * ry;
    case 4: return pre * 3.0 * rx * rz;
    default: return pre * 3.0 * ry * rz;
    }
}

// ---------------------------------------------------------------------------
// Thin layers of unequal height (Sec. 4.4, non-equidistant case).  Along an
// axis where the target spans [0, t] and the source [B, B + s], the double
// integral of a second derivative F'' is F(B + s) - F(B + s - t) - F(B) +
// F(B - t); with t = s it is the second difference of the equal-cell stencil.
// The entry is normalised by the target volume.
struct AxisPts {
    dd x[4];
    double w[4];  // sign of Newell's equal-cell stencil (positive self term)
    int n;
};

// Equal cells along a lateral axis: offset I cells of size a (source minus
// target), the three points (I - 1) a, I a, (I + 1) a, exact in double-double.
__host__ __device__ inline AxisPts axis_equal(int I, double a)
{
    AxisPts r;
    r.n = 3;
    r.x[0] = two_prod((double)(I - 1), a);
    r.w[0] = -1.0;
    r.x[1] = two_prod((double)I, a);
    r.w[1] = 2.0;
    r.x[2] = two_prod((double)(I + 1), a);
    r.w[2] = -1.0;
    r.x[3] = dd_from(0.0);
    r.w[3] = 0.0;
    return r;
}

// Unequal heights: source bottom B above the target bottom, target height t,
// source height s.
__host__ __device__ inline AxisPts axis_layer(dd B, double t, double s)
{
    AxisPts r;
    r.n = 4;
    r.x[0] = dd_add(B, dd_from(s));
    r.w[0] = -1.0;
    r.x[1] = dd_sub(dd_add(B, dd_from(s)), dd_from(t));
    r.w[1] = 1.0;
    r.x[2] = B;
    r.w[2] = 1.0;
    r.x[3] = dd_sub(B, dd_from(t));
    r.w[3] = -1.0;
    return r;
}

// Stencil sum of f (which 0) or g (which 1) over the argument slots (u, v, q)
// divided by den; g is odd in its first two arguments, f even in all.
__host__ __device__ inline double box_component(int which, const AxisPts& u, const AxisPts& v,
                                                const AxisPts& q, dd den)
{
    dd acc = dd_from(0.0);
    for (int a = 0; a < u.n; ++a)
        for (int b = 0; b < v.n; ++b)
            for (int e = 0; e < q.n; ++e) {
                dd X = u.x[a], Y = v.x[b], Z = q.x[e];
                double sg = u.w[a] * v.w[b] * q.w[e];
                if (X.hi < 0.0) {
                    X = dd_neg(X);
                    if (which == 1) sg = -sg;
                }
                if (Y.hi < 0.0) {
                    Y = dd_neg(Y);
                    if (which == 1) sg = -sg;
                }
                if (Z.hi < 0.0) Z = dd_neg(Z);
                dd val = which == 0 ? newell_f(X, Y, Z) : newell_g(X, Y, Z);
                acc = dd_add(acc, dd_mul_d(val, sg));
            }
    dd r = dd_div(acc, den);
    return r.hi + r.lo;
}

// Layered demag kernel entry K^{ts}_s (h_t = sum K M_s) near field, -N, for
// the lateral offset I = i_t - i_s, J = j_t - j_s and the layer bottoms zb.
__host__ __device__ inline double kernel_near_layer(int comp, int I, int J, const double* zb, int t,
                                                    int s, double dx, double dy)
{
    const double ct = zb[t + 1] - zb[t], cs = zb[s + 1] - zb[s];
    const AxisPts X = axis_equal(-I, dx), Y = axis_equal(-J, dy);
    const AxisPts Z = axis_layer(two_sum(zb[s], -zb[t]), ct, cs);
    const dd den = dd_mul_d(dd_mul_d(dd_mul_d(dd_mul_d(dd_pi(), 4.0), dx), dy), ct);
    switch (comp) {
    case 0: return -box_component(0, X, Y, Z, den);
    case 1: return -box_component(0, Y, X, Z, den);
    case 2: return -box_component(0, Z, Y, X, den);
    case 3: return -box_component(1, X, Y, Z, den);
    case 4: return -box_component(1, X, Z, Y, den);
    default: return -box_component(1, Y, Z, X, den);
    }
}

// Layered far field: the dipole of the source cell's moment (volume
// dx dy dz_s) at the centre offset (target minus source).
__host__ __device__ inline double kernel_dipole_layer(int comp, int I, int J, const double* zb,
                                                      int t, int s, double dx, double dy)
{
    const double rx = I * dx, ry = J * dy;
    const double rz = 0.5 * (zb[t] + zb[t + 1]) - 0.5 * (zb[s] + zb[s + 1]);
    const double r2 = rx * rx + ry * ry + rz * rz;
    const double pre = dx * dy * (zb[s + 1] - zb[s]) / (4.0 * M_PI) / (r2 * r2 * sqrt(r2));
    switch (comp) {
    case 0: return pre * (3.0 * rx * rx - r2);
    case 1: return pre * (3.0 * ry * ry - r2);
    case 2: return pre * (3.0 * rz * rz - r2);
    case 3: return pre * 3.0 * rx * ry;
    case 4: return pre * 3.0 * rx * rz;
    default: return pre * 3.0 * ry * rz;
    }
}

// ---------------------------------------------------------------------------
// Oersted kernel (Sec. 4.5): h_t = sum_s j_s x G(X_t - X_s), G the average over
// the target cell of the Biot-Savart vector (x - x')/(4 pi |x - x'|^3) of a
// uniform source cell.  G_l is a first derivative along l, so its 27-point
// stencil (Newell's weights, divided by 4 pi V) runs over Fo, the
// antiderivative of Newell's f along l:
//   Fo(x,y,z) = x R^3/12 - 5/24 (y^2+z^2) x R
//             + (y^2 z^2/3 - (y^2+z^2)^2/24) asinh(x / sqrt(y^2+z^2))
//             + y/2 (x z^2 - x^3/3) asinh(y / sqrt(x^2+z^2))
//             + z/2 (x y^2 - x^3/3) asinh(z / sqrt(x^2+y^2))
//             - x^2 y z/2 atan(y z/(x R)) - y z^3/6 atan(x y/(z R))
//             - y^3 z/6 atan(x z/(y R)),
// odd in x, even in y and z.
// ---------------------------------------------------------------------------
__host__ __device__ inline dd oersted_Fo(dd x, dd y, dd z)
{
    // x, y, z >= 0 (the caller applies the odd parity in x)
    dd x2 = dd_mul(x, x), y2 = dd_mul(y, y), z2 = dd_mul(z, z);
    dd r2 = dd_add(y2, z2);
    dd R2 = dd_add(x2, r2);
    if (R2.hi == 0.0) return dd_from(0.0);
    dd R = dd_sqrt(R2);
    dd xR = dd_mul(x, R);
    // x R^3 / 12 - 5/24 r2 x R
    dd s = dd_sub(dd_div_d(dd_mul(xR, R2), 12.0), dd_div_d(dd_mul_d(dd_mul(r2, xR), 5.0), 24.0));
    if (r2.hi > 0.0) {
        dd c = dd_sub(dd_div_d(dd_mul(y2, z2), 3.0), dd_div_d(dd_mul(r2, r2), 24.0));
        s = dd_add(s, dd_mul(c, dd_asinh_pos(dd_div(x, dd_sqrt(r2)))));
    }
    dd x3_3 = dd_div_d(dd_mul(x2, x), 3.0);
    dd xz2 = dd_add(x2, z2);
    if (xz2.hi > 0.0) {
        dd c = dd_mul_d(dd_mul(y, dd_sub(dd_mul(x, z2), x3_3)), 0.5);
        s = dd_add(s, dd_mul(c, dd_asinh_pos(dd_div(y, dd_sqrt(xz2)))));
    }
    dd xy2 = dd_add(x2, y2);
    if (xy2.hi > 0.0) {
        dd c = dd_mul_d(dd_mul(z, dd_sub(dd_mul(x, y2), x3_3)), 0.5);
        s = dd_add(s, dd_mul(c, dd_asinh_pos(dd_div(z, dd_sqrt(xy2)))));
    }
    dd yz = dd_mul(y, z);
    if (x.hi > 0.0)
        s = dd_sub(s, dd_mul(dd_mul_d(dd_mul(x2, yz), 0.5), dd_atan(dd_div(yz, xR))));
    if (z.hi > 0.0)
        s = dd_sub(s, dd_mul(dd_div_d(dd_mul(yz, z2), 6.0), dd_atan(dd_div(dd_mul(x, y), dd_mul(z, R)))));
    if (y.hi > 0.0)
        s = dd_sub(s, dd_mul(dd_div_d(dd_mul(yz, y2), 6.0), dd_atan(dd_div(dd_mul(x, z), dd_mul(y, R)))));
    return s;
}

// Near-field G_comp for the cell offset (I, J, K) (target minus source).
__host__ __device__ inline double oersted_near(int comp, int I, int J, int K, double dx, double dy,
                                               double dz)
{
    const int off[3] = {I, J, K};
    const double d[3] = {dx, dy, dz};
    const int l = comp, u = (comp + 1) % 3, v = (comp + 2) % 3;
    dd acc = dd_from(0.0);
    for (int e0 = -1; e0 <= 1; ++e0)
        for (int e1 = -1; e1 <= 1; ++e1)
            for (int e2 = -1; e2 <= 1; ++e2) {
                const double w = (e0 == 0 ? 2.0 : -1.0) * (e1 == 0 ? 2.0 : -1.0) *
                                 (e2 == 0 ? 2.0 : -1.0);
                int a = off[l] + e0, b = off[u] + e1, c = off[v] + e2;
                double sg = w;
                if (a < 0) {  // Fo is odd in its first argument
                    a = -a;
                    sg = -sg;
                }
                b = b < 0 ? -b : b;
                c = c < 0 ? -c : c;
                dd val = oersted_Fo(two_prod((double)a, d[l]), two_prod((double)b, d[u]),
                                    two_prod((double)c, d[v]));
                acc = dd_add(acc, dd_mul_d(val, sg));
            }
    dd den = dd_mul_d(dd_mul_d(dd_mul_d(dd_mul_d(dd_pi(), 4.0), dx), dy), dz);
    dd r = dd_div(acc, den);
    return r.hi + r.lo;
}

// Far field: the singular current, G = V D / (4 pi |D|^3).
__host__ __device__ inline double oersted_point(int comp, int I, int J, int K, double dx, double dy,
                                                double dz)
{
    const double D[3] = {I * dx, J * dy, K * dz};
    const double r2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
    return dx * dy * dz / (4.0 * M_PI) / (r2 * sqrt(r2)) * D[comp];
}

}  // namespace mmx

// restore the compiler default for the code that follows
#pragma clang fp contract(fast)

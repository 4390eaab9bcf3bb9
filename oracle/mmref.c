/*
 * mmref.c -- CPU reference ("oracle") for the finite-difference micromagnetic
 * hot path of Bruckner et al., "magnum.np -- A PyTorch based GPU enhanced
 * Finite Difference Micromagnetic Simulation Framework" (arXiv:2302.08843).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * loaded by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  The product library never links, loads or calls it, and the two
 * share no source: every formula here is written out again from the paper and
 * from the works it cites.
 *
 * Plain, slow, obviously correct: FP64 everywhere except the near-field Newell
 * tensor, which is evaluated in x87 long double and rounded to double because
 * Newell's f and g cancel catastrophically at a distance of a few cells.
 * OpenMP only splits independent rows / cells across threads; it reorders no
 * arithmetic inside a row or a cell.
 *
 * Parity status of each part (what pins it) is listed with each function.
 * Parity unpinned: the opposite-sign branch of the DMI coupling average
 * (dmi_avg below) -- only its symmetry and its bounds are checked.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Constants                                                                  */
/* ------------------------------------------------------------------------- */

/* Vacuum permeability.  The paper does not print it; the classical exact
 * value 4*pi*1e-7 is used. */
#define OR_MU0 (4.0e-7 * 3.14159265358979323846)
/* Reduced gyromagnetic ratio as printed with the LLG equation (Sec. 3). */
#define OR_GAMMA 2.21e5
#define OR_PI_L 3.141592653589793238462643383279502884L

enum { OR_DEMAG = 1, OR_EXCH = 2, OR_ANIS = 4, OR_ZEEMAN = 8, OR_DMI = 16, OR_OERSTED = 32 };

/* ------------------------------------------------------------------------- */
/* Newell, Williams & Dunlop (1993) cell-averaged demagnetisation tensor,     */
/* cited in Sec. 4.4 for the near field.  Pinned by: self term 1/3 of a cube, */
/* trace identities, Aharoni's prism factors, the dipole limit, the uniform-  */
/* cube field, and the box demag factors (tests/test_oracle_tensor.py).       */
/* ------------------------------------------------------------------------- */

/* Newell's f: even in each argument. */
static long double newell_f(long double x, long double y, long double z)
{
    x = fabsl(x);
    y = fabsl(y);
    z = fabsl(z);
    long double x2 = x * x, y2 = y * y, z2 = z * z;
    long double R = sqrtl(x2 + y2 + z2);
    if (R == 0.0L)
        return 0.0L;
    long double s = (2.0L * x2 - y2 - z2) * R / 6.0L;
    /* A term whose logarithm / arctangent argument is singular has a vanishing
     * prefactor there; dropping it is the exact limit. */
    if (x2 + z2 > 0.0L)
        s += 0.5L * y * (z2 - x2) * asinhl(y / sqrtl(x2 + z2));
    if (x2 + y2 > 0.0L)
        s += 0.5L * z * (y2 - x2) * asinhl(z / sqrtl(x2 + y2));
    if (x > 0.0L)
        s -= x * y * z * atanl(y * z / (x * R));
    return s;
}

/* Newell's g: odd in x and in y, even in z. */
static long double newell_g(long double x, long double y, long double z)
{
    long double sg = 1.0L;
    if (x < 0.0L) { x = -x; sg = -sg; }
    if (y < 0.0L) { y = -y; sg = -sg; }
    z = fabsl(z);
    long double x2 = x * x, y2 = y * y, z2 = z * z;
    long double R = sqrtl(x2 + y2 + z2);
    if (R == 0.0L)
        return 0.0L;
    long double s = -x * y * R / 3.0L;
    if (x2 + y2 > 0.0L)
        s += x * y * z * asinhl(z / sqrtl(x2 + y2));
    if (y2 + z2 > 0.0L)
        s += y / 6.0L * (3.0L * z2 - y2) * asinhl(x / sqrtl(y2 + z2));
    if (x2 + z2 > 0.0L)
        s += x / 6.0L * (3.0L * z2 - x2) * asinhl(y / sqrtl(x2 + z2));
    if (z > 0.0L)
        s -= z * z2 / 6.0L * atanl(x * y / (z * R));
    if (y > 0.0L)
        s -= z * y2 / 2.0L * atanl(x * z / (y * R));
    if (x > 0.0L)
        s -= z * x2 / 2.0L * atanl(y * z / (x * R));
    return sg * s;
}

/* Second-difference stencil over the 27 neighbours of (X,Y,Z) with cell size
 * (a,b,c): weight 2 for a zero shift and -1 for a +-1 shift, per axis.
 * which: 0 -> f, 1 -> g. */
static long double newell_stencil(int which, long double X, long double Y, long double Z,
                                  long double a, long double b, long double c)
{
    long double acc = 0.0L;
    for (int e1 = -1; e1 <= 1; e1++)
        for (int e2 = -1; e2 <= 1; e2++)
            for (int e3 = -1; e3 <= 1; e3++) {
                long double w = (e1 == 0 ? 2.0L : -1.0L) * (e2 == 0 ? 2.0L : -1.0L) *
                                (e3 == 0 ? 2.0L : -1.0L);
                long double u = X + e1 * a, v = Y + e2 * b, q = Z + e3 * c;
                acc += w * (which == 0 ? newell_f(u, v, q) : newell_g(u, v, q));
            }
    return acc / (4.0L * OR_PI_L * a * b * c);
}

/* Newell tensor N (positive self term) between cells offset by (I,J,K) cells.
 * out = {Nxx, Nyy, Nzz, Nxy, Nxz, Nyz}. */
void or_newell(const double d[3], long oi, long oj, long ok, double out[6])
{
    long double dx = d[0], dy = d[1], dz = d[2];
    long double X = oi * dx, Y = oj * dy, Z = ok * dz;
    out[0] = (double)newell_stencil(0, X, Y, Z, dx, dy, dz);
    out[1] = (double)newell_stencil(0, Y, X, Z, dy, dx, dz);
    out[2] = (double)newell_stencil(0, Z, Y, X, dz, dy, dx);
    out[3] = (double)newell_stencil(1, X, Y, Z, dx, dy, dz);
    out[4] = (double)newell_stencil(1, X, Z, Y, dx, dz, dy);
    out[5] = (double)newell_stencil(1, Y, Z, X, dy, dz, dx);
}

/* Point-dipole kernel of Eq. (dipole): the field of the moment V*Ms*m at the
 * cell-centre distance r.  out in the same component order, positive sign
 * (it multiplies M to give h). */
void or_dipole(const double d[3], long oi, long oj, long ok, double out[6])
{
    double r[3] = {oi * d[0], oj * d[1], ok * d[2]};
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double r5 = r2 * r2 * sqrt(r2);
    double pre = d[0] * d[1] * d[2] / (4.0 * M_PI) / r5;
    out[0] = pre * (3.0 * r[0] * r[0] - r2);
    out[1] = pre * (3.0 * r[1] * r[1] - r2);
    out[2] = pre * (3.0 * r[2] * r[2] - r2);
    out[3] = pre * 3.0 * r[0] * r[1];
    out[4] = pre * 3.0 * r[0] * r[2];
    out[5] = pre * 3.0 * r[1] * r[2];
}

/* Demag kernel K with h_i = sum_j K_{i-j} Ms_j m_j (Sec. 4.4, discrete
 * convolution).  Near field (Chebyshev index distance <= p): K = -N_Newell.
 * Far field: the dipole kernel.  p < 0 means Newell everywhere. */
void or_tensor_entry(const double d[3], long oi, long oj, long ok, int p, double out[6])
{
    long cheb = labs(oi);
    if (labs(oj) > cheb) cheb = labs(oj);
    if (labs(ok) > cheb) cheb = labs(ok);
    if (p < 0 || cheb <= p) {
        or_newell(d, oi, oj, ok, out);
        for (int c = 0; c < 6; c++)
            out[c] = -out[c];
    } else {
        or_dipole(d, oi, oj, ok, out);
    }
}

/* ------------------------------------------------------------------------- */
/* Thin layers of unequal thickness (Sec. 4.4, the non-equidistant case):     */
/* the cell-averaged tensor between a target box and a source box of another  */
/* height.  Along an axis where the target spans [0, t] and the source        */
/* [B, B + s], the double integral of a second derivative F'' over the pair   */
/* is F(B + s) - F(B + s - t) - F(B) + F(B - t); for t = s it is the second   */
/* difference of Newell's equal-cell stencil.  The result is normalised by    */
/* the target volume (the field is averaged over the target).  Pinned by the  */
/* equal-height limit, additivity in the source, volume-weighted averaging    */
/* over the target and the dipole limit (tests/test_oracle_layers.py).        */
/* ------------------------------------------------------------------------- */

/* Points and weights of one axis: bottom offset B, target size t, source
 * size s.  The weights carry the sign of Newell's equal-cell stencil
 * (positive self term). */
static void axis_points(long double B, long double t, long double s, long double pt[4],
                        long double w[4])
{
    pt[0] = B + s;
    w[0] = -1.0L;
    pt[1] = B + s - t;
    w[1] = 1.0L;
    pt[2] = B;
    w[2] = 1.0L;
    pt[3] = B - t;
    w[3] = -1.0L;
}

/* One component from f (which 0) or g (which 1) with the argument slots
 * (u, v, q): bottom offsets Bu, Bv, Bq, target sizes tu, tv, tq, source sizes
 * su, sv, sq. */
static long double box_stencil(int which, const long double B[3], const long double tz[3],
                               const long double sz[3])
{
    long double pu[4], wu[4], pv[4], wv[4], pq[4], wq[4];
    axis_points(B[0], tz[0], sz[0], pu, wu);
    axis_points(B[1], tz[1], sz[1], pv, wv);
    axis_points(B[2], tz[2], sz[2], pq, wq);
    long double acc = 0.0L;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            for (int e = 0; e < 4; e++)
                acc += wu[a] * wv[b] * wq[e] *
                       (which == 0 ? newell_f(pu[a], pv[b], pq[e]) : newell_g(pu[a], pv[b], pq[e]));
    return acc / (4.0L * OR_PI_L * tz[0] * tz[1] * tz[2]);
}

/* Newell tensor N between a target cell of height ct and a source cell of
 * height cs whose bottom lies Bz above the target's bottom and which sits
 * (oi dx, oj dy) from the target laterally (source minus target).
 * out = {Nxx, Nyy, Nzz, Nxy, Nxz, Nyz}. */
void or_newell_box(double dx, double dy, long oi, long oj, double Bz, double ct, double cs,
                   double out[6])
{
    long double X = oi * (long double)dx, Y = oj * (long double)dy;
    long double a = dx, b = dy;
    /* slot orders as in or_newell: xx f(x,y,z), yy f(y,x,z), zz f(z,y,x),
     * xy g(x,y,z), xz g(x,z,y), yz g(y,z,x) */
    long double B[3], T[3], S[3];
#define SLOT(k, base, tt, ss) (B[k] = (base), T[k] = (tt), S[k] = (ss))
    SLOT(0, X, a, a); SLOT(1, Y, b, b); SLOT(2, Bz, ct, cs);
    out[0] = (double)box_stencil(0, B, T, S);
    out[3] = (double)box_stencil(1, B, T, S);
    SLOT(0, Y, b, b); SLOT(1, X, a, a); SLOT(2, Bz, ct, cs);
    out[1] = (double)box_stencil(0, B, T, S);
    SLOT(0, Bz, ct, cs); SLOT(1, Y, b, b); SLOT(2, X, a, a);
    out[2] = (double)box_stencil(0, B, T, S);
    SLOT(0, X, a, a); SLOT(1, Bz, ct, cs); SLOT(2, Y, b, b);
    out[4] = (double)box_stencil(1, B, T, S);
    SLOT(0, Y, b, b); SLOT(1, Bz, ct, cs); SLOT(2, X, a, a);
    out[5] = (double)box_stencil(1, B, T, S);
#undef SLOT
}

/* Layered demag kernel entry K^{ts}(I, J) (h_t = sum K M_s) for the lateral
 * offset I = i_t - i_s, J = j_t - j_s: -N within Chebyshev index distance p
 * in (I, J, s - t), else the dipole of the source cell's moment (volume
 * dx dy dz_s) at the centre offset.  zb: layer bottoms (nz + 1 values,
 * zb[0] = 0). */
void or_layer_entry(double dx, double dy, const double *zb, long t, long s, long oi, long oj, int p,
                    double out[6])
{
    double ct = zb[t + 1] - zb[t], cs = zb[s + 1] - zb[s];
    long cheb = labs(oi);
    if (labs(oj) > cheb) cheb = labs(oj);
    if (labs(s - t) > cheb) cheb = labs(s - t);
    if (p < 0 || cheb <= p) {
        or_newell_box(dx, dy, -oi, -oj, zb[s] - zb[t], ct, cs, out);
        for (int q = 0; q < 6; q++)
            out[q] = -out[q];
        return;
    }
    /* r from the source centre to the target centre */
    double r[3] = {oi * dx, oj * dy, 0.5 * (zb[t] + zb[t + 1]) - 0.5 * (zb[s] + zb[s + 1])};
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double pre = dx * dy * cs / (4.0 * M_PI) / (r2 * r2 * sqrt(r2));
    out[0] = pre * (3.0 * r[0] * r[0] - r2);
    out[1] = pre * (3.0 * r[1] * r[1] - r2);
    out[2] = pre * (3.0 * r[2] * r[2] - r2);
    out[3] = pre * 3.0 * r[0] * r[1];
    out[4] = pre * 3.0 * r[0] * r[2];
    out[5] = pre * 3.0 * r[1] * r[2];
}

/* ------------------------------------------------------------------------- */
/* Oersted field (Sec. 4.5): the Biot-Savart field of a current density j,    */
/* h(x) = (1/4 pi) int j(x') x (x - x') / |x - x'|^3 dx'.  For cells of       */
/* uniform j the cell-averaged field is h_t = sum_s j_s x G(X_t - X_s) with   */
/* G(D) = (1/(4 pi V)) int_t int_s (x - x') / |x - x'|^3 dx' dx, the average  */
/* over the target of the field of a uniformly "charged" source box.  Along   */
/* its own axis G_l is a first derivative, so its stencil uses the            */
/* antiderivative F = int f dx of Newell's f along that axis, with Newell's   */
/* 27-point second-difference weights (Krueger et al. solve the same         */
/* integrals analytically).  Far field: the singular current density,        */
/* G = V D / (4 pi |D|^3).  Pinned by the point-current limit, the self term, */
/* antisymmetry, refinement consistency and the finite straight wire          */
/* (tests/test_oracle_oersted.py).                                            */
/* ------------------------------------------------------------------------- */

/* F(x, y, z) = int_0^x f(u, y, z) du for y, z >= 0: odd in x. */
static long double oersted_F(long double x, long double y, long double z)
{
    y = fabsl(y);
    z = fabsl(z);
    long double x2 = x * x, y2 = y * y, z2 = z * z, r2 = y2 + z2;
    long double R = sqrtl(x2 + y2 + z2);
    if (R == 0.0L)
        return 0.0L;
    long double s = x * R * R * R / 12.0L - 5.0L / 24.0L * r2 * x * R;
    if (r2 > 0.0L)
        s += (y2 * z2 / 3.0L - r2 * r2 / 24.0L) * asinhl(x / sqrtl(r2));
    if (x2 + z2 > 0.0L)
        s += 0.5L * y * (x * z2 - x * x2 / 3.0L) * asinhl(y / sqrtl(x2 + z2));
    if (x2 + y2 > 0.0L)
        s += 0.5L * z * (x * y2 - x * x2 / 3.0L) * asinhl(z / sqrtl(x2 + y2));
    if (x != 0.0L)
        s -= 0.5L * x2 * y * z * atanl(y * z / (x * R));
    if (z != 0.0L)
        s -= y * z * z2 / 6.0L * atanl(x * y / (z * R));
    if (y != 0.0L)
        s -= y * y2 * z / 6.0L * atanl(x * z / (y * R));
    return s;
}

/* G_l(D) for the cell offset D = (I dx, J dy, K dz) (target minus source),
 * near field. */
static void oersted_near(const double d[3], long oi, long oj, long ok, double out[3])
{
    long double D[3] = {oi * (long double)d[0], oj * (long double)d[1], ok * (long double)d[2]};
    for (int l = 0; l < 3; l++) {
        int u = (l + 1) % 3, v = (l + 2) % 3;
        long double acc = 0.0L;
        for (int e0 = -1; e0 <= 1; e0++)
            for (int e1 = -1; e1 <= 1; e1++)
                for (int e2 = -1; e2 <= 1; e2++) {
                    long double w = (e0 == 0 ? 2.0L : -1.0L) * (e1 == 0 ? 2.0L : -1.0L) *
                                    (e2 == 0 ? 2.0L : -1.0L);
                    acc += w * oersted_F(D[l] + e0 * (long double)d[l], D[u] + e1 * (long double)d[u],
                                         D[v] + e2 * (long double)d[v]);
                }
        out[l] = (double)(acc / (4.0L * OR_PI_L * d[0] * d[1] * d[2]));
    }
}

/* Oersted kernel G(I, J, K): near field within Chebyshev index distance p
 * (p < 0: everywhere), else the singular current density. */
void or_oersted_entry(const double d[3], long oi, long oj, long ok, int p, double out[3])
{
    long cheb = labs(oi);
    if (labs(oj) > cheb) cheb = labs(oj);
    if (labs(ok) > cheb) cheb = labs(ok);
    if (p < 0 || cheb <= p) {
        oersted_near(d, oi, oj, ok, out);
        return;
    }
    double D[3] = {oi * d[0], oj * d[1], ok * d[2]};
    double r2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
    double pre = d[0] * d[1] * d[2] / (4.0 * M_PI) / (r2 * sqrt(r2));
    for (int l = 0; l < 3; l++)
        out[l] = pre * D[l];
}

/* Demagnetisation field at selected target cells by direct summation of the
 * discrete convolution h_i = sum_j K_{i-j} Ms_j m_j (Sec. 4.4) over every
 * source cell -- no padded grid and no FFT, so it serves grids far too large
 * for the FFT path.  Near-field entries (Chebyshev index distance <= p) are
 * tabulated once; the rest are dipole entries.  Ms: per cell, or NULL for the
 * uniform value Ms0.  m is [3][N], x fastest; cells holds ncell linear cell
 * indices; out receives 3 values (x, y, z) per target.  Returns 0, or -1 for
 * p < 0 (Newell everywhere is not tabulated here). */
int or_demag_at(const long n[3], const double d[3], int p, const double *Ms, double Ms0,
                const double *m, long ncell, const long *cells, double *out)
{
    if (p < 0)
        return -1;
    long nx = n[0], ny = n[1], nz = n[2], N = nx * ny * nz;
    long rx = p < nx - 1 ? p : nx - 1, ry = p < ny - 1 ? p : ny - 1, rz = p < nz - 1 ? p : nz - 1;
    long tx = 2 * rx + 1, ty = 2 * ry + 1, tz = 2 * rz + 1, nt = tx * ty * tz;
    double *T = malloc(sizeof(double) * 6 * nt);
#pragma omp parallel for schedule(dynamic, 64)
    for (long q = 0; q < nt; q++) {
        long oi = q % tx - rx, oj = (q / tx) % ty - ry, ok = q / (tx * ty) - rz;
        or_tensor_entry(d, oi, oj, ok, p, T + 6 * q);
    }
    for (long s = 0; s < ncell; s++) {
        long t = cells[s];
        long i = t % nx, j = (t / nx) % ny, k = t / (nx * ny);
        long double hx = 0.0L, hy = 0.0L, hz = 0.0L;
#pragma omp parallel for reduction(+ : hx, hy, hz) schedule(static)
        for (long src = 0; src < N; src++) {
            long si = src % nx, sj = (src / nx) % ny, sk = src / (nx * ny);
            long oi = i - si, oj = j - sj, ok = k - sk;
            double e[6];
            /* |oi| <= nx - 1 always, so |oi| <= rx exactly when |oi| <= p */
            if (labs(oi) <= rx && labs(oj) <= ry && labs(ok) <= rz) {
                const double *te = T + 6 * ((oi + rx) + tx * ((oj + ry) + ty * (ok + rz)));
                for (int c = 0; c < 6; c++)
                    e[c] = te[c];
            } else {
                or_dipole(d, oi, oj, ok, e);
            }
            double ms = Ms ? Ms[src] : Ms0;
            double Mx = ms * m[src], My = ms * m[N + src], Mz = ms * m[2 * N + src];
            hx += e[0] * Mx + e[3] * My + e[4] * Mz;
            hy += e[3] * Mx + e[1] * My + e[5] * Mz;
            hz += e[4] * Mx + e[5] * My + e[2] * Mz;
        }
        out[3 * s] = (double)hx;
        out[3 * s + 1] = (double)hy;
        out[3 * s + 2] = (double)hz;
    }
    free(T);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* FFT: iterative radix-2 Cooley-Tukey with bit reversal, twiddles from long  */
/* double sin/cos.  sign = -1 forward, +1 inverse (unnormalised).  Pinned by  */
/* the naive DFT below at every power-of-two length up to 1024.              */
/* ------------------------------------------------------------------------- */

static void fft_pow2(long n, double complex *x, const double complex *tw /* n/2 roots */)
{
    for (long i = 1, j = 0; i < n; i++) {
        long bit = n >> 1;
        for (; j & bit; bit >>= 1)
            j ^= bit;
        j ^= bit;
        if (i < j) {
            double complex t = x[i];
            x[i] = x[j];
            x[j] = t;
        }
    }
    for (long len = 2; len <= n; len <<= 1) {
        long half = len >> 1, step = n / len;
        for (long s = 0; s < n; s += len)
            for (long k = 0; k < half; k++) {
                double complex w = tw[k * step];
                double complex u = x[s + k], v = x[s + k + half] * w;
                x[s + k] = u + v;
                x[s + k + half] = u - v;
            }
    }
}

static double complex *make_twiddles(long n, int sign)
{
    double complex *tw = malloc(sizeof(double complex) * (n > 1 ? n / 2 : 1));
    for (long k = 0; k < n / 2; k++) {
        long double ang = sign * 2.0L * OR_PI_L * (long double)k / (long double)n;
        tw[k] = (double)cosl(ang) + I * (double)sinl(ang);
    }
    return tw;
}

void or_fft1d(long n, double complex *x, int sign)
{
    if (n <= 1)
        return;
    double complex *tw = make_twiddles(n, sign);
    fft_pow2(n, x, tw);
    free(tw);
}

/* Naive O(n^2) DFT with long-double accumulation (the definition). */
void or_dft1d(long n, const double complex *x, double complex *X, int sign)
{
    for (long k = 0; k < n; k++) {
        long double re = 0.0L, im = 0.0L;
        for (long j = 0; j < n; j++) {
            long double ang = sign * 2.0L * OR_PI_L * (long double)((j * k) % n) / (long double)n;
            long double c = cosl(ang), s = sinl(ang);
            long double xr = creal(x[j]), xi = cimag(x[j]);
            re += xr * c - xi * s;
            im += xr * s + xi * c;
        }
        X[k] = (double)re + I * (double)im;
    }
}

/* 3-D transform of a complex array a[k][j][i] of extent P (x fastest), done
 * as 1-D transforms along x, then y, then z. */
static void fft3d(const long P[3], double complex *a, int sign)
{
    for (int ax = 0; ax < 3; ax++) {
        long n = P[ax];
        if (n <= 1)
            continue;
        long stride = ax == 0 ? 1 : (ax == 1 ? P[0] : P[0] * P[1]);
        long nlines = P[0] * P[1] * P[2] / n;
        double complex *tw = make_twiddles(n, sign);
#pragma omp parallel
        {
            double complex *buf = malloc(sizeof(double complex) * n);
#pragma omp for schedule(static)
            for (long l = 0; l < nlines; l++) {
                long base;
                if (ax == 0)
                    base = l * P[0];
                else if (ax == 1)
                    base = (l / P[0]) * P[0] * P[1] + (l % P[0]);
                else
                    base = l;
                for (long e = 0; e < n; e++)
                    buf[e] = a[base + e * stride];
                fft_pow2(n, buf, tw);
                for (long e = 0; e < n; e++)
                    a[base + e * stride] = buf[e];
            }
            free(buf);
        }
        free(tw);
    }
}

/* Padded extent for the zero-padded (aperiodic) convolution: 1 for a single
 * layer, else the next power of two >= 2n-1. */
long or_padded(long n)
{
    if (n <= 1)
        return 1;
    long p = 1;
    while (p < 2 * n - 1)
        p <<= 1;
    return p;
}

/* ------------------------------------------------------------------------- */
/* Problem context                                                            */
/* ------------------------------------------------------------------------- */

typedef struct or_ctx {
    long n[3];
    double d[3];
    long N;
    int p;
    double *Ms;      /* per cell, A/m; 0 marks a vacuum cell               */
    double *A;       /* per cell exchange constant, J/m                    */
    double Ku;       /* first-order uniaxial anisotropy constant, J/m^3    */
    double *Kuc;     /* per-cell first-order constant, or NULL (uniform Ku) */
    double eu[3];    /* easy axis (unit)                                   */
    double Ku2;      /* second-order uniaxial constant, J/m^3              */
    double Kc1, Kc2; /* first- and second-order cubic constants, J/m^3     */
    double ec[3][3]; /* cubic principal axes (orthonormal)                 */
    double *D;       /* per-cell DMI strength, J/m^2, or NULL               */
    double edmi[3][3]; /* DMI vectors e^dmi_x, e^dmi_y, e^dmi_z             */
    double alpha;
    double Hext[3];  /* uniform external field, A/m                        */
    /* sinusoidal drive: H += mask_i * amp * sin(2 pi f t) */
    double drive_amp[3];
    double drive_freq;
    unsigned char *drive_mask;
    int demag_direct;          /* 1: O(N^2) direct sum, 0: FFT            */
    /* FFT path */
    long P[3];
    long PN;
    double complex *Khat;      /* 6 x PN spectra of the padded kernel     */
    /* direct path: kernel per offset, (2nx-1)(2ny-1)(2nz-1) x 6            */
    double *Koff;
    /* thin layers of unequal height (or_set_layers): layer bottoms zb
     * (nz + 1 values) and the kernel per (component, t, s, I, J) */
    double *zb;
    double *Klay;
    /* Oersted field of the set current density (or_set_current), scaled by
     * sin(2 pi oe_freq t) when oe_freq != 0 */
    double *h_oe;
    double oe_freq;
    int terms;                 /* field-term mask used by heff            */
} or_ctx;

/* Height of layer k (d[2] without layers). */
static double layer_dz(const or_ctx *c, long k) { return c->zb ? c->zb[k + 1] - c->zb[k] : c->d[2]; }

/* Volume of the cells of layer k. */
static double layer_volume(const or_ctx *c, long k) { return c->d[0] * c->d[1] * layer_dz(c, k); }

static long cidx(const or_ctx *c, long i, long j, long k) { return i + c->n[0] * (j + c->n[1] * k); }

static void build_kernel(or_ctx *c)
{
    long nx = c->n[0], ny = c->n[1], nz = c->n[2];
    long ox = 2 * nx - 1, oy = 2 * ny - 1, oz = 2 * nz - 1;
    long noff = ox * oy * oz;
    double *Koff = malloc(sizeof(double) * 6 * noff);
#pragma omp parallel for schedule(dynamic, 16)
    for (long q = 0; q < noff; q++) {
        long oi = q % ox - (nx - 1);
        long oj = (q / ox) % oy - (ny - 1);
        long ok = q / (ox * oy) - (nz - 1);
        double e[6];
        or_tensor_entry(c->d, oi, oj, ok, c->p, e);
        for (int s = 0; s < 6; s++)
            Koff[s * noff + q] = e[s];
    }
    if (c->demag_direct) {
        c->Koff = Koff;
        return;
    }
    /* Place K(I,J,K) at (I mod Px, J mod Py, K mod Pz); all other entries are
     * zero.  Then transform each of the six components. */
    for (int a = 0; a < 3; a++)
        c->P[a] = or_padded(c->n[a]);
    c->PN = c->P[0] * c->P[1] * c->P[2];
    c->Khat = calloc(6 * c->PN, sizeof(double complex));
    for (long q = 0; q < noff; q++) {
        long oi = q % ox - (nx - 1);
        long oj = (q / ox) % oy - (ny - 1);
        long ok = q / (ox * oy) - (nz - 1);
        long pi = ((oi % c->P[0]) + c->P[0]) % c->P[0];
        long pj = ((oj % c->P[1]) + c->P[1]) % c->P[1];
        long pk = ((ok % c->P[2]) + c->P[2]) % c->P[2];
        long pidx = pi + c->P[0] * (pj + c->P[1] * pk);
        for (int s = 0; s < 6; s++)
            c->Khat[s * c->PN + pidx] = Koff[s * noff + q];
    }
    free(Koff);
    for (int s = 0; s < 6; s++)
        fft3d(c->P, c->Khat + s * c->PN, -1);
}

or_ctx *or_create(const long n[3], const double d[3], int p, const double *Ms, const double *A,
                  double Ku, const double eu[3], double alpha, int demag_direct)
{
    or_ctx *c = calloc(1, sizeof(or_ctx));
    for (int a = 0; a < 3; a++) {
        c->n[a] = n[a];
        c->d[a] = d[a];
        c->eu[a] = eu[a];
    }
    c->N = n[0] * n[1] * n[2];
    c->p = p;
    c->Ms = malloc(sizeof(double) * c->N);
    c->A = malloc(sizeof(double) * c->N);
    memcpy(c->Ms, Ms, sizeof(double) * c->N);
    memcpy(c->A, A, sizeof(double) * c->N);
    c->Ku = Ku;
    for (int i = 0; i < 3; i++)
        for (int a = 0; a < 3; a++)
            c->ec[i][a] = i == a ? 1.0 : 0.0;
    c->alpha = alpha;
    c->demag_direct = demag_direct;
    c->drive_mask = calloc(c->N, 1);
    c->terms = OR_DEMAG | OR_EXCH | OR_ANIS | OR_ZEEMAN | OR_DMI | OR_OERSTED;
    /* demag_direct 2: no demag kernel at all (local terms only, for grids
     * whose kernel the oracle cannot hold) */
    if (demag_direct != 2)
        build_kernel(c);
    return c;
}

/* Higher-order anisotropy (Sec. 4.3): second-order uniaxial Ku2 along the
 * easy axis of Ku, and cubic Kc1, Kc2 with principal axes c1, c2 and
 * c3 = c1 x c2 (c1, c2 orthonormalised here). */
void or_set_anisotropy2(or_ctx *c, double Ku2, double Kc1, double Kc2, const double c1[3],
                        const double c2[3])
{
    c->Ku2 = Ku2;
    c->Kc1 = Kc1;
    c->Kc2 = Kc2;
    double n1 = sqrt(c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
    for (int a = 0; a < 3; a++)
        c->ec[0][a] = c1[a] / n1;
    double dp = c2[0] * c->ec[0][0] + c2[1] * c->ec[0][1] + c2[2] * c->ec[0][2];
    double v[3], nv = 0.0;
    for (int a = 0; a < 3; a++) {
        v[a] = c2[a] - dp * c->ec[0][a];
        nv += v[a] * v[a];
    }
    nv = sqrt(nv);
    for (int a = 0; a < 3; a++)
        c->ec[1][a] = v[a] / nv;
    c->ec[2][0] = c->ec[0][1] * c->ec[1][2] - c->ec[0][2] * c->ec[1][1];
    c->ec[2][1] = c->ec[0][2] * c->ec[1][0] - c->ec[0][0] * c->ec[1][2];
    c->ec[2][2] = c->ec[0][0] * c->ec[1][1] - c->ec[0][1] * c->ec[1][0];
}

/* DMI (Sec. 4.3, Table of DMI types): per-cell strength D (NULL removes the
 * term) and the type's DMI vectors (e^dmi_x, e^dmi_y, e^dmi_z):
 * 0 interface (C_nv): (e_y, -e_x, 0); 1 bulk: (e_x, e_y, e_z);
 * 2 D_2d: (-e_x, e_y, 0). */
void or_set_dmi(or_ctx *c, const double *D, int type)
{
    free(c->D);
    c->D = NULL;
    memset(c->edmi, 0, sizeof(c->edmi));
    if (!D)
        return;
    c->D = malloc(sizeof(double) * c->N);
    memcpy(c->D, D, sizeof(double) * c->N);
    if (type == 0) {
        c->edmi[0][1] = 1.0;
        c->edmi[1][0] = -1.0;
    } else if (type == 1) {
        c->edmi[0][0] = c->edmi[1][1] = c->edmi[2][2] = 1.0;
    } else {
        c->edmi[0][0] = -1.0;
        c->edmi[1][1] = 1.0;
    }
}

/* Thin layers of unequal height dz[0..nz) stacked from z = 0 (Sec. 4.4, the
 * non-equidistant case): the demag field becomes the direct sum with the
 * layered kernel, the z exchange and DMI couplings use the layer heights, and
 * energies use each layer's cell volume.  dz = NULL restores equal layers. */
void or_set_layers(or_ctx *c, const double *dz)
{
    free(c->zb);
    free(c->Klay);
    c->zb = NULL;
    c->Klay = NULL;
    if (!dz)
        return;
    long nx = c->n[0], ny = c->n[1], nz = c->n[2];
    c->zb = malloc(sizeof(double) * (nz + 1));
    c->zb[0] = 0.0;
    for (long k = 0; k < nz; k++)
        c->zb[k + 1] = c->zb[k] + dz[k];
    long ox = 2 * nx - 1, oy = 2 * ny - 1, nl = ox * oy;
    long total = nz * nz * nl;
    c->Klay = malloc(sizeof(double) * 6 * total);
#pragma omp parallel for schedule(dynamic, 16)
    for (long q = 0; q < total; q++) {
        long l = q % nl, ts = q / nl;
        long t = ts / nz, s = ts % nz;
        long oi = l % ox - (nx - 1), oj = l / ox - (ny - 1);
        double e[6];
        or_layer_entry(c->d[0], c->d[1], c->zb, t, s, oi, oj, c->p, e);
        for (int a = 0; a < 6; a++)
            c->Klay[a * total + q] = e[a];
    }
}

/* Oersted field at selected target cells by direct summation over every
 * source cell (no table of all offsets), for grids too large for or_oersted:
 * near-field entries (Chebyshev index distance <= p) are tabulated once, the
 * rest are the singular current.  j is [3][N]; out receives 3 values per
 * target.  Returns -1 for p < 0. */
int or_oersted_at(const long n[3], const double d[3], int p, const double *j, long ncell,
                  const long *cells, double *out)
{
    if (p < 0)
        return -1;
    long nx = n[0], ny = n[1], nz = n[2], N = nx * ny * nz;
    long rx = p < nx - 1 ? p : nx - 1, ry = p < ny - 1 ? p : ny - 1, rz = p < nz - 1 ? p : nz - 1;
    long tx = 2 * rx + 1, ty = 2 * ry + 1, tz = 2 * rz + 1, nt = tx * ty * tz;
    double *T = malloc(sizeof(double) * 3 * nt);
#pragma omp parallel for schedule(dynamic, 64)
    for (long q = 0; q < nt; q++)
        or_oersted_entry(d, q % tx - rx, (q / tx) % ty - ry, q / (tx * ty) - rz, p, T + 3 * q);
    for (long c = 0; c < ncell; c++) {
        long t = cells[c];
        long i = t % nx, jj = (t / nx) % ny, k = t / (nx * ny);
        long double hx = 0.0L, hy = 0.0L, hz = 0.0L;
#pragma omp parallel for reduction(+ : hx, hy, hz) schedule(static)
        for (long src = 0; src < N; src++) {
            long oi = i - src % nx, oj = jj - (src / nx) % ny, ok = k - src / (nx * ny);
            double g[3];
            if (labs(oi) <= rx && labs(oj) <= ry && labs(ok) <= rz) {
                const double *te = T + 3 * ((oi + rx) + tx * ((oj + ry) + ty * (ok + rz)));
                g[0] = te[0];
                g[1] = te[1];
                g[2] = te[2];
            } else {
                or_oersted_entry(d, oi, oj, ok, p, g);
            }
            double jx = j[src], jy = j[N + src], jz = j[2 * N + src];
            hx += jy * g[2] - jz * g[1];
            hy += jz * g[0] - jx * g[2];
            hz += jx * g[1] - jy * g[0];
        }
        out[3 * c] = (double)hx;
        out[3 * c + 1] = (double)hy;
        out[3 * c + 2] = (double)hz;
    }
    free(T);
    return 0;
}

/* Layered demag field at selected target cells by direct summation (layer
 * heights dz[0..nz) stacked from 0): near-field entries (Chebyshev index
 * distance <= p in (i, j, layer)) tabulated per layer pair, dipoles beyond.
 * Ms per cell or NULL for Ms0.  Returns -1 for p < 0. */
int or_layer_demag_at(const long n[3], const double d[3], const double *dz, int p,
                      const double *Ms, double Ms0, const double *m, long ncell, const long *cells,
                      double *out)
{
    if (p < 0)
        return -1;
    long nx = n[0], ny = n[1], nz = n[2], N = nx * ny * nz;
    double *zb = malloc(sizeof(double) * (nz + 1));
    zb[0] = 0.0;
    for (long k = 0; k < nz; k++)
        zb[k + 1] = zb[k] + dz[k];
    long rx = p < nx - 1 ? p : nx - 1, ry = p < ny - 1 ? p : ny - 1;
    long tx = 2 * rx + 1, ty = 2 * ry + 1, nl = tx * ty, nt = nl * nz * nz;
    double *T = malloc(sizeof(double) * 6 * nt);
#pragma omp parallel for schedule(dynamic, 64)
    for (long q = 0; q < nt; q++) {
        long l = q % nl, ts = q / nl;
        or_layer_entry(d[0], d[1], zb, ts / nz, ts % nz, l % tx - rx, l / tx - ry, p, T + 6 * q);
    }
    for (long c = 0; c < ncell; c++) {
        long t = cells[c];
        long i = t % nx, jj = (t / nx) % ny, k = t / (nx * ny);
        long double hx = 0.0L, hy = 0.0L, hz = 0.0L;
#pragma omp parallel for reduction(+ : hx, hy, hz) schedule(static)
        for (long src = 0; src < N; src++) {
            long sk = src / (nx * ny);
            long oi = i - src % nx, oj = jj - (src / nx) % ny;
            double e[6];
            if (labs(oi) <= rx && labs(oj) <= ry) {
                const double *te = T + 6 * (((k * nz + sk) * nl) + (oi + rx) + tx * (oj + ry));
                for (int a = 0; a < 6; a++)
                    e[a] = te[a];
            } else {
                or_layer_entry(d[0], d[1], zb, k, sk, oi, oj, p, e);
            }
            double ms = Ms ? Ms[src] : Ms0;
            double Mx = ms * m[src], My = ms * m[N + src], Mz = ms * m[2 * N + src];
            hx += e[0] * Mx + e[3] * My + e[4] * Mz;
            hy += e[3] * Mx + e[1] * My + e[5] * Mz;
            hz += e[4] * Mx + e[5] * My + e[2] * Mz;
        }
        out[3 * c] = (double)hx;
        out[3 * c + 1] = (double)hy;
        out[3 * c + 2] = (double)hz;
    }
    free(T);
    free(zb);
    return 0;
}

/* Oersted field h = sum_s j_s x G(X_t - X_s) of a current density j ([3][N],
 * A/m^2) by direct summation over every source cell (Sec. 4.5), at every
 * cell.  Equal cells only (returns -1 with layers). */
int or_oersted(const or_ctx *c, const double *j, double *h)
{
    if (c->zb)
        return -1;
    long N = c->N, nx = c->n[0], ny = c->n[1], nz = c->n[2];
    long ox = 2 * nx - 1, oy = 2 * ny - 1, oz = 2 * nz - 1, noff = ox * oy * oz;
    double *G = malloc(sizeof(double) * 3 * noff);
#pragma omp parallel for schedule(dynamic, 16)
    for (long q = 0; q < noff; q++) {
        double e[3];
        or_oersted_entry(c->d, q % ox - (nx - 1), (q / ox) % oy - (ny - 1), q / (ox * oy) - (nz - 1),
                         c->p, e);
        for (int l = 0; l < 3; l++)
            G[l * noff + q] = e[l];
    }
#pragma omp parallel for schedule(static)
    for (long t = 0; t < N; t++) {
        long i = t % nx, jj = (t / nx) % ny, k = t / (nx * ny);
        double hx = 0, hy = 0, hz = 0;
        for (long s = 0; s < N; s++) {
            long si = s % nx, sj = (s / nx) % ny, sk = s / (nx * ny);
            long q = (i - si + nx - 1) + ox * ((jj - sj + ny - 1) + oy * (k - sk + nz - 1));
            double gx = G[q], gy = G[noff + q], gz = G[2 * noff + q];
            double jx = j[s], jy = j[N + s], jz = j[2 * N + s];
            hx += jy * gz - jz * gy;
            hy += jz * gx - jx * gz;
            hz += jx * gy - jy * gx;
        }
        h[t] = hx;
        h[N + t] = hy;
        h[2 * N + t] = hz;
    }
    (void)oz;
    free(G);
    return 0;
}

/* Current density for the Oersted term (OR_OERSTED): its field is computed
 * once and added, times sin(2 pi freq t) if freq != 0, on magnetic cells.
 * j = NULL removes it. */
int or_set_current(or_ctx *c, const double *j, double freq)
{
    free(c->h_oe);
    c->h_oe = NULL;
    c->oe_freq = 0.0;
    if (!j)
        return 0;
    c->h_oe = malloc(sizeof(double) * 3 * c->N);
    c->oe_freq = freq;
    if (or_oersted(c, j, c->h_oe) != 0) {
        free(c->h_oe);
        c->h_oe = NULL;
        return -1;
    }
    return 0;
}

/* Per-cell first-order uniaxial anisotropy constant (J/m^3, N values along
 * the common easy axis); NULL restores the uniform Ku.  The material of
 * Sec. 2 may vary per cell for every parameter. */
void or_set_ku(or_ctx *c, const double *Ku)
{
    free(c->Kuc);
    c->Kuc = NULL;
    if (!Ku)
        return;
    c->Kuc = malloc(sizeof(double) * c->N);
    memcpy(c->Kuc, Ku, sizeof(double) * c->N);
}

void or_destroy(or_ctx *c)
{
    if (!c)
        return;
    free(c->Kuc);
    free(c->h_oe);
    free(c->zb);
    free(c->Klay);
    free(c->D);
    free(c->Ms);
    free(c->A);
    free(c->drive_mask);
    free(c->Khat);
    free(c->Koff);
    free(c);
}

void or_set_field(or_ctx *c, const double H[3], unsigned terms)
{
    for (int a = 0; a < 3; a++)
        c->Hext[a] = H[a];
    c->terms = (int)terms;
}

void or_set_drive(or_ctx *c, const double amp[3], double freq, const unsigned char *mask)
{
    for (int a = 0; a < 3; a++)
        c->drive_amp[a] = amp[a];
    c->drive_freq = freq;
    memcpy(c->drive_mask, mask, c->N);
}

/* Replace the per-cell saturation magnetisation (the kernel is unchanged). */
void or_set_Ms(or_ctx *c, const double *Ms) { memcpy(c->Ms, Ms, sizeof(double) * c->N); }

/* ------------------------------------------------------------------------- */
/* Field terms (Sec. 4).  m and h are [3][N] arrays, x fastest.               */
/* ------------------------------------------------------------------------- */

/* Demagnetisation field, h_i = sum_j K_{i-j} Ms_j m_j (Sec. 4.4). */
void or_demag(const or_ctx *c, const double *m, double *h)
{
    long N = c->N, nx = c->n[0], ny = c->n[1], nz = c->n[2];
    if (c->demag_direct == 2 && !c->zb) {
        /* created without a demag kernel: a loud NaN field */
        for (long q = 0; q < 3 * N; q++)
            h[q] = NAN;
        return;
    }
    if (c->zb) {
        /* layers: h_t(i, j) = sum_s sum K^{ts}(i - i', j - j') Ms m (direct) */
        long ox = 2 * nx - 1, oy = 2 * ny - 1, nl = ox * oy, total = nz * nz * nl;
        const double *K = c->Klay;
#pragma omp parallel for schedule(static)
        for (long t = 0; t < N; t++) {
            long i = t % nx, j = (t / nx) % ny, k = t / (nx * ny);
            double hx = 0, hy = 0, hz = 0;
            for (long s = 0; s < N; s++) {
                long si = s % nx, sj = (s / nx) % ny, sk = s / (nx * ny);
                long q = (k * nz + sk) * nl + (i - si + nx - 1) + ox * (j - sj + ny - 1);
                double Mx = c->Ms[s] * m[s], My = c->Ms[s] * m[N + s], Mz = c->Ms[s] * m[2 * N + s];
                double kxx = K[q], kyy = K[total + q], kzz = K[2 * total + q];
                double kxy = K[3 * total + q], kxz = K[4 * total + q], kyz = K[5 * total + q];
                hx += kxx * Mx + kxy * My + kxz * Mz;
                hy += kxy * Mx + kyy * My + kyz * Mz;
                hz += kxz * Mx + kyz * My + kzz * Mz;
            }
            h[t] = hx;
            h[N + t] = hy;
            h[2 * N + t] = hz;
        }
        return;
    }
    if (c->demag_direct) {
        long ox = 2 * nx - 1, oy = 2 * ny - 1, oz = 2 * nz - 1, noff = ox * oy * oz;
        const double *K = c->Koff;
#pragma omp parallel for schedule(static)
        for (long t = 0; t < N; t++) {
            long i = t % nx, j = (t / nx) % ny, k = t / (nx * ny);
            double hx = 0, hy = 0, hz = 0;
            for (long s = 0; s < N; s++) {
                long si = s % nx, sj = (s / nx) % ny, sk = s / (nx * ny);
                long q = (i - si + nx - 1) + ox * ((j - sj + ny - 1) + oy * (k - sk + nz - 1));
                double Mx = c->Ms[s] * m[s], My = c->Ms[s] * m[N + s], Mz = c->Ms[s] * m[2 * N + s];
                double kxx = K[q], kyy = K[noff + q], kzz = K[2 * noff + q];
                double kxy = K[3 * noff + q], kxz = K[4 * noff + q], kyz = K[5 * noff + q];
                hx += kxx * Mx + kxy * My + kxz * Mz;
                hy += kxy * Mx + kyy * My + kyz * Mz;
                hz += kxz * Mx + kyz * My + kzz * Mz;
            }
            h[t] = hx;
            h[N + t] = hy;
            h[2 * N + t] = hz;
        }
        (void)oz;
        return;
    }
    long PN = c->PN;
    double complex *Mh = calloc(3 * PN, sizeof(double complex));
    for (long k = 0; k < nz; k++)
        for (long j = 0; j < ny; j++)
            for (long i = 0; i < nx; i++) {
                long t = cidx(c, i, j, k);
                long pidx = i + c->P[0] * (j + c->P[1] * k);
                for (int a = 0; a < 3; a++)
                    Mh[a * PN + pidx] = c->Ms[t] * m[a * N + t];
            }
    for (int a = 0; a < 3; a++)
        fft3d(c->P, Mh + a * PN, -1);
    /* full symmetric 3x3 product per frequency: index of K_ab in the six */
    static const int comp[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma omp parallel for schedule(static)
    for (long q = 0; q < PN; q++) {
        double complex M0 = Mh[q], M1 = Mh[PN + q], M2 = Mh[2 * PN + q];
        double complex H[3];
        for (int a = 0; a < 3; a++)
            H[a] = c->Khat[comp[a][0] * PN + q] * M0 + c->Khat[comp[a][1] * PN + q] * M1 +
                   c->Khat[comp[a][2] * PN + q] * M2;
        for (int a = 0; a < 3; a++)
            Mh[a * PN + q] = H[a];
    }
    for (int a = 0; a < 3; a++)
        fft3d(c->P, Mh + a * PN, +1);
    double scale = 1.0 / (double)PN;
    for (long k = 0; k < nz; k++)
        for (long j = 0; j < ny; j++)
            for (long i = 0; i < nx; i++) {
                long t = cidx(c, i, j, k);
                long pidx = i + c->P[0] * (j + c->P[1] * k);
                for (int a = 0; a < 3; a++)
                    h[a * N + t] = creal(Mh[a * PN + pidx]) * scale;
            }
    free(Mh);
}

/* Exchange field with the harmonic mean of A between neighbours (Sec. 4.2,
 * the discrete form for spatially varying A).  A is taken as zero outside the
 * grid, which gives dm/dn = 0.  A harmonic mean with A_i + A_j = 0 is 0.
 * Cells with Ms = 0 get h = 0. */
void or_exchange(const or_ctx *c, const double *m, double *h)
{
    long N = c->N;
    long nx = c->n[0], ny = c->n[1], nz = c->n[2];
#pragma omp parallel for schedule(static)
    for (long t = 0; t < N; t++) {
        long i = t % nx, j = (t / nx) % ny, k = t / (nx * ny);
        double acc[3] = {0, 0, 0};
        if (c->Ms[t] != 0.0) {
            long nb[6][3] = {{i + 1, j, k}, {i - 1, j, k}, {i, j + 1, k},
                             {i, j - 1, k}, {i, j, k + 1}, {i, j, k - 1}};
            for (int q = 0; q < 6; q++) {
                long a = nb[q][0], b = nb[q][1], e = nb[q][2];
                if (a < 0 || a >= nx || b < 0 || b >= ny || e < 0 || e >= nz)
                    continue; /* A = 0 outside: the harmonic mean vanishes */
                long s = cidx(c, a, b, e);
                double Ai = c->A[t], As = c->A[s];
                double hm = (Ai + As) != 0.0 ? Ai * As / (Ai + As) : 0.0;
                double dk = c->d[q / 2];
                double w = 2.0 / (dk * dk) * hm;
                if (q / 2 == 2 && c->zb) {
                    /* layers: the flux between the centres, per height of
                     * this cell: 2 / (dz_k (dz_k + dz_e)) in place of 1/dz^2 */
                    double hk = layer_dz(c, k), he = layer_dz(c, e);
                    w = 2.0 * hm * 2.0 / (hk * (hk + he));
                }
                for (int comp = 0; comp < 3; comp++)
                    acc[comp] += w * (m[comp * N + s] - m[comp * N + t]);
            }
            for (int comp = 0; comp < 3; comp++)
                acc[comp] *= 2.0 / (OR_MU0 * c->Ms[t]);
        }
        for (int comp = 0; comp < 3; comp++)
            h[comp * N + t] = acc[comp];
    }
}

/* First-order uniaxial anisotropy field, h = 2 Ku/(mu0 Ms) e (e.m)
 * (Sec. 4.1); zero where Ms = 0 (the listing's nan_to_num). */
void or_anisotropy(const or_ctx *c, const double *m, double *h)
{
    long N = c->N;
    for (long t = 0; t < N; t++) {
        if (c->Ms[t] == 0.0) {
            h[t] = h[N + t] = h[2 * N + t] = 0.0;
            continue;
        }
        double M[3] = {m[t], m[N + t], m[2 * N + t]};
        double em = c->eu[0] * M[0] + c->eu[1] * M[1] + c->eu[2] * M[2];
        /* uniaxial: (2 Ku1 em + 4 Ku2 em^3) e / (mu0 Ms) */
        double ku = c->Kuc ? c->Kuc[t] : c->Ku;
        double pu = (2.0 * ku * em + 4.0 * c->Ku2 * em * em * em) / (OR_MU0 * c->Ms[t]);
        /* cubic, in the principal axes: -2 Kc1 m_i (m_j^2 + m_k^2) - 2 Kc2 m_i m_j^2 m_k^2,
         * over mu0 Ms, mapped back along c_i */
        double p[3];
        for (int i = 0; i < 3; i++)
            p[i] = c->ec[i][0] * M[0] + c->ec[i][1] * M[1] + c->ec[i][2] * M[2];
        double hc[3];
        for (int i = 0; i < 3; i++) {
            double pj = p[(i + 1) % 3], pk = p[(i + 2) % 3];
            hc[i] = -(2.0 * c->Kc1 * p[i] * (pj * pj + pk * pk) +
                      2.0 * c->Kc2 * p[i] * pj * pj * pk * pk) /
                    (OR_MU0 * c->Ms[t]);
        }
        for (int a = 0; a < 3; a++)
            h[a * N + t] = pu * c->eu[a] + hc[0] * c->ec[0][a] + hc[1] * c->ec[1][a] +
                           hc[2] * c->ec[2][a];
    }
}

/* Anisotropy energy from its density (the linear-term formula of Sec. 4 does
 * not apply to the higher orders):
 * V sum_i [-Ku1 (e.m)^2 - Ku2 (e.m)^4 + Kc1 (m1^2 m2^2 + m2^2 m3^2 + m3^2 m1^2)
 *          + Kc2 m1^2 m2^2 m3^2] over magnetic cells. */
static double anisotropy_energy(const or_ctx *c, const double *m)
{
    long N = c->N;
    long double acc = 0.0L;
    for (long t = 0; t < N; t++) {
        if (c->Ms[t] == 0.0)
            continue;
        double M[3] = {m[t], m[N + t], m[2 * N + t]};
        double em = c->eu[0] * M[0] + c->eu[1] * M[1] + c->eu[2] * M[2];
        double p[3];
        for (int i = 0; i < 3; i++)
            p[i] = c->ec[i][0] * M[0] + c->ec[i][1] * M[1] + c->ec[i][2] * M[2];
        double q1 = p[0] * p[0], q2 = p[1] * p[1], q3 = p[2] * p[2];
        acc += (long double)layer_volume(c, t / (c->n[0] * c->n[1])) *
               (-(c->Kuc ? c->Kuc[t] : c->Ku) * em * em - c->Ku2 * em * em * em * em +
                c->Kc1 * (q1 * q2 + q2 * q3 + q3 * q1) + c->Kc2 * q1 * q2 * q3);
    }
    return (double)acc;
}

/* Effective DMI coupling between two cells (Eq. D_avg).  Pinned for equal
 * signs (the uniform limit and a two-cell value follow from the stencil
 * closed forms); the opposite-sign branch is parity unpinned.  The harmonic mean
 * 2 Da Db / (Da + Db) for equal signs (the printed denominator Da Db is read
 * as Da + Db; 0 when both vanish), otherwise sign(Da Db) times the geometric
 * mean of the geometric mean sqrt(-Da Db) and the mean |Da + Db| / 2. */
static double dmi_avg(double a, double b)
{
    if (a * b >= 0.0)
        return (a + b) != 0.0 ? 2.0 * a * b / (a + b) : 0.0;
    return -sqrt(sqrt(-a * b) * fabs(a + b) / 2.0);
}

/* DMI field by central differences (Sec. 4.3).  Pinned by the spiral and
 * helix closed forms of each tabulated type, the Ms-weighted symmetry of the
 * operator and dE/dm = -mu0 V Ms h (tests/test_oracle_dmi.py):
 * h_i = 2/(mu0 Ms_i) sum_{k = +-x, +-y, +-z} D~_{i,k} (e^dmi_k x m_{i+e_k}) / (2 Delta_k),
 * e^dmi_{-k} = -e^dmi_k; neighbours outside the grid or in vacuum are
 * ignored (the open boundary of Sec. 4.3).  Vacuum cells: h = 0. */
void or_dmi(const or_ctx *c, const double *m, double *h)
{
    long N = c->N, nx = c->n[0], ny = c->n[1], nz = c->n[2];
    memset(h, 0, sizeof(double) * 3 * N);
    if (!c->D)
        return;
    for (long t = 0; t < N; t++) {
        if (c->Ms[t] == 0.0)
            continue;
        long i = t % nx, j = (t / nx) % ny, k = t / (nx * ny);
        double acc[3] = {0, 0, 0};
        for (int q = 0; q < 6; q++) {
            int ax = q / 2;
            long sgn = (q % 2 == 0) ? 1 : -1;
            long a = i + (ax == 0 ? sgn : 0), b = j + (ax == 1 ? sgn : 0), e = k + (ax == 2 ? sgn : 0);
            if (a < 0 || a >= nx || b < 0 || b >= ny || e < 0 || e >= nz)
                continue;
            long s = cidx(c, a, b, e);
            if (c->Ms[s] == 0.0)
                continue;
            double Dt = dmi_avg(c->D[t], c->D[s]);
            double ev[3] = {sgn * c->edmi[ax][0], sgn * c->edmi[ax][1], sgn * c->edmi[ax][2]};
            double ms[3] = {m[s], m[N + s], m[2 * N + s]};
            double cr[3] = {ev[1] * ms[2] - ev[2] * ms[1], ev[2] * ms[0] - ev[0] * ms[2],
                            ev[0] * ms[1] - ev[1] * ms[0]};
            /* layers: the height of this cell's layer in place of dz (the
             * finite-volume form: face values averaged, divided by the
             * cell height, which keeps the operator Ms V-weighted symmetric) */
            double two_delta = 2.0 * (ax == 2 ? layer_dz(c, k) : c->d[ax]);
            for (int comp = 0; comp < 3; comp++)
                acc[comp] += Dt / two_delta * cr[comp];
        }
        for (int comp = 0; comp < 3; comp++)
            h[comp * N + t] = 2.0 / (OR_MU0 * c->Ms[t]) * acc[comp];
    }
}

/* Zeeman field at time t: uniform Hext plus the masked sinusoidal drive. */
void or_zeeman(const or_ctx *c, double t, double *h)
{
    long N = c->N;
    double s = c->drive_freq != 0.0 ? sin(2.0 * M_PI * c->drive_freq * t) : 0.0;
    for (long q = 0; q < N; q++)
        for (int a = 0; a < 3; a++)
            h[a * N + q] = c->Ms[q] != 0.0 ? c->Hext[a] + (c->drive_mask[q] ? c->drive_amp[a] * s : 0.0) : 0.0;
}

/* Effective field: sum of the terms selected by mask (bit 0 demag, 1 exchange,
 * 2 anisotropy, 3 Zeeman).  Vacuum cells get h = 0. */
void or_heff(const or_ctx *c, const double *m, double t, unsigned mask, double *h)
{
    long N = c->N;
    double *tmp = malloc(sizeof(double) * 3 * N);
    memset(h, 0, sizeof(double) * 3 * N);
    if (mask & OR_DEMAG) {
        or_demag(c, m, tmp);
        for (long q = 0; q < 3 * N; q++)
            h[q] += c->Ms[q % N] != 0.0 ? tmp[q] : 0.0;
    }
    if (mask & OR_EXCH) {
        or_exchange(c, m, tmp);
        for (long q = 0; q < 3 * N; q++)
            h[q] += tmp[q];
    }
    if (mask & OR_ANIS) {
        or_anisotropy(c, m, tmp);
        for (long q = 0; q < 3 * N; q++)
            h[q] += tmp[q];
    }
    if (mask & OR_ZEEMAN) {
        or_zeeman(c, t, tmp);
        for (long q = 0; q < 3 * N; q++)
            h[q] += tmp[q];
    }
    if ((mask & OR_DMI) && c->D) {
        or_dmi(c, m, tmp);
        for (long q = 0; q < 3 * N; q++)
            h[q] += tmp[q];
    }
    if ((mask & OR_OERSTED) && c->h_oe) {
        double s = c->oe_freq != 0.0 ? sin(2.0 * M_PI * c->oe_freq * t) : 1.0;
        for (long q = 0; q < 3 * N; q++)
            h[q] += c->Ms[q % N] != 0.0 ? s * c->h_oe[q] : 0.0;
    }
    free(tmp);
}

/* ------------------------------------------------------------------------- */
/* LLG right-hand side (Sec. 3, Eq. llg):                                     */
/*   dm/dt = -gamma/(1+alpha^2) [ m x h + alpha m x (m x h) ]                 */
/* precess = 0 drops the m x h term (relaxation).  Vacuum cells: dm = 0.      */
/* ------------------------------------------------------------------------- */

void or_llg_rhs(const or_ctx *c, const double *m, const double *h, double alpha, int precess,
                double *dm)
{
    long N = c->N;
    double g = OR_GAMMA / (1.0 + alpha * alpha);
    for (long q = 0; q < N; q++) {
        if (c->Ms[q] == 0.0) {
            dm[q] = dm[N + q] = dm[2 * N + q] = 0.0;
            continue;
        }
        double mx = m[q], my = m[N + q], mz = m[2 * N + q];
        double hx = h[q], hy = h[N + q], hz = h[2 * N + q];
        double px = my * hz - mz * hy, py = mz * hx - mx * hz, pz = mx * hy - my * hx; /* m x h */
        double dx = my * pz - mz * py, dy = mz * px - mx * pz, dz = mx * py - my * px;  /* m x (m x h) */
        double pf = precess ? 1.0 : 0.0;
        dm[q] = -g * (pf * px + alpha * dx);
        dm[N + q] = -g * (pf * py + alpha * dy);
        dm[2 * N + q] = -g * (pf * pz + alpha * dz);
    }
}

static void rhs_at(const or_ctx *c, const double *m, double t, double alpha, int precess,
                   double *h, double *dm)
{
    or_heff(c, m, t, (unsigned)c->terms, h);
    or_llg_rhs(c, m, h, alpha, precess, dm);
}

/* ------------------------------------------------------------------------- */
/* Energies (Sec. 4, Eqs. linear_energy / linear_energy_discrete).            */
/* E_t = -1/2 mu0 V sum Ms m.h_t for the linear terms (demag, exchange,       */
/* anisotropy); Zeeman E = -mu0 V sum Ms m.H.  E[4] is the total.             */
/* Accumulated in long double.                                               */
/* ------------------------------------------------------------------------- */

void or_energy(const or_ctx *c, const double *m, double t, double E[6])
{
    long N = c->N, nxy = c->n[0] * c->n[1];
    double *h = malloc(sizeof(double) * 3 * N);
    /* slots: 0 demag, 1 exchange, 2 anisotropy, 3 Zeeman, 5 DMI; 4 total */
    /* the Oersted field is an applied field: its energy joins the Zeeman slot */
    unsigned masks[6] = {OR_DEMAG, OR_EXCH, OR_ANIS, OR_ZEEMAN | OR_OERSTED, 0, OR_DMI};
    double tot = 0;
    for (int e = 0; e < 6; e++) {
        if (e == 4)
            continue;
        long double acc = 0.0L;
        if (e == 2) {
            E[e] = (c->terms & (int)masks[e]) ? anisotropy_energy(c, m) : 0.0;
            tot += E[e];
            continue;
        }
        if (c->terms & (int)masks[e]) {
            or_heff(c, m, t, masks[e] & (unsigned)c->terms, h);
            for (long q = 0; q < N; q++)
                acc += (long double)layer_volume(c, q / nxy) * c->Ms[q] *
                       ((long double)m[q] * h[q] + (long double)m[N + q] * h[N + q] +
                        (long double)m[2 * N + q] * h[2 * N + q]);
        }
        double pre = (e == 3 ? -1.0 : -0.5) * OR_MU0;
        E[e] = (double)(pre * acc);
        tot += E[e];
    }
    E[4] = tot;
    free(h);
}

/* ------------------------------------------------------------------------- */
/* Dormand-Prince 5(4) with first-same-as-last (Dormand & Prince, 1980).      */
/* The paper's default is Fehlberg's RK45 (Sec. 3); this hot path uses the    */
/* Dormand-Prince pair.  Controller reading: Hairer RMS norm over magnetic    */
/* components with sc = atol + rtol*max(|y|,|y1|); accept iff err <= 1;       */
/* dt *= min(facmax, max(0.2, 0.9 err^-1/5)), facmax = 10 (1 after a reject). */
/* ------------------------------------------------------------------------- */

static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
/* 5th-order weights (= last row of A) and the embedded 4th-order weights. */
static const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                               -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double DP_BS[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

/* Runge-Kutta-Fehlberg 4(5) (Fehlberg 1969), the paper's default (Sec. 3):
 * six stages, the 4th-order solution is propagated and the difference to the
 * 5th-order one is the error estimate; no first-same-as-last stage. */
static const double RKF_C[6] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
static const double RKF_A[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 4.0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
static const double RKF_B4[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0};
static const double RKF_B5[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0,
                                 -9.0 / 50.0, 2.0 / 55.0};

/* An embedded explicit pair: stages, nodes c, coefficients a (row s uses
 * a[s][0..s-1]), propagated weights b, error weights e (b minus the other
 * solution's weights); fsal: the last stage is evaluated at the propagated
 * solution, so it is the next step's first stage. */
typedef struct {
    int stages, fsal;
    double c[7], a[7][6], b[7], e[7];
} or_tableau;

static void tableau(int method, or_tableau *T)
{
    memset(T, 0, sizeof(*T));
    if (method == 1) {
        T->stages = 6;
        T->fsal = 0;
        for (int s = 0; s < 6; s++) {
            T->c[s] = RKF_C[s];
            for (int j = 0; j < 5; j++)
                T->a[s][j] = RKF_A[s][j];
            T->b[s] = RKF_B4[s];
            T->e[s] = RKF_B4[s] - RKF_B5[s];
        }
    } else {
        T->stages = 7;
        T->fsal = 1;
        for (int s = 0; s < 7; s++) {
            T->c[s] = DP_C[s];
            for (int j = 0; j < 6; j++)
                T->a[s][j] = DP_A[s][j];
            T->b[s] = DP_B[s];
            T->e[s] = DP_B[s] - DP_BS[s];
        }
    }
}

enum { OR_OK = 0, OR_EDTMIN = -5, OR_ENOTCONV = -6, OR_ENONFINITE = -4 };

typedef struct {
    long accepted, rejected, rhs_evals;
    double t, dt, err_last;
} or_stats;

static double err_norm(const or_ctx *c, const double *y, const double *y1, const double *e,
                       double rtol, double atol)
{
    long N = c->N;
    long double acc = 0.0L;
    long cnt = 0;
    for (long q = 0; q < N; q++) {
        if (c->Ms[q] == 0.0)
            continue;
        for (int a = 0; a < 3; a++) {
            double ya = fabs(y[a * N + q]), yb = fabs(y1[a * N + q]);
            double sc = atol + rtol * (ya > yb ? ya : yb);
            long double r = e[a * N + q] / sc;
            acc += r * r;
            cnt++;
        }
    }
    if (cnt == 0)
        return 0.0;
    return sqrt((double)(acc / cnt));
}

static void renormalise(const or_ctx *c, double *m)
{
    long N = c->N;
    for (long q = 0; q < N; q++) {
        if (c->Ms[q] == 0.0) {
            m[q] = m[N + q] = m[2 * N + q] = 0.0;
            continue;
        }
        double nrm = sqrt(m[q] * m[q] + m[N + q] * m[N + q] + m[2 * N + q] * m[2 * N + q]);
        for (int a = 0; a < 3; a++)
            m[a * N + q] /= nrm;
    }
}

/* Hairer-Norsett-Wanner starting step size (Solving ODEs I, Sec. II.4). */
static double initial_dt(const or_ctx *c, const double *y, const double *f0, double t, double alpha,
                         int precess, double rtol, double atol, long *evals)
{
    long N = c->N, n3 = 3 * N;
    double *y1 = malloc(sizeof(double) * n3), *f1 = malloc(sizeof(double) * n3);
    double *h = malloc(sizeof(double) * n3);
    long double s0 = 0, s1 = 0;
    long cnt = 0;
    for (long q = 0; q < N; q++) {
        if (c->Ms[q] == 0.0)
            continue;
        for (int a = 0; a < 3; a++) {
            double sc = atol + rtol * fabs(y[a * N + q]);
            s0 += (long double)(y[a * N + q] / sc) * (y[a * N + q] / sc);
            s1 += (long double)(f0[a * N + q] / sc) * (f0[a * N + q] / sc);
            cnt++;
        }
    }
    double d0 = cnt ? sqrt((double)(s0 / cnt)) : 0.0, d1 = cnt ? sqrt((double)(s1 / cnt)) : 0.0;
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    for (long q = 0; q < n3; q++)
        y1[q] = y[q] + h0 * f0[q];
    rhs_at(c, y1, t + h0, alpha, precess, h, f1);
    (*evals)++;
    long double s2 = 0;
    for (long q = 0; q < N; q++) {
        if (c->Ms[q] == 0.0)
            continue;
        for (int a = 0; a < 3; a++) {
            double sc = atol + rtol * fabs(y[a * N + q]);
            double r = (f1[a * N + q] - f0[a * N + q]) / sc;
            s2 += (long double)r * r;
        }
    }
    double d2 = (cnt ? sqrt((double)(s2 / cnt)) : 0.0) / h0;
    double mx = d1 > d2 ? d1 : d2;
    double h1 = mx <= 1e-15 ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / mx, 1.0 / 5.0);
    free(y1);
    free(f1);
    free(h);
    return fmin(100.0 * h0, h1);
}

/* Integrate the LLG from *t until t_end or until max_steps steps have been
 * accepted.  m is updated in place.  renorm != 0 renormalises m after each
 * accepted step (then FSAL cannot be used and k1 is re-evaluated).
 * fixed != 0 disables error control (every step accepted, dt constant): used
 * by the order test only.  *dt <= 0 asks for the automatic initial step. */
int or_rk_adaptive(or_ctx *c, int method, double *m, double *t, double *dt, double rtol,
                   double atol, double t_end, long max_steps, int renorm, int precess, double alpha,
                   int fixed, or_stats *st, double torque_tol);

int or_dp45(or_ctx *c, double *m, double *t, double *dt, double rtol, double atol, double t_end,
            long max_steps, int renorm, int precess, double alpha, int fixed, or_stats *st,
            double torque_tol)
{
    return or_rk_adaptive(c, 0, m, t, dt, rtol, atol, t_end, max_steps, renorm, precess, alpha,
                          fixed, st, torque_tol);
}

/* The same integration with the pair chosen by method: 0 Dormand-Prince 5(4),
 * 1 Runge-Kutta-Fehlberg 4(5).  Same controller for both. */
int or_rk_adaptive(or_ctx *c, int method, double *m, double *t, double *dt, double rtol,
                   double atol, double t_end, long max_steps, int renorm, int precess, double alpha,
                   int fixed, or_stats *st, double torque_tol)
{
    or_tableau T;
    tableau(method, &T);
    const int S = T.stages;
    long N = c->N, n3 = 3 * N;
    double *k[7];
    for (int s = 0; s < 7; s++)
        k[s] = malloc(sizeof(double) * n3);
    double *y = malloc(sizeof(double) * n3), *ys = malloc(sizeof(double) * n3);
    double *h = malloc(sizeof(double) * n3), *e = malloc(sizeof(double) * n3);
    double *yn = malloc(sizeof(double) * n3);
    memset(st, 0, sizeof(*st));
    int status = OR_OK;

    memcpy(y, m, sizeof(double) * n3);
    rhs_at(c, y, *t, alpha, precess, h, k[0]);
    st->rhs_evals++;
    if (*dt <= 0.0) {
        *dt = initial_dt(c, y, k[0], *t, alpha, precess, rtol, atol, &st->rhs_evals);
    }
    int last_rejected = 0;
    /* relaxation mode: stop when the torque criterion holds (checked on the
     * current state before every step) */
    while (st->accepted < max_steps && *t < t_end) {
        if (torque_tol > 0.0) {
            double mxt = 0.0;
            for (long q = 0; q < N; q++) {
                if (c->Ms[q] == 0.0)
                    continue;
                double mx_ = y[q], my_ = y[N + q], mz_ = y[2 * N + q];
                double hx = h[q], hy = h[N + q], hz = h[2 * N + q];
                double px = my_ * hz - mz_ * hy, py = mz_ * hx - mx_ * hz, pz = mx_ * hy - my_ * hx;
                double tq = sqrt(px * px + py * py + pz * pz) / c->Ms[q];
                if (tq > mxt)
                    mxt = tq;
            }
            if (mxt < torque_tol)
                break;
        }
        double hstep = *dt;
        if (*t + hstep > t_end)
            hstep = t_end - *t;
        for (int s = 1; s < S; s++) {
            for (long q = 0; q < n3; q++) {
                double acc = 0.0;
                for (int j = 0; j < s; j++)
                    acc += T.a[s][j] * k[j][q];
                ys[q] = y[q] + hstep * acc;
            }
            rhs_at(c, ys, *t + T.c[s] * hstep, alpha, precess, h, k[s]);
            st->rhs_evals++;
        }
        /* the propagated solution: with FSAL it is the last stage's input */
        if (T.fsal) {
            memcpy(yn, ys, sizeof(double) * n3);
        } else {
            for (long q = 0; q < n3; q++) {
                double acc = 0.0;
                for (int j = 0; j < S; j++)
                    acc += T.b[j] * k[j][q];
                yn[q] = y[q] + hstep * acc;
            }
        }
        for (long q = 0; q < n3; q++) {
            double acc = 0.0;
            for (int j = 0; j < S; j++)
                acc += T.e[j] * k[j][q];
            e[q] = hstep * acc;
        }
        double err = fixed ? 0.0 : err_norm(c, y, yn, e, rtol, atol);
        st->err_last = err;
        if (!isfinite(err)) {
            /* A trial step that overflows is rejected like any too-large step
             * (minimum factor 0.2); only a non-finite current state is an
             * error. */
            int bad = 0;
            for (long q = 0; q < n3; q++)
                if (!isfinite(y[q])) {
                    bad = 1;
                    break;
                }
            if (bad) {
                status = OR_ENONFINITE;
                break;
            }
            err = INFINITY;
        }
        if (err <= 1.0) {
            *t += hstep;
            memcpy(y, yn, sizeof(double) * n3);
            st->accepted++;
            if (renorm) {
                renormalise(c, y);
                rhs_at(c, y, *t, alpha, precess, h, k[0]);
                st->rhs_evals++;
            } else if (T.fsal) {
                double *tmp = k[0];
                k[0] = k[S - 1];
                k[S - 1] = tmp; /* first same as last; h holds the field at y */
            } else {
                rhs_at(c, y, *t, alpha, precess, h, k[0]);
                st->rhs_evals++;
            }
            if (!fixed) {
                double fac = err == 0.0 ? 10.0 : fmin(10.0, fmax(0.2, 0.9 * pow(err, -0.2)));
                if (last_rejected && fac > 1.0)
                    fac = 1.0;
                /* a step clipped to t_end keeps the unclipped proposal */
                if (!(hstep < *dt))
                    *dt = fac * hstep;
            }
            last_rejected = 0;
        } else {
            st->rejected++;
            double fac = fmax(0.2, 0.9 * pow(err, -0.2));
            *dt = fac * hstep;
            last_rejected = 1;
            /* field h was overwritten by the stages; restore the one at y */
            or_heff(c, y, *t, (unsigned)c->terms, h);
        }
        if (*dt < 1e-20) {
            status = OR_EDTMIN;
            break;
        }
    }
    if (torque_tol > 0.0 && status == OR_OK && st->accepted >= max_steps) {
        /* converged only if the criterion holds on the final state */
        double mxt = 0.0;
        for (long q = 0; q < N; q++) {
            if (c->Ms[q] == 0.0)
                continue;
            double px = y[N + q] * h[2 * N + q] - y[2 * N + q] * h[N + q];
            double py = y[2 * N + q] * h[q] - y[q] * h[2 * N + q];
            double pz = y[q] * h[N + q] - y[N + q] * h[q];
            double tq = sqrt(px * px + py * py + pz * pz) / c->Ms[q];
            if (tq > mxt)
                mxt = tq;
        }
        if (!(mxt < torque_tol))
            status = OR_ENOTCONV;
    }
    memcpy(m, y, sizeof(double) * n3);
    st->t = *t;
    st->dt = *dt;
    for (int s = 0; s < 7; s++)
        free(k[s]);
    free(y);
    free(ys);
    free(yn);
    free(h);
    free(e);
    return status;
}

/* Relaxation (Sec. 3): high damping (alpha = 1) without the precession term,
 * renormalised Dormand-Prince steps, until max_i |m_i x h_i| / Ms_i < tol. */
int or_relax(or_ctx *c, double *m, double tol, long max_steps, double rtol, or_stats *st)
{
    double t = 0.0, dt = -1.0;
    return or_dp45(c, m, &t, &dt, rtol, rtol, INFINITY, max_steps, 1, 0, 1.0, 0, st, tol);
}

/* Maximum torque max_i |m_i x h_i| / Ms_i over magnetic cells. */
double or_max_torque(const or_ctx *c, const double *m, double t)
{
    long N = c->N;
    double *h = malloc(sizeof(double) * 3 * N);
    or_heff(c, m, t, (unsigned)c->terms, h);
    double mxt = 0.0;
    for (long q = 0; q < N; q++) {
        if (c->Ms[q] == 0.0)
            continue;
        double px = m[N + q] * h[2 * N + q] - m[2 * N + q] * h[N + q];
        double py = m[2 * N + q] * h[q] - m[q] * h[2 * N + q];
        double pz = m[q] * h[N + q] - m[N + q] * h[q];
        double tq = sqrt(px * px + py * py + pz * pz) / c->Ms[q];
        if (tq > mxt)
            mxt = tq;
    }
    free(h);
    return mxt;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing harness only; n < 1 leaves the
   OpenMP default).  No arithmetic depends on it. */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* Differentiation: transposed field operator, LLG vector-Jacobian product,   */
/* classical RK4 with a time-averaged region loss and its discrete adjoint.  */
/* Supports the inverse-design use of the method (Sec. 5.2): gradients of a  */
/* scalar objective with respect to the magnetisation and to the per-cell    */
/* saturation magnetisation.  Pinned by dot-product tests against the        */
/* forward operators and by central finite differences                       */
/* (tests/test_oracle_adjoint.py).                                            */
/* ------------------------------------------------------------------------- */

/* (A~ v)_i = sum_nb (2/D^2) harmonic(A_i, A_nb) (v_nb - v_i): the symmetric
 * part of the exchange operator, h_ex = diag(2/(mu0 Ms)) A~ m. */
static void exch_core(const or_ctx *c, const double *v, double *out)
{
    long N = c->N, nx = c->n[0], ny = c->n[1], nz = c->n[2];
    for (long t = 0; t < N; t++) {
        long i = t % nx, j = (t / nx) % ny, k = t / (nx * ny);
        double acc[3] = {0, 0, 0};
        long nb[6][3] = {{i + 1, j, k}, {i - 1, j, k}, {i, j + 1, k},
                         {i, j - 1, k}, {i, j, k + 1}, {i, j, k - 1}};
        for (int q = 0; q < 6; q++) {
            long a = nb[q][0], b = nb[q][1], e = nb[q][2];
            if (a < 0 || a >= nx || b < 0 || b >= ny || e < 0 || e >= nz)
                continue;
            long s = cidx(c, a, b, e);
            double Ai = c->A[t], As = c->A[s];
            double hm = (Ai + As) != 0.0 ? Ai * As / (Ai + As) : 0.0;
            double dk = c->d[q / 2];
            double w = 2.0 / (dk * dk) * hm;
            for (int comp = 0; comp < 3; comp++)
                acc[comp] += w * (v[comp * N + s] - v[comp * N + t]);
        }
        for (int comp = 0; comp < 3; comp++)
            out[comp * N + t] = acc[comp];
    }
}

/* Demag kernel applied to a field without the Ms factor: (K w)_i. */
static void demag_raw(or_ctx *c, const double *w, double *out)
{
    double *Ms = c->Ms;
    double *ones = malloc(sizeof(double) * c->N);
    for (long q = 0; q < c->N; q++)
        ones[q] = 1.0;
    c->Ms = ones;
    or_demag(c, w, out);
    c->Ms = Ms;
    free(ones);
}

/* Transposed (linear part of the) effective field: for the terms in mask
 * (demag, exchange, first-order uniaxial anisotropy -- the higher-order
 * anisotropy terms are not linear in m and are not covered; the Zeeman field
 * does not depend on m),
 * grad_m = H^T w and grad_ms_i += d(w . h)/d Ms_i at fixed m.  grad_ms may be
 * NULL. */
void or_heff_vjp(or_ctx *c, const double *m, const double *w, unsigned mask, double *grad_m,
                 double *grad_ms)
{
    long N = c->N;
    double *tmp = malloc(sizeof(double) * 3 * N), *tmp2 = malloc(sizeof(double) * 3 * N);
    memset(grad_m, 0, sizeof(double) * 3 * N);
    if (mask & OR_DEMAG) {
        /* h = K (Ms m) on magnetic targets (zero on vacuum targets):
         * H^T w = Ms (K w') with w' = w masked to magnetic cells, since
         * K_ab(r) = K_ba(r) = K_ab(-r); d(w.h)/dMs_j = m_j . (K w')_j */
        for (long q = 0; q < N; q++)
            for (int a = 0; a < 3; a++)
                tmp2[a * N + q] = c->Ms[q] != 0.0 ? w[a * N + q] : 0.0;
        demag_raw(c, tmp2, tmp);
        for (long q = 0; q < N; q++) {
            for (int a = 0; a < 3; a++)
                grad_m[a * N + q] += c->Ms[q] * tmp[a * N + q];
            if (grad_ms)
                grad_ms[q] += m[q] * tmp[q] + m[N + q] * tmp[N + q] + m[2 * N + q] * tmp[2 * N + q];
        }
    }
    if (mask & OR_EXCH) {
        /* h = diag(2/(mu0 Ms)) A~ m: H^T w = A~ (2 w/(mu0 Ms));
         * d(w.h)/dMs_i = -2/(mu0 Ms_i^2) w_i . (A~ m)_i */
        for (long q = 0; q < N; q++)
            for (int a = 0; a < 3; a++)
                tmp[a * N + q] = c->Ms[q] != 0.0 ? 2.0 * w[a * N + q] / (OR_MU0 * c->Ms[q]) : 0.0;
        exch_core(c, tmp, tmp2);
        for (long q = 0; q < 3 * N; q++)
            grad_m[q] += tmp2[q];
        if (grad_ms) {
            exch_core(c, m, tmp2);
            for (long q = 0; q < N; q++)
                if (c->Ms[q] != 0.0)
                    grad_ms[q] -= 2.0 / (OR_MU0 * c->Ms[q] * c->Ms[q]) *
                                  (w[q] * tmp2[q] + w[N + q] * tmp2[N + q] + w[2 * N + q] * tmp2[2 * N + q]);
        }
    }
    if (mask & OR_ANIS) {
        for (long q = 0; q < N; q++) {
            if (c->Ms[q] == 0.0)
                continue;
            double ew = c->eu[0] * w[q] + c->eu[1] * w[N + q] + c->eu[2] * w[2 * N + q];
            double em = c->eu[0] * m[q] + c->eu[1] * m[N + q] + c->eu[2] * m[2 * N + q];
            double pre = 2.0 * (c->Kuc ? c->Kuc[q] : c->Ku) / (OR_MU0 * c->Ms[q]);
            for (int a = 0; a < 3; a++)
                grad_m[a * N + q] += pre * c->eu[a] * ew;
            if (grad_ms)
                grad_ms[q] -= pre / c->Ms[q] * ew * em;
        }
    }
    free(tmp);
    free(tmp2);
}

/* Exact Jacobian-vector product of the LLG right-hand side at (m, t) along v
 * (forward mode of Eq. llg with h = H m + h_zee(t)). */
void or_llg_jvp(or_ctx *c, const double *m, const double *v, double t, double *out)
{
    long N = c->N;
    double *h = malloc(sizeof(double) * 3 * N), *hv = malloc(sizeof(double) * 3 * N);
    or_heff(c, m, t, (unsigned)c->terms, h);
    or_heff(c, v, t, (unsigned)c->terms & ~(unsigned)OR_ZEEMAN, hv);
    double g = OR_GAMMA / (1.0 + c->alpha * c->alpha), al = c->alpha;
    for (long q = 0; q < N; q++) {
        double M[3] = {m[q], m[N + q], m[2 * N + q]}, V[3] = {v[q], v[N + q], v[2 * N + q]};
        double H[3] = {h[q], h[N + q], h[2 * N + q]}, HV[3] = {hv[q], hv[N + q], hv[2 * N + q]};
        if (c->Ms[q] == 0.0) {
            out[q] = out[N + q] = out[2 * N + q] = 0.0;
            continue;
        }
        double mh[3], vh[3], mhv[3];
#define CROSS(o, a, b) o[0] = a[1] * b[2] - a[2] * b[1], o[1] = a[2] * b[0] - a[0] * b[2], o[2] = a[0] * b[1] - a[1] * b[0]
        CROSS(mh, M, H);
        CROSS(vh, V, H);
        CROSS(mhv, M, HV);
        double dmh[3] = {vh[0] + mhv[0], vh[1] + mhv[1], vh[2] + mhv[2]}; /* d(m x h) */
        double t1[3], t2[3];
        CROSS(t1, V, mh);  /* v x (m x h) */
        CROSS(t2, M, dmh); /* m x d(m x h) */
#undef CROSS
        for (int a = 0; a < 3; a++)
            out[a * N + q] = -g * (dmh[a] + al * (t1[a] + t2[a]));
    }
    free(h);
    free(hv);
}

/* Vector-Jacobian product of the LLG right-hand side at (m, t): grad_m =
 * J^T w, and grad_ms += d(w . f)/dMs at fixed m (grad_ms may be NULL). */
void or_llg_vjp(or_ctx *c, const double *m, double t, const double *w, double *grad_m,
                double *grad_ms)
{
    long N = c->N;
    double *h = malloc(sizeof(double) * 3 * N), *z = malloc(sizeof(double) * 3 * N);
    double *hz = malloc(sizeof(double) * 3 * N);
    or_heff(c, m, t, (unsigned)c->terms, h);
    double g = OR_GAMMA / (1.0 + c->alpha * c->alpha), al = c->alpha;
    for (long q = 0; q < N; q++) {
        double M[3] = {m[q], m[N + q], m[2 * N + q]}, W[3] = {w[q], w[N + q], w[2 * N + q]};
        double H[3] = {h[q], h[N + q], h[2 * N + q]};
        if (c->Ms[q] == 0.0) {
            for (int a = 0; a < 3; a++)
                grad_m[a * N + q] = z[a * N + q] = 0.0;
            continue;
        }
        double mh = M[0] * H[0] + M[1] * H[1] + M[2] * H[2];
        double wm = W[0] * M[0] + W[1] * M[1] + W[2] * M[2];
        double wh = W[0] * H[0] + W[1] * H[1] + W[2] * H[2];
        double mm = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
        double hxw[3] = {H[1] * W[2] - H[2] * W[1], H[2] * W[0] - H[0] * W[2], H[0] * W[1] - H[1] * W[0]};
        double wxm[3] = {W[1] * M[2] - W[2] * M[1], W[2] * M[0] - W[0] * M[2], W[0] * M[1] - W[1] * M[0]};
        for (int a = 0; a < 3; a++) {
            /* d(w.f)/dm at fixed h, and z = d(w.f)/dh */
            grad_m[a * N + q] = -g * (hxw[a] + al * (W[a] * mh + H[a] * wm - 2.0 * M[a] * wh));
            z[a * N + q] = -g * (wxm[a] + al * (M[a] * wm - W[a] * mm));
        }
    }
    or_heff_vjp(c, m, z, (unsigned)c->terms & ~(unsigned)OR_ZEEMAN, hz, grad_ms);
    for (long q = 0; q < 3 * N; q++)
        grad_m[q] += hz[q];
    free(h);
    free(z);
    free(hz);
}

static double region_mz(const or_ctx *c, const double *m, const unsigned char *region, long nreg)
{
    long double acc = 0.0L;
    for (long q = 0; q < c->N; q++)
        if (region[q])
            acc += m[2 * c->N + q];
    return (double)(acc / nreg);
}

static void rk4_step(or_ctx *c, const double *m, double t, double dt, double *out, double *ys[4])
{
    long n3 = 3 * c->N;
    double *h = malloc(sizeof(double) * n3), *k = malloc(sizeof(double) * n3);
    double *y = malloc(sizeof(double) * n3);
    const double cs[4] = {0.0, 0.5, 0.5, 1.0}, wts[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    memcpy(y, m, sizeof(double) * n3);
    memcpy(out, m, sizeof(double) * n3);
    for (int s = 0; s < 4; s++) {
        if (ys)
            memcpy(ys[s], y, sizeof(double) * n3);
        rhs_at(c, y, t + cs[s] * dt, c->alpha, 1, h, k);
        for (long q = 0; q < n3; q++)
            out[q] += dt * wts[s] * k[q];
        if (s < 3)
            for (long q = 0; q < n3; q++)
                y[q] = m[q] + (s == 2 ? dt : 0.5 * dt) * k[q];
    }
    free(h);
    free(k);
    free(y);
}

/* Classical RK4 with fixed dt from t0; loss = (1/nsteps) sum_{n=1..nsteps}
 * mean over the region of m_z(t_n).  m is advanced in place. */
double or_rk4(or_ctx *c, double *m, double t0, double dt, long nsteps, const unsigned char *region)
{
    long n3 = 3 * c->N, nreg = 0;
    for (long q = 0; q < c->N; q++)
        nreg += region[q] ? 1 : 0;
    double *nxt = malloc(sizeof(double) * n3);
    long double loss = 0.0L;
    for (long n = 0; n < nsteps; n++) {
        rk4_step(c, m, t0 + n * dt, dt, nxt, NULL);
        memcpy(m, nxt, sizeof(double) * n3);
        loss += region_mz(c, m, region, nreg);
    }
    free(nxt);
    return (double)(loss / nsteps);
}

/* Discrete adjoint of or_rk4: gradient of the loss with respect to the
 * per-cell Ms (grad_ms, N values) and to the initial state (grad_m0, 3N,
 * may be NULL).  Every state is kept (no checkpointing): plain reverse-mode
 * differentiation of each step y1 = m, y2 = m + dt/2 k1, y3 = m + dt/2 k2,
 * y4 = m + dt k3, m' = m + dt (k1 + 2 k2 + 2 k3 + k4)/6. */
double or_rk4_adjoint(or_ctx *c, const double *m0, double t0, double dt, long nsteps,
                      const unsigned char *region, double *grad_ms, double *grad_m0)
{
    long N = c->N, n3 = 3 * N, nreg = 0;
    for (long q = 0; q < N; q++)
        nreg += region[q] ? 1 : 0;
    double *traj = malloc(sizeof(double) * n3 * (nsteps + 1));
    memcpy(traj, m0, sizeof(double) * n3);
    long double loss = 0.0L;
    for (long n = 0; n < nsteps; n++) {
        rk4_step(c, traj + n * n3, t0 + n * dt, dt, traj + (n + 1) * n3, NULL);
        loss += region_mz(c, traj + (n + 1) * n3, region, nreg);
    }
    double *lam = calloc(n3, sizeof(double)), *kap = malloc(sizeof(double) * n3);
    double *nu[4], *ys[4];
    for (int s = 0; s < 4; s++) {
        nu[s] = malloc(sizeof(double) * n3);
        ys[s] = malloc(sizeof(double) * n3);
    }
    double *scratch = malloc(sizeof(double) * n3);
    memset(grad_ms, 0, sizeof(double) * N);
    const double cs[4] = {0.0, 0.5, 0.5, 1.0};
    const double dL = 1.0 / ((double)nsteps * (double)nreg);
    for (long n = nsteps - 1; n >= 0; n--) {
        /* explicit dependence of the loss on m_{n+1} */
        for (long q = 0; q < N; q++)
            if (region[q])
                lam[2 * N + q] += dL;
        rk4_step(c, traj + n * n3, t0 + n * dt, dt, scratch, ys);
        double tn = t0 + n * dt;
        /* stage 4, 3, 2, 1 */
        for (long q = 0; q < n3; q++)
            kap[q] = dt / 6.0 * lam[q];
        or_llg_vjp(c, ys[3], tn + cs[3] * dt, kap, nu[3], grad_ms);
        for (long q = 0; q < n3; q++)
            kap[q] = dt / 3.0 * lam[q] + dt * nu[3][q];
        or_llg_vjp(c, ys[2], tn + cs[2] * dt, kap, nu[2], grad_ms);
        for (long q = 0; q < n3; q++)
            kap[q] = dt / 3.0 * lam[q] + 0.5 * dt * nu[2][q];
        or_llg_vjp(c, ys[1], tn + cs[1] * dt, kap, nu[1], grad_ms);
        for (long q = 0; q < n3; q++)
            kap[q] = dt / 6.0 * lam[q] + 0.5 * dt * nu[1][q];
        or_llg_vjp(c, ys[0], tn + cs[0] * dt, kap, nu[0], grad_ms);
        for (long q = 0; q < n3; q++)
            lam[q] += nu[0][q] + nu[1][q] + nu[2][q] + nu[3][q];
    }
    if (grad_m0)
        memcpy(grad_m0, lam, sizeof(double) * n3);
    for (int s = 0; s < 4; s++) {
        free(nu[s]);
        free(ys[s]);
    }
    free(traj);
    free(lam);
    free(kap);
    free(scratch);
    return (double)(loss / nsteps);
}

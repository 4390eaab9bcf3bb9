// dd.h -- double-double arithmetic (about 106-bit significands) for the
// cancellation-prone Newell functions of the demag kernel set-up.
//
// Error-free transformations: Knuth's TwoSum and Dekker's FastTwoSum, and the
// exact product via fused multiply-add (Dekker 1971, "A floating-point
// technique for extending the available precision").  Addition, product,
// quotient and square root follow the double-double schemes analysed by
// Hida, Li & Bailey (2001).  The elementary functions are written here from
// their series:
//   exp  -- reduction x = k ln2 + 512 r, Taylor series of expm1(r), nine
//           doublings expm1(2u) = 2 expm1(u) + expm1(u)^2;
//   log  -- one Newton step y <- y + a exp(-y) - 1 from the double log;
//   atan -- reflection to [0, 1], angle halving
//           atan(x) = 2 atan(x / (1 + sqrt(1 + x^2))) down to x < 1/64, then
//           the alternating Taylor series;
//   asinh -- log(x + sqrt(x^2 + 1)) for x >= 0.
// All functions are usable on host and device.
//
// Error-free transformations only hold if every product is rounded on its
// own: HIP compiles with floating-point contraction on by default, which would
// fuse the product of TwoProd into the following FastTwoSum and destroy the
// error term.  Contraction is therefore switched off for this header and for
// newell.h, and switched back on at the end of newell.h.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

#pragma clang fp contract(off)

namespace mmx {

struct dd {
    double hi, lo;
};

__host__ __device__ inline dd dd_from(double a) { return {a, 0.0}; }

__host__ __device__ inline dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

// requires |a| >= |b| (or a == 0)
__host__ __device__ inline dd fast_two_sum(double a, double b)
{
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}

__host__ __device__ inline dd two_prod(double a, double b)
{
    double p = a * b;
    double e = fma(a, b, -p);
    return {p, e};
}

__host__ __device__ inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }

__host__ __device__ inline dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

__host__ __device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

__host__ __device__ inline dd dd_mul(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}

__host__ __device__ inline dd dd_mul_d(dd a, double b)
{
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return fast_two_sum(p.hi, p.lo);
}

// exact scaling by a power of two
__host__ __device__ inline dd dd_ldexp(dd a, int e) { return {ldexp(a.hi, e), ldexp(a.lo, e)}; }

__host__ __device__ inline dd dd_div(dd a, dd b)
{
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd q = fast_two_sum(q1, q2);
    return dd_add(q, dd_from(q3));
}

__host__ __device__ inline dd dd_div_d(dd a, double b) { return dd_div(a, dd_from(b)); }

// sqrt(a) = s + (a - s^2)/(2 s) with s = a.hi * rsqrt(a.hi) (one Newton
// correction evaluated in double-double).
__host__ __device__ inline dd dd_sqrt(dd a)
{
    if (!(a.hi > 0.0)) return {0.0, 0.0};
    double x = 1.0 / sqrt(a.hi);
    double s = a.hi * x;
    dd r = dd_sub(a, two_prod(s, s));
    return two_sum(s, r.hi * (0.5 * x));
}

__host__ __device__ inline dd dd_ln2() { return {0.6931471805599453, 2.3190468138462996e-17}; }
__host__ __device__ inline dd dd_pi() { return {3.141592653589793, 1.2246467991473532e-16}; }
__host__ __device__ inline dd dd_pi_2() { return {1.5707963267948966, 6.123233995736766e-17}; }

__host__ __device__ inline dd dd_exp(dd a)
{
    if (a.hi == 0.0 && a.lo == 0.0) return dd_from(1.0);
    double k = floor(a.hi / 0.6931471805599453 + 0.5);
    dd r = dd_sub(a, dd_mul_d(dd_ln2(), k));
    r = dd_ldexp(r, -9);  // |r| <= ln2/1024
    // expm1(r) by Taylor: r + r^2/2! + ... ; |r|^11/11! < 1e-40
    dd term = r, s = r;
    for (int n = 2; n <= 11; ++n) {
        term = dd_div_d(dd_mul(term, r), (double)n);
        s = dd_add(s, term);
    }
    for (int i = 0; i < 9; ++i) s = dd_add(dd_ldexp(s, 1), dd_mul(s, s));
    s = dd_add(s, dd_from(1.0));
    return dd_ldexp(s, (int)k);
}

__host__ __device__ inline dd dd_log(dd a)
{
    if (!(a.hi > 0.0)) return {0.0, 0.0};
    dd y = dd_from(log(a.hi));
    // y <- y + a exp(-y) - 1
    dd e = dd_exp(dd_neg(y));
    return dd_sub(dd_add(y, dd_mul(a, e)), dd_from(1.0));
}

__host__ __device__ inline dd dd_atan(dd x)
{
    bool neg = x.hi < 0.0;
    if (neg) x = dd_neg(x);
    bool inv = x.hi > 1.0;
    if (inv) x = dd_div(dd_from(1.0), x);
    int halvings = 0;
    while (x.hi > 0.015625) {
        dd root = dd_sqrt(dd_add(dd_from(1.0), dd_mul(x, x)));
        x = dd_div(x, dd_add(dd_from(1.0), root));
        ++halvings;
    }
    // atan(x) = x - x^3/3 + x^5/5 - ...; x^2 < 2.5e-4, 12 terms reach 1e-40
    dd x2 = dd_mul(x, x);
    dd pw = x, s = x;
    for (int n = 1; n <= 12; ++n) {
        pw = dd_mul(pw, x2);
        dd t = dd_div_d(pw, (double)(2 * n + 1));
        s = (n & 1) ? dd_sub(s, t) : dd_add(s, t);
    }
    s = dd_ldexp(s, halvings);
    if (inv) s = dd_sub(dd_pi_2(), s);
    return neg ? dd_neg(s) : s;
}

// asinh for x >= 0
__host__ __device__ inline dd dd_asinh_pos(dd x)
{
    dd root = dd_sqrt(dd_add(dd_mul(x, x), dd_from(1.0)));
    return dd_log(dd_add(x, root));
}

}  // namespace mmx

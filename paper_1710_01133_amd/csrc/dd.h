// Double-double arithmetic on the device: a value is the unevaluated sum
// hi + lo of two doubles with |lo| <= ulp(hi)/2, about 106 significant bits.
// The building blocks are the error-free transformations of Knuth (TwoSum:
// the exact rounding error of a sum) and Dekker (Fast2Sum for |a| >= |b|, and
// the exact product error, here by one fused multiply-add); the compound
// operations follow the double-double algorithms of Hida, Li and Bailey
// ("Algorithms for quad-double precision floating point arithmetic", 2001):
// the accurate sum, the product with its cross terms, long division.
// Elementary functions are written here from their mathematics:
//   exp: x = k ln2 + r, e^r by Taylor series on r / 2^10, squared back as
//        (1 + s)^2 = 1 + (2s + s^2);
//   log: one Newton step y + x e^-y - 1 from the double logarithm;
//   expm1: Taylor series (small arguments, no cancellation);
//   Gamma: shifted to w >= 40 by Gamma(z) = Gamma(z + n) / (z (z+1) ... (z+n-1)),
//          ln Gamma(w) by Stirling's series with Bernoulli numbers B_2..B_32;
//   sin, cos: reduction by pi/2 (double-double), Taylor series on |r| <= pi/4.
// The error-free transformations hold only if every sum and product rounds
// on its own: a multiply fused into a following add by contraction (hipcc
// contracts across statements by default) breaks them, so contraction is
// switched off for everything after this header in the translation unit, and
// the library builds the file that includes it with -ffp-contract=off as well.
// Included only by libabm's own .hip files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace abm {

struct dd {
    double hi, lo;
};

__host__ __device__ __forceinline__ dd dd_make(double x) { return dd{x, 0.0}; }

// |a| >= |b|: a + b = s + e exactly
__host__ __device__ __forceinline__ dd fast_two_sum(double a, double b)
{
    const double s = a + b;
    return dd{s, b - (s - a)};
}

// a + b = s + e exactly, any order of magnitude
__host__ __device__ __forceinline__ dd two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    return dd{s, (a - (s - bb)) + (b - bb)};
}

// a * b = p + e exactly (the fused multiply-add rounds a*b - p once, exactly)
__host__ __device__ __forceinline__ dd two_prod(double a, double b)
{
    const double p = a * b;
    return dd{p, fma(a, b, -p)};
}

__host__ __device__ __forceinline__ dd dd_add(dd x, dd y)
{
    dd s = two_sum(x.hi, y.hi);
    const dd t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

__host__ __device__ __forceinline__ dd dd_neg(dd x) { return dd{-x.hi, -x.lo}; }
__host__ __device__ __forceinline__ dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }

__host__ __device__ __forceinline__ dd dd_add_d(dd x, double y)
{
    dd s = two_sum(x.hi, y);
    s.lo += x.lo;
    return fast_two_sum(s.hi, s.lo);
}

__host__ __device__ __forceinline__ dd dd_mul(dd x, dd y)
{
    dd p = two_prod(x.hi, y.hi);
    p.lo = fma(x.hi, y.lo, fma(x.lo, y.hi, p.lo));
    return fast_two_sum(p.hi, p.lo);
}

__host__ __device__ __forceinline__ dd dd_mul_d(dd x, double y)
{
    dd p = two_prod(x.hi, y);
    p.lo = fma(x.lo, y, p.lo);
    return fast_two_sum(p.hi, p.lo);
}

// exact scaling by a power of two
__host__ __device__ __forceinline__ dd dd_ldexp(dd x, int e) { return dd{ldexp(x.hi, e), ldexp(x.lo, e)}; }

__host__ __device__ __forceinline__ dd dd_div(dd x, dd y)
{
    const double q1 = x.hi / y.hi;
    dd r = dd_sub(x, dd_mul_d(y, q1));
    const double q2 = r.hi / y.hi;
    r = dd_sub(r, dd_mul_d(y, q2));
    const double q3 = r.hi / y.hi;
    return dd_add_d(fast_two_sum(q1, q2), q3);
}

// x / y for a double y: q1 = x.hi / y, the remainder x - q1 y exactly
// (two_prod), q2 = remainder / y (two divisions against dd_div's three; about
// the same accuracy, a few units of 2^-104)
__host__ __device__ __forceinline__ dd dd_div_d(dd x, double y)
{
    const double q1 = x.hi / y;
    const dd p = two_prod(q1, y);
    const dd s = two_sum(x.hi, -p.hi);
    const double t = (s.lo - p.lo) + x.lo;
    const double q2 = (s.hi + t) / y;
    return fast_two_sum(q1, q2);
}

// acc + w * f
__host__ __device__ __forceinline__ dd dd_fma(dd w, dd f, dd acc) { return dd_add(acc, dd_mul(w, f)); }

__host__ __device__ __forceinline__ bool dd_le(dd x, double c) { return x.hi < c || (x.hi == c && x.lo <= 0.0); }
__host__ __device__ __forceinline__ bool dd_ge(dd x, double c) { return x.hi > c || (x.hi == c && x.lo >= 0.0); }
__host__ __device__ __forceinline__ bool dd_isfinite(dd x) { return isfinite(x.hi) && isfinite(x.lo); }

// constants: the double pair nearest each value
__host__ __device__ __forceinline__ dd dd_ln2() { return dd{0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56}; }
__host__ __device__ __forceinline__ dd dd_pi_2() { return dd{0x1.921fb54442d18p+0, 0x1.1a62633145c07p-54}; }
__host__ __device__ __forceinline__ dd dd_half_ln_2pi()
{
    return dd{0x1.d67f1c864beb5p-1, -0x1.65b5a1b7ff5dfp-55};
}

// e^x - 1 for |x| <= 2 by its Taylor series (terms below 2^-110 of the sum end it)
__host__ __device__ inline dd dd_expm1_series(dd x)
{
    dd term = x, sum = x;
    for (int n = 2; n < 60; ++n) {
        term = dd_div(dd_mul(term, x), dd_make((double)n));
        sum = dd_add(sum, term);
        if (fabs(term.hi) <= 1e-34 * fabs(sum.hi)) break;
    }
    return sum;
}

__host__ __device__ inline dd dd_exp(dd x)
{
    if (x.hi == 0.0) return dd_make(1.0);
    const double k = rint(x.hi / 0x1.62e42fefa39efp-1);
    dd r = dd_sub(x, dd_mul_d(dd_ln2(), k));        // |r| <= ln2/2 (+ rounding)
    r = dd_ldexp(r, -10);
    dd s = dd_expm1_series(r);                         // e^(r/1024) - 1
    for (int i = 0; i < 10; ++i) s = dd_add(dd_ldexp(s, 1), dd_mul(s, s));   // (1+s)^2 - 1
    return dd_ldexp(dd_add_d(s, 1.0), (int)k);
}

__host__ __device__ inline dd dd_log(dd x)
{
    const dd y = dd_make(log(x.hi));
    // y + x e^-y - 1
    return dd_add(y, dd_add_d(dd_mul(x, dd_exp(dd_neg(y))), -1.0));
}

// x^a for x > 0 (a a double)
__host__ __device__ inline dd dd_pow(dd x, double a) { return dd_exp(dd_mul_d(dd_log(x), a)); }

// Gamma(z) for 1 <= z <= 4
__host__ __device__ inline dd dd_gamma(dd z)
{
    // Bernoulli numbers B_2k = num / den, k = 1..16
    const double num[16] = {1.0, -1.0, 1.0, -1.0, 5.0, -691.0, 7.0, -3617.0, 43867.0, -174611.0,
                            854513.0, -236364091.0, 8553103.0, -23749461029.0, 8615841276005.0,
                            -7709321041217.0};
    const double den[16] = {6.0, 30.0, 42.0, 30.0, 66.0, 2730.0, 6.0, 510.0, 798.0, 330.0,
                            138.0, 2730.0, 6.0, 870.0, 14322.0, 510.0};
    const int n = 40;
    dd prod = z;                                       // z (z+1) ... (z+n-1)
    for (int i = 1; i < n; ++i) prod = dd_mul(prod, dd_add_d(z, (double)i));
    const dd w = dd_add_d(z, (double)n);
    const dd lw = dd_log(w);
    // (w - 1/2) ln w - w + ln(2 pi)/2 + sum_k B_2k / (2k (2k-1) w^(2k-1))
    dd lg = dd_add(dd_sub(dd_mul(dd_add_d(w, -0.5), lw), w), dd_half_ln_2pi());
    const dd winv = dd_div(dd_make(1.0), w);
    const dd winv2 = dd_mul(winv, winv);
    dd wp = winv;                                      // w^-(2k-1)
    for (int k = 1; k <= 16; ++k) {
        const double c = (2.0 * k) * (2.0 * k - 1.0);
        const dd bk = dd_div(dd_make(num[k - 1]), dd_make(den[k - 1] * c));
        lg = dd_add(lg, dd_mul(bk, wp));
        wp = dd_mul(wp, winv2);
    }
    return dd_div(dd_exp(lg), prod);
}

// sin and cos of x (|x| up to ~1e6) by reduction with pi/2
__host__ __device__ inline void dd_sincos(dd x, dd* sn, dd* cs)
{
    const double k = rint(x.hi / 0x1.921fb54442d18p+0);
    const dd r = dd_sub(x, dd_mul_d(dd_pi_2(), k));
    const dd r2 = dd_mul(r, r);
    // sin r = r - r^3/3! + ..., cos r = 1 - r^2/2! + ...
    dd ts = r, s = r, tc = dd_make(1.0), c = dd_make(1.0);
    for (int n = 1; n < 30; ++n) {
        ts = dd_neg(dd_div_d(dd_mul(ts, r2), (2.0 * n) * (2.0 * n + 1.0)));
        tc = dd_neg(dd_div_d(dd_mul(tc, r2), (2.0 * n - 1.0) * (2.0 * n)));
        s = dd_add(s, ts);
        c = dd_add(c, tc);
        if (fabs(ts.hi) <= 1e-34 * fabs(s.hi) + 1e-300 && fabs(tc.hi) <= 1e-34) break;
    }
    const int q = (int)(((int64_t)k) & 3);
    switch (q) {
    case 0: *sn = s; *cs = c; break;
    case 1: *sn = c; *cs = dd_neg(s); break;
    case 2: *sn = dd_neg(s); *cs = dd_neg(c); break;
    default: *sn = dd_neg(c); *cs = s; break;
    }
}

}  // namespace abm

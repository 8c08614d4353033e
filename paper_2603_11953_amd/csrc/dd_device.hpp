// Double-double arithmetic on the gfx950 FP64 VALU.
//
// A value is the unevaluated sum hi + lo of two doubles with |lo| <= ulp(hi)/2
// after normalisation.  The building blocks are the classic error-free
// transformations: Knuth's TwoSum, Dekker's FastTwoSum and the FMA form of
// TwoProduct.  The library is built with -ffp-contract=off so that no a*b+c
// is silently fused; FMA appears only where __builtin_fma is written.
#pragma once

#include <hip/hip_runtime.h>

namespace gsvd {

struct dd_t {
    double hi, lo;
};

__device__ __forceinline__ dd_t dd_make(double h, double l) { return dd_t{h, l}; }

// s + e == a + b exactly, s = fl(a + b)   (Knuth, 6 flops)
__device__ __forceinline__ dd_t two_sum(double a, double b) {
    double s = a + b;
    double bv = s - a;
    double e = (a - (s - bv)) + (b - bv);
    return dd_t{s, e};
}

// exact when |a| >= |b|   (Dekker, 3 flops)
__device__ __forceinline__ dd_t quick_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    return dd_t{s, e};
}

// p + e == a * b exactly (no underflow)
__device__ __forceinline__ dd_t two_prod(double a, double b) {
    double p = a * b;
    double e = __builtin_fma(a, b, -p);
    return dd_t{p, e};
}

__device__ __forceinline__ dd_t dd_add(dd_t x, dd_t y) {
    dd_t s = two_sum(x.hi, y.hi);
    dd_t t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd_t dd_neg(dd_t x) { return dd_t{-x.hi, -x.lo}; }

// x - y with the error bound relative to |x| + |y| (one TwoSum on the high
// parts, low parts added in FP64): enough where the backward error model is
// componentwise in the operands, as in a Cholesky update.
__device__ __forceinline__ dd_t dd_sub_fast(dd_t x, dd_t y) {
    dd_t s = two_sum(x.hi, -y.hi);
    s.lo += x.lo - y.lo;
    return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd_t dd_sub(dd_t x, dd_t y) { return dd_add(x, dd_neg(y)); }

__device__ __forceinline__ dd_t dd_mul(dd_t x, dd_t y) {
    dd_t p = two_prod(x.hi, y.hi);
    p.lo = __builtin_fma(x.hi, y.lo, p.lo);
    p.lo = __builtin_fma(x.lo, y.hi, p.lo);
    return quick_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd_t dd_mul_d(dd_t x, double y) {
    dd_t p = two_prod(x.hi, y);
    p.lo = __builtin_fma(x.lo, y, p.lo);
    return quick_two_sum(p.hi, p.lo);
}

// x / y: two quotient digits corrected against the dd remainder, then a third.
__device__ __forceinline__ dd_t dd_div(dd_t x, dd_t y) {
    double q1 = x.hi / y.hi;
    dd_t r = dd_sub(x, dd_mul_d(y, q1));
    double q2 = r.hi / y.hi;
    r = dd_sub(r, dd_mul_d(y, q2));
    double q3 = r.hi / y.hi;
    dd_t q = quick_two_sum(q1, q2);
    return dd_add(q, dd_t{q3, 0.0});
}

// sqrt(x) for x > 0: the FP64 root refined by two Newton corrections
// y <- y + (x - y^2) / (2 y) carried out in dd.
__device__ __forceinline__ dd_t dd_sqrt(dd_t x) {
    if (!(x.hi > 0.0)) return dd_t{x.hi == 0.0 ? 0.0 : __builtin_nan(""), 0.0};
    double y = __builtin_sqrt(x.hi);
    dd_t r = dd_sub(x, two_prod(y, y));
    dd_t s = quick_two_sum(y, r.hi / (2.0 * y));
    dd_t r2 = dd_sub(x, dd_mul(s, s));
    return dd_add(s, dd_t{r2.hi / (2.0 * s.hi), 0.0});
}

// acc += a * b with the exact product folded in: TwoProduct + TwoSum, and the
// two error terms collected in acc.lo (10 FP64 operations).
__device__ __forceinline__ void dd_mac(double &hi, double &lo, double a, double b) {
    double p = a * b;
    double e = __builtin_fma(a, b, -p);
    double s = hi + p;
    double bv = s - hi;
    double err = (hi - (s - bv)) + (p - bv);
    hi = s;
    lo += e + err;
}

}  // namespace gsvd

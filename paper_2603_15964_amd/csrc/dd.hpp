// Double-double arithmetic: a value is the unevaluated sum hi + lo of two
// doubles with |lo| <= ulp(hi) / 2, about 106 significant bits.  The
// error-free transformations are Knuth's two-sum and the fma-based two-product
// (Dekker's products without splitting); the compound operations follow the
// usual double-double algorithms (e.g. Hida, Li and Bailey's QD library).
// Nothing here may be reassociated or contracted: the code relies on IEEE
// round-to-nearest evaluation of each operation in the order written.  Every
// body turns contraction off (device code is compiled with fp-contract=fast,
// which would otherwise fuse the product of two_prod into the following sum).
#pragma once

#include <hip/hip_runtime.h>

#define LMEP_DD_EXACT _Pragma("clang fp contract(off)")

namespace lmep {

struct dd {
    double hi, lo;
};

__host__ __device__ __forceinline__ dd dd_of(double x) { return {x, 0.0}; }

// s + e = a + b exactly
__host__ __device__ __forceinline__ dd two_sum(double a, double b) {
    LMEP_DD_EXACT
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
// the same when |a| >= |b|
__host__ __device__ __forceinline__ dd quick_two_sum(double a, double b) {
    LMEP_DD_EXACT
    const double s = a + b;
    return {s, b - (s - a)};
}
// p + e = a * b exactly
__host__ __device__ __forceinline__ dd two_prod(double a, double b) {
    LMEP_DD_EXACT
    const double p = a * b;
    return {p, fma(a, b, -p)};
}

__host__ __device__ __forceinline__ dd dd_add(dd a, dd b) {
    LMEP_DD_EXACT
    dd s = two_sum(a.hi, b.hi);
    const dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__host__ __device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__host__ __device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

__host__ __device__ __forceinline__ dd dd_mul(dd a, dd b) {
    LMEP_DD_EXACT
    dd p = two_prod(a.hi, b.hi);
    p.lo = fma(a.hi, b.lo, p.lo);
    p.lo = fma(a.lo, b.hi, p.lo);
    return quick_two_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ dd dd_mul_d(dd a, double b) {
    LMEP_DD_EXACT
    dd p = two_prod(a.hi, b);
    p.lo = fma(a.lo, b, p.lo);
    return quick_two_sum(p.hi, p.lo);
}
// a + b * c
__host__ __device__ __forceinline__ dd dd_fma(dd b, dd c, dd a) { return dd_add(a, dd_mul(b, c)); }

// a / b for a double b: one correction of the leading quotient
__host__ __device__ __forceinline__ dd dd_div_d(dd a, double b) {
    LMEP_DD_EXACT
    const double q1 = a.hi / b;
    const dd p = two_prod(q1, b);
    const dd r = dd_sub(a, p);
    const double q2 = r.hi / b;
    return quick_two_sum(q1, q2);
}
__host__ __device__ __forceinline__ dd dd_div(dd a, dd b) {
    LMEP_DD_EXACT
    const double q1 = a.hi / b.hi;
    const dd r = dd_sub(a, dd_mul_d(b, q1));
    const double q2 = r.hi / b.hi;
    const dd r2 = dd_sub(r, dd_mul_d(b, q2));
    const double q3 = r2.hi / b.hi;
    return dd_add(quick_two_sum(q1, q2), dd_of(q3));
}

// nearest double
__host__ __device__ __forceinline__ double dd_round(dd a) {
    LMEP_DD_EXACT
    return a.hi + a.lo;
}

}  // namespace lmep

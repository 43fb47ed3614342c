// Double-double ("dd") arithmetic on the GPU: a value is the unevaluated sum
// hi + lo of two doubles with |lo| <= ulp(hi) / 2, about 106 significant bits
// (unit roundoff ~1.1e-32).  Built from error-free transformations:
//   TwoSum (Knuth, TAOCP vol. 2, 4.2.2): s + e = a + b exactly;
//   FastTwoSum (Dekker 1971), valid when |a| >= |b|;
//   TwoProd with a fused multiply-add: p + e = a * b exactly.
// Addition is the accurate two-TwoSum form (Hida, Li and Bailey, 2001), which
// keeps a relative error of a few units of 2^-106 even under cancellation;
// multiplication adds the cross terms to the exact product of the high parts;
// division and square root take one Newton correction of the double result.
// Complex dd values hold a dd real and a dd imaginary part.
//
// The error-free transformations require every + and * to round on its own:
// floating-point contraction (fusing a product into a following add, which the
// device compiler does by default) would silently break them, so it is turned
// off for every file that includes this header.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace gbs {

struct dd {
    double hi, lo;
};
struct cdd {
    dd re, im;
};

__device__ __forceinline__ dd dd_make(double x) { return dd{x, 0.0}; }

__device__ __forceinline__ dd two_sum_dd(double a, double b) {
    const double s = a + b;
    const double v = s - a;
    return dd{s, (a - (s - v)) + (b - v)};
}

__device__ __forceinline__ dd fast_two_sum_dd(double a, double b) {
    const double s = a + b;
    return dd{s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod_dd(double a, double b) {
    const double p = a * b;
    return dd{p, fma(a, b, -p)};
}

__device__ __forceinline__ dd dd_add(dd x, dd y) {
    dd s = two_sum_dd(x.hi, y.hi);
    const dd t = two_sum_dd(x.lo, y.lo);
    s.lo += t.hi;
    s = fast_two_sum_dd(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum_dd(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_neg(dd x) { return dd{-x.hi, -x.lo}; }
__device__ __forceinline__ dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }

__device__ __forceinline__ dd dd_mul(dd x, dd y) {
    dd p = two_prod_dd(x.hi, y.hi);
    p.lo = fma(x.hi, y.lo, fma(x.lo, y.hi, p.lo));
    return fast_two_sum_dd(p.hi, p.lo);
}

__device__ __forceinline__ dd dd_mul_d(dd x, double b) {
    dd p = two_prod_dd(x.hi, b);
    p.lo = fma(x.lo, b, p.lo);
    return fast_two_sum_dd(p.hi, p.lo);
}

// x / y: q1 = x.hi / y.hi, then one correction from the dd residual x - q1 y.
__device__ __forceinline__ dd dd_div(dd x, dd y) {
    const double q1 = x.hi / y.hi;
    const dd r = dd_sub(x, dd_mul_d(y, q1));
    const double q2 = r.hi / y.hi;
    return fast_two_sum_dd(q1, q2);
}

__device__ __forceinline__ dd dd_sqrt(dd x) {
    if (!(x.hi > 0.0)) return dd{0.0, 0.0};
    const double y = sqrt(x.hi);
    const dd r = dd_sub(x, two_prod_dd(y, y));
    return fast_two_sum_dd(y, r.hi * (0.5 / y));
}

__device__ __forceinline__ cdd cdd_make(double re, double im) { return cdd{dd{re, 0.0}, dd{im, 0.0}}; }
__device__ __forceinline__ cdd cdd_zero() { return cdd{dd{0.0, 0.0}, dd{0.0, 0.0}}; }
__device__ __forceinline__ cdd cdd_add(cdd a, cdd b) { return cdd{dd_add(a.re, b.re), dd_add(a.im, b.im)}; }
__device__ __forceinline__ cdd cdd_sub(cdd a, cdd b) { return cdd{dd_sub(a.re, b.re), dd_sub(a.im, b.im)}; }
__device__ __forceinline__ cdd cdd_conj(cdd a) { return cdd{a.re, dd_neg(a.im)}; }
__device__ __forceinline__ cdd cdd_mul(cdd a, cdd b) {
    return cdd{dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
}
// conj(a) * b
__device__ __forceinline__ cdd cdd_cmul(cdd a, cdd b) {
    return cdd{dd_add(dd_mul(a.re, b.re), dd_mul(a.im, b.im)), dd_sub(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
}
__device__ __forceinline__ cdd cdd_mul_dd(cdd a, dd b) { return cdd{dd_mul(a.re, b), dd_mul(a.im, b)}; }
__device__ __forceinline__ cdd cdd_mul_d(cdd a, double b) { return cdd{dd_mul_d(a.re, b), dd_mul_d(a.im, b)}; }
__device__ __forceinline__ dd cdd_abs2(cdd a) { return dd_add(dd_mul(a.re, a.re), dd_mul(a.im, a.im)); }

}  // namespace gbs

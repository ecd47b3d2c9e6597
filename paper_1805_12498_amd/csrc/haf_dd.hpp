// Double-double arithmetic (a value is an unevaluated sum hi + lo with
// |lo| <= ulp(hi) / 2, about 106 significant bits) and complex double-double,
// for the per-term precision mode.  Built from the error-free transformations
// of Knuth (two-sum) and Dekker (two-product, here with a fused multiply-add),
// with the division and square root refined by one Newton step.  Every
// function is exact-rounding-free C++ that must be compiled without
// floating-point contraction, so that no a * b + c is fused behind its back.
#pragma once
#include <hip/hip_runtime.h>

#include "haf_common.hpp"

namespace hafgpu {

__device__ __forceinline__ dd dd_of(double a) { return dd{ a, 0.0 }; }
// a + b for |a| >= |b| (or a == 0)
__device__ __forceinline__ dd dd_quick(double a, double b) {
    const double s = a + b;
    return dd{ s, b - (s - a) };
}
__device__ __forceinline__ dd dd_neg(dd a) { return dd{ -a.hi, -a.lo }; }
__device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
    const double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e = fma(a.hi, b.lo, e);
    e = fma(a.lo, b.hi, e);
    return dd_quick(p, e);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
    const double p = a.hi * b;
    double e = fma(a.hi, b, -p);
    e = fma(a.lo, b, e);
    return dd_quick(p, e);
}
// exact scaling by a power of two
__device__ __forceinline__ dd dd_ldexp(dd a, int e) { return dd{ ldexp(a.hi, e), ldexp(a.lo, e) }; }
__device__ __forceinline__ dd dd_div(dd a, dd b) {
    const double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    const double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    const double q3 = r.hi / b.hi;
    return dd_add(dd_quick(q1, q2), dd_of(q3));
}
// sqrt(a), a >= 0: the double root x and one Newton step x + (a - x^2) / (2 x)
__device__ __forceinline__ dd dd_sqrt(dd a) {
    if (!(a.hi > 0.0)) return dd_of(0.0);
    const double x = sqrt(a.hi);
    const double p = x * x;
    const dd x2 = dd_quick(p, fma(x, x, -p));
    const dd d = dd_sub(a, x2);
    return dd_quick(x, d.hi / (2.0 * x));
}
__device__ __forceinline__ bool dd_is_zero(dd a) { return a.hi == 0.0 && a.lo == 0.0; }

struct cdd {
    dd re, im;
};
__device__ __forceinline__ cdd cdd_zero() { return cdd{ dd_of(0.0), dd_of(0.0) }; }
__device__ __forceinline__ cdd cdd_one() { return cdd{ dd_of(1.0), dd_of(0.0) }; }
__device__ __forceinline__ cdd cdd_of(double2 z) { return cdd{ dd_of(z.x), dd_of(z.y) }; }
__device__ __forceinline__ cdd cdd_add(cdd a, cdd b) { return cdd{ dd_add(a.re, b.re), dd_add(a.im, b.im) }; }
__device__ __forceinline__ cdd cdd_sub(cdd a, cdd b) { return cdd{ dd_sub(a.re, b.re), dd_sub(a.im, b.im) }; }
__device__ __forceinline__ cdd cdd_conj(cdd a) { return cdd{ a.re, dd_neg(a.im) }; }
__device__ __forceinline__ cdd cdd_mul(cdd a, cdd b) {
    return cdd{ dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re)) };
}
__device__ __forceinline__ cdd cdd_mul_dd(cdd a, dd b) { return cdd{ dd_mul(a.re, b), dd_mul(a.im, b) }; }
__device__ __forceinline__ cdd cdd_ldexp(cdd a, int e) { return cdd{ dd_ldexp(a.re, e), dd_ldexp(a.im, e) }; }
// acc + a * b, acc + conj(a) * b, acc - a * b
__device__ __forceinline__ cdd cdd_fma(cdd acc, cdd a, cdd b) { return cdd_add(acc, cdd_mul(a, b)); }
__device__ __forceinline__ cdd cdd_fma_cj(cdd acc, cdd a, cdd b) { return cdd_add(acc, cdd_mul(cdd_conj(a), b)); }
__device__ __forceinline__ cdd cdd_fms(cdd acc, cdd a, cdd b) { return cdd_sub(acc, cdd_mul(a, b)); }
// 1 / z for z != 0
__device__ __forceinline__ cdd cdd_recip(cdd z) {
    const dd d = dd_add(dd_mul(z.re, z.re), dd_mul(z.im, z.im));
    return cdd{ dd_div(z.re, d), dd_neg(dd_div(z.im, d)) };
}
__device__ __forceinline__ dd dd_shfl_xor(dd a, int o) { return dd{ __shfl_xor(a.hi, o, 64), __shfl_xor(a.lo, o, 64) }; }
__device__ __forceinline__ dd dd_readlane(dd a, int lane) { return dd{ readlane_d(a.hi, lane), readlane_d(a.lo, lane) }; }
__device__ __forceinline__ cdd cdd_readlane(cdd a, int lane) {
    return cdd{ dd_readlane(a.re, lane), dd_readlane(a.im, lane) };
}
// butterfly sum over the 64 lanes: every lane adds the same operands at every stage
__device__ __forceinline__ dd dd_wave_sum(dd a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a = dd_add(a, dd_shfl_xor(a, o));
    return a;
}

}  // namespace hafgpu

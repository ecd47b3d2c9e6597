// Shared device helpers for the hafnian kernels: complex double arithmetic,
// wave-level primitives and the subset enumeration.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hafgpu {

constexpr int kMaxN = 64;          // matrix size limit
constexpr int kMaxPairs = 32;      // n / 2

// ---------------------------------------------------------------- complex double
__device__ __forceinline__ double2 cz() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 cone() { return make_double2(1.0, 0.0); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// acc += a * b
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
// acc -= a * b
__device__ __forceinline__ void cfms(double2& acc, double2 a, double2 b) {
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}
// acc += conj(a) * b
__device__ __forceinline__ void cfma_cj(double2& acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}
// acc -= a * conj(b)
__device__ __forceinline__ void cfms_cj(double2& acc, double2 a, double2 b) {
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}
__device__ __forceinline__ double2 crecip(double2 z) {
    double d = 1.0 / fma(z.x, z.x, z.y * z.y);
    return make_double2(z.x * d, -z.y * d);
}

// ---------------------------------------------------------------- wave primitives
__device__ __forceinline__ double readlane_d(double x, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double2 readlane_c(double2 z, int lane) {
    return make_double2(readlane_d(z.x, lane), readlane_d(z.y, lane));
}
// Butterfly all-reduce over the 64 lanes: every lane adds the same two operands
// at every stage, so all lanes end with bitwise the same sum.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}

// Columns whose largest entry is below this are treated as already reduced.
constexpr double kTinyColumn = 0x1p-960;

// ---------------------------------------------------------------- DPP / swizzle moves of a double
// (a lane whose source is outside the wave reads 0; no register has to be zeroed first)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <int PATTERN>
__device__ __forceinline__ double swizzle_d(double x) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(x), PATTERN);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(x), PATTERN);
    return __hiloint2double(hi, lo);
}
// value of lane i ^ 32
__device__ __forceinline__ double xor32_d(double x) {
    int lo = __double2loint(x), hi = __double2hiint(x);
    auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    // after the swap the first result holds lanes 0..31 of x twice, the second lanes 32..63 twice
    const bool upper = (threadIdx.x & 32) != 0;
    return __hiloint2double(upper ? h[0] : h[1], upper ? l[0] : l[1]);
}

// x(lanes 0..31) + x(lanes 32..63) for a value that is uniform within each half:
// the swap hands every lane both halves, and every lane adds them in the same order
__device__ __forceinline__ double halves_sum(double x) {
    const auto l = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(x), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(x), false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}

// Sum over aligned groups of L lanes (L = 4, 8, 16, 32, 64); every lane of a
// group gets bitwise the same total (each stage adds the same two values).
template <int L>
__device__ __forceinline__ double group_sum(double x) {
    x += dpp_d<0xB1>(x);                    // quad_perm [1,0,3,2]: lane ^ 1
    x += dpp_d<0x4E>(x);                    // quad_perm [2,3,0,1]: lane ^ 2
    if (L >= 8) x += dpp_d<0x141>(x);       // row_half_mirror: the other quad of the 8-group
    if (L >= 16) x += dpp_d<0x140>(x);      // row_mirror: the other 8-group of the row
    if (L >= 32) x += swizzle_d<0x401F>(x); // lane ^ 16 within 32
    if (L >= 64) x = halves_sum(x);         // + lane ^ 32
    return x;
}

// sqrt(x) for normal x > 0: the hardware reciprocal square root refined by one
// Goldschmidt step and a final Newton correction (within an ulp or two)
__device__ __forceinline__ double sqrt_pos(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    double g = x * r, h = 0.5 * r;
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    return fma(fma(-g, g, x), h, g);
}
// 1 / x for normal x whose reciprocal is normal: the hardware reciprocal and two
// Newton steps (within an ulp)
__device__ __forceinline__ double rcp_normal(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// Maximum over aligned groups of L lanes (same exchange pattern as group_sum).
template <int L>
__device__ __forceinline__ double group_max(double x) {
    x = fmax(x, dpp_d<0xB1>(x));
    x = fmax(x, dpp_d<0x4E>(x));
    if (L >= 8) x = fmax(x, dpp_d<0x141>(x));
    if (L >= 16) x = fmax(x, dpp_d<0x140>(x));
    if (L >= 32) x = fmax(x, swizzle_d<0x401F>(x));
    if (L >= 64) x = fmax(x, xor32_d(x));
    return x;
}

// ---------------------------------------------------------------- double-double
struct dd { double hi, lo; };
__device__ __forceinline__ dd dd_two_sum(double a, double b) {
    double s = a + b, bb = s - a;
    return dd{ s, (a - (s - bb)) + (b - bb) };
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    dd s = dd_two_sum(a.hi, b.hi), t = dd_two_sum(a.lo, b.lo);
    s.lo += t.hi;
    double h = s.hi + s.lo;
    s.lo = s.lo - (h - s.hi);
    s.hi = h;
    s.lo += t.lo;
    h = s.hi + s.lo;
    return dd{ h, s.lo - (h - s.hi) };
}

// ---------------------------------------------------------------- subsets
// The rank-th m-subset of {0..N-1} in the combinatorial number system:
// rank = sum_i C(c_i, i) over the chosen elements c_m > ... > c_1 >= 0,
// taken greedily from the largest element.  C(c, k) is carried along with
// C(c-1, k) = C(c, k) (c-k)/c and C(c-1, k-1) = C(c, k) k/c (exact in 64 bits
// for c <= 32).
__device__ __forceinline__ uint32_t unrank_subset(uint64_t rank, int m, int N) {
    uint64_t b = 1;                                   // C(N-1, m)
    if (m > N - 1) b = 0;
    else
        for (int i = 1; i <= m; ++i) b = b * (uint64_t)(N - m - 1 + i) / (uint64_t)i;
    uint32_t mask = 0;
    int k = m;
    for (int c = N - 1; c >= 0 && k > 0; --c) {
        if (rank >= b) {
            mask |= 1u << c;
            rank -= b;
            b = c > 0 ? b * (uint64_t)k / (uint64_t)c : 0;
            --k;
        } else {
            b = c > 0 ? b * (uint64_t)(c - k) / (uint64_t)c : 0;
        }
    }
    return mask;
}

// Vertex of row r of the subset matrix: the (r/2)-th chosen pair, member r&1.
__device__ __forceinline__ int subset_vertex(uint32_t mask, int r) {
    uint32_t mm = mask;
    for (int t = 0; t < (r >> 1); ++t) mm &= mm - 1;
    return 2 * __builtin_ctz(mm) + (r & 1);
}

}  // namespace hafgpu

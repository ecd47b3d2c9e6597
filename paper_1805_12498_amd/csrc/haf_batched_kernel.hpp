// Persistent batched kernel: many hafnians / loop hafnians of different sizes
// in one launch (the work layout is described in haf_batch.hpp).
//
// Each one-wave workgroup loops: take the next chunk number from a global
// counter, find its class, run the register-tiled per-subset stage (gather,
// loop moments, Householder Hessenberg, characteristic polynomial; App. B,
// Sec. 3.3) for the chunk's subsets with their coefficients in a per-wave
// scratch area, then one lane per subset runs the series (Newton's identities
// and the exponential series, Eq. haffinal), the wave adds the signed terms
// (Eq. Pset) in double-double by a fixed tree and stores the chunk's partial.
// The wave that finishes an item's last chunk folds the item's partials in slot
// order and writes the result, scaled back by 2^(2eN) (the exact input scaling).
// Every wave leaves the loop once the counter passes the chunk count.
#pragma once
#include "haf_batch.hpp"
#include "haf_coef_reg.hpp"
#include "haf_series.hpp"

namespace hafgpu {

// Layout tables of the batched kernels: (P, Q, R, C, CP) for s in (lo, hi].
// Table 0: the default layouts up to s = 32; 1: one full wave per matrix above
// s = 16 (up to 32); 2: subsets of 34..48 rows.  A launch runs the chunks of
// s <= 32 with table 0 or 1 and those above 32 with table 2.
#define HAF_BATCH_T0(X) X(4, 4, 2, 2, 0, 0, 8) X(4, 4, 4, 4, 0, 8, 16) X(8, 4, 3, 6, 0, 16, 24) \
                        X(8, 4, 4, 8, 1, 24, 32)
#define HAF_BATCH_T1(X) X(4, 4, 2, 2, 0, 0, 8) X(4, 4, 4, 4, 0, 8, 16) X(8, 8, 3, 3, 2, 16, 24) \
                        X(8, 8, 4, 4, 2, 24, 32)
#define HAF_BATCH_T2(X) X(8, 8, 5, 5, 2, 32, 40) X(8, 8, 6, 6, 2, 40, 48)

constexpr int cmax_list(const int* v, int n) {
    int r = 0;
    for (int i = 0; i < n; ++i) r = v[i] > r ? v[i] : r;
    return r;
}
#define HAF_LDS_OF(P, Q, R, C, CP, LO, HI) , RegShape<P, Q, R, C>::W * RegShape<P, Q, R, C>::PER
#define HAF_W_OF(P, Q, R, C, CP, LO, HI) if (s > LO && s <= HI) return RegShape<P, Q, R, C>::W;
constexpr int kLds0[] = { 2 * kBatchMaxCap HAF_BATCH_T0(HAF_LDS_OF) };
constexpr int kLds1[] = { 2 * kBatchMaxCap HAF_BATCH_T1(HAF_LDS_OF) };
constexpr int kLds2[] = { 2 * kBatchMaxCap HAF_BATCH_T2(HAF_LDS_OF) };
template <int T> struct BatchTable;
template <> struct BatchTable<0> { static constexpr int LDS = cmax_list(kLds0, sizeof kLds0 / sizeof(int)); };
template <> struct BatchTable<1> { static constexpr int LDS = cmax_list(kLds1, sizeof kLds1 / sizeof(int)); };
template <> struct BatchTable<2> { static constexpr int LDS = cmax_list(kLds2, sizeof kLds2 / sizeof(int)); };

// Signed double-double sum of one value per lane by a fixed tree; lane 0 gets it.
__device__ __forceinline__ void wave_dd_sum(double* sh, dd& r, dd& i) {
    const int l = threadIdx.x;
    sh[l] = r.hi; sh[64 + l] = r.lo; sh[128 + l] = i.hi; sh[192 + l] = i.lo;
    __syncthreads();
    for (int st = 32; st > 0; st >>= 1) {
        if (l < st) {
            r = dd_add(dd{ sh[l], sh[64 + l] }, dd{ sh[l + st], sh[64 + l + st] });
            i = dd_add(dd{ sh[128 + l], sh[192 + l] }, dd{ sh[128 + l + st], sh[192 + l + st] });
            sh[l] = r.hi; sh[64 + l] = r.lo; sh[128 + l] = i.hi; sh[192 + l] = i.lo;
        }
        __syncthreads();
    }
    r = dd{ sh[0], sh[64] };
    i = dd{ sh[128], sh[192] };
    __syncthreads();
}

// T: layout table; WPE: resident waves per SIMD the register allocation must
// allow; NMAX: the largest N = n/2 of an item the series stage handles.
template <int T, int WPE, int NMAX>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_batched(const BatchItem* __restrict__ items, const BatchClass* __restrict__ classes, int ncls, int nchunks,
               int* __restrict__ cursor, int* __restrict__ done, const int* __restrict__ exps,
               double* __restrict__ partials, double2* __restrict__ coefscr) {
    __shared__ double2 lds[BatchTable<T>::LDS];
    double* shd = (double*)lds;
    const int lane = threadIdx.x;
    double2* cbuf = coefscr + (int64_t)blockIdx.x * (kBatchMaxCap * 2 * NMAX);

    for (;;) {
        int k = 0;
        if (lane == 0) k = atomicAdd(cursor, 1);
        k = __builtin_amdgcn_readfirstlane(__shfl(k, 0));
        if (k >= nchunks) break;
        // class of chunk k: the last class whose chunk_base <= k
        int lo = 0, hi = ncls - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (classes[mid].chunk_base <= k) lo = mid;
            else hi = mid - 1;
        }
        const BatchClass cl = classes[lo];
        const BatchItem& it = items[cl.item];
        const int j = cl.j0 + (k - cl.chunk_base);
        const int m = cl.m, s = 2 * m, N = it.n / 2;
        const uint64_t rank0 = (uint64_t)j * (uint64_t)cl.cap;
        const int count = (int)min((uint64_t)cl.cap, (uint64_t)cl.total - rank0);
        const int e = exps[cl.item];
        const double off_scale = ldexp(1.0, -2 * e), diag_scale = ldexp(1.0, -e);
        const bool loops = it.loops != 0;

        // ---- per-subset stage: coefficients of the chunk's subsets -> cbuf[k][subset]
#define HAF_BATCH_CASE(P, Q, R, C, CP, LO, HI)                                                                  \
        if (s > LO && s <= HI) {                                                                                \
            constexpr int W = RegShape<P, Q, R, C>::W;                                                          \
            const int span = (count + W - 1) / W;                                                               \
            /* an opaque copy of the lane index keeps each layout's lane-dependent */                           \
            /* addresses inside its own branch instead of live across the loop */                               \
            int tid;                                                                                            \
            asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(lane));                                           \
            if (loops)                                                                                          \
                coef_reg_span<P, Q, R, C, CP, true>(lds, it.A, it.lda, N, m, rank0, count, nullptr, off_scale,  \
                                                    diag_scale, cbuf, kBatchMaxCap, 0, span, tid);              \
            else                                                                                                \
                coef_reg_span<P, Q, R, C, CP, false>(lds, it.A, it.lda, N, m, rank0, count, nullptr, off_scale, \
                                                     diag_scale, cbuf, kBatchMaxCap, 0, span, tid);             \
        } else
        if (T == 0) { HAF_BATCH_T0(HAF_BATCH_CASE) {} }
        else if (T == 1) { HAF_BATCH_T1(HAF_BATCH_CASE) {} }
        else { HAF_BATCH_T2(HAF_BATCH_CASE) {} }
#undef HAF_BATCH_CASE
        __syncthreads();

        // ---- series, one lane per subset, and the chunk's signed partial
        double2 f = cz();
        if (lane < count) {
            if (loops) f = subset_series_upto<NMAX, true>(cbuf, kBatchMaxCap, lane, N);
            else f = subset_series_upto<NMAX, false>(cbuf, kBatchMaxCap, lane, N);
        }
        const double sign = ((N - m) & 1) ? -1.0 : 1.0;
        dd r{ sign * f.x, 0.0 }, im{ sign * f.y, 0.0 };
        wave_dd_sum(shd, r, im);
        const int64_t slot = it.slot0 + cl.slot_base + j;
        if (lane == 0) {
            double* o = partials + 4 * slot;
            o[0] = r.hi; o[1] = r.lo; o[2] = im.hi; o[3] = im.lo;
        }
        __threadfence();                      // the partial is visible device-wide before the count
        int last = 0;
        if (lane == 0) last = atomicAdd(&done[cl.item], 1) == it.nslots - 1;
        last = __builtin_amdgcn_readfirstlane(__shfl(last, 0));
        if (!last) continue;

        // ---- the item is complete: fold its partials in slot order
        __threadfence();
        dd rr{ 0.0, 0.0 }, ii{ 0.0, 0.0 };
        for (int q = lane; q < it.nslots; q += 64) {
            const double* p = partials + 4 * (it.slot0 + q);
            rr = dd_add(rr, dd{ p[0], p[1] });
            ii = dd_add(ii, dd{ p[2], p[3] });
        }
        wave_dd_sum(shd, rr, ii);
        if (lane == 0) {
            const int e2n = 2 * N * e;
            const double rh = ldexp(rr.hi, e2n), rl = ldexp(rr.lo, e2n);
            const double ih = ldexp(ii.hi, e2n), il = ldexp(ii.lo, e2n);
            if (it.out_dd) { it.out_dd[0] = rh; it.out_dd[1] = rl; it.out_dd[2] = ih; it.out_dd[3] = il; }
            if (it.out) *it.out = make_double2(rh + rl, ih + il);
        }
    }
}

// Kernel variants (id, table, waves per SIMD, NMAX): the small-subset kernels
// come with series bounds 16 (items up to 32 rows) and 24 (up to 48); for a
// given N both give bitwise the same terms.
#define HAF_BATCH_VARIANTS16(X) X(0, 0, 2, 16) X(1, 1, 2, 16) X(3, 0, 1, 16)
#define HAF_BATCH_VARIANTS24(X) X(2, 2, 1, 24) X(4, 0, 2, 24) X(5, 1, 2, 24) X(6, 0, 1, 24)

}  // namespace hafgpu

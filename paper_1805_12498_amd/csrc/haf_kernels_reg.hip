// One-size-class launch of the register-tiled per-subset stage: the grid's
// groups split the chunk's subsets into equal contiguous runs.
#include <algorithm>

#include "haf_coef_reg.hpp"
#include "haf_launch.hpp"

namespace hafgpu {

// Lower bound on waves per SIMD that the compiler must keep room for: two for the
// tiles of 36 entries and more; three for the 3 x 3 tile, which the compiler then
// fits in 168 registers with a few spilled bytes (the batched call 1.4-2% faster,
// bitwise-equal results; the 2 x 2 tile at four waves and the 4 x 4 tile at three
// were no faster); no bound otherwise.
#define HAF_REG_WAVES(R, C) ((R) * (C) >= 36 ? 2 : ((R) * (C) == 9 ? 3 : 1))

template <int P, int Q, int R, int C, int CP, bool LOOPS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(HAF_REG_WAVES(R, C)))) void k_coef_reg(const double2* __restrict__ A, int lda, int N, int m,
                                                 uint64_t rank0, int count, const uint32_t* __restrict__ masks,
                                                 const int* __restrict__ d_exp, double2* __restrict__ coef,
                                                 int64_t cstride) {
    using S = RegShape<P, Q, R, C>;
    __shared__ double2 lds[S::W * S::PER];
    const int e = d_exp ? *d_exp : 0;
    const int groups = gridDim.x * S::W;
    const int span = (count + groups - 1) / groups;
    coef_reg_span<P, Q, R, C, CP, LOOPS>(lds, A, lda, N, m, rank0, count, masks, ldexp(1.0, -2 * e),
                                               ldexp(1.0, -e), coef, cstride, blockIdx.x * S::W, span, threadIdx.x);
}

#define HAF_INST_REG(P, Q, R, C, CP, LO, HI)                                                                \
    template __global__ void k_coef_reg<P, Q, R, C, CP, false>(const double2*, int, int, int, uint64_t, int,     \
                                                               const uint32_t*, const int*, double2*, int64_t); \
    template __global__ void k_coef_reg<P, Q, R, C, CP, true>(const double2*, int, int, int, uint64_t, int,      \
                                                              const uint32_t*, const int*, double2*, int64_t);
HAF_REG_TABLE(HAF_INST_REG)

int reg_max_s() { return 48; }

// Several chunks of one matrix: the workgroup finds its chunk in the table (a
// short uniform scan), then runs the same per-subset body as k_coef_reg.
template <int P, int Q, int R, int C, int CP, bool LOOPS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(HAF_REG_WAVES(R, C)))) void k_coef_reg_multi(
    const double2* __restrict__ A, int lda, int N, const int* __restrict__ d_exp, double2* __restrict__ coef,
    MultiChunks mc) {
    using S = RegShape<P, Q, R, C>;
    __shared__ double2 lds[S::W * S::PER];
    const int e = d_exp ? *d_exp : 0;
    int c = 0;
    while (c + 1 < mc.nc && (int)blockIdx.x >= mc.gstart[c + 1]) ++c;
    const int groups = (mc.gstart[c + 1] - mc.gstart[c]) * S::W;
    const int count = mc.count[c];
    const int span = (count + groups - 1) / groups;
    coef_reg_span<P, Q, R, C, CP, LOOPS>(lds, A, lda, N, mc.m[c], mc.rank0[c], count, nullptr,
                                                ldexp(1.0, -2 * e), ldexp(1.0, -e), coef + mc.coff[c], count,
                                                ((int)blockIdx.x - mc.gstart[c]) * S::W, span, threadIdx.x);
}

#define HAF_INST_REG_MULTI(P, Q, R, C, CP, LO, HI)                                                           \
    template __global__ void k_coef_reg_multi<P, Q, R, C, CP, false>(const double2*, int, int, const int*,   \
                                                                     double2*, MultiChunks);                 \
    template __global__ void k_coef_reg_multi<P, Q, R, C, CP, true>(const double2*, int, int, const int*,    \
                                                                    double2*, MultiChunks);
HAF_REG_TABLE(HAF_INST_REG_MULTI)

// Matrices of a batch: the workgroup finds its chunk by a binary search over
// the launch's chunk table (uniform), then runs the per-subset body for the
// chunk's matrix (its own N, exponent and subset ranks).
template <int P, int Q, int R, int C, int CP, bool LOOPS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(HAF_REG_WAVES(R, C)))) void k_coef_reg_group(
    const GroupItem* __restrict__ items, const GroupChunk* __restrict__ chunks, int nchunks,
    double2* __restrict__ coef) {
    using S = RegShape<P, Q, R, C>;
    __shared__ double2 lds[S::W * S::PER];
    const int blk = (int)blockIdx.x;
    int lo = 0, hi = nchunks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunks[mid].gstart <= blk) lo = mid;
        else hi = mid - 1;
    }
    const GroupChunk ch = chunks[lo];
    const int gend = lo + 1 < nchunks ? chunks[lo + 1].gstart : (int)gridDim.x;
    const int groups = (gend - ch.gstart) * S::W;
    const int span = (ch.count + groups - 1) / groups;
    const GroupItem it = items[ch.item];
    const int e = *it.exp;
    coef_reg_span<P, Q, R, C, CP, LOOPS, false>(lds, it.A, it.lda, ch.N, ch.m, ch.rank0, ch.count, nullptr,
                                                ldexp(1.0, -2 * e), ldexp(1.0, -e), coef + ch.coff, ch.count,
                                                (blk - ch.gstart) * S::W, span, threadIdx.x);
}

#define HAF_INST_REG_GROUP(P, Q, R, C, CP, LO, HI)                                                          \
    template __global__ void k_coef_reg_group<P, Q, R, C, CP, false>(const GroupItem*, const GroupChunk*,   \
                                                                     int, double2*);                        \
    template __global__ void k_coef_reg_group<P, Q, R, C, CP, true>(const GroupItem*, const GroupChunk*,    \
                                                                    int, double2*);
HAF_REG_TABLE(HAF_INST_REG_GROUP)

int reg_layout_count() {
    int i = 0;
#define HAF_CNT(P, Q, R, C, CP, LO, HI) ++i;
    HAF_REG_TABLE(HAF_CNT)
#undef HAF_CNT
    return i;
}

int reg_layout_sm(int layout) {
    int i = 0;
#define HAF_SM_OF(P, Q, R, C, CP, LO, HI) \
    if (i++ == layout) return RegShape<P, Q, R, C>::SM;
    HAF_REG_TABLE(HAF_SM_OF)
#undef HAF_SM_OF
    return 0;
}

int reg_layout_groups(int layout) {
    int i = 0;
#define HAF_W_OF(P, Q, R, C, CP, LO, HI) \
    if (i++ == layout) return RegShape<P, Q, R, C>::W;
    HAF_REG_TABLE(HAF_W_OF)
#undef HAF_W_OF
    return 0;
}

int reg_layout_family(int layout) {
    int i = 0;
#define HAF_FAMILY_OF(P, Q, R, C, CP, LO, HI) \
    if (i++ == layout) return (P << 16) | (Q << 8) | CP;
    HAF_REG_TABLE(HAF_FAMILY_OF)
#undef HAF_FAMILY_OF
    return -1;
}

int group_coef_blocks(int layout, int count, int span) {
    const int w = reg_layout_groups(layout) * (span > 0 ? span : 1);
    return w > 0 ? (count + w - 1) / w : 0;
}

hipError_t launch_coef_reg_group(int layout, bool loops, int blocks, hipStream_t st, const GroupItem* items,
                                 const GroupChunk* chunks, int nchunks, double2* coef) {
    if (nchunks < 1 || blocks < 1) return hipErrorInvalidValue;
    int i = 0;
#define HAF_TRY_GROUP(P, Q, R, C, CP, LO, HI)                                                                 \
    if (i++ == layout) {                                                                                      \
        if (loops) hipLaunchKernelGGL((k_coef_reg_group<P, Q, R, C, CP, true>), dim3(blocks), dim3(64), 0, st, \
                                      items, chunks, nchunks, coef);                                          \
        else hipLaunchKernelGGL((k_coef_reg_group<P, Q, R, C, CP, false>), dim3(blocks), dim3(64), 0, st,     \
                                items, chunks, nchunks, coef);                                                \
        return hipGetLastError();                                                                             \
    }
    HAF_REG_TABLE(HAF_TRY_GROUP)
#undef HAF_TRY_GROUP
    return hipErrorInvalidValue;
}

int reg_layout_index(int s) {
    int i = 0;
#define HAF_IDX(P, Q, R, C, CP, LO, HI) \
    if (s > LO && s <= HI) return i;    \
    ++i;
    HAF_REG_TABLE(HAF_IDX)
#undef HAF_IDX
    return -1;
}

hipError_t launch_coef_reg_multi(int s_max, bool loops, int grid_waves, hipStream_t st, const double2* A, int lda,
                                 int N, const int* d_exp, double2* coef, MultiChunks mc) {
    if (mc.nc < 1 || mc.nc > kMultiMax) return hipErrorInvalidValue;
#define HAF_TRY_MULTI(P, Q, R, C, CP, LO, HI)                                                                 \
    if (s_max > LO && s_max <= HI) {                                                                          \
        constexpr int W = RegShape<P, Q, R, C>::W;                                                            \
        int g = 0;                                                                                            \
        for (int c = 0; c < mc.nc; ++c) {                                                                     \
            const int s = 2 * mc.m[c];                                                                        \
            if (s <= LO || s > HI || mc.count[c] <= 0) return hipErrorInvalidValue;                           \
            mc.gstart[c] = g;                                                                                 \
            const int b = (mc.count[c] + W - 1) / W;                                                          \
            g += b < grid_waves ? b : grid_waves;                                                             \
        }                                                                                                     \
        mc.gstart[mc.nc] = g;                                                                                 \
        if (loops) hipLaunchKernelGGL((k_coef_reg_multi<P, Q, R, C, CP, true>), dim3(g), dim3(64), 0, st, A,   \
                                      lda, N, d_exp, coef, mc);                                               \
        else hipLaunchKernelGGL((k_coef_reg_multi<P, Q, R, C, CP, false>), dim3(g), dim3(64), 0, st, A, lda,  \
                                N, d_exp, coef, mc);                                                          \
        return hipGetLastError();                                                                             \
    }
    HAF_REG_TABLE(HAF_TRY_MULTI)
#undef HAF_TRY_MULTI
    return hipErrorInvalidValue;
}

// Workgroups of one launch: whole rounds of the kernel's resident one-wave workgroups
// (a partial last round leaves SIMDs idle while it drains), as many rounds as keep at
// least 32 subsets per lane group, up to eight (shorter workgroups also end more evenly).
template <int P, int Q, int R, int C, int CP, bool LOOPS>
static int coef_reg_grid(int cus, int count) {
    constexpr int W = RegShape<P, Q, R, C>::W;
    static const int per_cu = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_coef_reg<P, Q, R, C, CP, LOOPS>, 64, 0) != hipSuccess) {
            (void)hipGetLastError();          // not the launch's error: fall back to two waves per SIMD
            b = 0;
        }
        return b < 1 ? 8 : b;
    }();
    const int64_t slots = (int64_t)per_cu * cus;
    int64_t rounds = 1;
    while (rounds < 8 && slots * W * 32 * (rounds * 2) <= (int64_t)count) rounds *= 2;
    return (int)std::min<int64_t>(rounds * slots, ((int64_t)count + W - 1) / W);
}

hipError_t launch_coef_reg(int s, bool loops, int cus, hipStream_t st, const double2* A, int lda, int N,
                           int m, uint64_t rank0, int count, const uint32_t* masks, const int* d_exp,
                           double2* coef, int64_t cstride) {
    if (count <= 0) return hipSuccess;
#define HAF_TRY_REG(P, Q, R, C, CP, LO, HI)                                                                   \
    if (s > LO && s <= HI) {                                                                                  \
        if (loops)                                                                                            \
            hipLaunchKernelGGL((k_coef_reg<P, Q, R, C, CP, true>),                                            \
                               dim3(coef_reg_grid<P, Q, R, C, CP, true>(cus, count)), dim3(64), 0, st, A, lda, \
                               N, m, rank0, count, masks, d_exp, coef, cstride);                              \
        else                                                                                                  \
            hipLaunchKernelGGL((k_coef_reg<P, Q, R, C, CP, false>),                                           \
                               dim3(coef_reg_grid<P, Q, R, C, CP, false>(cus, count)), dim3(64), 0, st, A,    \
                               lda, N, m, rank0, count, masks, d_exp, coef, cstride);                         \
        return hipGetLastError();                                                                             \
    }
    HAF_REG_TABLE(HAF_TRY_REG)
#undef HAF_TRY_REG
    return hipErrorInvalidValue;
}

}  // namespace hafgpu

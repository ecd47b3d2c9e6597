// One-size-class launch of the register-tiled per-subset stage: the grid's
// groups split the chunk's subsets into equal contiguous runs.
#include "haf_coef_reg.hpp"
#include "haf_launch.hpp"

namespace hafgpu {

template <int P, int Q, int R, int C, int CP, bool LOOPS, bool ELIM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((ELIM || R * C >= 36) ? 2 : 1))) void k_coef_reg(const double2* __restrict__ A, int lda, int N, int m,
                                                 uint64_t rank0, int count, const uint32_t* __restrict__ masks,
                                                 const int* __restrict__ d_exp, double2* __restrict__ coef,
                                                 int64_t cstride) {
    using S = RegShape<P, Q, R, C>;
    __shared__ double2 lds[S::W * S::PER];
    const int e = d_exp ? *d_exp : 0;
    const int groups = gridDim.x * S::W;
    const int span = (count + groups - 1) / groups;
    coef_reg_span<P, Q, R, C, CP, LOOPS, ELIM>(lds, A, lda, N, m, rank0, count, masks, ldexp(1.0, -2 * e),
                                               ldexp(1.0, -e), coef, cstride, blockIdx.x * S::W, span, threadIdx.x);
}

#define HAF_INST_REG_E(P, Q, R, C, CP, LO, HI, E)                                                             \
    template __global__ void k_coef_reg<P, Q, R, C, CP, false, E>(const double2*, int, int, int, uint64_t, int,   \
                                                                  const uint32_t*, const int*, double2*, int64_t); \
    template __global__ void k_coef_reg<P, Q, R, C, CP, true, E>(const double2*, int, int, int, uint64_t, int,    \
                                                                 const uint32_t*, const int*, double2*, int64_t);
#define HAF_INST_REG_H(P, Q, R, C, CP, LO, HI) HAF_INST_REG_E(P, Q, R, C, CP, LO, HI, false)
#define HAF_INST_REG_EL(P, Q, R, C, CP, LO, HI) HAF_INST_REG_E(P, Q, R, C, CP, LO, HI, true)
HAF_REG_SHAPES(HAF_INST_REG_H)
HAF_REG_NARROW(HAF_INST_REG_EL)

int reg_max_s() { return 48; }

hipError_t launch_coef_reg(int s, bool loops, int grid_waves, hipStream_t st, const double2* A, int lda, int N,
                           int m, uint64_t rank0, int count, const uint32_t* masks, const int* d_exp,
                           double2* coef, int64_t cstride, bool wide, bool elim) {
    if (count <= 0) return hipSuccess;
#define HAF_TRY_REG(P, Q, R, C, CP, LO, HI, E)                                                                \
    if (s > LO && s <= HI) {                                                                                  \
        constexpr int W = RegShape<P, Q, R, C>::W;                                                            \
        int grid = (count + W - 1) / W;                                                                       \
        if (grid > grid_waves) grid = grid_waves;                                                             \
        if (loops) hipLaunchKernelGGL((k_coef_reg<P, Q, R, C, CP, true, E>), dim3(grid), dim3(64), 0, st, A,  \
                                      lda, N, m, rank0, count, masks, d_exp, coef, cstride);                  \
        else hipLaunchKernelGGL((k_coef_reg<P, Q, R, C, CP, false, E>), dim3(grid), dim3(64), 0, st, A, lda,  \
                                N, m, rank0, count, masks, d_exp, coef, cstride);                             \
        return hipGetLastError();                                                                             \
    }
#define HAF_TRY_REG_H(P, Q, R, C, CP, LO, HI) HAF_TRY_REG(P, Q, R, C, CP, LO, HI, false)
#define HAF_TRY_REG_EL(P, Q, R, C, CP, LO, HI) HAF_TRY_REG(P, Q, R, C, CP, LO, HI, true)
    if (elim) { HAF_REG_NARROW(HAF_TRY_REG_EL) }
    if (wide) { HAF_REG_WIDE(HAF_TRY_REG_H) }
    HAF_REG_NARROW(HAF_TRY_REG_H)
#undef HAF_TRY_REG_EL
#undef HAF_TRY_REG_H
#undef HAF_TRY_REG
    return hipErrorInvalidValue;
}

}  // namespace hafgpu

// Host-side launch wrappers around the kernels (each defined in the
// translation unit that instantiates its kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hafgpu {

// Per-subset coefficients (LDS-resident kernel): a_1..a_N of det(I - lambda B)
// at coef[(k-1) * cstride + i] and, for loops, l_1..l_N at coef[(N+k-1) * cstride + i],
// for subsets i = 0..count-1 (ranks rank0.. of size class m, or masks[i]).
// smax >= the largest subset size; grid = number of workgroups.
hipError_t launch_coef_lds(int smax, bool loops, int grid, hipStream_t st, const double2* A, int lda, int N,
                           int m, uint64_t rank0, int count, const uint32_t* masks, const int* d_exp, double2* coef,
                           int64_t cstride);

// Register-tiled coefficient kernel for subsets of s <= reg_max_s() rows (same
// outputs).  grid_waves bounds the number of one-wave workgroups.
hipError_t launch_coef_reg(int s, bool loops, int grid_waves, hipStream_t st, const double2* A, int lda, int N,
                           int m, uint64_t rank0, int count, const uint32_t* masks, const int* d_exp,
                           double2* coef, int64_t cstride, bool wide);
int reg_max_s();

// Exponent e of the exact input scaling (off-diagonal by 2^-2e, diagonal by
// 2^-e; the result is multiplied back by 2^(2eN)), written to *d_exp.
hipError_t launch_prescale(hipStream_t st, const double2* A, int n, int lda, int* d_exp);

// Series + signed block sums (terms == nullptr) or unsigned terms.
hipError_t launch_series(int N, bool loops, int count, hipStream_t st, const double2* coef, int64_t cstride,
                         double sign, double* partials, int64_t slot0, double2* terms, const int* d_exp);
int series_block();

hipError_t launch_reduce(hipStream_t st, const double* partials, int64_t nslots, double* out_dd, double2* out,
                         const int* d_exp, int N);
// out[perm[i]] = in[i], i < count
hipError_t launch_scatter(hipStream_t st, const double2* in, const int* perm, int count, double2* out);
hipError_t launch_write_const(hipStream_t st, double re, double* out_dd, double2* out);
hipError_t launch_pad_odd(hipStream_t st, const double2* A, int n, int lda, double2* out);

}  // namespace hafgpu

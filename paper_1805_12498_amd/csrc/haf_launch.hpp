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
// outputs).  grid_waves bounds the number of one-wave workgroups.  elim selects
// the Hessenberg reduction by elimination with exchanges (default layouts only),
// otherwise Householder reflections (wide: one wave per matrix above s = 16).
hipError_t launch_coef_reg(int s, bool loops, int grid_waves, hipStream_t st, const double2* A, int lda, int N,
                           int m, uint64_t rank0, int count, const uint32_t* masks, const int* d_exp,
                           double2* coef, int64_t cstride, bool wide, bool elim);
int reg_max_s();

// Several chunks of one matrix in one launch (each chunk: one size class m,
// ranks rank0 .. rank0 + count - 1).  Chunk c owns the workgroups
// gstart[c] .. gstart[c+1] - 1; the launch wrappers fill gstart.  Each chunk's
// coefficients sit at coef + coff[c] with stride count[c], exactly as a
// one-chunk launch would write them, and each series block of a chunk leaves its
// partial in the slot a one-chunk launch would use, so the results are bitwise
// those of one launch per chunk.
constexpr int kMultiMax = 16;
struct MultiChunks {
    int nc;                              // chunks in the launch (1..kMultiMax)
    int gstart[kMultiMax + 1];
    int m[kMultiMax];
    int count[kMultiMax];
    int64_t coff[kMultiMax];             // offset of the chunk's coefficients (complex values)
    uint64_t rank0[kMultiMax];
    int64_t slot0[kMultiMax];            // first partial slot (series)
    double sign[kMultiMax];              // (-1)^(N - m) (series)
};
// Register-tiled coefficients of several chunks whose sizes s = 2m all fall in
// the range of one default layout (s_max names it).
hipError_t launch_coef_reg_multi(int s_max, bool loops, int grid_waves, hipStream_t st, const double2* A, int lda,
                                 int N, const int* d_exp, double2* coef, MultiChunks mc);
// Index of the default layout that serves subsets of s rows (-1 above the table).
int reg_layout_index(int s);
// Series + signed block partials of several chunks (N <= 16).
hipError_t launch_series_multi(int N, bool loops, hipStream_t st, const double2* coef, double* partials,
                               MultiChunks mc);

// Same-size matrices of a batch in shared launches.  Matrix j of a group is
// items[j]; chunk c of a launch covers subsets 0..count-1 of size class m of
// matrix `item` (N <= 16: one chunk per class), owns the workgroups gstart ..
// (next chunk's gstart or the grid) - 1, keeps its coefficients at coef + coff
// (stride count) and, for the series, writes partial slots slot, slot + 1, ...
// Every matrix's coefficients, partial slots and reduction are those of the
// single-matrix path, so its result is bitwise the same.
struct GroupItem {
    const double2* A;                    // matrix the kernels read (the dense copy for odd-n loop hafnians)
    const double2* src;                  // caller's matrix; the prologue pads it into A when they differ
    double2* out;                        // result
    int n, lda, src_n, src_lda;
    int64_t slot_base;                   // the matrix's first partial slot
    int64_t nslots;                      // its partial slots
};
struct GroupChunk {
    int item, m, count, gstart;
    int64_t coff, slot;
    double sign;                         // (-1)^(N - m)
};
// One workgroup per matrix: pad odd-n loop hafnians into A, exponent of the
// exact input scaling into exps[j] (as the prescale kernel computes it).
hipError_t launch_group_prologue(hipStream_t st, const GroupItem* items, int nitems, int* exps);
// Coefficients of the chunks of one launch (all s = 2m in the range of the
// default layout named by s_max); blocks = the launch's grid, as planned by the
// host with group_coef_blocks.
int group_coef_blocks(int s_max, int count);
hipError_t launch_coef_reg_group(int s_max, bool loops, int blocks, hipStream_t st, const GroupItem* items,
                                 const GroupChunk* chunks, int nchunks, int N, const int* exps, double2* coef);
// Series + signed block partials of the chunks of one launch (N <= 16).
int group_series_blocks(int count);
hipError_t launch_series_group(int N, bool loops, int blocks, hipStream_t st, const GroupChunk* chunks, int nchunks,
                               const double2* coef, double* partials);
// One workgroup per matrix: its partials reduced as the single-matrix path does.
hipError_t launch_reduce_group(hipStream_t st, const GroupItem* items, int nitems, const double* partials,
                               const int* exps, int N);

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
// B = [[0, W], [W^T, 0]] (2n x 2n, dense) from the n x n matrix W (leading dimension ldw).
hipError_t launch_bipartite(hipStream_t st, const double2* W, int n, int ldw, double2* B);

}  // namespace hafgpu

#include "haf_batch.hpp"

namespace hafgpu {

// Persistent batched kernel.  Variants (layout table, waves per SIMD, series
// bound): 0 = (0, 2, 16), 1 = (1, 2, 16), 2 = (2, 1, 24), 3 = (0, 1, 16),
// 4 = (0, 2, 24), 5 = (1, 2, 24), 6 = (0, 1, 24).  Table 0: the default layouts
// up to s = 32; 1: one wave per matrix above s = 16, up to 32; 2: s = 34..48.
int batch_group_count(int table, int s);       // matrices per wave of table's layout for s rows
int batch_variant_table(int v);
int batch_variant_nmax(int v);
int batch_coef_per_wave(int v);                // coefficient scratch per wave (complex values)
int batch_waves_per_cu(int v);                 // resident one-wave workgroups per CU
const void* batched_kernel16(int v);
bool launch_batched16(int v, int grid, hipStream_t st, const BatchItem* items, const BatchClass* classes, int ncls,
                      int nchunks, int* cursor, int* done, const int* exps, double* partials, double2* coefscr);
hipError_t launch_batch_prologue(hipStream_t st, const BatchItem* items, const int* new_items, int nnew, int* exps,
                                 int* done, int* cursor);
hipError_t launch_batched(int v, int grid, hipStream_t st, const BatchItem* items, const BatchClass* classes,
                          int ncls, int nchunks, int* cursor, int* done, const int* exps, double* partials,
                          double2* coefscr);

}  // namespace hafgpu

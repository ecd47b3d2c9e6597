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
// outputs).  cus is the device's compute-unit count; the launch sizes its grid
// of one-wave workgroups from it and the kernel's occupancy.
hipError_t launch_coef_reg(int s, bool loops, int cus, hipStream_t st, const double2* A, int lda, int N,
                           int m, uint64_t rank0, int count, const uint32_t* masks, const int* d_exp,
                           double2* coef, int64_t cstride);
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

// Matrices of a batch in shared launches (any mix of sizes n <= 32 after the
// odd-n padding).  Chunk c of a launch covers subsets rank0 .. rank0 + count - 1
// of size class m of matrix `item` (which has N pairs), owns the workgroups
// gstart .. (next chunk's gstart or the grid) - 1, keeps its coefficients at
// coef + coff (stride count) and, for the series, writes partial slots slot,
// slot + 1, ...  Every matrix's coefficients, partial slots and reduction are
// those of the single-matrix path, so its result is bitwise the same.
constexpr int kGroupComputed = -1;       // GroupItem::cval of a matrix the kernels compute
constexpr int kGroupConstZero = 0;       // haf of odd n
constexpr int kGroupConstOne = 1;        // n = 0
struct GroupItem {
    const double2* A;                    // matrix the kernels read (the dense copy for odd-n loop hafnians)
    const double2* src;                  // caller's matrix; the prologue pads it into A when they differ
    double2* out;                        // result, or null
    double* out_dd;                      // double-double result (re_hi, re_lo, im_hi, im_lo), or null
    int n, lda, src_n, src_lda;
    int cval, pad_;                      // kGroupComputed, or the constant result the prologue writes
    int* exp;                            // exponent of the matrix's exact input scaling (the prologue writes it)
    int64_t slot_base;                   // the matrix's first partial slot
    int64_t nslots;                      // its partial slots
};
struct GroupChunk {
    int item, m, count, gstart;
    int N, pad_;
    uint64_t rank0;
    int64_t coff, slot;
    double sign;                         // (-1)^(N - m)
};
// One workgroup per matrix: write constant results, pad odd-n loop hafnians
// into A, exponent of the exact input scaling into *exp (as the prescale
// kernel computes it).
hipError_t launch_group_prologue(hipStream_t st, const GroupItem* items, int nitems);
// Coefficients of the chunks of one launch, all served by register layout
// `layout` (an index into the layout table; every chunk's s = 2m must lie in
// the layout's range (SM - 8, SM]); blocks = the launch's grid, as planned by
// the host with group_coef_blocks.
int reg_layout_count();
int reg_layout_sm(int layout);           // largest s of the layout
int reg_layout_groups(int layout);       // matrices per wave
int reg_layout_family(int layout);       // (P, Q, CP) packed: layouts of one family agree bit for bit
int group_coef_blocks(int layout, int count, int span);
hipError_t launch_coef_reg_group(int layout, bool loops, int blocks, hipStream_t st, const GroupItem* items,
                                 const GroupChunk* chunks, int nchunks, double2* coef);
// Series + signed block partials of the chunks of one launch (every N <= nmax <= 32).
int group_series_blocks(int count);
hipError_t launch_series_group(bool loops, int nmax, int blocks, hipStream_t st, const GroupChunk* chunks,
                               int nchunks, const double2* coef, double* partials);
// One workgroup per matrix: its partials reduced as the single-matrix path does.
hipError_t launch_reduce_group(hipStream_t st, const GroupItem* items, int nitems, const double* partials);

// Per-term double-double mode: coefficients of det(I - lambda B) (and loop
// moments) as complex double-double, hi parts at coef[(k-1) cstride + i] and lo
// parts at coef[lo_plane + (k-1) cstride + i]; then series and signed
// double-double block partials (slots slot0 + b).
hipError_t launch_coef_dd(int s, bool loops, int grid, hipStream_t st, const double2* A, int lda, int N, int m,
                          uint64_t rank0, int count, const int* d_exp, double2* coef, int64_t cstride,
                          int64_t lo_plane);
hipError_t launch_series_dd(bool loops, int count, int N, double sign, hipStream_t st, const double2* coef,
                            int64_t cstride, int64_t lo_plane, double* partials, int64_t slot0);

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


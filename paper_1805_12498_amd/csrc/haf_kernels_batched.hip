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
//
// This unit: the prologue, the variants with series bound 16 and the dispatch.
#include "haf_batched_kernel.hpp"
#include "haf_launch.hpp"

namespace hafgpu {

#define HAF_INST_BATCH(V, T, WPE, NM)                                                                          \
    template __global__ void k_batched<T, WPE, NM>(const BatchItem*, const BatchClass*, int, int, int*, int*,  \
                                                   const int*, double*, double2*);
HAF_BATCH_VARIANTS16(HAF_INST_BATCH)

const void* batched_kernel16(int v) {
#define HAF_KPTR(V, T, WPE, NM) if (v == V) return (const void*)k_batched<T, WPE, NM>;
    HAF_BATCH_VARIANTS16(HAF_KPTR)
#undef HAF_KPTR
    return nullptr;
}

bool launch_batched16(int v, int grid, hipStream_t st, const BatchItem* items, const BatchClass* classes, int ncls,
                      int nchunks, int* cursor, int* done, const int* exps, double* partials, double2* coefscr) {
#define HAF_KLAUNCH(V, T, WPE, NM)                                                                             \
    if (v == V) {                                                                                              \
        hipLaunchKernelGGL((k_batched<T, WPE, NM>), dim3(grid), dim3(64), 0, st, items, classes, ncls,         \
                           nchunks, cursor, done, exps, partials, coefscr);                                    \
        return true;                                                                                           \
    }
    HAF_BATCH_VARIANTS16(HAF_KLAUNCH)
#undef HAF_KLAUNCH
    return false;
}

// Matrices per wave of the layout that table t uses for subsets of s rows.
int batch_group_count(int t, int s) {
    if (t == 0) { HAF_BATCH_T0(HAF_W_OF) }
    if (t == 1) { HAF_BATCH_T1(HAF_W_OF) }
    if (t == 2) { HAF_BATCH_T2(HAF_W_OF) }
    return 0;
}

int batch_variant_table(int v) { return (v == 1 || v == 5) ? 1 : (v == 2 ? 2 : 0); }
int batch_variant_nmax(int v) { return (v == 0 || v == 1 || v == 3) ? 16 : 24; }
int batch_coef_per_wave(int v) { return kBatchMaxCap * 2 * batch_variant_nmax(v); }

const void* batched_kernel24(int v);
bool launch_batched24(int v, int grid, hipStream_t st, const BatchItem* items, const BatchClass* classes, int ncls,
                      int nchunks, int* cursor, int* done, const int* exps, double* partials, double2* coefscr);

int batch_waves_per_cu(int v) {
    int blocks = 0;
    const void* k = batched_kernel16(v);
    if (!k) k = batched_kernel24(v);
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, 64, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks > 0 ? blocks : 1;
}

// One block per item listed in new_items (block 0 also resets the two chunk
// counters, one per launch of a batch): constant results are written, odd-n loop hafnians are padded into
// their dense copy, and the exponent e of the exact input scaling (from the
// largest |Re|, |Im| of an off-diagonal entry f: e = floor(ilogb(f) / 2)) and
// the item's completion counter are set.
__global__ __launch_bounds__(256) void k_batch_prologue(const BatchItem* __restrict__ items,
                                                        const int* __restrict__ new_items, int nnew,
                                                        int* __restrict__ exps, int* __restrict__ done,
                                                        int* __restrict__ cursor) {
    if (blockIdx.x == 0 && threadIdx.x < 2) cursor[threadIdx.x] = 0;
    if ((int)blockIdx.x >= nnew) return;
    const int t = new_items[blockIdx.x];
    const BatchItem it = items[t];
    if (it.kind == kItemExternal) return;
    if (it.kind != kItemComputed) {
        if (threadIdx.x == 0) {
            const double v = it.kind == kItemOne ? 1.0 : 0.0;
            if (it.out) *it.out = make_double2(v, 0.0);
            if (it.out_dd) { it.out_dd[0] = v; it.out_dd[1] = 0.0; it.out_dd[2] = 0.0; it.out_dd[3] = 0.0; }
            exps[t] = 0;
            done[t] = 0;
        }
        return;
    }
    if (it.src != it.A) {                      // pad with an isolated vertex of loop weight 1
        double2* dst = const_cast<double2*>(it.A);
        for (int e = threadIdx.x; e < it.n * it.n; e += blockDim.x) {
            const int i = e / it.n, j = e % it.n;
            double2 v = cz();
            if (i < it.src_n && j < it.src_n) v = it.src[(int64_t)i * it.src_lda + j];
            else if (i == it.src_n && j == it.src_n) v = cone();
            dst[(int64_t)i * it.lda + j] = v;
        }
    }
    __shared__ double sh[256];
    double f = 0.0;
    for (int e = threadIdx.x; e < it.src_n * it.src_n; e += blockDim.x) {
        const int i = e / it.src_n, j = e % it.src_n;
        if (i != j) {
            const double2 v = it.src[(int64_t)i * it.src_lda + j];
            f = fmax(f, fmax(fabs(v.x), fabs(v.y)));
        }
    }
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = sh[0];
        int e = 0;
        if (m > 0.0 && m <= 1.7e308) e = ilogb(m) >> 1;
        exps[t] = e;
        done[t] = 0;
    }
}

hipError_t launch_batch_prologue(hipStream_t st, const BatchItem* items, const int* new_items, int nnew, int* exps,
                                 int* done, int* cursor) {
    const int grid = nnew > 0 ? nnew : 1;
    hipLaunchKernelGGL(k_batch_prologue, dim3(grid), dim3(256), 0, st, items, new_items, nnew, exps, done, cursor);
    return hipGetLastError();
}

hipError_t launch_batched(int v, int grid, hipStream_t st, const BatchItem* items, const BatchClass* classes,
                          int ncls, int nchunks, int* cursor, int* done, const int* exps, double* partials,
                          double2* coefscr) {
    if (nchunks <= 0) return hipSuccess;
    if (!launch_batched16(v, grid, st, items, classes, ncls, nchunks, cursor, done, exps, partials, coefscr) &&
        !launch_batched24(v, grid, st, items, classes, ncls, nchunks, cursor, done, exps, partials, coefscr))
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace hafgpu

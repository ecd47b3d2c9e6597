// Instantiations of the persistent batched kernel (series bound 24) and
// their launch wrappers.
#include "haf_batched_kernel.hpp"
#include "haf_launch.hpp"

namespace hafgpu {

#define HAF_INST_BATCH(V, T, WPE, NM)                                                                          \
    template __global__ void k_batched<T, WPE, NM>(const BatchItem*, const BatchClass*, int, int, int*, int*,  \
                                                   const int*, double*, double2*);
HAF_BATCH_VARIANTS24(HAF_INST_BATCH)

const void* batched_kernel24(int v) {
#define HAF_KPTR(V, T, WPE, NM) if (v == V) return (const void*)k_batched<T, WPE, NM>;
    HAF_BATCH_VARIANTS24(HAF_KPTR)
#undef HAF_KPTR
    return nullptr;
}

bool launch_batched24(int v, int grid, hipStream_t st, const BatchItem* items, const BatchClass* classes, int ncls,
                      int nchunks, int* cursor, int* done, const int* exps, double* partials, double2* coefscr) {
#define HAF_KLAUNCH(V, T, WPE, NM)                                                                             \
    if (v == V) {                                                                                              \
        hipLaunchKernelGGL((k_batched<T, WPE, NM>), dim3(grid), dim3(64), 0, st, items, classes, ncls,         \
                           nchunks, cursor, done, exps, partials, coefscr);                                    \
        return true;                                                                                           \
    }
    HAF_BATCH_VARIANTS24(HAF_KLAUNCH)
#undef HAF_KLAUNCH
    return false;
}

}  // namespace hafgpu

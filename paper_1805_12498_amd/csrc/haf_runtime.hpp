// Internal host-side interfaces shared by the runtime, batched and serving code.
#pragma once
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "hafgpu.h"

namespace hafgpu {

constexpr int64_t kChunk = 1 << 20;   // subsets per coefficient launch

struct Chunk {
    int m;            // subset size |Z|
    uint64_t rank0;   // first rank within the size class
    int count;        // subsets in the chunk
    int64_t slot0;    // first partial slot
    int64_t nslots;   // series blocks = partial slots
};

struct Plan {
    int n, N, kind, ncoef;
    int64_t max_chunk, nslots;
    std::vector<Chunk> chunks;
};

struct Workspace {
    double2* coef = nullptr; size_t coef_cap = 0;   // per-subset coefficients
    double* part = nullptr; size_t part_cap = 0;    // double-double partial slots
    void* aux = nullptr; size_t aux_cap = 0;        // small scratch
    double2* pad = nullptr; size_t pad_cap = 0;     // padded odd-n matrix
    void* in = nullptr; size_t in_cap = 0;          // uploaded host matrix + result
    double2* emb = nullptr; size_t emb_cap = 0;     // bipartite embedding of a permanent's matrix
};

int set_error(int code, const char* fmt, ...);
void clear_error();
const char* last_error();
int kernel_path();

uint64_t binom(int a, int b);
Plan make_plan(int n, int kind, int64_t chunk);
int ensure_device(int* dev_out);
int device_cus(int dev);
int workspace_for(hipStream_t st, Workspace** out);
int workspace_reserve(Workspace* w, hipStream_t st, size_t coef_bytes, size_t part_bytes, size_t aux_bytes);
int check_dims(const void* p, int n, int lda, int kind);
int check_values(const haf_cplx* A, int n, int lda);
int launch_coef_chunk(int dev, const double2* dA, int lda, int N, int m, uint64_t rank0, int count,
                      const uint32_t* masks, bool loops, const int* d_exp, double2* coef, int64_t cstride,
                      hipStream_t st);
int run_dev(const double2* dA, int n, int lda, int kind, double* out_dd, double2* out, hipStream_t st,
            int prec = 0);   // prec 1: every step of each term in double-double
double now_seconds();
int grow(void** p, size_t* cap, size_t need, hipStream_t st);   // (re)allocate device memory, 1.25x headroom
int hip_check(hipError_t e, const char* what);
int prof_begin(hipStream_t st, int what, double flops, int64_t subsets);
void prof_end(int idx, hipStream_t st);
double coef_model_flops(int s, int N, bool loops);
void release_batch_workspaces();
void release_stream_workspace(hipStream_t st);   // free the workspace kept for one stream (current device)
int noalloc_setup(int dev);   // device address of the allocation-free entry point's scratch array
int batched_load_cache(bool quiet);   // batched configuration from HAF_AUTOTUNE_CACHE, if it has this device

// A named range of host work for rocprofv3's marker trace (a no-op without a tool attached).
struct HostRange {
    explicit HostRange(const char* what) { roctxRangePushA(what); }
    ~HostRange() { roctxRangePop(); }
    HostRange(const HostRange&) = delete;
    HostRange& operator=(const HostRange&) = delete;
};

}  // namespace hafgpu

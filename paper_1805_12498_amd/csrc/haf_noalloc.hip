// The allocation-free variant of the device entry point: the same launch
// sequence as haf_c128x2_dev, with every work buffer (exponent, padded odd-n
// matrix, partial slots, per-subset coefficients) carved from one fixed array
// in device memory instead of the per-stream workspaces.  Nothing here calls
// hipMalloc, hipFree or any other allocating routine, and the plan is walked
// on the fly instead of being stored, so a caller under stream capture or in a
// loop that must not allocate can use it.
//
// The array is a file-scope __device__ variable: each device that loads the
// library holds its own copy until the process ends.  Host code never takes
// its address directly (that would be a host-side stand-in); the device address
// is looked up once per device with hipGetSymbolAddress and kept.
//
// Chunks of a size class are cut at multiples of the 256-subset series block,
// so every series block covers the subsets it covers in the ordinary path and
// the partial slots come out in the same order: results are bitwise those of
// haf_c128x2_dev.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "haf_launch.hpp"
#include "haf_runtime.hpp"

namespace hafgpu {

constexpr size_t kScratchExp = 256;                          // exponent of the input scaling
constexpr size_t kScratchPad = 64 * 64 * sizeof(double2);    // padded odd-n matrix (n + 1 <= 64)
constexpr size_t kScratchPart = size_t(36) << 20;            // double-double partial slots
constexpr size_t kScratchCoef = size_t(44) << 20;            // per-subset coefficients
constexpr size_t kScratchBytes = kScratchExp + kScratchPad + kScratchPart + kScratchCoef;

static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static char* g_scratch_ptr[64];                              // device address of `scratch`, per device

// Look up (once per device, with that device current) the device address of
// the scratch array.
int noalloc_setup(int dev) {
    if (dev < 0 || dev >= 64) return set_error(HAF_E_DEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return HAF_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(HAF_E_DEVICE, "hipGetSymbolAddress of the scratch array: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
    return HAF_OK;
}

int coef_grid(int dev, int count);

// One size-class chunk: the coefficient launch (register-tiled or LDS kernel,
// chosen as the ordinary path chooses) and its series launch.
static int noalloc_chunk(int dev, const double2* dA, int lda, int N, int m, uint64_t rank0, int count, bool loops,
                         const int* d_exp, double2* coef, double* part, int64_t slot0, hipStream_t st) {
    const int s = 2 * m;
    hipError_t e;
    if (kernel_path() != 1 && s <= reg_max_s())
        e = launch_coef_reg(s, loops, device_cus(dev), st, dA, lda, N, m, rank0, count, nullptr, d_exp, coef,
                            count);
    else
        e = launch_coef_lds(s, loops, coef_grid(dev, count), st, dA, lda, N, m, rank0, count, nullptr, d_exp, coef,
                            count);
    int rc = hip_check(e, "coefficient kernel launch");
    if (rc) return rc;
    const double sign = ((N - m) & 1) ? -1.0 : 1.0;
    return hip_check(launch_series(N, loops, count, st, coef, count, sign, part, slot0, nullptr, nullptr),
                     "series kernel launch");
}

static int noalloc_run(const double2* dA, int n, int lda, int kind, double* out_dd, hipStream_t st) {
    int dev = 0;
    int rc = ensure_device(&dev);
    if (rc) return rc;
    if ((rc = noalloc_setup(dev))) return rc;
    if (n == 0) return hip_check(launch_write_const(st, 1.0, out_dd, nullptr), "write kernel launch");
    if (n % 2 == 1 && kind == HAF_KIND_HAF)
        return hip_check(launch_write_const(st, 0.0, out_dd, nullptr), "write kernel launch");
    char* base = g_scratch_ptr[dev];
    int* d_exp = (int*)base;
    double2* pad = (double2*)(base + kScratchExp);
    double* part = (double*)(base + kScratchExp + kScratchPad);
    double2* coef = (double2*)(base + kScratchExp + kScratchPad + kScratchPart);
    if (n % 2 == 1) {                          // odd-n loop hafnian: lhaf(A (+) [1])
        if ((rc = hip_check(launch_pad_odd(st, dA, n, lda, pad), "pad kernel launch"))) return rc;
        dA = pad;
        n += 1;
        lda = n;
    }
    const int N = n / 2;
    const bool loops = kind == HAF_KIND_LHAF;
    const int ncoef = loops ? 2 * N : N;
    const int sb = series_block();
    const int64_t coef_cap = (int64_t)(kScratchCoef / sizeof(double2));
    const int64_t slot_cap = (int64_t)(kScratchPart / (4 * sizeof(double)));
    // chunk size: the ordinary one, cut to the coefficient area at a multiple of the series block
    int64_t chunk = std::min<int64_t>(kChunk, coef_cap / ncoef);
    chunk -= chunk % sb;
    if (chunk < sb) return set_error(HAF_E_TOO_LARGE, "n = %d: the scratch array holds too few coefficients", n);
    // partial slots of the plan (a chunk of `chunk` ranks is a whole number of series blocks)
    int64_t nslots = 0, total_coef = 0;
    for (int m = 1; m <= N; ++m) {
        const uint64_t cnt = binom(N, m);
        nslots += (int64_t)((cnt + sb - 1) / sb);
        total_coef += (int64_t)cnt * ncoef;
    }
    if (nslots > slot_cap)
        return set_error(HAF_E_TOO_LARGE, "n = %d needs %lld partial slots, the scratch array holds %lld", n,
                         (long long)nslots, (long long)slot_cap);
    if ((rc = hip_check(launch_prescale(st, dA, n, lda, d_exp), "prescale kernel launch"))) return rc;

    if (kernel_path() == 0 && N <= 16 && N <= kMultiMax && total_coef <= coef_cap) {
        // all classes resident: one coefficient launch per run of classes that share a
        // layout, one series launch (as the ordinary path does for N <= 16)
        int64_t coff[kMultiMax + 1];
        int64_t slot0[kMultiMax + 1];
        coff[0] = 0;
        slot0[0] = 0;
        for (int m = 1; m <= N; ++m) {
            const int64_t cnt = (int64_t)binom(N, m);
            coff[m] = coff[m - 1] + cnt * ncoef;
            slot0[m] = slot0[m - 1] + (cnt + sb - 1) / sb;
        }
        for (int m0 = 1; m0 <= N;) {
            const int lay = reg_layout_index(2 * m0);
            MultiChunks mc{};
            int m1 = m0;
            for (; m1 <= N && reg_layout_index(2 * m1) == lay; ++m1) {
                const int k = mc.nc++;
                mc.m[k] = m1;
                mc.count[k] = (int)binom(N, m1);
                mc.coff[k] = coff[m1 - 1];
                mc.rank0[k] = 0;
            }
            if ((rc = hip_check(launch_coef_reg_multi(2 * (m1 - 1), loops, device_cus(dev) * 16, st, dA, lda, N, d_exp,
                                                      coef, mc),
                                "coefficient kernel launch")))
                return rc;
            m0 = m1;
        }
        MultiChunks ms{};
        for (int m = 1; m <= N; ++m) {
            const int k = ms.nc++;
            ms.m[k] = m;
            ms.count[k] = (int)binom(N, m);
            ms.coff[k] = coff[m - 1];
            ms.slot0[k] = slot0[m - 1];
            ms.sign[k] = ((N - m) & 1) ? -1.0 : 1.0;
        }
        if ((rc = hip_check(launch_series_multi(N, loops, st, coef, part, ms), "series kernel launch"))) return rc;
    } else {
        int64_t slot = 0;
        for (int m = 1; m <= N; ++m) {
            const uint64_t cnt = binom(N, m);
            for (uint64_t r0 = 0; r0 < cnt; r0 += (uint64_t)chunk) {
                const int count = (int)std::min<uint64_t>((uint64_t)chunk, cnt - r0);
                if ((rc = noalloc_chunk(dev, dA, lda, N, m, r0, count, loops, d_exp, coef, part, slot, st)))
                    return rc;
                slot += (count + sb - 1) / sb;
            }
        }
    }
    return hip_check(launch_reduce(st, part, nslots, out_dd, nullptr, d_exp, N), "reduce kernel launch");
}

}  // namespace hafgpu

using namespace hafgpu;

extern "C" int haf_c128x2_dev_noalloc(const haf_cplx* dA, int n, int lda, int kind, haf_cplx2* d_out,
                                      void* stream) {
    clear_error();
    int rc = check_dims(dA, n, lda, kind);
    if (rc) return rc;
    if (!d_out) return set_error(HAF_E_INVALID_ARG, "null output");
    return noalloc_run((const double2*)dA, n, lda, kind, (double*)d_out, (hipStream_t)stream);
}

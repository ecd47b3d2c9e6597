// Host runtime behind the C ABI: argument checks, the plan over size classes,
// per-(device, stream) workspaces, and the launch sequence of one hafnian.
//
// Plan of one hafnian (Sec. 3.2, Eq. Pset): the 2^N - 1 nonempty subsets are
// grouped by size m = |Z| (all subsets of a class share s = 2m and the sign
// (-1)^(N-m)); each class is cut into chunks of at most kChunk ranks.  A chunk
// is one coefficient launch (Hessenberg + characteristic polynomial per subset)
// followed by one series launch that leaves one double-double partial per
// series block in a fixed slot.  A final one-block launch folds the slots in
// slot order.  The chunking depends only on n, so results are bitwise
// reproducible run to run.
#include "haf_runtime.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "haf_launch.hpp"
#include "hafgpu.h"

namespace hafgpu {

static thread_local std::string g_err;
// HAF_KERNEL_PATH (0, 1 or 2) selects the initial kernel path
static int initial_kernel_path() {
    const char* e = std::getenv("HAF_KERNEL_PATH");
    const int p = e ? std::atoi(e) : 0;
    return (p >= 0 && p <= 2) ? p : 0;
}
static int g_kernel_path = initial_kernel_path();

static bool debug_enabled() {
    static const bool on = [] {
        const char* e = std::getenv("HAF_DEBUG");
        return e && *e && std::strcmp(e, "0") != 0;
    }();
    return on;
}

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    if (debug_enabled()) std::fprintf(stderr, "hafgpu: error %d: %s\n", code, buf);
    return code;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }
int kernel_path() { return g_kernel_path; }
void set_kernel_path(int p) { g_kernel_path = p; }

uint64_t binom(int a, int b) {
    if (b < 0 || b > a) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= b; ++i) r = r * (uint64_t)(a - b + i) / (uint64_t)i;
    return r;
}

Plan make_plan(int n, int kind, int64_t chunk) {
    Plan p;
    p.n = n;
    p.N = n / 2;
    p.kind = kind;
    p.ncoef = kind == HAF_KIND_LHAF ? 2 * p.N : p.N;
    p.max_chunk = 0;
    int64_t slot = 0;
    const int sb = series_block();
    for (int m = 1; m <= p.N; ++m) {
        const uint64_t cnt = binom(p.N, m);
        for (uint64_t r0 = 0; r0 < cnt; r0 += (uint64_t)chunk) {
            Chunk c;
            c.m = m;
            c.rank0 = r0;
            c.count = (int)std::min<uint64_t>((uint64_t)chunk, cnt - r0);
            c.slot0 = slot;
            c.nslots = (c.count + sb - 1) / sb;
            slot += c.nslots;
            p.max_chunk = std::max<int64_t>(p.max_chunk, c.count);
            p.chunks.push_back(c);
        }
    }
    p.nslots = slot;
    return p;
}

// ------------------------------------------------------------------ devices
struct DeviceState {
    std::mutex mu;
    bool ready = false;
    int cus = 0;
    size_t lds_per_block = 0;
    std::string name;
    std::map<hipStream_t, Workspace*> ws;
};
static std::mutex g_dev_mu;
static DeviceState* g_dev[64];

static DeviceState* device_state(int dev) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (dev < 0 || dev >= 64) return nullptr;
    if (!g_dev[dev]) g_dev[dev] = new DeviceState();
    return g_dev[dev];
}

int ensure_device(int* dev_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(HAF_E_DEVICE, "hipGetDevice failed (no GPU?)");
    DeviceState* ds = device_state(dev);
    if (!ds) return set_error(HAF_E_DEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(ds->mu);
    if (!ds->ready) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return set_error(HAF_E_DEVICE, "hipGetDeviceProperties failed on device %d", dev);
        ds->cus = prop.multiProcessorCount;
        ds->lds_per_block = prop.sharedMemPerBlock;
        ds->name = prop.gcnArchName;
        ds->ready = true;
    }
    if (dev_out) *dev_out = dev;
    return HAF_OK;
}

int device_cus(int dev) {
    DeviceState* ds = device_state(dev);
    return ds && ds->cus > 0 ? ds->cus : 256;
}

std::string device_description() {
    int dev = 0;
    if (ensure_device(&dev) != HAF_OK) return std::string("no device: ") + g_err;
    DeviceState* ds = device_state(dev);
    char buf[256];
    snprintf(buf, sizeof buf, "device %d arch %s CUs %d lds/block %zu kernel_path %d", dev, ds->name.c_str(),
             ds->cus, ds->lds_per_block, g_kernel_path);
    return buf;
}

int grow(void** p, size_t* cap, size_t need, hipStream_t st) {
    if (need <= *cap) return HAF_OK;
    if (*p) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(*p);
        *p = nullptr;
        *cap = 0;
    }
    size_t sz = need + need / 4;
    if (hipMalloc(p, sz) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(HAF_E_NOMEM, "hipMalloc of %zu bytes failed", sz);
    }
    *cap = sz;
    return HAF_OK;
}

int workspace_for(hipStream_t st, Workspace** out) {
    int dev = 0;
    int rc = ensure_device(&dev);
    if (rc) return rc;
    DeviceState* ds = device_state(dev);
    std::lock_guard<std::mutex> lk(ds->mu);
    Workspace*& w = ds->ws[st];
    if (!w) w = new Workspace();
    *out = w;
    return HAF_OK;
}

int workspace_reserve(Workspace* w, hipStream_t st, size_t coef_bytes, size_t part_bytes, size_t aux_bytes) {
    int rc;
    if ((rc = grow((void**)&w->coef, &w->coef_cap, coef_bytes, st))) return rc;
    if ((rc = grow((void**)&w->part, &w->part_cap, part_bytes, st))) return rc;
    if ((rc = grow((void**)&w->aux, &w->aux_cap, aux_bytes, st))) return rc;
    return HAF_OK;
}

int release_workspaces() {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (int d = 0; d < 64; ++d) {
        DeviceState* ds = g_dev[d];
        if (!ds) continue;
        std::lock_guard<std::mutex> lk2(ds->mu);
        if (ds->ws.empty()) continue;
        (void)hipSetDevice(d);
        (void)hipDeviceSynchronize();
        for (auto& kv : ds->ws) {
            Workspace* w = kv.second;
            if (w->coef) (void)hipFree(w->coef);
            if (w->part) (void)hipFree(w->part);
            if (w->aux) (void)hipFree(w->aux);
            if (w->pad) (void)hipFree(w->pad);
            if (w->in) (void)hipFree(w->in);
            if (w->emb) (void)hipFree(w->emb);
            delete w;
        }
        ds->ws.clear();
    }
    (void)hipSetDevice(cur);
    release_batch_workspaces();
    return HAF_OK;
}

void release_stream_workspace(hipStream_t st) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    DeviceState* ds = device_state(dev);
    if (!ds) return;
    std::lock_guard<std::mutex> lk(ds->mu);
    auto it = ds->ws.find(st);
    if (it == ds->ws.end()) return;
    (void)hipStreamSynchronize(st);
    Workspace* w = it->second;
    if (w->coef) (void)hipFree(w->coef);
    if (w->part) (void)hipFree(w->part);
    if (w->aux) (void)hipFree(w->aux);
    if (w->pad) (void)hipFree(w->pad);
    if (w->in) (void)hipFree(w->in);
    if (w->emb) (void)hipFree(w->emb);
    delete w;
    ds->ws.erase(it);
}

int hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return HAF_OK;
    return set_error(HAF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------------ timing
struct ProfRec {
    hipEvent_t a, b;
    int what;           // 0 = coefficient launch, 1 = series launch, 2 = persistent batched launch
    double flops;
    int64_t subsets;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;

bool profiling() { return g_prof_on; }

// Record events around a launch when profiling; returns the record index or -1.
int prof_begin(hipStream_t st, int what, double flops, int64_t subsets) {
    if (!g_prof_on) return -1;
    ProfRec r{ nullptr, nullptr, what, flops, subsets };
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
    (void)hipEventRecord(r.a, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back(r);
    return (int)g_prof.size() - 1;
}
void prof_end(int idx, hipStream_t st) {
    if (idx < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (idx < (int)g_prof.size()) (void)hipEventRecord(g_prof[idx].b, st);
}

double coef_model_flops(int s, int N, bool loops) {
    const double sd = s;
    double f = 44.0 / 3.0 * sd * sd * sd;
    if (loops) f += 8.0 * (N - 1) * sd * sd;
    return f;
}

int coef_grid(int dev, int count) {
    const int g = device_cus(dev) * 8;
    return count < g ? count : g;
}

// Coefficient launch of one chunk of subsets that all have m pairs (s = 2m
// rows): ranks rank0.. of the size class, or the given masks.  The
// register-tiled kernel takes every s it has a layout for; the LDS kernel
// takes the rest (and everything when forced).
int launch_coef_chunk(int dev, const double2* dA, int lda, int N, int m, uint64_t rank0, int count,
                      const uint32_t* masks, bool loops, const int* d_exp, double2* coef, int64_t cstride,
                      hipStream_t st) {
    const int s = 2 * m;
    const int pidx = prof_begin(st, 0, (double)count * coef_model_flops(s, N, loops), count);
    hipError_t e;
    if (g_kernel_path != 1 && s <= reg_max_s())
        e = launch_coef_reg(s, loops, device_cus(dev), st, dA, lda, N, m, rank0, count, masks, d_exp, coef,
                            cstride);
    else
        e = launch_coef_lds(s, loops, coef_grid(dev, count), st, dA, lda, N, m, rank0, count, masks, d_exp, coef,
                            cstride);
    prof_end(pidx, st);
    return hip_check(e, "coefficient kernel launch");
}

// The same work as the per-chunk loop below, in fewer launches: chunk c's
// coefficients at coef + coff[c] (stride count[c]), partial slots as planned.
static int enqueue_haf_multi(int dev, Workspace* w, const Plan& plan, const double2* dA, int lda, bool loops,
                             double* out_dd, double2* out, hipStream_t st) {
    std::vector<int64_t> coff(plan.chunks.size());
    int64_t total = 0;
    for (size_t c = 0; c < plan.chunks.size(); ++c) {
        coff[c] = total;
        total += (int64_t)plan.chunks[c].count * plan.ncoef;
    }
    int rc = workspace_reserve(w, st, (size_t)total * sizeof(double2), (size_t)plan.nslots * 4 * sizeof(double), 64);
    if (rc) return rc;
    int* d_exp = (int*)w->aux;
    if ((rc = hip_check(launch_prescale(st, dA, plan.n, lda, d_exp), "prescale kernel launch"))) return rc;
    // coefficients: one launch per run of consecutive chunks that share a layout
    for (size_t c0 = 0; c0 < plan.chunks.size();) {
        const int lay = reg_layout_index(2 * plan.chunks[c0].m);
        MultiChunks mc{};
        double flops = 0.0;
        int64_t subsets = 0;
        size_t c1 = c0;
        for (; c1 < plan.chunks.size() && reg_layout_index(2 * plan.chunks[c1].m) == lay; ++c1) {
            const Chunk& ch = plan.chunks[c1];
            const int k = mc.nc++;
            mc.m[k] = ch.m;
            mc.count[k] = ch.count;
            mc.coff[k] = coff[c1];
            mc.rank0[k] = ch.rank0;
            flops += (double)ch.count * coef_model_flops(2 * ch.m, plan.N, loops);
            subsets += ch.count;
        }
        const int pidx = prof_begin(st, 0, flops, subsets);
        const hipError_t e = launch_coef_reg_multi(2 * plan.chunks[c1 - 1].m, loops, device_cus(dev) * 16, st, dA,
                                                   lda, plan.N, d_exp, w->coef, mc);
        prof_end(pidx, st);
        if ((rc = hip_check(e, "coefficient kernel launch"))) return rc;
        c0 = c1;
    }
    MultiChunks ms{};
    int64_t subsets = 0;
    for (size_t c = 0; c < plan.chunks.size(); ++c) {
        const Chunk& ch = plan.chunks[c];
        ms.m[c] = ch.m;
        ms.count[c] = ch.count;
        ms.coff[c] = coff[c];
        ms.slot0[c] = ch.slot0;
        ms.sign[c] = ((plan.N - ch.m) & 1) ? -1.0 : 1.0;
        subsets += ch.count;
    }
    ms.nc = (int)plan.chunks.size();
    const int pidx = prof_begin(st, 1, 0.0, subsets);
    const hipError_t e = launch_series_multi(plan.N, loops, st, w->coef, w->part, ms);
    prof_end(pidx, st);
    if ((rc = hip_check(e, "series kernel launch"))) return rc;
    return hip_check(launch_reduce(st, w->part, plan.nslots, out_dd, out, d_exp, plan.N), "reduce kernel launch");
}

constexpr int64_t kChunkDD = 1 << 18;   // subsets per launch of the double-double mode

// The per-term double-double mode: the same plan over size classes (smaller
// chunks), every coefficient and term in complex double-double, the same
// partial slots and reduction.
static int enqueue_haf_dd(int dev, Workspace* w, const double2* dA, int n, int lda, int kind, double* out_dd,
                          double2* out, hipStream_t st) {
    const Plan plan = make_plan(n, kind, kChunkDD);
    const bool loops = kind == HAF_KIND_LHAF;
    const int64_t lo_plane = plan.max_chunk * plan.ncoef;
    int rc = workspace_reserve(w, st, (size_t)(2 * lo_plane) * sizeof(double2), (size_t)plan.nslots * 4 * sizeof(double),
                               64);
    if (rc) return rc;
    int* d_exp = (int*)w->aux;
    if ((rc = hip_check(launch_prescale(st, dA, n, lda, d_exp), "prescale kernel launch"))) return rc;
    for (const Chunk& c : plan.chunks) {
        const int pidx = prof_begin(st, 0, (double)c.count * coef_model_flops(2 * c.m, plan.N, loops), c.count);
        rc = hip_check(launch_coef_dd(2 * c.m, loops, coef_grid(dev, c.count), st, dA, lda, plan.N, c.m, c.rank0,
                                      c.count, d_exp, w->coef, c.count, lo_plane),
                       "double-double coefficient kernel launch");
        prof_end(pidx, st);
        if (rc) return rc;
        const double sign = ((plan.N - c.m) & 1) ? -1.0 : 1.0;
        if ((rc = hip_check(launch_series_dd(loops, c.count, plan.N, sign, st, w->coef, c.count, lo_plane, w->part,
                                             c.slot0),
                            "double-double series kernel launch")))
            return rc;
    }
    return hip_check(launch_reduce(st, w->part, plan.nslots, out_dd, out, d_exp, plan.N), "reduce kernel launch");
}

// Enqueue one hafnian of an n x n device matrix (n even, 2 <= n <= 64).
int enqueue_haf(const double2* dA, int n, int lda, int kind, double* out_dd, double2* out, hipStream_t st,
                int prec = 0) {
    int dev = 0;
    int rc = ensure_device(&dev);
    if (rc) return rc;
    Workspace* w = nullptr;
    if ((rc = workspace_for(st, &w))) return rc;
    if (prec == 1) return enqueue_haf_dd(dev, w, dA, n, lda, kind, out_dd, out, st);
    const Plan plan = make_plan(n, kind, kChunk);
    const bool loops = kind == HAF_KIND_LHAF;
    // Small matrices (N <= 16, one chunk per size class) on the default path: all
    // coefficients stay resident, one launch per layout and one series launch
    // replace a launch pair per size class (launch overhead dominates there)
    if (g_kernel_path == 0 && plan.N <= 16 && (int)plan.chunks.size() <= kMultiMax)
        return enqueue_haf_multi(dev, w, plan, dA, lda, loops, out_dd, out, st);
    const size_t coef_bytes = (size_t)plan.max_chunk * plan.ncoef * sizeof(double2);
    const size_t part_bytes = (size_t)plan.nslots * 4 * sizeof(double);
    if ((rc = workspace_reserve(w, st, coef_bytes, part_bytes, 64))) return rc;
    int* d_exp = (int*)w->aux;
    if ((rc = hip_check(launch_prescale(st, dA, n, lda, d_exp), "prescale kernel launch"))) return rc;
    for (const Chunk& c : plan.chunks) {
        if ((rc = launch_coef_chunk(dev, dA, lda, plan.N, c.m, c.rank0, c.count, nullptr, loops, d_exp, w->coef,
                                    c.count, st)))
            return rc;
        const double sign = ((plan.N - c.m) & 1) ? -1.0 : 1.0;
        const int pidx = prof_begin(st, 1, 0.0, c.count);
        rc = hip_check(launch_series(plan.N, loops, c.count, st, w->coef, c.count, sign, w->part, c.slot0, nullptr,
                                     nullptr),
                       "series kernel launch");
        prof_end(pidx, st);
        if (rc) return rc;
    }
    return hip_check(launch_reduce(st, w->part, plan.nslots, out_dd, out, d_exp, plan.N), "reduce kernel launch");
}

// Device-side entry: handles n = 0, odd n and the padding for odd-n lhaf.
int run_dev(const double2* dA, int n, int lda, int kind, double* out_dd, double2* out, hipStream_t st, int prec) {
    HostRange range("hafgpu: enqueue one matrix");
    int rc = ensure_device(nullptr);
    if (rc) return rc;
    if (n == 0) return hip_check(launch_write_const(st, 1.0, out_dd, out), "write kernel launch");
    if (n % 2 == 1) {
        if (kind == HAF_KIND_HAF) return hip_check(launch_write_const(st, 0.0, out_dd, out), "write kernel launch");
        Workspace* w = nullptr;
        if ((rc = workspace_for(st, &w))) return rc;
        const size_t need = (size_t)(n + 1) * (n + 1) * sizeof(double2);
        if ((rc = grow((void**)&w->pad, &w->pad_cap, need, st))) return rc;
        if ((rc = hip_check(launch_pad_odd(st, dA, n, lda, w->pad), "pad kernel launch"))) return rc;
        return enqueue_haf(w->pad, n + 1, n + 1, kind, out_dd, out, st, prec);
    }
    return enqueue_haf(dA, n, lda, kind, out_dd, out, st, prec);
}

int check_dims(const void* p, int n, int lda, int kind) {
    if (!p) return set_error(HAF_E_INVALID_ARG, "null pointer");
    if (n < 0) return set_error(HAF_E_INVALID_ARG, "n = %d < 0", n);
    if (n > 0 && lda < n) return set_error(HAF_E_INVALID_ARG, "lda = %d < n = %d", lda, n);
    if (kind != HAF_KIND_HAF && kind != HAF_KIND_LHAF) return set_error(HAF_E_INVALID_ARG, "unknown kind %d", kind);
    const int eff = (n % 2 == 1 && kind == HAF_KIND_LHAF) ? n + 1 : n;
    if (eff > HAF_MAX_N) return set_error(HAF_E_TOO_LARGE, "n = %d exceeds the limit %d", n, HAF_MAX_N);
    return HAF_OK;
}

int check_values(const haf_cplx* A, int n, int lda) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const haf_cplx a = A[(int64_t)i * lda + j];
            if (!std::isfinite(a.re) || !std::isfinite(a.im))
                return set_error(HAF_E_NONFINITE, "non-finite entry at (%d, %d)", i, j);
        }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const haf_cplx a = A[(int64_t)i * lda + j], b = A[(int64_t)j * lda + i];
            if (a.re != b.re || a.im != b.im)
                return set_error(HAF_E_NOT_SYMMETRIC, "A[%d][%d] != A[%d][%d]", i, j, j, i);
        }
    return HAF_OK;
}

static hipStream_t host_stream() {
    static thread_local hipStream_t s = nullptr;
    static thread_local int sdev = -1;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (!s || sdev != dev) {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
        sdev = dev;
    }
    return s;
}

int run_host(const haf_cplx* A, int n, int lda, int kind, haf_cplx2* out, int prec = 0) {
    int rc = check_dims(A, n, lda, kind);
    if (rc) return rc;
    if (!out) return set_error(HAF_E_INVALID_ARG, "null output");
    if ((rc = check_values(A, n, lda))) return rc;
    if ((rc = ensure_device(nullptr))) return rc;
    hipStream_t st = host_stream();
    if (!st) return set_error(HAF_E_DEVICE, "hipStreamCreate failed");
    Workspace* w = nullptr;
    if ((rc = workspace_for(st, &w))) return rc;
    const size_t mat = (size_t)std::max(n, 1) * std::max(n, 1) * sizeof(double2);
    if ((rc = grow((void**)&w->in, &w->in_cap, mat + 64, st))) return rc;
    double2* dA = (double2*)w->in;
    double* dout = (double*)((char*)w->in + mat);
    if (n > 0 && (rc = hip_check(hipMemcpy2DAsync(dA, (size_t)n * sizeof(double2), A, (size_t)lda * sizeof(double2),
                                                  (size_t)n * sizeof(double2), (size_t)n, hipMemcpyHostToDevice, st),
                                 "matrix upload")))
        return rc;
    if ((rc = run_dev(dA, n, n, kind, dout, nullptr, st, prec))) return rc;
    double h[4];
    if ((rc = hip_check(hipMemcpyAsync(h, dout, sizeof h, hipMemcpyDeviceToHost, st), "result download"))) return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "stream synchronize"))) return rc;
    out->re_hi = h[0];
    out->re_lo = h[1];
    out->im_hi = h[2];
    out->im_lo = h[3];
    return HAF_OK;
}

// Unsigned terms f(Z) for a list of masks.  The masks are copied to the host
// and grouped by size so every launch sees one subset size (as in the full
// sum); results are scattered back to the caller's order.
int run_terms(const double2* dA, int n, int lda, int kind, const uint32_t* d_masks, int count, double2* d_terms,
              hipStream_t st) {
    int rc = check_dims(dA, n, lda, kind);
    if (rc) return rc;
    if (!d_masks || !d_terms) return set_error(HAF_E_INVALID_ARG, "null pointer");
    if (n % 2 || n < 2) return set_error(HAF_E_INVALID_ARG, "terms need an even n >= 2");
    if (count < 0) return set_error(HAF_E_INVALID_ARG, "count < 0");
    if (count == 0) return HAF_OK;
    int dev = 0;
    if ((rc = ensure_device(&dev))) return rc;
    Workspace* w = nullptr;
    if ((rc = workspace_for(st, &w))) return rc;
    const int N = n / 2;
    const bool loops = kind == HAF_KIND_LHAF;
    const int ncoef = loops ? 2 * N : N;
    std::vector<uint32_t> hm((size_t)count);
    if ((rc = hip_check(hipMemcpyAsync(hm.data(), d_masks, sizeof(uint32_t) * count, hipMemcpyDeviceToHost, st),
                        "mask download")))
        return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "stream synchronize"))) return rc;
    std::vector<int> order((size_t)count);
    for (int i = 0; i < count; ++i) {
        if (hm[i] == 0u || (N < 32 && (hm[i] >> N) != 0u))
            return set_error(HAF_E_INVALID_ARG, "mask %d = %#x is empty or has bits beyond n/2 = %d", i, hm[i], N);
        order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return __builtin_popcount(hm[x]) < __builtin_popcount(hm[y]); });
    std::vector<uint32_t> sorted((size_t)count);
    std::vector<int> perm((size_t)count);
    for (int i = 0; i < count; ++i) { sorted[i] = hm[order[i]]; perm[i] = order[i]; }
    // aux: [exponent (256 B)] [sorted masks] [permutation] ; coef: coefficients then terms
    const size_t off_m = 256, off_p = off_m + ((sizeof(uint32_t) * count + 255) & ~(size_t)255);
    const size_t aux_need = off_p + sizeof(int) * count;
    const size_t coef_need = (size_t)count * (ncoef + 1) * sizeof(double2);
    if ((rc = workspace_reserve(w, st, coef_need, 64, aux_need))) return rc;
    int* d_exp = (int*)w->aux;
    uint32_t* d_sorted = (uint32_t*)((char*)w->aux + off_m);
    int* d_perm = (int*)((char*)w->aux + off_p);
    if ((rc = hip_check(hipMemcpyAsync(d_sorted, sorted.data(), sizeof(uint32_t) * count, hipMemcpyHostToDevice, st),
                        "mask upload")))
        return rc;
    if ((rc = hip_check(hipMemcpyAsync(d_perm, perm.data(), sizeof(int) * count, hipMemcpyHostToDevice, st),
                        "permutation upload")))
        return rc;
    if ((rc = hip_check(launch_prescale(st, dA, n, lda, d_exp), "prescale kernel launch"))) return rc;
    double2* tmp_terms = w->coef + (size_t)count * ncoef;
    for (int i0 = 0; i0 < count;) {
        const int m = __builtin_popcount(sorted[i0]);
        int i1 = i0;
        while (i1 < count && __builtin_popcount(sorted[i1]) == m) ++i1;
        const int cnt = i1 - i0;
        if ((rc = launch_coef_chunk(dev, dA, lda, N, m, 0, cnt, d_sorted + i0, loops, d_exp, w->coef + 0, cnt, st)))
            return rc;
        if ((rc = hip_check(launch_series(N, loops, cnt, st, w->coef, cnt, 1.0, nullptr, 0, tmp_terms + i0, d_exp),
                            "series kernel launch")))
            return rc;
        i0 = i1;
    }
    return hip_check(launch_scatter(st, tmp_terms, d_perm, count, d_terms), "scatter kernel launch");
}

double now_seconds() {
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace hafgpu

// ======================================================================== C ABI
using namespace hafgpu;

extern "C" {

const char* haf_last_error(void) { return last_error(); }
const char* haf_version(void) { return "hafgpu 0.1 (gfx950)"; }

int haf_init(int device) {
    clear_error();
    if (hipSetDevice(device) != hipSuccess) return set_error(HAF_E_DEVICE, "hipSetDevice(%d) failed", device);
    int rc = ensure_device(nullptr);
    if (!rc) rc = noalloc_setup(device);
    if (!rc) rc = batched_load_cache(true);
    return rc;
}

int haf_device_info(char* buf, int buflen) {
    if (!buf || buflen <= 0) return set_error(HAF_E_INVALID_ARG, "null buffer");
    std::string d = device_description();
    snprintf(buf, (size_t)buflen, "%s", d.c_str());
    return HAF_OK;
}

int haf_c128x2_host(const haf_cplx* A, int n, int lda, int kind, haf_cplx2* out) {
    clear_error();
    return run_host(A, n, lda, kind, out);
}

int haf_c128(const haf_cplx* A, int n, int lda, haf_cplx* out) {
    clear_error();
    if (!out) return set_error(HAF_E_INVALID_ARG, "null output");
    haf_cplx2 r;
    int rc = run_host(A, n, lda, HAF_KIND_HAF, &r);
    if (rc) return rc;
    out->re = r.re_hi + r.re_lo;
    out->im = r.im_hi + r.im_lo;
    return HAF_OK;
}

int lhaf_c128(const haf_cplx* A, int n, int lda, haf_cplx* out) {
    clear_error();
    if (!out) return set_error(HAF_E_INVALID_ARG, "null output");
    haf_cplx2 r;
    int rc = run_host(A, n, lda, HAF_KIND_LHAF, &r);
    if (rc) return rc;
    out->re = r.re_hi + r.re_lo;
    out->im = r.im_hi + r.im_lo;
    return HAF_OK;
}

static int dev_entry(const haf_cplx* dA, int n, int lda, int kind, double* out_dd, double2* out, void* stream) {
    clear_error();
    int rc = check_dims(dA, n, lda, kind);
    if (rc) return rc;
    if (!out_dd && !out) return set_error(HAF_E_INVALID_ARG, "null output");
    return run_dev((const double2*)dA, n, lda, kind, out_dd, out, (hipStream_t)stream);
}

int haf_c128_dev(const haf_cplx* dA, int n, int lda, haf_cplx* d_out, void* stream) {
    return dev_entry(dA, n, lda, HAF_KIND_HAF, nullptr, (double2*)d_out, stream);
}

int lhaf_c128_dev(const haf_cplx* dA, int n, int lda, haf_cplx* d_out, void* stream) {
    return dev_entry(dA, n, lda, HAF_KIND_LHAF, nullptr, (double2*)d_out, stream);
}

int haf_c128x2_dev(const haf_cplx* dA, int n, int lda, int kind, haf_cplx2* d_out, void* stream) {
    return dev_entry(dA, n, lda, kind, (double*)d_out, nullptr, stream);
}

int haf_dd_c128x2_dev(const haf_cplx* dA, int n, int lda, int kind, haf_cplx2* d_out, void* stream) {
    clear_error();
    int rc = check_dims(dA, n, lda, kind);
    if (rc) return rc;
    if (!d_out) return set_error(HAF_E_INVALID_ARG, "null output");
    return run_dev((const double2*)dA, n, lda, kind, (double*)d_out, nullptr, (hipStream_t)stream, 1);
}

int haf_dd_c128x2_host(const haf_cplx* A, int n, int lda, int kind, haf_cplx2* out) {
    clear_error();
    return run_host(A, n, lda, kind, out, 1);
}

int perm_c128(const haf_cplx* W, int n, int ldw, haf_cplx* out) {
    clear_error();
    if (!W || !out) return set_error(HAF_E_INVALID_ARG, "null pointer");
    if (n < 0) return set_error(HAF_E_INVALID_ARG, "n = %d < 0", n);
    if (n > 0 && ldw < n) return set_error(HAF_E_INVALID_ARG, "ldw = %d < n = %d", ldw, n);
    if (2 * n > HAF_MAX_N) return set_error(HAF_E_TOO_LARGE, "n = %d exceeds the limit %d", n, HAF_MAX_N / 2);
    const int m = 2 * n;
    std::vector<haf_cplx> B((size_t)std::max(m, 1) * std::max(m, 1), haf_cplx{ 0.0, 0.0 });
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const haf_cplx w = W[(int64_t)i * ldw + j];
            if (!std::isfinite(w.re) || !std::isfinite(w.im))
                return set_error(HAF_E_NONFINITE, "non-finite entry at (%d, %d)", i, j);
            B[(size_t)i * m + (n + j)] = w;
            B[(size_t)(n + j) * m + i] = w;
        }
    haf_cplx2 r;
    const int rc = run_host(B.data(), m, std::max(m, 1), HAF_KIND_HAF, &r);
    if (rc) return rc;
    out->re = r.re_hi + r.re_lo;
    out->im = r.im_hi + r.im_lo;
    return HAF_OK;
}

int perm_c128_dev(const haf_cplx* dW, int n, int ldw, haf_cplx* d_out, void* stream) {
    clear_error();
    if (!dW || !d_out) return set_error(HAF_E_INVALID_ARG, "null pointer");
    if (n < 0) return set_error(HAF_E_INVALID_ARG, "n = %d < 0", n);
    if (n > 0 && ldw < n) return set_error(HAF_E_INVALID_ARG, "ldw = %d < n = %d", ldw, n);
    if (2 * n > HAF_MAX_N) return set_error(HAF_E_TOO_LARGE, "n = %d exceeds the limit %d", n, HAF_MAX_N / 2);
    hipStream_t st = (hipStream_t)stream;
    int rc = ensure_device(nullptr);
    if (rc) return rc;
    if (n == 0) return hip_check(launch_write_const(st, 1.0, nullptr, (double2*)d_out), "write kernel launch");
    Workspace* w = nullptr;
    if ((rc = workspace_for(st, &w))) return rc;
    const int m = 2 * n;
    if ((rc = grow((void**)&w->emb, &w->emb_cap, sizeof(double2) * (size_t)m * m, st))) return rc;
    if ((rc = hip_check(launch_bipartite(st, (const double2*)dW, n, ldw, w->emb), "bipartite kernel launch")))
        return rc;
    return run_dev(w->emb, m, m, HAF_KIND_HAF, nullptr, (double2*)d_out, st);
}

int haf_terms_dev(const haf_cplx* dA, int n, int lda, int kind, const uint32_t* d_masks, int count,
                  haf_cplx* d_terms, void* stream) {
    clear_error();
    return run_terms((const double2*)dA, n, lda, kind, d_masks, count, (double2*)d_terms, (hipStream_t)stream);
}

int haf_release_workspaces(void) {
    clear_error();
    return release_workspaces();
}

int haf_set_kernel_path(int path) {
    clear_error();
    if (path < 0 || path > 2) return set_error(HAF_E_INVALID_ARG, "kernel path %d not in 0..2", path);
    set_kernel_path(path);
    return HAF_OK;
}

double haf_now(void) { return now_seconds(); }

int haf_profile_enable(int on) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (ProfRec& r : g_prof) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    g_prof_on = on != 0;
    return HAF_OK;
}

int haf_profile_read(haf_profile* out) {
    clear_error();
    if (!out) return set_error(HAF_E_INVALID_ARG, "null output");
    memset(out, 0, sizeof *out);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (ProfRec& r : g_prof) {
        if (hipEventSynchronize(r.b) != hipSuccess) return set_error(HAF_E_DEVICE, "event synchronize failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return set_error(HAF_E_DEVICE, "event time failed");
        if (r.what == 0) {
            out->coef_launches++;
            out->coef_ms += ms;
            out->coef_model_flops += r.flops;
            out->coef_subsets += r.subsets;
        } else if (r.what == 2) {
            out->batched_launches++;
            out->batched_ms += ms;
            out->batched_model_flops += r.flops;
        } else {
            out->series_launches++;
            out->series_ms += ms;
        }
    }
    return HAF_OK;
}

}  // extern "C"

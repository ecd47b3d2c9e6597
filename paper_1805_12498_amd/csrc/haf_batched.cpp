// Batched hafnians: the host planner, the workspaces, the configuration and
// autotuner, and the C ABI of the batched path.
//
// A batch is run as shared launches.  Every matrix with at most 32 rows (after
// padding an odd-n loop hafnian) contributes one chunk per subset size class m
// (Sec. 3.2, Eq. Pset: the subsets of one size share s = 2m and the sign
// (-1)^(N-m)).  The chunks are grouped into stages, one per (register layout,
// kind): a stage is one coefficient launch over the chunks of every matrix
// whose subset size that layout serves, followed by one series launch over the
// same chunks, so the coefficients of one stage are reused by the next.  One
// reduction launch per batch then folds each matrix's partial slots.  Each
// matrix keeps the single-matrix path's per-subset arithmetic (same layout
// P, Q and polynomial split for every s), its partial slots and its reduction
// order, so every result is bitwise the single-matrix result.  Matrices above
// 32 rows run the single-matrix path on up to four library streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <unistd.h>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "haf_launch.hpp"
#include "haf_runtime.hpp"

namespace hafgpu {

constexpr int kGroupMaxN = 32;        // largest matrix (after padding) that takes the shared launches
constexpr int kMaxPoolStreams = 4;    // hardware queues per process on the target

// ------------------------------------------------------------------ configuration
static std::mutex g_bcfg_mu;
static haf_batched_config g_bcfg = { 0, 4, kMaxPoolStreams, 1, 8192 };

haf_batched_config batch_config() {
    std::lock_guard<std::mutex> lk(g_bcfg_mu);
    return g_bcfg;
}

static void set_batch_config(const haf_batched_config& c) {
    std::lock_guard<std::mutex> lk(g_bcfg_mu);
    g_bcfg = c;
}

static int check_config(const haf_batched_config& c) {
    if (c.table < 0 || c.table > 1) return set_error(HAF_E_INVALID_ARG, "table %d not 0 or 1", c.table);
    if (c.span < 1 || c.span > 64) return set_error(HAF_E_INVALID_ARG, "span %d not in 1..64", c.span);
    if (c.streams < 1 || c.streams > kMaxPoolStreams)
        return set_error(HAF_E_INVALID_ARG, "streams %d not in 1..%d", c.streams, kMaxPoolStreams);
    if (c.grouped != 0 && c.grouped != 1) return set_error(HAF_E_INVALID_ARG, "grouped %d not 0 or 1", c.grouped);
    if (c.coef_budget_mb < 64 || c.coef_budget_mb > (1 << 18))
        return set_error(HAF_E_INVALID_ARG, "coef_budget_mb %d not in 64..262144", c.coef_budget_mb);
    return HAF_OK;
}

// Layout that serves subsets of s rows under table t: the single-matrix layout
// (t = 0) or the first layout of the same family (P, Q and polynomial split)
// with a multiple of 8 rows at or above s, if there is one (t = 1).  Layouts of
// one family give bitwise the same results; the coarse table has fewer stages
// and more padding.
static int stage_layout(int table, int s) {
    const int fine = reg_layout_index(s);
    if (table == 0 || fine < 0) return fine;
    for (int l = fine; l < reg_layout_count(); ++l)
        if (reg_layout_family(l) == reg_layout_family(fine) && reg_layout_sm(l) % 8 == 0) return l;
    return fine;
}

// ------------------------------------------------------------------ autotune cache
// A text file named by HAF_AUTOTUNE_CACHE, one line per device:
//   <arch>:<compute units> <table> <span> <streams> <grouped> <coef_budget_mb>
// written by the autotuner and read by haf_batched_load_cache (and haf_init).
static std::string device_key() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return std::string();
    std::string arch = p.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    return arch + ":" + std::to_string(p.multiProcessorCount);
}

static int cache_read(const char* path, const std::string& key, haf_batched_config* out, bool* found) {
    *found = false;
    std::ifstream f(path);
    if (!f) return HAF_OK;                                  // no file yet: nothing cached
    std::string line;
    for (int ln = 1; std::getline(f, line); ++ln) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string k;
        haf_batched_config c{};
        if (!(is >> k >> c.table >> c.span >> c.streams >> c.grouped >> c.coef_budget_mb))
            return set_error(HAF_E_INVALID_ARG, "%s:%d: malformed autotune cache line", path, ln);
        if (k != key) continue;
        if (check_config(c)) return set_error(HAF_E_INVALID_ARG, "%s:%d: %s", path, ln, last_error());
        *out = c;
        *found = true;
    }
    return HAF_OK;
}

static int cache_write(const char* path, const std::string& key, const haf_batched_config& c) {
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            std::istringstream is(line);
            std::string k;
            if (!line.empty() && line[0] != '#' && (is >> k) && k == key) continue;
            keep.push_back(line);
        }
    }
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream f(tmp);
        if (!f) return set_error(HAF_E_STATE, "cannot write autotune cache %s", tmp.c_str());
        for (const std::string& l : keep) f << l << "\n";
        f << key << ' ' << c.table << ' ' << c.span << ' ' << c.streams << ' ' << c.grouped << ' '
          << c.coef_budget_mb << "\n";
        if (!f) return set_error(HAF_E_STATE, "cannot write autotune cache %s", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0) return set_error(HAF_E_STATE, "cannot replace autotune cache %s", path);
    return HAF_OK;
}

int batched_load_cache(bool quiet) {
    const char* path = std::getenv("HAF_AUTOTUNE_CACHE");
    if (!path || !*path) return quiet ? HAF_OK : set_error(HAF_E_STATE, "HAF_AUTOTUNE_CACHE is not set");
    const std::string key = device_key();
    if (key.empty()) return set_error(HAF_E_DEVICE, "no current device");
    haf_batched_config c{};
    bool found = false;
    const int rc = cache_read(path, key, &c, &found);
    if (rc) return rc;
    if (!found) return quiet ? HAF_OK : set_error(HAF_E_STATE, "no entry for %s in %s", key.c_str(), path);
    set_batch_config(c);
    return HAF_OK;
}

// ------------------------------------------------------------------ planner
static int eff_n(int n, int kind) { return (n % 2 == 1 && kind == HAF_KIND_LHAF) ? n + 1 : n; }
static int constant_of(int n, int kind) {
    if (n == 0) return kGroupConstOne;
    if (n % 2 == 1 && kind == HAF_KIND_HAF) return kGroupConstZero;
    return kGroupComputed;
}
static bool groupable(int n, int kind) {
    return constant_of(n, kind) != kGroupComputed || eff_n(n, kind) <= kGroupMaxN;
}

struct StageLaunch {
    int what;            // 0 coefficients, 1 series
    int layout;
    bool loops;
    int blocks;
    size_t first;        // first chunk in GroupPlan::chunks
    int nch;
    int64_t coef_elems;  // complex values of coefficient storage the launch pair uses
    double flops;        // model flops of the coefficient launch
};

struct GroupPlan {
    std::vector<int> order;            // caller index of group item j
    std::vector<int> cval;             // kGroupComputed or the constant result
    std::vector<int> n_eff;
    std::vector<int64_t> slot_base, nslots;
    std::vector<GroupChunk> chunks;
    std::vector<StageLaunch> launches;
    int64_t coef_max = 0, slots = 0, pad_elems = 0;
};

static int plan_groups(const int32_t* ns, const uint8_t* kinds, const std::vector<int>& list,
                       const haf_batched_config& cfg, GroupPlan* gp) {
    gp->order = list;
    const int ni = (int)list.size();
    gp->cval.assign((size_t)ni, kGroupComputed);
    gp->n_eff.assign((size_t)ni, 0);
    gp->slot_base.assign((size_t)ni, 0);
    gp->nslots.assign((size_t)ni, 0);
    std::vector<Plan> plans((size_t)ni);
    for (int j = 0; j < ni; ++j) {
        const int t = list[(size_t)j];
        gp->cval[(size_t)j] = constant_of(ns[t], kinds[t]);
        gp->n_eff[(size_t)j] = eff_n(ns[t], kinds[t]);
        if (gp->cval[(size_t)j] != kGroupComputed) continue;
        if (gp->n_eff[(size_t)j] != ns[t]) gp->pad_elems += (int64_t)gp->n_eff[(size_t)j] * gp->n_eff[(size_t)j];
        plans[(size_t)j] = make_plan(gp->n_eff[(size_t)j], kinds[t], kChunk);
        gp->slot_base[(size_t)j] = gp->slots;
        gp->nslots[(size_t)j] = plans[(size_t)j].nslots;
        gp->slots += plans[(size_t)j].nslots;
    }
    const int64_t budget = (int64_t)cfg.coef_budget_mb * (1 << 20) / (int64_t)sizeof(double2);
    // stages: one per (layout, kind), larger layouts first
    for (int loops = 0; loops < 2; ++loops)
        for (int lay = reg_layout_count() - 1; lay >= 0; --lay) {
            std::vector<GroupChunk> cur;
            std::vector<int64_t> size;
            for (int j = 0; j < ni; ++j) {
                if (gp->cval[(size_t)j] != kGroupComputed) continue;
                const int t = list[(size_t)j];
                if ((kinds[t] == HAF_KIND_LHAF) != (loops == 1)) continue;
                const Plan& p = plans[(size_t)j];
                for (const Chunk& c : p.chunks) {
                    if (stage_layout(cfg.table, 2 * c.m) != lay) continue;
                    GroupChunk ch{};
                    ch.item = j;
                    ch.m = c.m;
                    ch.count = c.count;
                    ch.N = p.N;
                    ch.rank0 = c.rank0;
                    ch.slot = gp->slot_base[(size_t)j] + c.slot0;
                    ch.sign = ((p.N - c.m) & 1) ? -1.0 : 1.0;
                    cur.push_back(ch);
                    size.push_back((int64_t)c.count * p.ncoef);
                }
            }
            // cut the stage into launch pairs whose coefficients fit the budget
            for (size_t c0 = 0; c0 < cur.size();) {
                int64_t used = 0;
                size_t c1 = c0;
                while (c1 < cur.size() && (c1 == c0 || used + size[c1] <= budget)) used += size[c1++];
                StageLaunch co{ 0, lay, loops == 1, 0, gp->chunks.size(), (int)(c1 - c0), used, 0.0 };
                StageLaunch se{ 1, lay, loops == 1, 0, gp->chunks.size() + (c1 - c0), (int)(c1 - c0), used, 0.0 };
                int64_t off = 0;
                for (size_t c = c0; c < c1; ++c) {
                    cur[c].coff = off;
                    off += size[c];
                }
                for (size_t c = c0; c < c1; ++c) {
                    GroupChunk ch = cur[c];
                    ch.gstart = co.blocks;
                    co.blocks += group_coef_blocks(lay, ch.count, cfg.span);
                    co.flops += (double)ch.count * coef_model_flops(2 * ch.m, ch.N, loops == 1);
                    gp->chunks.push_back(ch);
                }
                for (size_t c = c0; c < c1; ++c) {
                    GroupChunk ch = cur[c];
                    ch.gstart = se.blocks;
                    se.blocks += group_series_blocks(ch.count);
                    gp->chunks.push_back(ch);
                }
                gp->launches.push_back(co);
                gp->launches.push_back(se);
                gp->coef_max = std::max(gp->coef_max, used);
                c0 = c1;
            }
        }
    return HAF_OK;
}

// ------------------------------------------------------------------ workspaces
struct BatchWS {
    char* dmeta = nullptr; size_t dmeta_cap = 0;   // items | chunks
    char* hmeta = nullptr; size_t hmeta_cap = 0;   // pinned staging of the same
    hipEvent_t staged = nullptr;                   // the last upload out of hmeta
    bool staged_used = false;
    int* dstate = nullptr; size_t dstate_cap = 0;  // exponents
    double* part = nullptr; size_t part_cap = 0;   // partial slots
    double2* coef = nullptr; size_t coef_cap = 0;  // coefficients of one launch pair
    double2* pad = nullptr; size_t pad_cap = 0;    // padded odd-n matrices
};
static std::mutex g_bws_mu;
static std::map<std::pair<int, hipStream_t>, BatchWS*> g_bws;

static int batch_ws(hipStream_t st, BatchWS** out) {
    int dev = 0;
    int rc = ensure_device(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_bws_mu);
    BatchWS*& w = g_bws[std::make_pair(dev, st)];
    if (!w) {
        w = new BatchWS();
        if (hipEventCreateWithFlags(&w->staged, hipEventDisableTiming) != hipSuccess)
            return set_error(HAF_E_DEVICE, "hipEventCreate failed");
    }
    *out = w;
    return HAF_OK;
}

static int grow_pinned(BatchWS* w, size_t need) {
    if (need <= w->hmeta_cap) return HAF_OK;
    if (w->hmeta) {
        if (w->staged_used) (void)hipEventSynchronize(w->staged);
        (void)hipHostFree(w->hmeta);
        w->hmeta = nullptr;
        w->hmeta_cap = 0;
    }
    const size_t sz = need + need / 4;
    if (hipHostMalloc((void**)&w->hmeta, sz, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        w->hmeta = nullptr;
        return set_error(HAF_E_NOMEM, "hipHostMalloc of %zu bytes failed", sz);
    }
    w->hmeta_cap = sz;
    return HAF_OK;
}

void release_batch_workspaces() {
    std::lock_guard<std::mutex> lk(g_bws_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_bws) {
        BatchWS* w = kv.second;
        (void)hipSetDevice(kv.first.first);
        (void)hipDeviceSynchronize();
        if (w->dmeta) (void)hipFree(w->dmeta);
        if (w->hmeta) (void)hipHostFree(w->hmeta);
        if (w->staged) (void)hipEventDestroy(w->staged);
        if (w->dstate) (void)hipFree(w->dstate);
        if (w->part) (void)hipFree(w->part);
        if (w->coef) (void)hipFree(w->coef);
        if (w->pad) (void)hipFree(w->pad);
        delete w;
    }
    g_bws.clear();
    (void)hipSetDevice(cur);
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int check_batch_args(const void* dA, const int64_t* offs, const int32_t* ns, const uint8_t* kinds, int count,
                            const void* d_out) {
    if (count < 0) return set_error(HAF_E_INVALID_ARG, "count = %d < 0", count);
    if (count == 0) return HAF_OK;
    if (!dA || !offs || !ns || !kinds || !d_out) return set_error(HAF_E_INVALID_ARG, "null pointer");
    for (int t = 0; t < count; ++t) {
        if (ns[t] < 0) return set_error(HAF_E_INVALID_ARG, "n[%d] = %d < 0", t, ns[t]);
        if (kinds[t] != HAF_KIND_HAF && kinds[t] != HAF_KIND_LHAF)
            return set_error(HAF_E_INVALID_ARG, "kind[%d] = %d unknown", t, kinds[t]);
        if (offs[t] < 0) return set_error(HAF_E_INVALID_ARG, "offset[%d] < 0", t);
        if (eff_n(ns[t], kinds[t]) > HAF_MAX_N)
            return set_error(HAF_E_TOO_LARGE, "n[%d] = %d exceeds the limit %d", t, ns[t], HAF_MAX_N);
    }
    return HAF_OK;
}

// ------------------------------------------------------------------ shared launches
static int run_grouped(const double2* dA, const int64_t* offs, const int32_t* ns, const uint8_t* kinds,
                       const std::vector<int>& list, double2* d_out, double* d_out_dd, hipStream_t st,
                       const haf_batched_config& cfg) {
    if (list.empty()) return HAF_OK;
    HostRange range("hafgpu: batched stage launches");
    BatchWS* w = nullptr;
    int rc = batch_ws(st, &w);
    if (rc) return rc;
    GroupPlan gp;
    if ((rc = plan_groups(ns, kinds, list, cfg, &gp))) return rc;
    const int ni = (int)list.size();

    // device buffers
    if (gp.pad_elems &&
        (rc = grow((void**)&w->pad, &w->pad_cap, sizeof(double2) * (size_t)gp.pad_elems, st)))
        return rc;
    if ((rc = grow((void**)&w->coef, &w->coef_cap, sizeof(double2) * (size_t)std::max<int64_t>(gp.coef_max, 1), st)))
        return rc;
    if ((rc = grow((void**)&w->part, &w->part_cap, sizeof(double) * 4 * (size_t)std::max<int64_t>(gp.slots, 1), st)))
        return rc;
    if ((rc = grow((void**)&w->dstate, &w->dstate_cap, sizeof(int) * (size_t)ni, st))) return rc;
    const size_t items_b = align256(sizeof(GroupItem) * (size_t)ni);
    const size_t meta_b = items_b + align256(sizeof(GroupChunk) * std::max<size_t>(gp.chunks.size(), 1));
    if ((rc = grow((void**)&w->dmeta, &w->dmeta_cap, meta_b, st))) return rc;
    if (w->staged_used && (rc = hip_check(hipEventSynchronize(w->staged), "event synchronize"))) return rc;
    if ((rc = grow_pinned(w, meta_b))) return rc;

    GroupItem* items = (GroupItem*)w->hmeta;
    int64_t pad_off = 0;
    for (int j = 0; j < ni; ++j) {
        const int t = list[(size_t)j];
        GroupItem& it = items[j];
        it.src = dA + offs[t];
        it.src_n = ns[t];
        it.src_lda = std::max(ns[t], 1);
        it.n = gp.n_eff[(size_t)j];
        it.A = it.src;
        it.lda = it.src_lda;
        it.cval = gp.cval[(size_t)j];
        it.pad_ = 0;
        it.exp = w->dstate + j;
        if (it.cval == kGroupComputed && it.n != ns[t]) {   // odd-n loop hafnian: dense padded copy
            it.A = w->pad + pad_off;
            it.lda = it.n;
            pad_off += (int64_t)it.n * it.n;
        }
        it.out = d_out ? d_out + t : nullptr;
        it.out_dd = d_out_dd ? d_out_dd + 4 * (int64_t)t : nullptr;
        it.slot_base = gp.slot_base[(size_t)j];
        it.nslots = gp.nslots[(size_t)j];
    }
    if (!gp.chunks.empty())
        std::memcpy(w->hmeta + items_b, gp.chunks.data(), sizeof(GroupChunk) * gp.chunks.size());
    if ((rc = hip_check(hipMemcpyAsync(w->dmeta, w->hmeta, meta_b, hipMemcpyHostToDevice, st), "batch table upload")))
        return rc;
    if ((rc = hip_check(hipEventRecord(w->staged, st), "event record"))) return rc;
    w->staged_used = true;
    const GroupItem* ditems = (const GroupItem*)w->dmeta;
    const GroupChunk* dch = (const GroupChunk*)(w->dmeta + items_b);

    if ((rc = hip_check(launch_group_prologue(st, ditems, ni), "batch prologue launch"))) return rc;
    for (const StageLaunch& L : gp.launches) {
        hipError_t e;
        if (L.what == 0) {
            int64_t subsets = 0;
            for (int c = 0; c < L.nch; ++c) subsets += gp.chunks[L.first + (size_t)c].count;
            const int pidx = prof_begin(st, 2, L.flops, subsets);
            e = launch_coef_reg_group(L.layout, L.loops, L.blocks, st, ditems, dch + L.first, L.nch, w->coef);
            prof_end(pidx, st);
        } else {
            e = launch_series_group(L.loops, 16, L.blocks, st, dch + L.first, L.nch, w->coef, w->part);
        }
        if ((rc = hip_check(e, "batch kernel launch"))) return rc;
    }
    return hip_check(launch_reduce_group(st, ditems, ni, w->part), "batch reduce launch");
}

// ------------------------------------------------------------------ stream pool
// Streams (default priority, non-blocking) owned by the library per device,
// with an event per stream for joining back into the caller's stream.
struct StreamPool {
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> done;
    hipEvent_t start = nullptr;
};
static std::mutex g_pool_mu;
static std::map<int, StreamPool*> g_pool;

static int stream_pool(int dev, int want, StreamPool** out) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    StreamPool*& p = g_pool[dev];
    if (!p) {
        p = new StreamPool();
        if (hipEventCreateWithFlags(&p->start, hipEventDisableTiming) != hipSuccess)
            return set_error(HAF_E_DEVICE, "hipEventCreate failed");
    }
    while ((int)p->st.size() < want) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return set_error(HAF_E_DEVICE, "hipStreamCreate failed");
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return set_error(HAF_E_DEVICE, "hipEventCreate failed");
        p->st.push_back(s);
        p->done.push_back(e);
    }
    *out = p;
    return HAF_OK;
}

// Model flops of one whole matrix (every subset through the coefficient stage).
double item_cost(int n, int kind) {
    double f = 2.0e5;                                   // launch and series overhead, in flop units
    if (constant_of(n, kind) != kGroupComputed) return f;
    const int N = eff_n(n, kind) / 2;
    for (int m = 1; m <= N; ++m) f += (double)binom(N, m) * coef_model_flops(2 * m, N, kind == HAF_KIND_LHAF);
    return f;
}

int run_batched(const double2* dA, const int64_t* offs, const int32_t* ns, const uint8_t* kinds, int count,
                double2* d_out, double* d_out_dd, hipStream_t st, const haf_batched_config& cfg) {
    HostRange range("hafgpu: batched call");
    int rc = check_batch_args(dA, offs, ns, kinds, count, d_out ? (const void*)d_out : (const void*)d_out_dd);
    if (rc || count == 0) return rc;
    int dev = 0;
    if ((rc = ensure_device(&dev))) return rc;

    std::vector<int> grouped, rest;
    for (int t = 0; t < count; ++t) (cfg.grouped && groupable(ns[t], kinds[t]) ? grouped : rest).push_back(t);
    // the rest: largest model cost first, each to the stream with the least work so far
    std::vector<double> cost((size_t)count, 0.0);
    for (int t : rest) cost[(size_t)t] = item_cost(ns[t], kinds[t]);
    std::stable_sort(rest.begin(), rest.end(), [&](int a, int b) { return cost[(size_t)a] > cost[(size_t)b]; });
    const int nst = std::max(1, std::min(cfg.streams, kMaxPoolStreams));
    std::vector<std::vector<int>> lists((size_t)nst);
    std::vector<double> load((size_t)nst, 0.0);
    for (int t : rest) {
        const int p = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lists[(size_t)p].push_back(t);
        load[(size_t)p] += cost[(size_t)t];
    }
    StreamPool* pool = nullptr;
    if (!rest.empty()) {
        if ((rc = stream_pool(dev, nst, &pool))) return rc;
        // the pool streams start after the work already on st
        if ((rc = hip_check(hipEventRecord(pool->start, st), "event record"))) return rc;
        for (int p = 0; p < nst; ++p)
            if ((rc = hip_check(hipStreamWaitEvent(pool->st[(size_t)p], pool->start, 0), "stream wait"))) return rc;
    }
    std::vector<int> rcs((size_t)nst, HAF_OK);
    std::vector<std::string> msgs((size_t)nst);
    auto worker = [&](int p) {
        if (hipSetDevice(dev) != hipSuccess) {
            rcs[(size_t)p] = HAF_E_DEVICE;
            msgs[(size_t)p] = "hipSetDevice failed";
            return;
        }
        for (int t : lists[(size_t)p]) {
            const int r = run_dev(dA + offs[t], ns[t], std::max(ns[t], 1), kinds[t],
                                  d_out_dd ? d_out_dd + 4 * (int64_t)t : nullptr, d_out ? d_out + t : nullptr,
                                  pool->st[(size_t)p]);
            if (r) {
                rcs[(size_t)p] = r;
                msgs[(size_t)p] = last_error();
                return;
            }
        }
    };
    std::vector<std::thread> th;
    if (!rest.empty())
        for (int p = 0; p < nst; ++p)
            if (!lists[(size_t)p].empty()) th.emplace_back(worker, p);
    const int grc = run_grouped(dA, offs, ns, kinds, grouped, d_out, d_out_dd, st, cfg);
    const std::string gmsg = grc ? last_error() : std::string();
    for (auto& x : th) x.join();
    if (!rest.empty()) {
        // join back: st waits for every pool stream (also after an error, so that
        // nothing enqueued so far is left unordered with the caller's stream)
        for (int p = 0; p < nst; ++p) {
            (void)hipEventRecord(pool->done[(size_t)p], pool->st[(size_t)p]);
            (void)hipStreamWaitEvent(st, pool->done[(size_t)p], 0);
        }
    }
    if (grc) return set_error(grc, "%s", gmsg.c_str());
    for (int p = 0; p < nst; ++p)
        if (rcs[(size_t)p]) return set_error(rcs[(size_t)p], "%s", msgs[(size_t)p].c_str());
    return HAF_OK;
}

}  // namespace hafgpu

// ======================================================================== C ABI
using namespace hafgpu;

extern "C" {

int haf_batched_c128(const haf_cplx* dA_packed, const int64_t* h_offsets, const int32_t* h_n,
                     const uint8_t* h_kind, int count, haf_cplx* d_out, void* stream) {
    clear_error();
    if (count > 0 && !d_out) return set_error(HAF_E_INVALID_ARG, "null output");
    return run_batched((const double2*)dA_packed, h_offsets, h_n, h_kind, count, (double2*)d_out, nullptr,
                       (hipStream_t)stream, batch_config());
}

int haf_batched_c128x2(const haf_cplx* dA_packed, const int64_t* h_offsets, const int32_t* h_n,
                       const uint8_t* h_kind, int count, haf_cplx2* d_out, void* stream) {
    clear_error();
    if (count > 0 && !d_out) return set_error(HAF_E_INVALID_ARG, "null output");
    return run_batched((const double2*)dA_packed, h_offsets, h_n, h_kind, count, nullptr, (double*)d_out,
                       (hipStream_t)stream, batch_config());
}

int haf_batched_get_config(haf_batched_config* cfg) {
    clear_error();
    if (!cfg) return set_error(HAF_E_INVALID_ARG, "null pointer");
    *cfg = batch_config();
    return HAF_OK;
}

int haf_batched_set_config(const haf_batched_config* cfg) {
    clear_error();
    if (!cfg) return set_error(HAF_E_INVALID_ARG, "null pointer");
    const int rc = check_config(*cfg);
    if (rc) return rc;
    set_batch_config(*cfg);
    return HAF_OK;
}

int haf_batched_tune(const haf_cplx* dA_packed, const int64_t* h_offsets, const int32_t* h_n,
                     const uint8_t* h_kind, int count, haf_cplx* d_out, void* stream, haf_batched_config* best,
                     double* best_ms) {
    clear_error();
    int rc = check_batch_args(dA_packed, h_offsets, h_n, h_kind, count, d_out);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return set_error(HAF_E_DEVICE, "hipEventCreate failed");
    const haf_batched_config keep = batch_config();
    haf_batched_config pick = keep;
    double pick_ms = 1e300;
    // one configuration: a warm run (workspaces), then a timed run
    auto trial = [&](const haf_batched_config& c) -> int {
        int r = run_batched((const double2*)dA_packed, h_offsets, h_n, h_kind, count, (double2*)d_out, nullptr, st,
                            c);
        if (!r) r = hip_check(hipEventRecord(a, st), "event record");
        if (!r)
            r = run_batched((const double2*)dA_packed, h_offsets, h_n, h_kind, count, (double2*)d_out, nullptr, st,
                            c);
        if (!r) r = hip_check(hipEventRecord(b, st), "event record");
        if (!r) r = hip_check(hipEventSynchronize(b), "event synchronize");
        float ms = 0.f;
        if (!r) r = hip_check(hipEventElapsedTime(&ms, a, b), "event time");
        if (!r && ms < pick_ms) {
            pick_ms = ms;
            pick = c;
        }
        return r;
    };
    // coordinate search: subsets per lane group, then the layout table, then the
    // streams of the large matrices; the single-matrix launches for reference
    for (int span : { 1, 2, 4, 8, 16 }) {
        haf_batched_config c = keep;
        c.grouped = 1;
        c.table = 0;
        c.span = span;
        if ((rc = trial(c))) break;
    }
    if (!rc) {
        haf_batched_config c = pick;
        c.table = 1 - pick.table;
        rc = trial(c);
    }
    for (int nst = 1; !rc && nst <= kMaxPoolStreams; nst *= 2) {
        haf_batched_config c = pick;
        c.streams = nst;
        if (c.streams != pick.streams) rc = trial(c);
    }
    if (!rc) {
        haf_batched_config c = pick;
        c.grouped = 0;
        c.streams = kMaxPoolStreams;
        rc = trial(c);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) {
        set_batch_config(keep);
        return rc;
    }
    set_batch_config(pick);
    if (best) *best = pick;
    if (best_ms) *best_ms = pick_ms;
    const char* path = std::getenv("HAF_AUTOTUNE_CACHE");
    if (path && *path) {
        const std::string key = device_key();
        if (key.empty()) return set_error(HAF_E_DEVICE, "no current device");
        return cache_write(path, key, pick);
    }
    return HAF_OK;
}

int haf_batched_load_cache(void) {
    clear_error();
    return batched_load_cache(false);
}

int haf_batched_plan(const int32_t* h_n, const uint8_t* h_kind, int count, int64_t* launches, int max_launches,
                     int* n_launches, int64_t* chunks, int max_chunks, int* n_chunks) {
    clear_error();
    if (count < 0 || (count > 0 && (!h_n || !h_kind)) || !n_launches || !n_chunks)
        return set_error(HAF_E_INVALID_ARG, "bad argument");
    for (int t = 0; t < count; ++t)
        if (h_n[t] < 0 || (h_kind[t] != HAF_KIND_HAF && h_kind[t] != HAF_KIND_LHAF) ||
            eff_n(h_n[t], h_kind[t]) > HAF_MAX_N)
            return set_error(HAF_E_INVALID_ARG, "bad item %d", t);
    const haf_batched_config cfg = batch_config();
    std::vector<int> list;
    for (int t = 0; t < count; ++t)
        if (cfg.grouped && groupable(h_n[t], h_kind[t])) list.push_back(t);
    GroupPlan gp;
    const int rc = plan_groups(h_n, h_kind, list, cfg, &gp);
    if (rc) return rc;
    *n_launches = (int)gp.launches.size();
    *n_chunks = (int)gp.chunks.size();
    for (size_t l = 0; l < gp.launches.size() && launches && (int)l < max_launches; ++l) {
        const StageLaunch& L = gp.launches[l];
        int64_t* o = launches + 8 * l;
        o[0] = L.what; o[1] = L.layout; o[2] = L.loops; o[3] = L.blocks;
        o[4] = (int64_t)L.first; o[5] = L.nch; o[6] = L.coef_elems; o[7] = reg_layout_sm(L.layout);
    }
    for (size_t c = 0; c < gp.chunks.size() && chunks && (int)c < max_chunks; ++c) {
        const GroupChunk& ch = gp.chunks[c];
        int64_t* o = chunks + 8 * c;
        o[0] = gp.order[(size_t)ch.item]; o[1] = ch.m; o[2] = ch.count; o[3] = ch.gstart;
        o[4] = ch.coff; o[5] = ch.slot; o[6] = ch.N; o[7] = (int64_t)ch.rank0;
    }
    return HAF_OK;
}

}  // extern "C"

// Continuous-batching request server.
//
// submit() validates and copies a host matrix into the host queue and returns
// at once.  One scheduler thread owns all device work and runs in ticks:
//
//  * admission: queued requests are admitted in arrival order while a request
//    slot is free and the device arena holds the request's whole state: its
//    matrix, the padded copy of an odd-n loop hafnian, the exponent of its
//    input scaling and its partial slots (one per 256-subset series block);
//  * a tick takes work from every admitted request with work left, round-robin
//    in admission order up to a tick budget of model flops and coefficient
//    memory: a piece is a run of subsets of one size class (Sec. 3.2, Eq. Pset)
//    cut at multiples of the series block, so each piece fills exactly the
//    partial slots the single-matrix path fills for those subsets;
//  * one tick is a handful of launches shared by all its pieces: the prologue
//    of the requests that start in it (padding, input scaling), one
//    coefficient launch per register layout and kind, one series launch per
//    kind, and one reduction launch for the requests whose last piece is in
//    the tick, whose results go to a pinned host slot behind an event;
//  * up to kTicksInFlight ticks are enqueued ahead on the server's stream, so
//    requests that arrive while a tick runs join the next one.
//
// A small request completes in the tick after its admission instead of queueing
// behind a large one, and the large ones proceed a budget's worth per tick.
// Each request keeps the single-matrix path's per-subset arithmetic, partial
// slots and reduction order, so a result is bitwise the single-matrix result,
// whatever else the server runs.  With continuous = 0 the server runs one
// request at a time through the single-matrix path (the plain server).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "haf_launch.hpp"
#include "haf_runtime.hpp"

using namespace hafgpu;

namespace {

constexpr int kTicksInFlight = 2;
constexpr int kSeriesBlockSubsets = 256;       // one partial slot per series block

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// First-fit allocator over [0, size) with coalescing of free blocks.
class Arena {
public:
    void reset(int64_t size) {
        free_.clear();
        if (size > 0) free_[0] = size;
    }
    int64_t alloc(int64_t bytes) {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                const int64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest > 0) free_[off + bytes] = rest;
                return off;
            }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<int64_t, int64_t> free_;
};

struct Request {
    uint64_t ticket = 0;
    int n = 0, kind = 0;
    std::vector<haf_cplx> A;        // dense copy, kept until the request completes
    double t_submit = 0, t_admit = 0;
    int ne = 0;                     // size after padding an odd-n loop hafnian
    int cval = kGroupComputed;      // constant result (n = 0, odd-n haf) or computed
    int64_t bytes = 0;              // arena block: matrix | padded copy | exponent | partial slots
    int64_t off = -1;
    int64_t off_pad = 0, off_exp = 0, off_part = 0;
    Plan plan;
    size_t chunk = 0;               // progress through the plan: next chunk, next rank within it
    uint64_t rank = 0;
    bool started = false;           // its prologue has been enqueued
    bool enqueued_all = false;      // its reduction has been enqueued
    int slot = -1;                  // request slot
};

bool has_work(const Request* r) { return r->cval == kGroupComputed && !r->enqueued_all; }

int64_t plan_bytes(int n, int kind, Plan* plan, int* ne) {
    *ne = (n % 2 == 1 && kind == HAF_KIND_LHAF) ? n + 1 : n;
    *plan = make_plan(*ne, kind, kChunk);
    int64_t b = align256((int64_t)n * n * (int64_t)sizeof(haf_cplx));
    if (*ne != n) b += align256((int64_t)*ne * *ne * (int64_t)sizeof(haf_cplx));
    b += 256;                                                   // exponent
    b += align256(plan->nslots * 4 * (int64_t)sizeof(double));  // partial slots
    return b;
}

struct TickSlot {
    char* hstage = nullptr;         // pinned: items | reduce items | chunks | matrices of starting requests
    char* dmeta = nullptr;          // device copy of the tables
    size_t cap = 0;
    double* dres = nullptr;         // device results of the requests finishing in the tick
    double* hres = nullptr;         // pinned copy of the same
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Request*> finishing;
};

}  // namespace

struct haf_server {
    haf_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_done;
    std::deque<Request*> queue;
    std::deque<haf_result> results;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, finished = 0;
    bool stop = false;
    std::thread thread;
    // owned by the scheduler thread after start-up
    char* arena = nullptr;
    Arena alloc;
    hipStream_t stream = nullptr;
    double2* coef = nullptr;                // coefficients of one tick
    std::vector<int> free_slots;
    std::deque<Request*> active;            // admitted, in admission order
    TickSlot ticks[kTicksInFlight];
    std::deque<int> inflight;               // tick slots in launch order
    size_t rr = 0;                          // round-robin start
    // plain server: one request at a time
    double* plain_res = nullptr;            // device result
    double* plain_host = nullptr;           // pinned
    hipEvent_t plain_ev = nullptr;
    Request* plain_cur = nullptr;
    std::string start_error;
    bool started = false;
    std::condition_variable cv_start;
    // test hook: this many of the next completed ticks (or plain-server requests)
    // are handled as failed launches
    std::atomic<int> inject_fail{0};
    bool broken = false;                    // no stream after a failed reset: requests fail at once
};

namespace {

void finish(haf_server* s, Request* r, int status, const double* res) {
    haf_result out{};
    out.ticket = r->ticket;
    out.status = status;
    out.n = r->n;
    out.kind = r->kind;
    if (res) {
        out.value.re = res[0] + res[1];
        out.value.im = res[2] + res[3];
    }
    out.t_submit = r->t_submit;
    out.t_admit = r->t_admit;
    out.t_done = now_seconds();
    if (r->off >= 0) s->alloc.release(r->off, r->bytes);
    if (r->slot >= 0) s->free_slots.push_back(r->slot);
    delete r;
    std::lock_guard<std::mutex> lk(s->mu);
    s->results.push_back(out);
    s->finished++;
    s->cv_done.notify_all();
}

// Piece: subsets [rank0, rank0 + count) of chunk `ci` of a request's plan.
struct Piece {
    Request* r;
    size_t ci;
    uint64_t rank0;
    int count;
};

double subset_flops(const Request* r, int m) { return coef_model_flops(2 * m, r->plan.N, r->kind == HAF_KIND_LHAF); }

// Take pieces from r worth at most `budget` flops and the coefficient room left,
// advancing its cursor; with `force`, at least one series block (if it fits).
double take(Request* r, double budget, int64_t* coef_left, bool force, std::vector<Piece>* out) {
    double used = 0.0;
    bool got = false;
    while (r->chunk < r->plan.chunks.size()) {
        const Chunk& c = r->plan.chunks[r->chunk];
        const double f = subset_flops(r, c.m);
        const int64_t left = (int64_t)((uint64_t)c.count - r->rank);
        const int64_t per = r->plan.ncoef;
        const int64_t room = *coef_left / per;
        int64_t want = std::min<int64_t>(left, room);
        want = std::min<int64_t>(want, (int64_t)std::max(0.0, (budget - used) / f));
        if (want < left) want -= want % kSeriesBlockSubsets;   // cut at a series block
        if (want <= 0) {
            if (!force || got) break;
            want = std::min<int64_t>(left, kSeriesBlockSubsets);
            if (want > room) break;
        }
        out->push_back(Piece{ r, r->chunk, r->rank, (int)want });
        got = true;
        used += f * (double)want;
        *coef_left -= want * per;
        r->rank += (uint64_t)want;
        if (r->rank >= (uint64_t)c.count) {
            r->chunk++;
            r->rank = 0;
        }
        if (want < left) break;
    }
    return used;
}

int grow_slot(TickSlot& t, size_t need, hipStream_t st) {
    if (need <= t.cap) return HAF_OK;
    if (t.hstage) (void)hipHostFree(t.hstage);
    if (t.dmeta) (void)hipFree(t.dmeta);
    t.hstage = nullptr;
    t.dmeta = nullptr;
    t.cap = 0;
    (void)st;
    const size_t sz = need + need / 2;
    if (hipHostMalloc((void**)&t.hstage, sz, hipHostMallocDefault) != hipSuccess)
        return set_error(HAF_E_NOMEM, "pinned tick table of %zu bytes", sz);
    if (hipMalloc((void**)&t.dmeta, sz) != hipSuccess) return set_error(HAF_E_NOMEM, "tick table of %zu bytes", sz);
    t.cap = sz;
    return HAF_OK;
}

// Build and enqueue one tick into slot `ti`.  Returns false if there was no work.
bool enqueue_tick(haf_server* s, int ti, int* rc_out) {
    HostRange range("hafgpu: server tick");
    TickSlot& T = s->ticks[ti];
    *rc_out = HAF_OK;
    const haf_server_config& c = s->cfg;
    std::vector<Request*> cand;
    for (Request* r : s->active)
        if (has_work(r)) cand.push_back(r);
    if (cand.empty()) return false;
    // ---- pieces: a fair share per request first, then the rest of the budget in order
    std::vector<Piece> pieces;
    int64_t coef_left = c.tick_coef_bytes / (int64_t)sizeof(double2);
    double budget = c.tick_flops;
    const size_t nc = cand.size();
    const double share = budget / (double)nc;
    for (size_t k = 0; k < nc; ++k) {
        Request* r = cand[(s->rr + k) % nc];
        budget -= take(r, share, &coef_left, true, &pieces);
    }
    for (size_t k = 0; k < nc && budget > 0.0 && coef_left > 0; ++k) {
        Request* r = cand[(s->rr + k) % nc];
        budget -= take(r, budget, &coef_left, false, &pieces);
    }
    s->rr = (s->rr + 1) % std::max<size_t>(nc, 1);
    // ---- items of the tick: starting requests first, then the others with pieces
    std::vector<Request*> items;
    std::map<Request*, int> index;
    for (Request* r : cand)
        if (!r->started) { index[r] = (int)items.size(); items.push_back(r); }
    const int nstart = (int)items.size();
    for (const Piece& p : pieces)
        if (!index.count(p.r)) { index[p.r] = (int)items.size(); items.push_back(p.r); }
    T.finishing.clear();
    for (Request* r : items)
        if (r->chunk >= r->plan.chunks.size()) T.finishing.push_back(r);
    // ---- tables
    auto make_item = [&](Request* r, int fin) {
        GroupItem it{};
        char* base = s->arena + r->off;
        it.src = (const double2*)base;
        it.A = r->ne != r->n ? (const double2*)(base + r->off_pad) : it.src;
        it.out = nullptr;
        it.out_dd = fin >= 0 ? T.dres + 4 * fin : nullptr;
        it.n = r->ne;
        it.lda = r->ne != r->n ? r->ne : std::max(r->n, 1);
        it.src_n = r->n;
        it.src_lda = std::max(r->n, 1);
        it.cval = kGroupComputed;
        it.exp = (int*)(base + r->off_exp);
        it.slot_base = (r->off + r->off_part) / (int64_t)(4 * sizeof(double));
        it.nslots = r->plan.nslots;
        return it;
    };
    std::vector<GroupItem> gitems;
    for (Request* r : items) gitems.push_back(make_item(r, -1));
    std::vector<GroupItem> fitems;
    for (size_t k = 0; k < T.finishing.size(); ++k) fitems.push_back(make_item(T.finishing[k], (int)k));
    // chunks: per (layout, kind) coefficient launches; a series launch per kind
    struct L { int layout; bool loops; size_t first; int nch; int blocks; int nmax; };
    std::vector<GroupChunk> chunks;
    std::vector<L> coefL, seriesL;
    std::vector<Piece> lds_pieces;
    std::vector<int64_t> lds_coff;
    int64_t coff_next = 0;
    std::map<const Piece*, int64_t> coff_of;
    for (int loops = 0; loops < 2; ++loops) {
        for (int lay = reg_layout_count() - 1; lay >= -1; --lay) {
            L cl{ lay, loops == 1, chunks.size(), 0, 0, 0 };
            for (const Piece& p : pieces) {
                if ((p.r->kind == HAF_KIND_LHAF) != (loops == 1)) continue;
                const Chunk& ch = p.r->plan.chunks[p.ci];
                if (reg_layout_index(2 * ch.m) != lay) continue;
                coff_of[&p] = coff_next;
                if (lay < 0) {                              // no register layout: LDS kernel per piece
                    lds_pieces.push_back(p);
                    lds_coff.push_back(coff_next);
                } else {
                    GroupChunk g{};
                    g.item = index[p.r];
                    g.m = ch.m;
                    g.count = p.count;
                    g.N = p.r->plan.N;
                    g.rank0 = ch.rank0 + p.rank0;
                    g.coff = coff_next;
                    g.gstart = cl.blocks;
                    cl.blocks += group_coef_blocks(lay, p.count, 4);
                    chunks.push_back(g);
                    cl.nch++;
                }
                coff_next += (int64_t)p.count * p.r->plan.ncoef;
            }
            if (cl.nch) coefL.push_back(cl);
        }
        L sl{ -1, loops == 1, chunks.size(), 0, 0, 0 };
        for (const Piece& p : pieces) {
            if ((p.r->kind == HAF_KIND_LHAF) != (loops == 1)) continue;
            const Chunk& ch = p.r->plan.chunks[p.ci];
            GroupChunk g{};
            g.item = index[p.r];
            g.m = ch.m;
            g.count = p.count;
            g.N = p.r->plan.N;
            g.rank0 = ch.rank0 + p.rank0;
            g.coff = coff_of[&p];
            g.slot = (p.r->off + p.r->off_part) / (int64_t)(4 * sizeof(double)) + ch.slot0 +
                     (int64_t)(p.rank0 / kSeriesBlockSubsets);
            g.sign = ((p.r->plan.N - ch.m) & 1) ? -1.0 : 1.0;
            g.gstart = sl.blocks;
            sl.blocks += group_series_blocks(p.count);
            sl.nmax = std::max(sl.nmax, p.r->plan.N);
            chunks.push_back(g);
            sl.nch++;
        }
        if (sl.nch) seriesL.push_back(sl);
    }
    // matrices of the starting requests are staged after the tables
    const size_t items_b = (size_t)align256((int64_t)(sizeof(GroupItem) * std::max<size_t>(gitems.size(), 1)));
    const size_t fitems_b = (size_t)align256((int64_t)(sizeof(GroupItem) * std::max<size_t>(fitems.size(), 1)));
    const size_t chunks_b = (size_t)align256((int64_t)(sizeof(GroupChunk) * std::max<size_t>(chunks.size(), 1)));
    size_t mats_b = 0;
    for (int k = 0; k < nstart; ++k) mats_b += (size_t)align256((int64_t)items[(size_t)k]->A.size() * 16);
    const size_t table_b = items_b + fitems_b + chunks_b;
    int rc = grow_slot(T, table_b + mats_b, s->stream);
    if (rc) { *rc_out = rc; return true; }
    std::memcpy(T.hstage, gitems.data(), sizeof(GroupItem) * gitems.size());
    std::memcpy(T.hstage + items_b, fitems.data(), sizeof(GroupItem) * fitems.size());
    std::memcpy(T.hstage + items_b + fitems_b, chunks.data(), sizeof(GroupChunk) * chunks.size());
    hipStream_t st = s->stream;
    auto chk = [&](hipError_t e, const char* what) {
        if (rc == HAF_OK) rc = hip_check(e, what);
        return rc == HAF_OK;
    };
    chk(hipMemcpyAsync(T.dmeta, T.hstage, table_b, hipMemcpyHostToDevice, st), "tick table upload");
    size_t mo = table_b;
    for (int k = 0; k < nstart && rc == HAF_OK; ++k) {
        Request* r = items[(size_t)k];
        const size_t b = r->A.size() * sizeof(haf_cplx);
        if (b) {
            std::memcpy(T.hstage + mo, r->A.data(), b);
            chk(hipMemcpyAsync(s->arena + r->off, T.hstage + mo, b, hipMemcpyHostToDevice, st), "matrix upload");
        }
        mo += (size_t)align256((int64_t)b);
        r->started = true;
    }
    const GroupItem* ditems = (const GroupItem*)T.dmeta;
    const GroupItem* dfin = (const GroupItem*)(T.dmeta + items_b);
    const GroupChunk* dch = (const GroupChunk*)(T.dmeta + items_b + fitems_b);
    double* partials = (double*)s->arena;
    if (nstart && rc == HAF_OK) chk(launch_group_prologue(st, ditems, nstart), "tick prologue launch");
    for (const L& l : coefL) {
        if (rc != HAF_OK) break;
        double flops = 0.0;
        int64_t subsets = 0;
        for (int k = 0; k < l.nch; ++k) {
            const GroupChunk& g = chunks[l.first + (size_t)k];
            flops += (double)g.count * coef_model_flops(2 * g.m, g.N, l.loops);
            subsets += g.count;
        }
        const int pidx = prof_begin(st, 2, flops, subsets);
        chk(launch_coef_reg_group(l.layout, l.loops, l.blocks, st, ditems, dch + l.first, l.nch, s->coef),
            "tick coefficient launch");
        prof_end(pidx, st);
    }
    for (size_t k = 0; k < lds_pieces.size() && rc == HAF_OK; ++k) {
        // subsets above the register layouts: the LDS kernel, reading the exponent the
        // prologue left in the request's arena block
        const Piece& p = lds_pieces[k];
        const Chunk& ch = p.r->plan.chunks[p.ci];
        const char* base = s->arena + p.r->off;
        const double2* A = p.r->ne != p.r->n ? (const double2*)(base + p.r->off_pad) : (const double2*)base;
        const int lda = p.r->ne != p.r->n ? p.r->ne : std::max(p.r->n, 1);
        chk(launch_coef_lds(2 * ch.m, p.r->kind == HAF_KIND_LHAF, std::min(p.count, 2048), st, A, lda, p.r->plan.N,
                            ch.m, ch.rank0 + p.rank0, p.count, nullptr, (const int*)(base + p.r->off_exp),
                            s->coef + lds_coff[k], p.count),
            "tick coefficient launch");
    }
    for (const L& l : seriesL) {
        if (rc != HAF_OK) break;
        chk(launch_series_group(l.loops, l.nmax, l.blocks, st, dch + l.first, l.nch, s->coef, partials),
            "tick series launch");
    }
    if (!fitems.empty() && rc == HAF_OK) {
        chk(launch_reduce_group(st, dfin, (int)fitems.size(), partials), "tick reduce launch");
        chk(hipMemcpyAsync(T.hres, T.dres, sizeof(double) * 4 * fitems.size(), hipMemcpyDeviceToHost, st),
            "result download");
    }
    if (rc == HAF_OK) chk(hipEventRecord(T.done, st), "event record");
    for (Request* r : T.finishing) r->enqueued_all = true;
    T.busy = true;
    *rc_out = rc;
    return true;
}

// A launch failed: wait for everything enqueued on the stream (no work may
// outlive the device memory of its request), fail every admitted request, and
// go on with a fresh stream.  Requests still queued are admitted afterwards.
void fail_all(haf_server* s, int status) {
    (void)hipStreamSynchronize(s->stream);
    for (int t = 0; t < kTicksInFlight; ++t) {
        s->ticks[t].busy = false;
        s->ticks[t].finishing.clear();
    }
    s->inflight.clear();
    std::deque<Request*> act;
    act.swap(s->active);
    for (Request* r : act) finish(s, r, status, nullptr);
    release_stream_workspace(s->stream);     // the plain server's single-matrix workspaces
    (void)hipStreamDestroy(s->stream);
    s->stream = nullptr;
    (void)hipGetLastError();                 // clear a sticky launch error before the new stream
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        s->stream = nullptr;
        s->broken = true;
    }
}

// hipEventQuery, or a failure forced by the test hook once the event has completed
hipError_t query_done(haf_server* s, hipEvent_t ev) {
    const hipError_t e = hipEventQuery(ev);
    if (e != hipSuccess) return e;
    int k = s->inject_fail.load();
    while (k > 0 && !s->inject_fail.compare_exchange_weak(k, k - 1)) {}
    return k > 0 ? hipErrorLaunchFailure : hipSuccess;
}

void scheduler(haf_server* s) {
    const haf_server_config& c = s->cfg;
    auto fail_start = [&](const char* what) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->start_error = what;
        s->started = true;
        s->cv_start.notify_all();
    };
    if (hipSetDevice(c.device) != hipSuccess || ensure_device(nullptr) != HAF_OK) return fail_start("hipSetDevice failed");
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
        return fail_start("stream creation failed");
    if (hipMalloc((void**)&s->arena, (size_t)c.arena_bytes) != hipSuccess) return fail_start("arena allocation failed");
    s->alloc.reset(c.arena_bytes);
    if (c.continuous) {
        if (hipMalloc((void**)&s->coef, (size_t)c.tick_coef_bytes) != hipSuccess)
            return fail_start("tick coefficient buffer allocation failed");
        for (int t = 0; t < kTicksInFlight; ++t) {
            TickSlot& T = s->ticks[t];
            if (hipMalloc((void**)&T.dres, sizeof(double) * 4 * (size_t)c.max_active) != hipSuccess ||
                hipHostMalloc((void**)&T.hres, sizeof(double) * 4 * (size_t)c.max_active, hipHostMallocDefault) !=
                    hipSuccess ||
                hipEventCreateWithFlags(&T.done, hipEventDisableTiming) != hipSuccess)
                return fail_start("tick buffers allocation failed");
        }
    } else {
        if (hipMalloc((void**)&s->plain_res, 4 * sizeof(double)) != hipSuccess ||
            hipHostMalloc((void**)&s->plain_host, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&s->plain_ev, hipEventDisableTiming) != hipSuccess)
            return fail_start("plain server buffers allocation failed");
    }
    for (int i = c.max_active - 1; i >= 0; --i) s->free_slots.push_back(i);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->started = true;
        s->cv_start.notify_all();
    }

    for (;;) {
        bool progress = false;
        // ---- admission in arrival order while a slot and arena room are free
        for (;;) {
            Request* r = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->stop || s->queue.empty() || s->free_slots.empty()) break;
                if (!c.continuous && (s->plain_cur || !s->active.empty())) break;
                r = s->queue.front();
                if (r->cval == kGroupComputed) {
                    const int64_t off = s->alloc.alloc(r->bytes);
                    if (off < 0) break;
                    r->off = off;
                }
                s->queue.pop_front();
            }
            r->slot = s->free_slots.back();
            s->free_slots.pop_back();
            r->t_admit = now_seconds();
            progress = true;
            if (s->broken && r->cval == kGroupComputed) {    // no stream to run it on
                finish(s, r, HAF_E_DEVICE, nullptr);
                continue;
            }
            if (r->cval != kGroupComputed) {                    // n = 0 or odd-n haf
                const double v[4] = { r->cval == kGroupConstOne ? 1.0 : 0.0, 0.0, 0.0, 0.0 };
                finish(s, r, HAF_OK, v);
                continue;
            }
            if (c.continuous) {
                s->active.push_back(r);
                continue;
            }
            // plain server: the whole single-matrix path for this request alone
            s->plain_cur = r;
            double2* dA = (double2*)(s->arena + r->off);
            int rc = HAF_OK;
            if (r->n > 0)
                rc = hip_check(hipMemcpyAsync(dA, r->A.data(), r->A.size() * sizeof(haf_cplx), hipMemcpyHostToDevice,
                                              s->stream),
                               "matrix upload");
            if (!rc) rc = run_dev(dA, r->n, std::max(r->n, 1), r->kind, s->plain_res, nullptr, s->stream);
            if (!rc)
                rc = hip_check(hipMemcpyAsync(s->plain_host, s->plain_res, 4 * sizeof(double), hipMemcpyDeviceToHost,
                                              s->stream),
                               "result download");
            if (!rc) rc = hip_check(hipEventRecord(s->plain_ev, s->stream), "event record");
            if (rc) {
                (void)hipStreamSynchronize(s->stream);   // nothing enqueued may outlive the request
                s->plain_cur = nullptr;
                finish(s, r, rc, nullptr);
            }
        }
        if (c.continuous) {
            // ---- completed ticks, in launch order
            while (!s->inflight.empty()) {
                TickSlot& T = s->ticks[s->inflight.front()];
                const hipError_t e = query_done(s, T.done);
                if (e == hipErrorNotReady) break;
                if (e != hipSuccess) {
                    fail_all(s, HAF_E_DEVICE);
                    break;
                }
                s->inflight.pop_front();
                T.busy = false;
                for (size_t k = 0; k < T.finishing.size(); ++k) {
                    Request* r = T.finishing[k];
                    s->active.erase(std::find(s->active.begin(), s->active.end(), r));
                    finish(s, r, HAF_OK, T.hres + 4 * k);
                }
                T.finishing.clear();
                progress = true;
            }
            // ---- the next tick, if a slot is free and there is work
            if ((int)s->inflight.size() < kTicksInFlight) {
                int ti = 0;
                while (s->ticks[ti].busy) ++ti;
                int rc = HAF_OK;
                if (enqueue_tick(s, ti, &rc)) {
                    progress = true;
                    if (rc) fail_all(s, rc);
                    else s->inflight.push_back(ti);
                }
            }
        } else if (s->plain_cur) {
            const hipError_t e = query_done(s, s->plain_ev);
            if (e != hipErrorNotReady) {
                Request* r = s->plain_cur;
                s->plain_cur = nullptr;
                if (e == hipSuccess) {
                    finish(s, r, HAF_OK, s->plain_host);
                } else {
                    s->active.push_back(r);          // fail_all fails it and resets the stream
                    fail_all(s, HAF_E_DEVICE);
                }
                progress = true;
            }
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->stop && s->active.empty() && s->inflight.empty() && !s->plain_cur) break;
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    // queued requests that were never admitted
    std::deque<Request*> left;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        left.swap(s->queue);
    }
    for (Request* r : left) finish(s, r, HAF_E_STATE, nullptr);
}

}  // namespace

extern "C" {

void haf_server_default_config(haf_server_config* cfg) {
    if (!cfg) return;
    cfg->device = 0;
    cfg->arena_bytes = (int64_t)1 << 30;
    // HAF_ARENA_BYTES overrides the arena size: an integer, optionally followed by K, M or G
    if (const char* e = std::getenv("HAF_ARENA_BYTES")) {
        char* end = nullptr;
        long long v = std::strtoll(e, &end, 10);
        const char u = end ? *end : 0;
        v <<= (u == 'K' || u == 'k') ? 10 : (u == 'M' || u == 'm') ? 20 : (u == 'G' || u == 'g') ? 30 : 0;
        if (v > 0) cfg->arena_bytes = v;
    }
    cfg->max_active = 256;
    cfg->max_queue = 1 << 20;
    cfg->tick_flops = 2.0e10;
    cfg->tick_coef_bytes = (int64_t)256 << 20;
    cfg->continuous = 1;
}

haf_server* haf_server_create(const haf_server_config* cfg) {
    clear_error();
    if (!cfg || cfg->arena_bytes < 4096 || cfg->max_active < 1 || cfg->max_queue < 1 || !(cfg->tick_flops > 0.0) ||
        cfg->tick_coef_bytes < (int64_t)(kSeriesBlockSubsets * 2 * HAF_MAX_N * sizeof(double2))) {
        set_error(HAF_E_INVALID_ARG, "bad server configuration");
        return nullptr;
    }
    haf_server* s = new haf_server();
    s->cfg = *cfg;
    s->thread = std::thread(scheduler, s);
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_start.wait(lk, [&] { return s->started || !s->start_error.empty(); });
    if (!s->start_error.empty()) {
        const std::string e = s->start_error;
        lk.unlock();
        s->thread.join();
        haf_server_destroy(s);
        set_error(HAF_E_DEVICE, "server start: %s", e.c_str());
        return nullptr;
    }
    return s;
}

int haf_server_submit(haf_server* s, const haf_cplx* A, int n, int lda, int kind, uint64_t* ticket) {
    clear_error();
    if (!s || !ticket) return set_error(HAF_E_INVALID_ARG, "null pointer");
    int rc = check_dims(A, n, lda, kind);
    if (rc) return rc;
    if ((rc = check_values(A, n, lda))) return rc;
    Request* r = new Request();
    r->n = n;
    r->kind = kind;
    if (n == 0) r->cval = kGroupConstOne;
    else if (n % 2 == 1 && kind == HAF_KIND_HAF) r->cval = kGroupConstZero;
    if (r->cval == kGroupComputed) {
        r->bytes = plan_bytes(n, kind, &r->plan, &r->ne);
        r->off_pad = align256((int64_t)n * n * (int64_t)sizeof(haf_cplx));
        r->off_exp = r->off_pad + (r->ne != n ? align256((int64_t)r->ne * r->ne * (int64_t)sizeof(haf_cplx)) : 0);
        r->off_part = r->off_exp + 256;
        if (r->bytes > s->cfg.arena_bytes) {
            delete r;
            return set_error(HAF_E_NOMEM, "request of n = %d needs %lld arena bytes, more than the arena", n,
                             (long long)plan_bytes(n, kind, &r->plan, &r->ne));
        }
    }
    r->A.resize((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) r->A[(size_t)i * n + j] = A[(int64_t)i * lda + j];
    r->t_submit = now_seconds();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        delete r;
        return set_error(HAF_E_STATE, "server stopped");
    }
    if ((int64_t)s->queue.size() >= s->cfg.max_queue) {
        delete r;
        return set_error(HAF_E_BUSY, "queue full (%d requests)", s->cfg.max_queue);
    }
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->queue.push_back(r);
    s->submitted++;
    return HAF_OK;
}

int haf_server_poll(haf_server* s, haf_result* out, int max, int* n_out) {
    clear_error();
    if (!s || !n_out || (max > 0 && !out)) return set_error(HAF_E_INVALID_ARG, "null pointer");
    std::lock_guard<std::mutex> lk(s->mu);
    int k = 0;
    while (k < max && !s->results.empty()) {
        out[k++] = s->results.front();
        s->results.pop_front();
    }
    *n_out = k;
    return HAF_OK;
}

int haf_server_debug_fail_ticks(haf_server* s, int count) {
    clear_error();
    if (!s || count < 0) return set_error(HAF_E_INVALID_ARG, "null server or negative count");
    s->inject_fail.store(count);
    return HAF_OK;
}

int haf_server_drain(haf_server* s) {
    clear_error();
    if (!s) return set_error(HAF_E_INVALID_ARG, "null pointer");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->finished == s->submitted || s->stop; });
    return HAF_OK;
}

void haf_server_destroy(haf_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    if (s->thread.joinable()) s->thread.join();
    if (s->stream) {
        (void)hipStreamSynchronize(s->stream);
        release_stream_workspace(s->stream);   // the plain server's single-matrix workspaces
        (void)hipStreamDestroy(s->stream);
    }
    for (TickSlot& T : s->ticks) {
        if (T.hstage) (void)hipHostFree(T.hstage);
        if (T.dmeta) (void)hipFree(T.dmeta);
        if (T.dres) (void)hipFree(T.dres);
        if (T.hres) (void)hipHostFree(T.hres);
        if (T.done) (void)hipEventDestroy(T.done);
    }
    for (Request* r : s->active) delete r;
    if (s->plain_cur) delete s->plain_cur;
    if (s->plain_res) (void)hipFree(s->plain_res);
    if (s->plain_host) (void)hipHostFree(s->plain_host);
    if (s->plain_ev) (void)hipEventDestroy(s->plain_ev);
    if (s->coef) (void)hipFree(s->coef);
    if (s->arena) (void)hipFree(s->arena);
    for (Request* r : s->queue) delete r;
    delete s;
}

}  // extern "C"

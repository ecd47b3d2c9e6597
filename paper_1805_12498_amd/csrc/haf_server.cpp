// Continuous-batching request server.
//
// submit() validates and copies a host matrix into the host queue and returns
// at once.  One scheduler thread owns all device work: between steps it admits
// queued requests in arrival order while a request slot is free and the device
// arena has room for the request's state (its matrix and its double-double
// result), copies the matrix into the arena and enqueues the whole hafnian
// (the single-matrix path) on the least-loaded of the server's streams,
// followed by the copy of the result into a pinned host slot and an event.
// Requests admitted while others run overlap with them on the device; a
// request's result does not depend on what else runs (the single-matrix path
// is deterministic).  Completions are found by polling the events, only the
// oldest unfinished request of each stream (a stream finishes in order); the result
// carries the host steady-clock times of submit, admission and completion.
// With continuous = 0 the server admits one request at a time on one stream,
// in arrival order (the plain server).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "haf_runtime.hpp"

using namespace hafgpu;

namespace {

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
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t off = -1, bytes = 0;    // arena block
    int slot = -1;                  // pinned result slot
    int stream = -1;
    hipEvent_t ev = nullptr;
};

int64_t request_bytes(int n) {
    const int64_t mat = (int64_t)n * n * (int64_t)sizeof(haf_cplx);
    return ((mat + 255) & ~(int64_t)255) + 256;     // matrix, then the 32-byte result
}

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
    double* pinned = nullptr;       // 4 doubles per request slot
    std::vector<int> free_slots;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;
    std::vector<hipEvent_t> events;
    // admitted requests per stream, in launch order: a stream completes them in
    // that order, so only the front of each queue needs polling
    std::vector<std::deque<Request*>> inflight;
    int n_active = 0;
    std::string start_error;
    bool started = false;
    std::condition_variable cv_start;
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
    if (r->stream >= 0) s->stream_load[r->stream]--;
    if (r->ev) s->events.push_back(r->ev);
    delete r;
    std::lock_guard<std::mutex> lk(s->mu);
    s->results.push_back(out);
    s->finished++;
    s->cv_done.notify_all();
}

// Enqueue one admitted request; returns an error code if nothing could be enqueued.
int launch(haf_server* s, Request* r) {
    int best = 0;
    for (int i = 1; i < (int)s->streams.size(); ++i)
        if (s->stream_load[i] < s->stream_load[best]) best = i;
    hipStream_t st = s->streams[best];
    r->stream = best;
    s->stream_load[best]++;
    double2* dA = (double2*)(s->arena + r->off);
    double* dres = (double*)(s->arena + r->off + r->bytes - 256);
    int rc = HAF_OK;
    if (r->n > 0 && hipMemcpyAsync(dA, r->A.data(), (size_t)r->n * r->n * sizeof(haf_cplx), hipMemcpyHostToDevice,
                                   st) != hipSuccess)
        return set_error(HAF_E_DEVICE, "matrix upload failed");
    if ((rc = run_dev(dA, r->n, std::max(r->n, 1), r->kind, dres, nullptr, st))) return rc;
    if (hipMemcpyAsync(s->pinned + 4 * r->slot, dres, 4 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
        return set_error(HAF_E_DEVICE, "result download failed");
    if (hipEventRecord(r->ev, st) != hipSuccess) return set_error(HAF_E_DEVICE, "event record failed");
    return HAF_OK;
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
    const int nst = c.continuous ? std::max(1, std::min(c.streams, 64)) : 1;
    if (hipMalloc((void**)&s->arena, (size_t)c.arena_bytes) != hipSuccess) return fail_start("arena allocation failed");
    s->alloc.reset(c.arena_bytes);
    if (hipHostMalloc((void**)&s->pinned, sizeof(double) * 4 * (size_t)c.max_active, hipHostMallocDefault) != hipSuccess)
        return fail_start("pinned result buffer allocation failed");
    for (int i = c.max_active - 1; i >= 0; --i) s->free_slots.push_back(i);
    for (int i = 0; i < nst; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return fail_start("stream creation failed");
        s->streams.push_back(st);
        s->stream_load.push_back(0);
        s->inflight.emplace_back();
    }
    for (int i = 0; i < c.max_active; ++i) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail_start("event creation failed");
        s->events.push_back(e);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->started = true;
        s->cv_start.notify_all();
    }

    for (;;) {
        bool progress = false;
        // ---- admit in arrival order while a slot and arena room are free
        for (;;) {
            Request* r = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->stop || s->queue.empty()) break;
                if (s->n_active >= c.max_active || s->free_slots.empty()) break;
                if (!c.continuous && s->n_active > 0) break;
                r = s->queue.front();
                const int64_t off = s->alloc.alloc(r->bytes);
                if (off < 0) break;
                s->queue.pop_front();
                r->off = off;
            }
            r->slot = s->free_slots.back();
            s->free_slots.pop_back();
            r->ev = s->events.back();
            s->events.pop_back();
            r->t_admit = now_seconds();
            const int rc = launch(s, r);
            if (rc) {
                finish(s, r, rc, nullptr);
            } else {
                s->inflight[r->stream].push_back(r);
                s->n_active++;
            }
            progress = true;
        }
        // ---- completions, in launch order per stream
        for (std::deque<Request*>& q : s->inflight) {
            while (!q.empty()) {
                Request* r = q.front();
                const hipError_t e = hipEventQuery(r->ev);
                if (e == hipErrorNotReady) break;
                q.pop_front();
                s->n_active--;
                if (e == hipSuccess) finish(s, r, HAF_OK, s->pinned + 4 * r->slot);
                else finish(s, r, HAF_E_DEVICE, nullptr);
                progress = true;
            }
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->stop && s->n_active == 0) break;
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
    cfg->max_active = 256;
    cfg->max_queue = 1 << 20;
    cfg->streams = 8;
    cfg->continuous = 1;
}

haf_server* haf_server_create(const haf_server_config* cfg) {
    clear_error();
    if (!cfg || cfg->arena_bytes < 4096 || cfg->max_active < 1 || cfg->max_queue < 1 || cfg->streams < 1) {
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
    const int64_t bytes = request_bytes(n);
    if (bytes > s->cfg.arena_bytes) return set_error(HAF_E_NOMEM, "request of n = %d does not fit the arena", n);
    Request* r = new Request();
    r->n = n;
    r->kind = kind;
    r->bytes = bytes;
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
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    for (std::deque<Request*>& q : s->inflight)
        for (Request* r : q) {
            if (r->ev) (void)hipEventDestroy(r->ev);
            delete r;
        }
    if (s->arena) (void)hipFree(s->arena);
    if (s->pinned) (void)hipHostFree(s->pinned);
    for (Request* r : s->queue) delete r;
    delete s;
}

}  // extern "C"

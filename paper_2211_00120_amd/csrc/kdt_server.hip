// kdt_server.hip -- the build server of include/kdt.h (request loop,
// continuous batching under an HBM budget).
//
// One worker thread per server owns the schedule.  Each pass of its loop
//   1. retires the batches whose completion event has fired (their requests
//      become done; their workspace goes back to the pool), and
//   2. while a batch slot is free, asks choose_batch for the next batch of
//      queued requests that fits the pool, carves its blocks and enqueues it
//      on the slot's stream: copy-in of every request's points, the batched
//      build, copy-back of the batch's status word and of each request's own
//      status word, completion event.
// Submitters, pollers and releasers only touch the queue and the request
// table under the server mutex; the worker enqueues device work outside it.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/kdt.h"
#include "kdt_admit.h"
#include "kdt_host.h"
#include "kdt_plan.h"

namespace {

using namespace kdt;

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum State { QUEUED, RUNNING, DONE };

struct Batch;

struct Request {
    uint64_t ticket = 0;
    const float* h_points = nullptr;
    uint32_t n = 0, k = 0;
    int mode = 0;
    State state = QUEUED;
    int status = KDT_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::shared_ptr<Batch> batch;
    uint64_t off = 0;                 // first entry of the request in its batch
};

struct Batch {
    std::vector<std::shared_ptr<Request>> reqs;
    Plan plan;
    size_t out_off = 0, out_bytes = 0;     // points + outputs block in the pool
    size_t ws_off = 0, ws_bytes = 0;       // workspace block in the pool
    uint32_t refs = 0;                     // requests not released yet
    float device_ms = 0.f;
    char* base = nullptr;                  // pool base
    float* points() const { return (float*)(base + out_off); }
    float* tree() const { return (float*)(base + out_off + align_up(plan.ntotal * plan.k * 4)); }
    uint32_t* perm() const { return (uint32_t*)(base + out_off + 2 * align_up(plan.ntotal * plan.k * 4)); }
    uint8_t* dim() const
    {
        return (uint8_t*)(base + out_off + 2 * align_up(plan.ntotal * plan.k * 4) + align_up(plan.ntotal * 4));
    }
    uint32_t* status() const { return (uint32_t*)(base + out_off + out_bytes - WS_ALIGN); }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t start = nullptr, done = nullptr;
    void* pinned = nullptr;                // share tables of the running batch
    size_t pinned_bytes = 0;
    uint32_t* h_status = nullptr;          // pinned: the batch status word, then one word per request
    size_t h_status_words = 0;
    std::shared_ptr<Batch> batch;          // running batch, if any
};

}  // namespace

struct kdt_server {
    kdt_server_config cfg{};
    int device = 0;
    char* pool_base = nullptr;
    ArenaAllocator pool;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;            // wakes the worker (submit, release, stop)
    std::condition_variable done_cv;       // wakes waiters
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> table;
    uint64_t next_ticket = 1;
    uint64_t gen = 0;                      // bumped by submit, release and stop
    bool stop = false;
    std::thread worker;

    void run();
    void retire(Slot& sl);
    void launch(Slot& sl, const std::shared_ptr<Batch>& b);
    void fail_batch(const std::shared_ptr<Batch>& b, int status);
};

void kdt_server::fail_batch(const std::shared_ptr<Batch>& b, int status)
{
    const double t = now_s();
    for (auto& r : b->reqs) {
        r->status = status;
        r->state = DONE;
        r->t_done = t;
    }
}

// Enqueue one batch on its slot (called without the mutex held; the batch
// and its requests belong to the worker until they are marked done).
void kdt_server::launch(Slot& sl, const std::shared_ptr<Batch>& b)
{
    const Plan& p = b->plan;
    hipStream_t st = sl.stream;
    bool ok = hipEventRecord(sl.start, st) == hipSuccess;
    if (ok && sl.h_status_words < 1 + b->reqs.size()) {
        // the slot has no batch in flight, so its status words are free
        if (sl.h_status) (void)hipHostFree(sl.h_status);
        sl.h_status = nullptr;
        sl.h_status_words = 0;
        ok = hipHostMalloc((void**)&sl.h_status, (1 + b->reqs.size()) * 4, hipHostMallocDefault) == hipSuccess;
        if (ok) sl.h_status_words = 1 + b->reqs.size();
    }
    for (auto& r : b->reqs)
        if (ok && r->n)
            ok = hipMemcpyAsync(b->points() + r->off * p.k, r->h_points, (size_t)r->n * r->k * 4,
                                hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok && p.tables) {
        if (sl.pinned_bytes < p.blob.size()) {
            if (sl.pinned) (void)hipHostFree(sl.pinned);
            sl.pinned = nullptr;
            sl.pinned_bytes = 0;
            ok = hipHostMalloc(&sl.pinned, p.blob.size(), hipHostMallocDefault) == hipSuccess;
            if (ok) sl.pinned_bytes = p.blob.size();
        }
        // the slot's previous batch has finished, so its tables are free
        if (ok) memcpy(sl.pinned, p.blob.data(), p.blob.size());
    }
    int rc = ok ? KDT_OK : KDT_EDEVICE;
    if (ok)
        rc = enqueue_plan(p, b->points(), b->tree(), b->perm(), b->dim(), b->status(), b->base + b->ws_off,
                          sl.pinned, st);
    if (rc == KDT_OK) {
        // the batch's status word, then each request's own (tree t of the
        // plan is request t of the batch), read by retire()
        const size_t nt = p.trees.size();
        ok = hipMemcpyAsync(sl.h_status, b->status(), 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
             hipMemcpyAsync(sl.h_status + 1, b->base + b->ws_off + p.o_tstatus, nt * 4, hipMemcpyDeviceToHost,
                            st) == hipSuccess &&
             hipEventRecord(sl.done, st) == hipSuccess;
        if (!ok) rc = KDT_EDEVICE;
    }
    if (rc != KDT_OK) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(st);
        std::lock_guard<std::mutex> lk(mu);
        fail_batch(b, rc);
        pool.release(b->ws_off, b->ws_bytes);
        sl.batch.reset();
        done_cv.notify_all();
    }
}

// A batch whose completion event fired: its requests are done.
void kdt_server::retire(Slot& sl)
{
    std::shared_ptr<Batch> b = sl.batch;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, sl.start, sl.done);
    b->device_ms = ms;
    // each request's result is its own build's: non-finite input is
    // reported per request; an internal failure of the batch fails them all
    const uint32_t dev_status = sl.h_status[0];
    const double t = now_s();
    for (size_t j = 0; j < b->reqs.size(); ++j) {
        auto& r = b->reqs[j];
        const uint32_t own = sl.h_status[1 + j];
        r->status = (dev_status & KDT_STATUS_INTERNAL) ? KDT_EDEVICE
                    : (own & KDT_ENONFINITE)          ? KDT_ENONFINITE
                                                       : KDT_OK;
        r->state = DONE;
        r->t_done = t;
    }
    pool.release(b->ws_off, b->ws_bytes);
    b->ws_bytes = 0;
    sl.batch.reset();
    done_cv.notify_all();
}

void kdt_server::run()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        const uint64_t seen = gen;
        bool progressed = false;
        bool busy = false;
        for (Slot& sl : slots) {
            if (!sl.batch) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                retire(sl);
                progressed = true;
            } else if (q == hipErrorNotReady) {
                busy = true;
            } else {
                // the device reported an error for this stream
                (void)hipGetLastError();
                std::shared_ptr<Batch> b = sl.batch;
                fail_batch(b, KDT_EDEVICE);
                pool.release(b->ws_off, b->ws_bytes);
                b->ws_bytes = 0;
                sl.batch.reset();
                done_cv.notify_all();
                progressed = true;
            }
        }
        for (Slot& sl : slots) {
            if (sl.batch || queue.empty()) continue;
            std::vector<QueuedShape> shapes;
            const size_t look = std::min<size_t>(queue.size(), 4u * cfg.max_batch_requests);
            for (size_t i = 0; i < look; ++i) shapes.push_back({queue[i]->n, queue[i]->k, queue[i]->mode});
            const BatchChoice c = choose_batch(shapes, pool, cfg.max_batch_requests, cfg.max_batch_points);
            if (c.picks.empty()) break;
            auto b = std::make_shared<Batch>();
            b->base = pool_base;
            b->out_bytes = c.out_bytes;
            b->ws_bytes = c.ws_bytes;
            b->out_off = pool.alloc(c.out_bytes);
            b->ws_off = pool.alloc(c.ws_bytes);
            if (b->out_off == ArenaAllocator::NPOS || b->ws_off == ArenaAllocator::NPOS) {
                // choose_batch checked both blocks on a copy of the pool
                if (b->out_off != ArenaAllocator::NPOS) pool.release(b->out_off, c.out_bytes);
                if (b->ws_off != ArenaAllocator::NPOS) pool.release(b->ws_off, c.ws_bytes);
                break;
            }
            std::vector<uint32_t> sizes;
            uint64_t off = 0;
            const double t = now_s();
            for (size_t j = c.picks.size(); j-- > 0;) {
                auto r = queue[c.picks[j]];
                queue.erase(queue.begin() + (long)c.picks[j]);
                b->reqs.insert(b->reqs.begin(), r);
            }
            for (auto& r : b->reqs) {
                r->state = RUNNING;
                r->t_admit = t;
                r->batch = b;
                r->off = off;
                off += r->n;
                sizes.push_back(r->n);
            }
            b->refs = (uint32_t)b->reqs.size();
            b->plan = make_plan(sizes, b->reqs[0]->k, b->reqs[0]->mode == KDT_DIM_WIDEST);
            sl.batch = b;
            lk.unlock();
            launch(sl, b);
            lk.lock();
            progressed = true;
            busy = true;
        }
        if (progressed) continue;
        if (stop && !busy) {
            if (queue.empty()) break;
            // nothing runs and the oldest request does not fit: results that
            // are never released hold the pool, so the rest cannot start
            const double t = now_s();
            for (auto& r : queue) {
                r->status = KDT_ENOMEM;
                r->state = DONE;
                r->t_done = t;
            }
            queue.clear();
            done_cv.notify_all();
            continue;
        }
        // wait for a device completion (polled) or for a submit / release
        if (busy) cv.wait_for(lk, std::chrono::microseconds(20), [&] { return gen != seen; });
        else cv.wait(lk, [&] { return gen != seen; });
    }
}

namespace {

void fill_result(const Request& r, kdt_result* out)
{
    memset(out, 0, sizeof *out);
    out->status = r.status;
    out->n = r.n;
    out->k = r.k;
    if (r.batch && r.n) {
        out->d_tree = r.batch->tree() + r.off * r.k;
        out->d_perm = r.batch->perm() + r.off;
        out->d_dim = r.batch->dim() + r.off;
        out->device_ms = r.batch->device_ms;
        out->batch_requests = (uint32_t)r.batch->reqs.size();
    }
    out->t_submit = r.t_submit;
    out->t_admit = r.t_admit;
    out->t_done = r.t_done;
}

}  // namespace

extern "C" {

double kdt_clock(void) { return now_s(); }

kdt_status kdt_server_create(const kdt_server_config* cfg, kdt_server** out)
{
    if (!cfg || !out || cfg->hbm_budget_bytes < (1u << 20) || cfg->max_inflight < 1 || cfg->max_inflight > 8 ||
        cfg->max_batch_requests < 1 || cfg->max_batch_points < 1) {
        set_last_error("bad server config (budget >= 1 MiB, 1 <= max_inflight <= 8, batch limits >= 1)");
        return KDT_EINVAL;
    }
    auto s = std::make_unique<kdt_server>();
    s->cfg = *cfg;
    if (hipGetDevice(&s->device) != hipSuccess) {
        set_last_error("no current HIP device");
        return KDT_EDEVICE;
    }
    const size_t bytes = cfg->hbm_budget_bytes & ~(WS_ALIGN - 1);
    if (hipMalloc((void**)&s->pool_base, bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_last_error("hipMalloc of the %zu-byte pool failed", bytes);
        return KDT_ENOMEM;
    }
    s->pool.reset(bytes);
    s->slots.resize(cfg->max_inflight);
    for (Slot& sl : s->slots) {
        bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreate(&sl.start) == hipSuccess && hipEventCreate(&sl.done) == hipSuccess &&
                  hipHostMalloc((void**)&sl.h_status, 2 * 4, hipHostMallocDefault) == hipSuccess;
        if (ok) sl.h_status_words = 2;
        if (!ok) {
            (void)hipGetLastError();
            set_last_error("could not create the server's streams or events");
            for (Slot& x : s->slots) {
                if (x.stream) (void)hipStreamDestroy(x.stream);
                if (x.start) (void)hipEventDestroy(x.start);
                if (x.done) (void)hipEventDestroy(x.done);
                if (x.h_status) (void)hipHostFree(x.h_status);
            }
            (void)hipFree(s->pool_base);
            return KDT_EDEVICE;
        }
    }
    kdt_server* raw = s.release();
    raw->worker = std::thread([raw] { raw->run(); });
    *out = raw;
    return KDT_OK;
}

kdt_status kdt_server_submit(kdt_server* s, const kdt_request* req, uint64_t* ticket)
{
    if (!s || !req || !ticket) {
        set_last_error("null server, request or ticket");
        return KDT_EINVAL;
    }
    if (req->k < 1 || req->k > 4 || (req->dim_mode != KDT_DIM_ROUND_ROBIN && req->dim_mode != KDT_DIM_WIDEST) ||
        req->n > KDT_MAX_POINTS || (req->n > 0 && !req->h_points)) {
        set_last_error("bad request (k in 1..4, valid dim_mode, n <= KDT_MAX_POINTS, points for n > 0)");
        return KDT_EINVAL;
    }
    if (request_footprint(req->n, req->k, req->dim_mode) > s->pool.capacity()) {
        set_last_error("request of %u points needs %zu bytes, more than the pool holds", req->n,
                       request_footprint(req->n, req->k, req->dim_mode));
        return KDT_ENOMEM;
    }
    auto r = std::make_shared<Request>();
    r->h_points = req->h_points;
    r->n = req->n;
    r->k = req->k;
    r->mode = req->dim_mode;
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    s->table[r->ticket] = r;
    if (r->n == 0) {
        r->state = DONE;
        r->t_admit = r->t_done = r->t_submit;
    } else {
        s->queue.push_back(r);
        ++s->gen;
        s->cv.notify_all();
    }
    *ticket = r->ticket;
    return KDT_OK;
}

kdt_status kdt_server_poll(kdt_server* s, uint64_t ticket, kdt_result* out)
{
    if (!s || !out) return KDT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return KDT_ENOTFOUND;
    if (it->second->state != DONE) return KDT_EBUSY;
    fill_result(*it->second, out);
    return KDT_OK;
}

kdt_status kdt_server_wait(kdt_server* s, uint64_t ticket, kdt_result* out)
{
    if (!s || !out) return KDT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return KDT_ENOTFOUND;
    std::shared_ptr<Request> r = it->second;
    s->done_cv.wait(lk, [&] { return r->state == DONE; });
    fill_result(*r, out);
    return KDT_OK;
}

kdt_status kdt_server_copy_out(kdt_server* s, uint64_t ticket, float* d_tree, uint32_t* d_perm, uint8_t* d_dim,
                               hipStream_t stream)
{
    if (!s) return KDT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return KDT_ENOTFOUND;
    const Request& r = *it->second;
    if (r.state != DONE) return KDT_EBUSY;
    if (!r.batch || r.n == 0) return KDT_OK;
    const Batch& b = *r.batch;
    bool ok = true;
    if (d_tree)
        ok = ok && hipMemcpyAsync(d_tree, b.tree() + r.off * r.k, (size_t)r.n * r.k * 4, hipMemcpyDeviceToDevice,
                                  stream) == hipSuccess;
    if (d_perm)
        ok = ok && hipMemcpyAsync(d_perm, b.perm() + r.off, (size_t)r.n * 4, hipMemcpyDeviceToDevice, stream) ==
                       hipSuccess;
    if (d_dim)
        ok = ok && hipMemcpyAsync(d_dim, b.dim() + r.off, r.n, hipMemcpyDeviceToDevice, stream) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        set_last_error("copy of a server result failed");
        return KDT_EDEVICE;
    }
    return KDT_OK;
}

kdt_status kdt_server_release(kdt_server* s, uint64_t ticket)
{
    if (!s) return KDT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->table.find(ticket);
    if (it == s->table.end()) return KDT_ENOTFOUND;
    std::shared_ptr<Request> r = it->second;
    if (r->state != DONE) return KDT_EBUSY;
    s->table.erase(it);
    if (r->batch) {
        std::shared_ptr<Batch> b = r->batch;
        r->batch.reset();
        if (--b->refs == 0) {
            s->pool.release(b->out_off, b->out_bytes);
            ++s->gen;
            s->cv.notify_all();
        }
    }
    return KDT_OK;
}

kdt_status kdt_server_destroy(kdt_server* s)
{
    if (!s) return KDT_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        ++s->gen;
        s->cv.notify_all();
    }
    s->worker.join();
    for (Slot& sl : s->slots) {
        (void)hipStreamSynchronize(sl.stream);
        (void)hipStreamDestroy(sl.stream);
        (void)hipEventDestroy(sl.start);
        (void)hipEventDestroy(sl.done);
        (void)hipHostFree(sl.h_status);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
    }
    (void)hipFree(s->pool_base);
    delete s;
    return KDT_OK;
}

}  // extern "C"

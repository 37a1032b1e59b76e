// Serving: hull requests of mixed sizes that arrive over time, computed with
// continuous batching on one GPU (the method of Section 2.1 per request).
//
// A request names its points in device memory and its output buffers; the
// server admits it against a memory budget and queues it.  Worker threads,
// each with its own HIP stream (and so its own library workspace), take the
// oldest pending work whenever they are free:
//   * a large request (more points than the tuned serve_batch_max, 2^18 by
//     default) alone, through the
//     single-hull path (`hull2d`), which uses the whole device;
//   * otherwise every pending small request (up to kServeBatchSets sets and
//     kServeBatchPoints points): their points are gathered into the
//     worker's staging buffer and computed by one `hull2d_batched` launch,
//     one workgroup per request, then copied out to each request's buffers.
// Requests that arrive while others run are admitted and batched as soon as
// a worker and budget free up; the workers' streams overlap on the device.
// Results do not depend on the mix: each request's hull is exactly the one
// `hull2d` gives for it alone.
//
// Admission: a request holds `need` bytes of the budget from admission to
// completion (12 bytes per point for a batched request's staging, the
// single-hull workspace bound for a large one).  Admission is first come,
// first served; a request that could never fit is refused with CH_EADMIT.
// The memory a worker keeps between requests (its stream's workspace and
// its staging buffers) counts against the budget too: when it would take
// the requests in flight and the workers' memory past the budget, the
// worker gives its memory back after its request.  The server's device
// memory then stays within the budget plus what the running requests
// allocate beyond their share.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "chainhull.h"

namespace chainhull {
namespace {

constexpr int32_t kServeBatchSets = 4096;           // requests per batched launch
constexpr int64_t kServeBatchPoints = 64ll << 20;   // points per batched launch
constexpr int32_t kServeMaxWorkers = 16;

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    const float* pts = nullptr;
    int64_t n = 0;
    int32_t* out_idx = nullptr;
    int32_t* out_count = nullptr;
    size_t need = 0;
    int status = CH_OK;
    int32_t hull = 0;
    bool done = false;
    bool claimed = false;  // a wait holds it
    Clock::time_point t_submit, t_done;
};

struct Worker {
    hipStream_t stream = nullptr;
    float* stage_pts = nullptr;  // gathered points of a batch
    int32_t* stage_out = nullptr;
    int32_t* stage_cnt = nullptr;
    int32_t* h_cnt = nullptr;    // pinned copy of the counts
    int64_t stage_cap = 0;       // points
    int32_t sets_cap = 0;
    int64_t ws_n = 0;            // the most points one call on its stream has had (its workspace)
    size_t retained = 0;         // device bytes it keeps between requests (workspace and staging)
    bool busy = false;           // running a request (under the server's lock)
    std::thread th;
};

// Device memory a worker keeps: its stream's workspace and its staging.
size_t retained_bytes(const Worker& w)
{
    return (w.ws_n ? chainhull_workspace_bytes(w.ws_n) : 0) + (size_t)w.stage_cap * 12 + (size_t)w.sets_cap * 4;
}

// Give a worker's memory back: its stream's workspace and its staging.
void release_worker(Worker& w)
{
    (void)hipStreamSynchronize(w.stream);
    (void)chainhull_release_stream(w.stream);
    if (w.stage_pts) (void)hipFree(w.stage_pts);
    if (w.stage_out) (void)hipFree(w.stage_out);
    if (w.stage_cnt) (void)hipFree(w.stage_cnt);
    if (w.h_cnt) (void)hipHostFree(w.h_cnt);
    w.stage_pts = nullptr;
    w.stage_out = nullptr;
    w.stage_cnt = nullptr;
    w.h_cnt = nullptr;
    w.stage_cap = 0;
    w.sets_cap = 0;
    w.ws_n = 0;
}

}  // namespace
}  // namespace chainhull

struct ch_server {
    int device = 0;
    int64_t batch_max = 0;  // requests of at most this many points are batched (the tuned shape)
    size_t budget = 0;
    size_t reserved = 0;
    size_t retained = 0;  // device bytes the workers keep between requests
    bool stop = false;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv_work;  // pending work or stop
    std::condition_variable cv_done;  // a request completed
    std::deque<chainhull::Request*> admission;     // waiting for budget
    std::deque<chainhull::Request*> small, large;  // admitted, not started
    std::unordered_map<uint64_t, chainhull::Request*> reqs;
    std::vector<chainhull::Worker> workers;
    // counters
    int64_t completed = 0, batches = 0, batched_requests = 0, single_requests = 0, points = 0;
    int32_t max_inflight = 0, inflight = 0;
};

namespace chainhull {
namespace {

size_t need_of(const ch_server* s, int64_t n)
{
    if (n <= s->batch_max) return (size_t)n * 12 + 64;
    return chainhull_workspace_bytes(n);
}

// Admit from the head of the admission queue while the budget allows: the
// requests in flight, the memory the workers keep and the head's need must
// fit.  When only the memory of idle workers stands in the way, they give
// it back first.  Caller holds s->mu.
void admit_locked(ch_server* s)
{
    bool any = false;
    while (!s->admission.empty()) {
        const size_t need = s->admission.front()->need;
        if (s->reserved + s->retained + need > s->budget) {
            for (auto& w : s->workers) {
                if (w.busy || !w.retained) continue;
                release_worker(w);
                s->retained -= w.retained;
                w.retained = 0;
            }
            if (s->reserved + s->retained + need > s->budget) break;
        }
        Request* r = s->admission.front();
        s->admission.pop_front();
        s->reserved += r->need;
        (r->n <= s->batch_max ? s->small : s->large).push_back(r);
        any = true;
    }
    if (any) s->cv_work.notify_all();
}

void finish_locked(ch_server* s, Request* r, int status, int32_t hull)
{
    r->status = status;
    r->hull = hull;
    r->done = true;
    r->t_done = Clock::now();
    s->reserved -= r->need;
    s->completed += 1;
    s->points += r->n;
    s->inflight -= 1;
}

int grow(Worker& w, int64_t pts, int32_t sets)
{
    if (pts > w.stage_cap) {
        if (w.stage_pts) (void)hipFree(w.stage_pts);
        if (w.stage_out) (void)hipFree(w.stage_out);
        w.stage_pts = nullptr;
        w.stage_out = nullptr;
        w.stage_cap = 0;
        const int64_t cap = std::max<int64_t>(pts, 1 << 20);
        if (hipMalloc(reinterpret_cast<void**>(&w.stage_pts), (size_t)cap * 8) != hipSuccess) return CH_ENOMEM;
        if (hipMalloc(reinterpret_cast<void**>(&w.stage_out), (size_t)cap * 4) != hipSuccess) return CH_ENOMEM;
        w.stage_cap = cap;
    }
    if (sets > w.sets_cap) {
        if (w.stage_cnt) (void)hipFree(w.stage_cnt);
        if (w.h_cnt) (void)hipHostFree(w.h_cnt);
        w.stage_cnt = nullptr;
        w.h_cnt = nullptr;
        w.sets_cap = 0;
        const int32_t cap = std::max<int32_t>(sets, 1024);
        if (hipMalloc(reinterpret_cast<void**>(&w.stage_cnt), (size_t)cap * 4) != hipSuccess) return CH_ENOMEM;
        if (hipHostMalloc(reinterpret_cast<void**>(&w.h_cnt), (size_t)cap * 4, hipHostMallocDefault) != hipSuccess)
            return CH_ENOMEM;
        w.sets_cap = cap;
    }
    return CH_OK;
}

// One batched launch over small requests; returns per-request statuses in
// place (status, hull).
void run_batch(Worker& w, std::vector<Request*>& batch)
{
    int64_t total = 0;
    for (Request* r : batch) {
        total += r->n;
        w.ws_n = std::max(w.ws_n, r->n);  // (a set the kernel hands back runs alone on this stream)
    }
    int rc = grow(w, total, (int32_t)batch.size());
    std::vector<int64_t> offs(batch.size() + 1, 0);
    for (size_t k = 0; k < batch.size(); ++k) offs[k + 1] = offs[k] + batch[k]->n;
    for (size_t k = 0; k < batch.size() && rc == CH_OK; ++k) {
        if (batch[k]->n > 0 &&
            hipMemcpyAsync(w.stage_pts + 2 * offs[k], batch[k]->pts, (size_t)batch[k]->n * 8,
                           hipMemcpyDeviceToDevice, w.stream) != hipSuccess)
            rc = CH_EHIP;
    }
    if (rc == CH_OK) {
        const int b = hull2d_batched(w.stage_pts, offs.data(), (int32_t)batch.size(), w.stage_out, w.stage_cnt,
                                     w.stream);
        // per-set failures come back in the counts; anything else fails all
        if (b != CH_OK && b != CH_EDOMAIN) rc = b;
    }
    if (rc == CH_OK && (hipMemcpyAsync(w.h_cnt, w.stage_cnt, batch.size() * 4, hipMemcpyDeviceToHost, w.stream) !=
                            hipSuccess ||
                        hipStreamSynchronize(w.stream) != hipSuccess))
        rc = CH_EHIP;
    for (size_t k = 0; k < batch.size(); ++k) {
        Request* r = batch[k];
        if (rc != CH_OK) {
            r->status = rc;
            r->hull = 0;
            continue;
        }
        const int32_t c = w.h_cnt[k];
        r->status = c < 0 ? c : CH_OK;
        r->hull = c < 0 ? 0 : c;
        // a failed request's count is 0, as hull2d leaves it; its status is
        // the ticket's
        bool ok = c < 0 ? hipMemsetAsync(r->out_count, 0, 4, w.stream) == hipSuccess
                        : hipMemcpyAsync(r->out_count, w.stage_cnt + k, 4, hipMemcpyDeviceToDevice, w.stream) ==
                              hipSuccess;
        if (c > 0)
            ok = ok && hipMemcpyAsync(r->out_idx, w.stage_out + offs[k], (size_t)c * 4, hipMemcpyDeviceToDevice,
                                      w.stream) == hipSuccess;
        if (!ok) r->status = CH_EHIP;
    }
    if (hipStreamSynchronize(w.stream) != hipSuccess) {
        for (Request* r : batch) r->status = CH_EHIP;
    }
}

void run_single(Worker& w, Request* r)
{
    w.ws_n = std::max(w.ws_n, r->n);
    int rc = hull2d(r->pts, r->n, r->out_idx, r->out_count, w.stream);
    int32_t h = 0;
    if (rc == CH_OK) {
        ch_stats st;
        if (chainhull_last_stats(&st) == CH_OK) h = (int32_t)st.hull;
    }
    if (hipStreamSynchronize(w.stream) != hipSuccess && rc == CH_OK) rc = CH_EHIP;
    r->status = rc;
    r->hull = rc == CH_OK ? h : 0;
}

void worker_loop(ch_server* s, Worker* w)
{
    (void)hipSetDevice(s->device);
    std::vector<Request*> batch;
    for (;;) {
        Request* single = nullptr;
        batch.clear();
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->small.empty() || !s->large.empty(); });
            if (s->small.empty() && s->large.empty()) return;  // stopping, nothing left
            // the oldest pending work first
            const bool take_large =
                !s->large.empty() && (s->small.empty() || s->large.front()->t_submit <= s->small.front()->t_submit);
            if (take_large) {
                single = s->large.front();
                s->large.pop_front();
                s->single_requests += 1;
            } else {
                int64_t pts = 0;
                while (!s->small.empty() && (int32_t)batch.size() < kServeBatchSets &&
                       (batch.empty() || pts + s->small.front()->n <= kServeBatchPoints)) {
                    pts += s->small.front()->n;
                    batch.push_back(s->small.front());
                    s->small.pop_front();
                }
                s->batches += 1;
                s->batched_requests += (int64_t)batch.size();
            }
            w->busy = true;
            s->inflight += single ? 1 : (int32_t)batch.size();
            s->max_inflight = std::max(s->max_inflight, s->inflight);
        }
        if (single) {
            run_single(*w, single);
        } else {
            run_batch(*w, batch);
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (single) {
                finish_locked(s, single, single->status, single->hull);
            } else {
                for (Request* r : batch) finish_locked(s, r, r->status, r->hull);
            }
            // the memory this worker keeps counts against the budget with the
            // requests in flight; beyond it, the worker gives its memory back
            w->busy = false;
            s->retained -= w->retained;
            w->retained = retained_bytes(*w);
            if (s->reserved + s->retained + w->retained > s->budget) {
                release_worker(*w);
                w->retained = 0;
            }
            s->retained += w->retained;
            admit_locked(s);  // (may release idle workers' memory for the next request)
        }
        s->cv_done.notify_all();
    }
}

}  // namespace
}  // namespace chainhull

using namespace chainhull;

extern "C" {

int chainhull_server_create(int32_t workers, size_t mem_budget, ch_server** out)
{
    if (!out || workers < 1 || workers > kServeMaxWorkers || mem_budget == 0) return CH_EINVAL;
    *out = nullptr;
    ch_server* s = new ch_server();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return CH_EHIP;
    }
    s->budget = mem_budget;
    ch_tuning tu;
    (void)chainhull_get_tuning(INT64_MAX, &tu);
    s->batch_max = tu.serve_batch_max;
    s->workers.resize((size_t)workers);
    for (auto& w : s->workers) {
        if (hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess) {
            for (auto& v : s->workers)
                if (v.stream) (void)hipStreamDestroy(v.stream);
            delete s;
            return CH_EHIP;
        }
    }
    for (auto& w : s->workers) w.th = std::thread(worker_loop, s, &w);
    *out = s;
    return CH_OK;
}

int chainhull_server_submit(ch_server* s, const float* points, int64_t n, int32_t* out_idx, int32_t* out_count,
                            uint64_t* ticket)
{
    if (!s || !ticket || !out_count || n < 0 || n > INT32_MAX || (n > 0 && (!points || !out_idx))) return CH_EINVAL;
    if (reinterpret_cast<uintptr_t>(points) & 7u) return CH_EINVAL;
    const size_t need = need_of(s, n);
    if (need > s->budget) return CH_EADMIT;
    Request* r = new Request();
    r->pts = points;
    r->n = n;
    r->out_idx = out_idx;
    r->out_count = out_count;
    r->need = need;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        delete r;
        return CH_EINVAL;
    }
    r->ticket = s->next_ticket++;
    s->reqs[r->ticket] = r;
    s->admission.push_back(r);
    admit_locked(s);
    *ticket = r->ticket;
    return CH_OK;
}

int chainhull_server_wait(ch_server* s, uint64_t ticket, int32_t* hull, double* latency_ms)
{
    if (!s) return CH_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return CH_EINVAL;
    Request* r = it->second;
    if (r->claimed) return CH_EINVAL;  // another thread waits for it
    r->claimed = true;
    s->cv_done.wait(lk, [&] { return r->done; });
    const int status = r->status;
    if (hull) *hull = r->hull;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    s->reqs.erase(it);
    delete r;
    return status;
}

int chainhull_server_stats(ch_server* s, ch_server_stats* out)
{
    if (!s || !out) return CH_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->completed = s->completed;
    out->batches = s->batches;
    out->batched_requests = s->batched_requests;
    out->single_requests = s->single_requests;
    out->points = s->points;
    out->pending = (int64_t)(s->admission.size() + s->small.size() + s->large.size());
    out->max_inflight = s->max_inflight;
    out->reserved_bytes = s->reserved;
    return CH_OK;
}

int chainhull_server_destroy(ch_server* s)
{
    if (!s) return CH_EINVAL;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        // everything admitted or waiting is computed first
        s->cv_done.wait(lk, [&] { return s->admission.empty() && s->small.empty() && s->large.empty() && s->inflight == 0; });
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& w : s->workers) {
        if (w.th.joinable()) w.th.join();
    }
    (void)hipSetDevice(s->device);
    for (auto& w : s->workers) {
        if (w.stream) (void)hipStreamSynchronize(w.stream);
        if (w.stage_pts) (void)hipFree(w.stage_pts);
        if (w.stage_out) (void)hipFree(w.stage_out);
        if (w.stage_cnt) (void)hipFree(w.stage_cnt);
        if (w.h_cnt) (void)hipHostFree(w.h_cnt);
        if (w.stream) {
            (void)chainhull_release_stream(w.stream);
            (void)hipStreamDestroy(w.stream);
        }
    }
    for (auto& kv : s->reqs) delete kv.second;
    delete s;
    return CH_OK;
}

}  // extern "C"

// Batched request server of the C ABI (rsvd_server_*): continuous batching
// of independent randomized SVD requests of uneven shape on one GPU.
//
// Requests are queued on submit and admitted in arrival order as soon as a
// stream slot is free and their workspace fits in the server's HBM budget
// (one device arena, sub-allocated first fit).  An admitted request is one
// rsvd_solve on its slot's stream, so requests that arrive while others run
// overlap on the device; each uses its own workspace and the same
// deterministic kernels, so its result is the same alone and in the mix.
// A scheduler thread admits, launches and retires requests (retirement:
// the request's completion event has fired; its workspace and slot return
// to the pools).  Latency is measured from submit to the scheduler seeing
// the completion.
//
// Launch graphs: by default an admitted request's kernels are captured from
// rsvd_solve into a HIP graph and launched as one graph.  Each slot keeps
// the executable graphs of its last few shape buckets (a bucket = every
// parameter that fixes the kernel sequence: precision, m, n, k, p, q and the
// options); a request of a cached bucket updates that executable graph in
// place with its own pointers and sizes (hipGraphExecUpdate), otherwise a new
// one is instantiated.  The captured kernels are exactly those rsvd_solve
// enqueues (no memset or copy nodes), so a graph computes what the direct
// launches compute.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/rsvd.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t kArenaAlign = 256;

// First-fit allocator over [0, size) with coalescing on free.
class Arena {
public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_[*off] = bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                prev->second += len;
                return;
            }
        }
        free_[start] = len;
    }

private:
    std::map<size_t, size_t> free_, used_;
};

// Everything about a request that decides which kernels rsvd_solve launches.
struct BucketKey {
    int64_t v[17];
    bool operator==(const BucketKey& o) const {
        for (int i = 0; i < 17; ++i)
            if (v[i] != o.v[i]) return false;
        return true;
    }
};

struct GraphEntry {
    BucketKey key;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};
constexpr size_t kGraphsPerSlot = 8;

struct Request {
    uint64_t ticket;
    rsvd_matrix A;
    rsvd_params params;
    rsvd_result out;
    size_t ws_bytes = 0;
    size_t ws_off = 0;
    int slot = -1;
    Clock::time_point t_submit, t_done;
    rsvd_status status = RSVD_OK;
    bool done = false;
};

}  // namespace

struct rsvd_server {
    int device = 0;
    rsvd_handle* h = nullptr;
    void* arena_base = nullptr;
    size_t arena_bytes = 0;
    Arena* arena = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<int> slot_busy;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::vector<Request*> running;
    std::map<uint64_t, Request*> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    // launch graphs, per slot
    std::atomic<bool> use_graphs{true};
    std::vector<std::vector<GraphEntry>> graphs;       // touched by the scheduler thread only
    uint64_t graph_clock = 0;
    std::atomic<int64_t> graph_launches{0}, graph_instantiations{0};

    // statistics
    std::vector<double> latencies_ms;
    Clock::time_point t_first{}, t_last{};
    bool any = false;

    void loop();
    rsvd_status launch(Request* r, int slot, void* ws);
};

namespace {

BucketKey bucket_of(const Request* r) {
    const rsvd_params& p = r->params;
    return BucketKey{{(int64_t)r->A.dtype, r->A.rows, r->A.cols, p.k, p.p, p.q, (int64_t)p.extra_power_pass,
                      (int64_t)p.residual, (int64_t)p.residual_iters, (int64_t)p.return_full_l,
                      (int64_t)p.orth, r->out.Q != nullptr, r->A.master != nullptr,
                      r->A.col_scale != nullptr, (int64_t)p.algorithm, (int64_t)p.jacobi_max_sweeps,
                      (int64_t)p.test_matrix}};
}

}  // namespace

// Enqueue one admitted request on its slot's stream: directly, or captured
// into a graph that replaces (or updates) the slot's graph of its bucket.
rsvd_status rsvd_server::launch(Request* r, int slot, void* ws) {
    hipStream_t st = streams[slot];
    if (!use_graphs) return rsvd_solve(h, &r->A, &r->params, &r->out, ws, r->ws_bytes, st);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) return RSVD_ERR_DEVICE;
    const rsvd_status rs = rsvd_solve(h, &r->A, &r->params, &r->out, ws, r->ws_bytes, st);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (rs != RSVD_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rs != RSVD_OK ? rs : RSVD_ERR_DEVICE;
    }
    const BucketKey key = bucket_of(r);
    std::vector<GraphEntry>& cache = graphs[slot];
    GraphEntry* ent = nullptr;
    for (auto& e : cache)
        if (e.key == key) ent = &e;
    bool ready = false;
    if (ent) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        if (hipGraphExecUpdate(ent->exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
            ready = true;
        } else {
            (void)hipGraphExecDestroy(ent->exec);
            ent->exec = nullptr;
        }
    } else {
        if (cache.size() >= kGraphsPerSlot) {         // evict the least recently used bucket
            auto lru = std::min_element(cache.begin(), cache.end(),
                                        [](const GraphEntry& a, const GraphEntry& b) { return a.last_use < b.last_use; });
            if (lru->exec) (void)hipGraphExecDestroy(lru->exec);
            cache.erase(lru);
        }
        cache.push_back(GraphEntry{key, nullptr, 0});
        ent = &cache.back();
    }
    if (!ready) {
        if (hipGraphInstantiate(&ent->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            ent->exec = nullptr;
            (void)hipGraphDestroy(g);
            return RSVD_ERR_DEVICE;
        }
        ++graph_instantiations;
    }
    ent->last_use = ++graph_clock;
    const hipError_t el = hipGraphLaunch(ent->exec, st);
    (void)hipGraphDestroy(g);
    if (el != hipSuccess) return RSVD_ERR_DEVICE;
    ++graph_launches;
    return RSVD_OK;
}

void rsvd_server::loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        // Retire finished requests.
        bool progressed = false;
        for (size_t i = 0; i < running.size();) {
            Request* r = running[i];
            const hipError_t q = hipEventQuery(events[r->slot]);
            if (q == hipErrorNotReady) { ++i; continue; }
            r->t_done = Clock::now();
            if (q != hipSuccess) r->status = RSVD_ERR_DEVICE;
            arena->release(r->ws_off);
            slot_busy[r->slot] = 0;
            r->done = true;
            latencies_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
            t_last = r->t_done;
            running[i] = running.back();
            running.pop_back();
            progressed = true;
        }
        if (progressed) cv_done.notify_all();
        // Admit in arrival order while a slot is free and the workspace fits.
        while (!pending.empty()) {
            Request* r = pending.front();
            int slot = -1;
            for (size_t s = 0; s < slot_busy.size(); ++s)
                if (!slot_busy[s]) { slot = (int)s; break; }
            if (slot < 0) break;
            size_t off = 0;
            if (!arena->alloc(r->ws_bytes, &off)) {
                if (running.empty()) {          // can never fit
                    r->status = RSVD_ERR_NO_MEMORY;
                    r->done = true;
                    pending.pop_front();
                    cv_done.notify_all();
                    continue;
                }
                break;
            }
            pending.pop_front();
            r->ws_off = off;
            r->slot = slot;
            slot_busy[slot] = 1;
            void* ws = static_cast<char*>(arena_base) + off;
            lk.unlock();                        // launch without holding the lock
            rsvd_status st = launch(r, slot, ws);
            hipError_t e = hipEventRecord(events[slot], streams[slot]);
            lk.lock();
            if (st != RSVD_OK || e != hipSuccess) {
                // nothing (or not all) was enqueued: retire on the spot once the stream drains
                r->status = st != RSVD_OK ? st : RSVD_ERR_DEVICE;
            }
            running.push_back(r);
        }
        if (stop && pending.empty() && running.empty()) break;
        if (running.empty() && pending.empty()) {
            cv_work.wait(lk, [&] { return stop || !pending.empty(); });
        } else {
            // poll the in-flight events at a short interval
            cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

extern "C" {

rsvd_status rsvd_server_create(rsvd_server** out, int device, size_t hbm_budget_bytes, int n_streams) {
    if (!out || n_streams < 1 || n_streams > 64 || hbm_budget_bytes < kArenaAlign) return RSVD_ERR_INVALID_ARG;
    *out = nullptr;
    rsvd_server* s = new (std::nothrow) rsvd_server;
    if (!s) return RSVD_ERR_NO_MEMORY;
    s->device = device;
    rsvd_status st = rsvd_create(&s->h, device);
    if (st != RSVD_OK) { delete s; return st; }
    if (hipSetDevice(device) != hipSuccess) { rsvd_destroy(s->h); delete s; return RSVD_ERR_DEVICE; }
    if (hipMalloc(&s->arena_base, hbm_budget_bytes) != hipSuccess) {
        rsvd_destroy(s->h);
        delete s;
        return RSVD_ERR_NO_MEMORY;
    }
    s->arena_bytes = hbm_budget_bytes;
    s->arena = new Arena(hbm_budget_bytes);
    s->streams.assign(n_streams, nullptr);
    s->events.assign(n_streams, nullptr);
    s->slot_busy.assign(n_streams, 0);
    s->graphs.assign(n_streams, {});
    for (int i = 0; i < n_streams; ++i) {
        // default priority: every stream of the server is an ordinary stream
        if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming) != hipSuccess) {
            s->stop = true;                 // no worker yet: destroy only releases
            rsvd_server_destroy(s);
            return RSVD_ERR_DEVICE;
        }
    }
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return RSVD_OK;
}

rsvd_status rsvd_server_submit(rsvd_server* s, const rsvd_matrix* A, const rsvd_params* params,
                               const rsvd_result* out, uint64_t* ticket) {
    if (!s || !A || !params || !out || !ticket) return RSVD_ERR_INVALID_ARG;
    size_t bytes = 0;
    rsvd_status st = rsvd_workspace_size(s->h, A, params, &bytes);
    if (st != RSVD_OK) return st;
    if (bytes > s->arena_bytes) return RSVD_ERR_NO_MEMORY;
    Request* r = new (std::nothrow) Request;
    if (!r) return RSVD_ERR_NO_MEMORY;
    r->A = *A;
    r->params = *params;
    r->out = *out;
    r->ws_bytes = bytes;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) { delete r; return RSVD_ERR_INVALID_ARG; }
        r->ticket = s->next_ticket++;
        if (!s->any) { s->t_first = r->t_submit; s->any = true; }
        s->all[r->ticket] = r;
        s->pending.push_back(r);
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return RSVD_OK;
}

rsvd_status rsvd_server_poll(rsvd_server* s, uint64_t ticket, int* done, rsvd_status* final_status) {
    if (!s || !done) return RSVD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return RSVD_ERR_INVALID_ARG;
    *done = it->second->done ? 1 : 0;
    if (final_status) *final_status = it->second->status;
    return RSVD_OK;
}

rsvd_status rsvd_server_wait(rsvd_server* s, uint64_t ticket, rsvd_status* final_status, double* latency_ms) {
    if (!s) return RSVD_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return RSVD_ERR_INVALID_ARG;
    Request* r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    if (final_status) *final_status = r->status;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    return RSVD_OK;
}

rsvd_status rsvd_server_drain(rsvd_server* s) {
    if (!s) return RSVD_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->pending.empty() && s->running.empty(); });
    return RSVD_OK;
}

rsvd_status rsvd_server_stats(rsvd_server* s, double* p50_ms, double* p99_ms, double* solves_per_s,
                              int64_t* completed) {
    if (!s) return RSVD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    std::vector<double> v = s->latencies_ms;
    const size_t nlat = v.size();
    auto pct = [&](double p) {
        if (v.empty()) return 0.0;
        const size_t i = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
        std::nth_element(v.begin(), v.begin() + (long)i, v.end());
        return v[i];
    };
    if (p50_ms) *p50_ms = pct(0.50);
    if (p99_ms) *p99_ms = pct(0.99);
    if (solves_per_s) {
        const double span = std::chrono::duration<double>(s->t_last - s->t_first).count();
        *solves_per_s = (nlat && span > 0) ? (double)nlat / span : 0.0;
    }
    if (completed) *completed = (int64_t)nlat;
    return RSVD_OK;
}

rsvd_status rsvd_server_use_graphs(rsvd_server* s, int32_t enable) {
    if (!s) return RSVD_ERR_INVALID_ARG;
    s->use_graphs = enable != 0;
    return RSVD_OK;
}

rsvd_status rsvd_server_graph_stats(rsvd_server* s, int64_t* launches, int64_t* instantiations) {
    if (!s) return RSVD_ERR_INVALID_ARG;
    if (launches) *launches = s->graph_launches;
    if (instantiations) *instantiations = s->graph_instantiations;
    return RSVD_OK;
}

rsvd_status rsvd_server_destroy(rsvd_server* s) {
    if (!s) return RSVD_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->all) delete kv.second;
    for (auto& cache : s->graphs)
        for (auto& e : cache)
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
    for (size_t i = 0; i < s->streams.size(); ++i) {
        if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
        if (s->events[i]) (void)hipEventDestroy(s->events[i]);
    }
    delete s->arena;
    if (s->arena_base) (void)hipFree(s->arena_base);
    rsvd_destroy(s->h);
    delete s;
    return RSVD_OK;
}

}  // extern "C"

// Batched request server of the C ABI (rsvd_server_*): continuous batching
// of independent randomized SVD requests of uneven shape on one GPU.
//
// Requests are queued on submit (at most max_pending) and admitted oldest
// first as soon as a stream slot is free and their workspace fits in the
// server's HBM budget (one device arena, sub-allocated first fit); younger
// requests that fit may pass an oldest one that does not, a bounded number of
// times.  An admitted request is one
// rsvd_solve on its slot's stream, so requests that arrive while others run
// overlap on the device; each uses its own workspace and the same
// deterministic kernels, so its result is the same alone and in the mix.
// A scheduler thread admits, launches and retires requests (retirement:
// the request's completion event has fired; its workspace and slot return
// to the pools).  Latency is measured from submit to the scheduler seeing
// the completion.
//
// Launch graphs (off by default, rsvd_server_use_graphs): an admitted
// request's kernels are captured from rsvd_solve into a HIP graph and
// launched as one graph.  HIP refuses a device-wide synchronisation from any
// thread while a stream of the device is capturing, so with graphs on the
// rest of the process must wait on streams or events, not on the device.  Executable graphs
// are pooled by bucket (a bucket = what fixes the kernel sequence:
// precision, l and the output width rounded to 16, q, the options, and
// whether each product is split along its reduction).  An admitted request
// takes an idle executable graph of its bucket, updates it in place with its
// own pointers, sizes and grids (hipGraphExecUpdate) and launches it; the
// graph returns to the pool when the request retires, so a graph never runs
// twice at once.  With no idle graph of the bucket, or when the runtime
// refuses the update, a new one is instantiated; the pool keeps at most
// kGraphPool idle graphs (least recently used evicted).  The captured kernels are exactly those rsvd_solve
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
#include "kernels.hpp"

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
constexpr int kKeyLen = 18;
struct BucketKey {
    int64_t v[kKeyLen];
    bool operator==(const BucketKey& o) const {
        for (int i = 0; i < kKeyLen; ++i)
            if (v[i] != o.v[i]) return false;
        return true;
    }
};

struct GraphEntry {
    BucketKey key;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};
constexpr size_t kGraphPool = 256;
constexpr int kMaxBypass = 8;             // times the oldest request may be passed over
constexpr size_t kAdmitWindow = 64;       // pending requests looked at per admission pass
constexpr size_t kLatencyWindow = 65536;  // latencies kept for the percentiles
constexpr int kDefaultMaxPending = 4096;

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
    hipEvent_t ready = nullptr;           // the caller's event the request's stream waits for
    int bypassed = 0;                     // younger requests admitted while this one was the oldest
    GraphEntry graph;                     // the executable graph it was launched as (exec null: direct)
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
    std::map<uint64_t, Request*> all;     // every request not yet released
    uint64_t next_ticket = 1;
    size_t max_pending = kDefaultMaxPending;
    bool stop = false, paused = false;
    std::thread worker;

    // launch graphs: the idle pool (touched by the scheduler thread only)
    std::atomic<bool> use_graphs{false};
    std::vector<GraphEntry> idle_graphs;
    uint64_t graph_clock = 0;
    std::atomic<int64_t> graph_launches{0}, graph_instantiations{0}, graph_fallbacks{0};

    // statistics: the last kLatencyWindow latencies (a ring) and a count
    std::vector<double> latencies_ms;
    size_t lat_next = 0;
    int64_t completed = 0;
    Clock::time_point t_first{}, t_last{};
    bool any = false;

    void loop();
    rsvd_status launch(Request* r, int slot, void* ws);
};

namespace {

// The kernels a solve launches depend on the shape only through l (their
// tile templates and the small-matrix kernels' forms), the output width and
// whether a product is split along its reduction (a reduction kernel
// follows); grids, sizes and pointers are launch arguments, which a graph
// update replaces.
BucketKey bucket_of(const Request* r) {
    const rsvd_params& p = r->params;
    const int64_t m = r->A.rows, n = r->A.cols;
    const int64_t l = std::min(p.k + p.p, std::min(m, n));
    const int L = (int)((l + 15) / 16 * 16);
    const int64_t width = p.return_full_l ? l : p.k;
    const bool lowp = r->A.dtype == RSVD_BF16 || r->A.dtype == RSVD_FP8_E4M3;
    const int wdt = lowp ? RSVD_F32 : r->A.dtype;
    int snn = 1, stn = 1;
    if (p.algorithm == 6) {
        snn = rsvd::dual_splits(wdt, m, n);
        rsvd::gemm_partials_elems(wdt, n, n, L, &stn);
    } else if (lowp) {
        rsvd::lp_partials_elems(m, n, L, &snn);
        rsvd::lp_partials_elems(n, m, L, &stn);
    } else {
        rsvd::gemm_partials_elems(wdt, m, n, L, &snn);
        rsvd::gemm_partials_elems(wdt, n, m, L, &stn);
    }
    int s16 = 0;
    if (p.residual & 1) {
        int a = 1, b = 1;
        rsvd::gemm_partials_elems(RSVD_F32, m, n, 16, &a);
        rsvd::gemm_partials_elems(RSVD_F32, n, m, 16, &b);
        s16 = (a > 1) + 2 * (b > 1);
    }
    return BucketKey{{(int64_t)r->A.dtype, L, (width + 15) / 16, p.q, (int64_t)p.extra_power_pass,
                      (int64_t)p.residual, (int64_t)p.residual_iters, (int64_t)p.return_full_l,
                      (int64_t)p.orth, r->out.Q != nullptr, r->A.master != nullptr,
                      r->A.col_scale != nullptr, (int64_t)p.algorithm, (int64_t)p.jacobi_max_sweeps,
                      (int64_t)p.test_matrix, snn > 1, stn > 1, s16}};
}

}  // namespace

// Enqueue one admitted request on its slot's stream: directly, or captured
// into a graph that replaces (or updates) the slot's graph of its bucket.
rsvd_status rsvd_server::launch(Request* r, int slot, void* ws) {
    hipStream_t st = streams[slot];
    // Order the request after the caller's work (outside any capture).
    if (r->ready && hipStreamWaitEvent(st, r->ready, 0) != hipSuccess) return RSVD_ERR_DEVICE;
    if (!use_graphs) return rsvd_solve(h, &r->A, &r->params, &r->out, ws, r->ws_bytes, st);
    // A capture that fails for any reason recorded nothing that ran: the
    // request is then launched directly (an invalid request gets the same
    // error from the direct call).
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        ++graph_fallbacks;
        return rsvd_solve(h, &r->A, &r->params, &r->out, ws, r->ws_bytes, st);
    }
    const rsvd_status rs = rsvd_solve(h, &r->A, &r->params, &r->out, ws, r->ws_bytes, st);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (rs != RSVD_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        if (rs == RSVD_OK) ++graph_fallbacks;
        return rsvd_solve(h, &r->A, &r->params, &r->out, ws, r->ws_bytes, st);
    }
    const BucketKey key = bucket_of(r);
    GraphEntry ent{key, nullptr, 0};
    for (size_t e = 0; e < idle_graphs.size(); ++e)
        if (idle_graphs[e].key == key) {          // take an idle graph of the bucket
            ent = idle_graphs[e];
            idle_graphs[e] = idle_graphs.back();
            idle_graphs.pop_back();
            break;
        }
    bool ready = false;
    if (ent.exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        if (hipGraphExecUpdate(ent.exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
            ready = true;
        } else {
            (void)hipGraphExecDestroy(ent.exec);
            ent.exec = nullptr;
        }
    }
    if (!ready) {
        if (hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return RSVD_ERR_DEVICE;
        }
        ++graph_instantiations;
    }
    ent.last_use = ++graph_clock;
    const hipError_t el = hipGraphLaunch(ent.exec, st);
    (void)hipGraphDestroy(g);
    r->graph = ent;                               // returned to the pool when the request retires
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
            if (r->graph.exec) {                // its graph is idle again
                if (idle_graphs.size() >= kGraphPool) {
                    auto lru = std::min_element(idle_graphs.begin(), idle_graphs.end(),
                                                [](const GraphEntry& a, const GraphEntry& b) {
                                                    return a.last_use < b.last_use;
                                                });
                    (void)hipGraphExecDestroy(lru->exec);
                    *lru = idle_graphs.back();
                    idle_graphs.pop_back();
                }
                idle_graphs.push_back(r->graph);
                r->graph.exec = nullptr;
            }
            r->done = true;
            const double lat = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
            if (latencies_ms.size() < kLatencyWindow) latencies_ms.push_back(lat);
            else latencies_ms[lat_next] = lat;
            lat_next = (lat_next + 1) % kLatencyWindow;
            ++completed;
            t_last = r->t_done;
            running[i] = running.back();
            running.pop_back();
            progressed = true;
        }
        if (progressed) cv_done.notify_all();
        // Admit oldest first while a slot is free and the workspace fits; when
        // the oldest does not fit, younger ones that fit may pass it, at most
        // kMaxBypass times in all.
        size_t scanned = 0;
        for (auto it = pending.begin(); !paused && it != pending.end() && scanned < kAdmitWindow; ++scanned) {
            Request* r = *it;
            const bool oldest = it == pending.begin();
            int slot = -1;
            for (size_t sl = 0; sl < slot_busy.size(); ++sl)
                if (!slot_busy[sl]) { slot = (int)sl; break; }
            if (slot < 0) break;
            if (!oldest && pending.front()->bypassed >= kMaxBypass) break;
            size_t off = 0;
            if (!arena->alloc(r->ws_bytes, &off)) {
                if (oldest && running.empty()) {       // can never fit
                    r->status = RSVD_ERR_NO_MEMORY;
                    r->done = true;
                    it = pending.erase(it);
                    cv_done.notify_all();
                    continue;
                }
                ++it;
                continue;
            }
            if (!oldest) ++pending.front()->bypassed;
            it = pending.erase(it);
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
            it = pending.begin();               // the queue changed while unlocked: rescan from the oldest
        }
        if (stop && pending.empty() && running.empty()) break;
        if (running.empty() && (pending.empty() || paused)) {
            cv_work.wait(lk, [&] { return stop || (!pending.empty() && !paused); });
        } else {
            // poll the in-flight events at a short interval
            cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

extern "C" {

rsvd_status rsvd_server_create(rsvd_server** out, int device, size_t hbm_budget_bytes, int n_streams,
                               int32_t max_pending) {
    if (!out || n_streams < 1 || n_streams > 64 || hbm_budget_bytes < kArenaAlign || max_pending < 0)
        return RSVD_ERR_INVALID_ARG;
    *out = nullptr;
    rsvd_server* s = new (std::nothrow) rsvd_server;
    if (!s) return RSVD_ERR_NO_MEMORY;
    s->device = device;
    s->max_pending = max_pending ? (size_t)max_pending : (size_t)kDefaultMaxPending;
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
                               const rsvd_result* out, void* ready_event, uint64_t* ticket) {
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
    r->ready = static_cast<hipEvent_t>(ready_event);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) { delete r; return RSVD_ERR_INVALID_ARG; }
        if (s->pending.size() >= s->max_pending) { delete r; return RSVD_ERR_QUEUE_FULL; }
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

rsvd_status rsvd_server_release(rsvd_server* s, uint64_t ticket) {
    if (!s) return RSVD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end() || !it->second->done) return RSVD_ERR_INVALID_ARG;
    delete it->second;
    s->all.erase(it);
    return RSVD_OK;
}

rsvd_status rsvd_server_pause(rsvd_server* s, int32_t paused) {
    if (!s) return RSVD_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->paused = paused != 0;
    }
    s->cv_work.notify_all();
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
    const int64_t nlat = s->completed;
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
    if (completed) *completed = nlat;
    return RSVD_OK;
}

rsvd_status rsvd_server_use_graphs(rsvd_server* s, int32_t enable) {
    if (!s) return RSVD_ERR_INVALID_ARG;
    s->use_graphs = enable != 0;
    return RSVD_OK;
}

rsvd_status rsvd_server_graph_stats(rsvd_server* s, int64_t* launches, int64_t* instantiations,
                                    int64_t* fallbacks) {
    if (!s) return RSVD_ERR_INVALID_ARG;
    if (launches) *launches = s->graph_launches;
    if (instantiations) *instantiations = s->graph_instantiations;
    if (fallbacks) *fallbacks = s->graph_fallbacks;
    return RSVD_OK;
}

rsvd_status rsvd_server_destroy(rsvd_server* s) {
    if (!s) return RSVD_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->paused = false;                  // queued requests still run before the thread ends
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->all) delete kv.second;
    for (auto& e : s->idle_graphs)
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

// Serving: a request loop over device-resident graphs with continuous batching.
//
// Requests arrive at any time (vdmc_serve_submit).  A worker thread admits them in
// arrival order while the number of requests on the GPU is below max_inflight and the
// device memory they touch (output matrix plus the graph's hub scratch) fits the
// budget; a request that could never fit is rejected at submit.  Admitted requests
// run concurrently: small graphs admitted in the same pass with the same k are fused
// into one batched launch, larger ones get a stream of their own, so new work joins
// the device while earlier work is still running.  Completion is observed through
// events; latency is submit -> completion seen by the worker.  Requests on the same
// graph are serialised (a graph's scratch belongs to one count at a time).  The
// arithmetic is the same as vdmc_count, so every result is identical alone and in
// the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <set>
#include <thread>
#include <unordered_map>

#include "vdmc_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double now_us() {
    return std::chrono::duration<double, std::micro>(Clock::now().time_since_epoch()).count();
}

constexpr int64_t kSmallGraph = 20000;   // graphs up to this many vertices are fused into batches

struct Request {
    uint64_t id = 0;
    vdmc_graph_s* g = nullptr;
    int k = 4;
    uint64_t* out = nullptr;
    size_t bytes = 0;
    double t_submit = 0, t_done = 0;
    int state = 0;   // 0 queued, 1 running, 2 done, 3 cancelled
    int slot = -1;
    int group = -1;  // launch group id (requests finishing together)
};

struct Group {
    int slot = -1;
    hipEvent_t ev = nullptr;
    std::vector<uint64_t> ids;
};

}  // namespace

struct vdmc_server_s {
    vdmc_serve_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;        // wakes the worker
    std::condition_variable done_cv;   // wakes waiters
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    std::unordered_map<int, Group> groups;
    std::vector<hipStream_t> streams;
    std::vector<int> slot_busy;
    std::set<vdmc_graph_s*> busy_graphs;
    size_t inflight_bytes = 0;
    int inflight_groups = 0;
    int inflight_reqs = 0;
    uint64_t next_id = 1;
    int next_group = 0;
    bool stop = false;
    std::thread worker;
    std::vector<double> lat_us;
    uint64_t sets = 0;
    double t_first_submit = -1, t_last_done = -1;
    std::string worker_error;
};

namespace vdmc {
namespace {

size_t request_bytes(vdmc_graph_s* g, int k) {
    return (size_t)std::max<int64_t>(g->n, 1) * (size_t)num_classes(k) * sizeof(uint64_t) + g->hub_scratch_bytes;
}

// Complete every launch group whose event has fired.  Called with the lock held.
void reap(vdmc_server_s* s) {
    for (auto it = s->groups.begin(); it != s->groups.end();) {
        Group& gr = it->second;
        hipError_t q = hipEventQuery(gr.ev);
        if (q == hipErrorNotReady) {
            ++it;
            continue;
        }
        const double t = now_us();
        for (uint64_t id : gr.ids) {
            Request& r = s->reqs[id];
            r.state = 2;
            r.t_done = t;
            s->lat_us.push_back(t - r.t_submit);
            uint64_t st[kShapes] = {0, 0, 0, 0, 0, 0};
            if (hipMemcpy(st, r.g->stats, sizeof(st), hipMemcpyDeviceToHost) == hipSuccess)
                s->sets += r.k == 3 ? st[0] + st[1] : st[2] + st[3] + st[4] + st[5];
            s->inflight_bytes -= r.bytes;
            s->inflight_reqs--;
            s->busy_graphs.erase(r.g);
        }
        s->t_last_done = t;
        s->slot_busy[gr.slot] = 0;
        s->inflight_groups--;
        (void)hipEventDestroy(gr.ev);
        it = s->groups.erase(it);
    }
    s->done_cv.notify_all();
}

// Pick the requests to start now, in arrival order.  Called with the lock held.
std::vector<std::vector<uint64_t>> admit(vdmc_server_s* s) {
    std::vector<std::vector<uint64_t>> launches;
    std::vector<uint64_t> small3, small4;
    int free_slots = 0;
    for (int b : s->slot_busy) free_slots += b == 0;
    auto slots_needed = [&] { return (int)launches.size() + (int)!small3.empty() + (int)!small4.empty(); };
    int reqs_room = s->cfg.max_inflight - s->inflight_reqs;
    std::set<vdmc_graph_s*> taken;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request& r = s->reqs[*it];
        if (r.state != 0) {
            it = s->queue.erase(it);
            continue;
        }
        if (reqs_room <= 0) break;
        if (s->busy_graphs.count(r.g) || taken.count(r.g)) {
            ++it;   // same graph still counting: later requests may go first
            continue;
        }
        if (s->inflight_bytes + r.bytes > s->cfg.mem_budget_bytes) break;   // arrival order: wait for memory
        const bool small = r.g->n <= kSmallGraph && r.g->nhub == 0;
        const bool new_launch = !small || (r.k == 3 ? small3.empty() : small4.empty());
        if (new_launch && slots_needed() + 1 > free_slots) break;   // no stream free: wait
        s->inflight_bytes += r.bytes;
        reqs_room--;
        taken.insert(r.g);
        if (small) (r.k == 3 ? small3 : small4).push_back(r.id);
        else launches.push_back({r.id});
        it = s->queue.erase(it);
    }
    if (!small3.empty()) launches.push_back(small3);
    if (!small4.empty()) launches.push_back(small4);
    return launches;
}

void worker_main(vdmc_server_s* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lock(s->mu);
    while (true) {
        reap(s);
        if (s->stop && s->inflight_groups == 0) break;
        std::vector<std::vector<uint64_t>> launches;
        if (!s->stop) launches = admit(s);
        for (auto& ids : launches) {
            int slot = -1;
            for (size_t i = 0; i < s->slot_busy.size(); i++)
                if (!s->slot_busy[i]) {
                    slot = (int)i;
                    break;
                }
            if (slot < 0) {   // cannot happen: admit() reserved the slots; requeue defensively
                for (uint64_t id : ids) {
                    Request& r = s->reqs[id];
                    s->inflight_bytes -= r.bytes;
                    s->queue.push_front(id);
                }
                continue;
            }
            Group gr;
            gr.slot = slot;
            gr.ids = ids;
            s->slot_busy[slot] = 1;
            s->inflight_groups++;
            for (uint64_t id : ids) {
                Request& r = s->reqs[id];
                r.state = 1;
                r.slot = slot;
                s->inflight_reqs++;
                s->busy_graphs.insert(r.g);
            }
            hipStream_t st = s->streams[slot];
            const int gid = s->next_group++;
            std::vector<vdmc_graph_s*> gs;
            std::vector<uint64_t*> outs;
            const int k = s->reqs[ids[0]].k;
            for (uint64_t id : ids) {
                gs.push_back(s->reqs[id].g);
                outs.push_back(s->reqs[id].out);
            }
            lock.unlock();
            std::string err;
            try {
                if (ids.size() == 1) {
                    launch_count(gs[0], k == 3, k == 4, k == 3 ? outs[0] : nullptr, k == 4 ? outs[0] : nullptr, st);
                } else {
                    count_batch_impl(gs.data(), (int32_t)gs.size(), k, outs.data(), st, false, nullptr);
                }
                VDMC_HIP(hipEventCreateWithFlags(&gr.ev, hipEventDisableTiming));
                VDMC_HIP(hipEventRecord(gr.ev, st));
            } catch (const Error& e) {
                err = e.msg;
            } catch (const std::exception& e) {
                err = e.what();
            }
            lock.lock();
            if (!err.empty()) {
                // mark the group as finished with an error: the requests report DEVICE on wait
                s->worker_error = err;
                if (!gr.ev) (void)hipEventCreateWithFlags(&gr.ev, hipEventDisableTiming);
                (void)hipEventRecord(gr.ev, st);
            }
            s->groups[gid] = gr;
        }
        if (s->groups.empty() && (s->queue.empty() || s->stop)) {
            if (s->stop) continue;
            s->cv.wait(lock);
        } else {
            s->cv.wait_for(lock, std::chrono::microseconds(50));
        }
    }
}

}  // namespace
}  // namespace vdmc

extern "C" {

vdmc_status vdmc_serve_create(const vdmc_serve_config* cfg, vdmc_server* out) {
    vdmc_server_s* s = nullptr;
    vdmc_status st = vdmc::guarded([&] {
        VDMC_REQUIRE(cfg != nullptr && out != nullptr, VDMC_ERR_INVALID_ARG, "cfg/out is NULL");
        *out = nullptr;
        VDMC_REQUIRE(cfg->mem_budget_bytes > 0, VDMC_ERR_INVALID_ARG, "mem_budget_bytes must be positive");
        VDMC_REQUIRE(cfg->max_inflight >= 1 && cfg->max_inflight <= 256, VDMC_ERR_INVALID_ARG,
                     "max_inflight must be in [1, 256]");
        s = new vdmc_server_s();
        s->cfg = *cfg;
        VDMC_HIP(hipGetDevice(&s->device));
        (void)vdmc::class_tables();
        const int nstreams = std::min(cfg->max_inflight, 16);
        for (int i = 0; i < nstreams; i++) {
            hipStream_t h = nullptr;
            VDMC_HIP(hipStreamCreateWithFlags(&h, hipStreamNonBlocking));
            s->streams.push_back(h);
            s->slot_busy.push_back(0);
        }
        s->worker = std::thread(vdmc::worker_main, s);
    });
    if (st != VDMC_OK) {
        if (s) {
            for (auto h : s->streams) (void)hipStreamDestroy(h);
            delete s;
        }
        return st;
    }
    *out = s;
    return VDMC_OK;
}

vdmc_status vdmc_serve_submit(vdmc_server s, vdmc_graph g, int32_t k, uint64_t* out, uint64_t* req_id) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(s != nullptr && g != nullptr && req_id != nullptr, VDMC_ERR_INVALID_ARG, "NULL argument");
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG, "k must be 3 or 4");
        VDMC_REQUIRE(out != nullptr || g->n == 0, VDMC_ERR_INVALID_ARG, "out is NULL");
        VDMC_REQUIRE(g->device == s->device, VDMC_ERR_INVALID_ARG, "graph lives on another device");
        {
            std::lock_guard<std::mutex> lock(s->mu);
            VDMC_REQUIRE(!s->stop, VDMC_ERR_INVALID_ARG, "server is shutting down");
        }
        // bins and hub scratch are built once per graph; their size is part of the request
        {
            std::lock_guard<std::mutex> lock(g->mu);
            if (g->bins_hub_min != g->hub_min) {
                hipStream_t st = nullptr;
                VDMC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
                try {
                    vdmc::ensure_bins(g, st);
                } catch (...) {
                    (void)hipStreamDestroy(st);
                    throw;
                }
                VDMC_HIP(hipStreamDestroy(st));
            }
        }
        const size_t bytes = vdmc::request_bytes(g, k);
        VDMC_REQUIRE(bytes <= s->cfg.mem_budget_bytes, VDMC_ERR_REJECTED,
                     "request needs " + std::to_string(bytes) + " bytes, budget is " +
                         std::to_string(s->cfg.mem_budget_bytes));
        std::lock_guard<std::mutex> lock(s->mu);
        Request r;
        r.id = s->next_id++;
        r.g = g;
        r.k = k;
        r.out = out;
        r.bytes = bytes;
        r.t_submit = now_us();
        if (s->t_first_submit < 0) s->t_first_submit = r.t_submit;
        s->reqs[r.id] = r;
        s->queue.push_back(r.id);
        *req_id = r.id;
        s->cv.notify_all();
    });
}

vdmc_status vdmc_serve_poll(vdmc_server s, uint64_t req_id, int32_t* done) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(s != nullptr && done != nullptr, VDMC_ERR_INVALID_ARG, "NULL argument");
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->reqs.find(req_id);
        VDMC_REQUIRE(it != s->reqs.end(), VDMC_ERR_NOT_FOUND, "unknown request id");
        *done = it->second.state == 2 ? 1 : 0;
    });
}

vdmc_status vdmc_serve_wait(vdmc_server s, uint64_t req_id, int64_t timeout_us) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(s != nullptr, VDMC_ERR_INVALID_ARG, "server is NULL");
        std::unique_lock<std::mutex> lock(s->mu);
        auto it = s->reqs.find(req_id);
        VDMC_REQUIRE(it != s->reqs.end(), VDMC_ERR_NOT_FOUND, "unknown request id");
        auto is_done = [&] {
            const int st = s->reqs[req_id].state;
            return st == 2 || st == 3;
        };
        if (timeout_us < 0) {
            s->done_cv.wait(lock, is_done);
        } else if (!s->done_cv.wait_for(lock, std::chrono::microseconds(timeout_us), is_done)) {
            throw vdmc::Error{VDMC_ERR_TIMEOUT, "request still running"};
        }
        VDMC_REQUIRE(s->reqs[req_id].state == 2, VDMC_ERR_DEVICE, "request was cancelled");
        VDMC_REQUIRE(s->worker_error.empty(), VDMC_ERR_DEVICE, "serving launch failed: " + s->worker_error);
    });
}

vdmc_status vdmc_serve_stats(vdmc_server s, double* p50_us, double* p99_us, double* req_per_s, uint64_t* sets) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(s != nullptr, VDMC_ERR_INVALID_ARG, "server is NULL");
        std::lock_guard<std::mutex> lock(s->mu);
        std::vector<double> l = s->lat_us;
        std::sort(l.begin(), l.end());
        auto pct = [&](double q) {
            if (l.empty()) return 0.0;
            size_t i = (size_t)std::ceil(q * (double)l.size()) - 1;   // nearest-rank percentile
            return l[std::min(i, l.size() - 1)];
        };
        if (p50_us) *p50_us = pct(0.50);
        if (p99_us) *p99_us = pct(0.99);
        if (req_per_s) {
            const double span = s->t_last_done - s->t_first_submit;
            *req_per_s = (span > 0 && !l.empty()) ? (double)l.size() / (span * 1e-6) : 0.0;
        }
        if (sets) *sets = s->sets;
    });
}

vdmc_status vdmc_serve_destroy(vdmc_server s) {
    if (!s) return VDMC_OK;
    return vdmc::guarded([&] {
        {
            std::lock_guard<std::mutex> lock(s->mu);
            s->stop = true;
            for (uint64_t id : s->queue) s->reqs[id].state = 3;   // never started: cancelled
            s->queue.clear();
            s->cv.notify_all();
            s->done_cv.notify_all();
        }
        if (s->worker.joinable()) s->worker.join();
        for (auto h : s->streams) (void)hipStreamDestroy(h);
        delete s;
    });
}

}  // extern "C"

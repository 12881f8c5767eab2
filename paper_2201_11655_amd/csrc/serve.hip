// Serving: a request loop over device-resident graphs with continuous batching.
//
// Requests arrive at any time (vdmc_serve_submit, which only queues them).  A worker
// thread admits them in arrival order while fewer than max_inflight requests are on the
// GPU, a stream slot is free and the device memory the server must allocate for them
// fits the budget:
//   * a request on a graph that the whole-graph kernel takes (small.hip) needs no memory
//     of its own; such requests admitted in one pass with the same k are fused into one
//     launch whose graph descriptors go through the slot's preallocated buffers;
//   * any other request needs its graph's hub-path scratch (sized when the graph's root
//     bins are built, at its first admission); the scratch is allocated at admission
//     inside the budget and freed when the request completes.  A request whose scratch
//     does not fit now waits (the queue keeps arrival order); one that can never fit is
//     rejected.
// Admitted requests run concurrently on separate streams, so new work joins the device
// while earlier work is still running.  Completion is observed through events; latency
// is submit -> completion seen by the worker.  Requests on the same graph run one at a
// time (later requests on other graphs may overtake them).  The arithmetic is the same
// as vdmc_count, so every result is identical alone and in the mix.
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

constexpr uint32_t kMaxFused = 256;   // requests fused into one whole-graph launch

enum ReqState { QUEUED = 0, RUNNING = 1, DONE = 2, FAILED = 3 };

struct Request {
    uint64_t id = 0;
    vdmc_graph_s* g = nullptr;
    int k = 4;
    uint64_t* out = nullptr;
    size_t bytes = 0;          // server-allocated device memory while it runs
    bool owns_scratch = false;
    bool fused = false;
    double t_submit = 0, t_done = 0;
    int state = QUEUED;
    vdmc_status status = VDMC_OK;
    std::string error;
};

struct Group {
    int slot = -1;
    hipEvent_t ev = nullptr;
    std::vector<uint64_t> ids;
};

struct Slot {
    hipStream_t stream = nullptr;
    bool busy = false;
    vdmc::SmallGraph* d_desc = nullptr;   // kMaxFused descriptors + a cursor word
    vdmc::SmallGraph* h_desc = nullptr;   // pinned staging of the same
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
    std::vector<Slot> slots;
    hipStream_t aux = nullptr;         // root binning of newly seen graphs
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
    // counters (vdmc_serve_counters)
    uint64_t n_submitted = 0, n_admitted = 0, n_completed = 0, n_rejected = 0, n_failed = 0, n_deferred = 0;
    uint64_t max_queue = 0, max_bytes = 0;
};

namespace vdmc {
namespace {

int g_ncu = -1;

void finish(vdmc_server_s* s, Request& r, int state, vdmc_status st, const std::string& err) {
    r.state = state;
    r.status = st;
    r.error = err;
    r.t_done = now_us();
    if (state == FAILED) {
        if (st == VDMC_ERR_REJECTED) s->n_rejected++;
        else s->n_failed++;
    }
}

// Complete every launch group whose event has fired.  Called with the lock held.
void reap(vdmc_server_s* s) {
    for (auto it = s->groups.begin(); it != s->groups.end();) {
        Group& gr = it->second;
        const hipError_t q = hipEventQuery(gr.ev);
        if (q == hipErrorNotReady) {
            ++it;
            continue;
        }
        const double t = now_us();
        for (uint64_t id : gr.ids) {
            Request& r = s->reqs[id];
            if (r.state == RUNNING) {
                if (q == hipSuccess) {
                    r.state = DONE;
                    r.t_done = t;
                    s->lat_us.push_back(t - r.t_submit);
                    s->n_completed++;
                    uint64_t st[kShapes] = {0, 0, 0, 0, 0, 0};
                    if (hipMemcpy(st, r.g->stats, sizeof(st), hipMemcpyDeviceToHost) == hipSuccess)
                        s->sets += r.k == 3 ? st[0] + st[1] : st[2] + st[3] + st[4] + st[5];
                } else {
                    finish(s, r, FAILED, VDMC_ERR_DEVICE, std::string("device error: ") + hipGetErrorString(q));
                }
            }
            if (r.owns_scratch) {   // the hub scratch allocated at admission goes back
                std::lock_guard<std::mutex> lock(r.g->mu);
                free_hub_scratch(r.g);
                r.owns_scratch = false;
            }
            s->inflight_bytes -= r.bytes;
            s->inflight_reqs--;
            s->busy_graphs.erase(r.g);
        }
        s->t_last_done = t;
        s->slots[gr.slot].busy = false;
        s->inflight_groups--;
        (void)hipEventDestroy(gr.ev);
        it = s->groups.erase(it);
    }
    s->done_cv.notify_all();
}

// Server-allocated bytes a request needs, building the graph's root bins if they are
// stale.  Called with the server lock held (by the worker).
size_t need_bytes(vdmc_server_s* s, Request& r) {
    std::lock_guard<std::mutex> lock(r.g->mu);
    if (r.g->bins_hub_min != r.g->hub_min) {
        ensure_bins(r.g, s->aux);
        VDMC_HIP(hipStreamSynchronize(s->aux));
    }
    return r.g->hub_scratch ? 0 : hub_scratch_need(r.g);
}

// Pick the launches to start now, in arrival order.  Called with the lock held.
std::vector<std::vector<uint64_t>> admit(vdmc_server_s* s) {
    std::vector<std::vector<uint64_t>> launches;
    std::vector<uint64_t> fused3, fused4;
    int free_slots = 0;
    for (const Slot& sl : s->slots) free_slots += !sl.busy;
    auto slots_needed = [&] { return (int)launches.size() + (int)!fused3.empty() + (int)!fused4.empty(); };
    int room = s->cfg.max_inflight - s->inflight_reqs;
    std::set<vdmc_graph_s*> taken;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request& r = s->reqs[*it];
        if (r.state != QUEUED) {
            it = s->queue.erase(it);
            continue;
        }
        if (room <= 0) break;
        if (s->busy_graphs.count(r.g) || taken.count(r.g)) {
            ++it;   // same graph still counting: later requests may go first
            continue;
        }
        r.fused = small_eligible(r.g->n, 2 * r.g->pairs, r.k);
        auto& fl = r.k == 3 ? fused3 : fused4;
        size_t need = 0;
        if (!r.fused) {
            try {
                need = need_bytes(s, r);
            } catch (const Error& e) {
                finish(s, r, FAILED, e.code, e.msg);
                it = s->queue.erase(it);
                continue;
            }
            if (need > s->cfg.mem_budget_bytes) {
                finish(s, r, FAILED, VDMC_ERR_REJECTED,
                       "request needs " + std::to_string(need) + " bytes of scratch, budget is " +
                           std::to_string(s->cfg.mem_budget_bytes));
                it = s->queue.erase(it);
                continue;
            }
            if (s->inflight_bytes + need > s->cfg.mem_budget_bytes) {
                s->n_deferred++;   // waits for memory; arrival order is kept
                break;
            }
        }
        const bool new_launch = !r.fused || fl.empty() || fl.size() >= kMaxFused;
        if (new_launch && slots_needed() + 1 > free_slots) break;   // no stream free: wait
        if (r.fused && fl.size() >= kMaxFused) break;
        r.bytes = need;
        s->inflight_bytes += need;
        s->max_bytes = std::max<uint64_t>(s->max_bytes, s->inflight_bytes);
        room--;
        taken.insert(r.g);
        if (r.fused) fl.push_back(r.id);
        else launches.push_back({r.id});
        it = s->queue.erase(it);
    }
    if (!fused3.empty()) launches.push_back(fused3);
    if (!fused4.empty()) launches.push_back(fused4);
    return launches;
}

// Launch a group on slot sl.  Called without the server lock.
void launch_group(vdmc_server_s* s, Slot& sl, std::vector<Request*>& rs) {
    const hipStream_t st = sl.stream;
    const int k = rs[0]->k;
    if (rs[0]->fused) {
        std::vector<vdmc_graph_s*> gs;
        size_t lds = 0;
        for (uint32_t i = 0; i < rs.size(); i++) {
            vdmc_graph_s* g = rs[i]->g;
            gs.push_back(g);
            sl.h_desc[i] = SmallGraph{g->off, g->adj, g->perm, (unsigned long long*)rs[i]->out, g->stats,
                                      (uint32_t)g->n, (uint32_t)(2 * g->pairs)};
            lds = std::max(lds, small_lds_bytes(g->n, 2 * g->pairs, k));
        }
        const uint32_t num = (uint32_t)rs.size();
        *reinterpret_cast<unsigned*>(sl.h_desc + kMaxFused) = 0u;
        GraphUse use(gs, st);
        VDMC_HIP(hipMemcpyAsync(sl.d_desc, sl.h_desc, sizeof(SmallGraph) * num, hipMemcpyHostToDevice, st));
        VDMC_HIP(hipMemcpyAsync(sl.d_desc + kMaxFused, sl.h_desc + kMaxFused, sizeof(unsigned), hipMemcpyHostToDevice,
                                st));
        const ClassTables& t = class_tables();
        SmallArgs a{};
        a.graphs = sl.d_desc;
        a.num = num;
        a.cursor = reinterpret_cast<unsigned*>(sl.d_desc + kMaxFused);
        a.table = k == 3 ? t.t3 : t.t4;
        a.comp_of = t.slot4;
        a.comp_cls = t.slotcls;
        const int fit = std::max(1, (int)(163840 / (lds + 9216)));
        const unsigned grid = (unsigned)std::min<int64_t>(num, (int64_t)g_ncu * fit);
        launch_small(a, k, 2, grid, lds, st);
    } else {
        Request& r = *rs[0];
        GraphUse use(r.g, st);
        if (r.bytes > 0 && !r.g->hub_scratch) {
            ensure_hub_scratch(r.g);   // inside the budget reserved at admission
            r.owns_scratch = true;
        }
        launch_count(r.g, k == 3, k == 4, k == 3 ? r.out : nullptr, k == 4 ? r.out : nullptr, st);
    }
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
            for (size_t i = 0; i < s->slots.size(); i++)
                if (!s->slots[i].busy) {
                    slot = (int)i;
                    break;
                }
            std::vector<Request*> rs;
            for (uint64_t id : ids) rs.push_back(&s->reqs[id]);
            if (slot < 0) {   // cannot happen: admit() counted the free slots; requeue
                for (auto it = rs.rbegin(); it != rs.rend(); ++it) {
                    s->inflight_bytes -= (*it)->bytes;
                    (*it)->bytes = 0;
                    s->queue.push_front((*it)->id);
                }
                continue;
            }
            Slot& sl = s->slots[slot];
            sl.busy = true;
            s->inflight_groups++;
            for (Request* r : rs) {
                r->state = RUNNING;
                s->inflight_reqs++;
                s->n_admitted++;
                s->busy_graphs.insert(r->g);
            }
            Group gr;
            gr.slot = slot;
            gr.ids = ids;
            lock.unlock();
            std::string err;
            vdmc_status code = VDMC_OK;
            try {
                launch_group(s, sl, rs);
            } catch (const Error& e) {
                err = e.msg;
                code = e.code;
            } catch (const std::exception& e) {
                err = e.what();
                code = VDMC_ERR_DEVICE;
            }
            (void)hipEventCreateWithFlags(&gr.ev, hipEventDisableTiming);
            (void)hipEventRecord(gr.ev, sl.stream);
            lock.lock();
            if (!err.empty())   // this group's requests fail; the others are unaffected
                for (Request* r : rs) finish(s, *r, FAILED, code, "serving launch failed: " + err);
            s->groups[s->next_group++] = gr;
        }
        if (s->groups.empty() && (s->queue.empty() || s->stop)) {
            if (s->stop) continue;
            s->cv.wait(lock);
        } else {
            s->cv.wait_for(lock, std::chrono::microseconds(50));
        }
    }
}

void destroy_slots(vdmc_server_s* s) {
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        (void)hipFree(sl.d_desc);
        (void)hipHostFree(sl.h_desc);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    s->slots.clear();
    if (s->aux) (void)hipStreamDestroy(s->aux);
    s->aux = nullptr;
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
        if (vdmc::g_ncu < 0) {
            hipDeviceProp_t prop;
            VDMC_HIP(hipGetDeviceProperties(&prop, s->device));
            vdmc::g_ncu = prop.multiProcessorCount;
        }
        VDMC_HIP(hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking));
        const int nslots = std::min(cfg->max_inflight, 16);
        s->slots.resize(nslots);
        for (Slot& sl : s->slots) {
            VDMC_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
            const size_t bytes = sizeof(vdmc::SmallGraph) * (kMaxFused + 1);
            VDMC_HIP(hipMalloc(&sl.d_desc, bytes));
            VDMC_HIP(hipHostMalloc(&sl.h_desc, bytes, hipHostMallocDefault));
        }
        s->worker = std::thread(vdmc::worker_main, s);
    });
    if (st != VDMC_OK) {
        if (s) {
            vdmc::destroy_slots(s);
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
        // a request whose graph is already binned and whose scratch can never fit is refused now
        {
            std::lock_guard<std::mutex> lock(g->mu);
            if (!vdmc::small_eligible(g->n, 2 * g->pairs, k) && g->bins_hub_min == g->hub_min && !g->hub_scratch) {
                const size_t need = vdmc::hub_scratch_need(g);
                VDMC_REQUIRE(need <= s->cfg.mem_budget_bytes, VDMC_ERR_REJECTED,
                             "request needs " + std::to_string(need) + " bytes of scratch, budget is " +
                                 std::to_string(s->cfg.mem_budget_bytes));
            }
        }
        std::lock_guard<std::mutex> lock(s->mu);
        VDMC_REQUIRE(!s->stop, VDMC_ERR_INVALID_ARG, "server is shutting down");
        Request r;
        r.id = s->next_id++;
        r.g = g;
        r.k = k;
        r.out = out;
        r.t_submit = now_us();
        if (s->t_first_submit < 0) s->t_first_submit = r.t_submit;
        s->reqs[r.id] = r;
        s->queue.push_back(r.id);
        s->n_submitted++;
        s->max_queue = std::max<uint64_t>(s->max_queue, s->queue.size());
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
        *done = it->second.state == DONE ? 1 : 0;
        VDMC_REQUIRE(it->second.state != FAILED, it->second.status, it->second.error);
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
            return st == DONE || st == FAILED;
        };
        if (timeout_us < 0) {
            s->done_cv.wait(lock, is_done);
        } else if (!s->done_cv.wait_for(lock, std::chrono::microseconds(timeout_us), is_done)) {
            throw vdmc::Error{VDMC_ERR_TIMEOUT, "request still running"};
        }
        const Request& r = s->reqs[req_id];
        VDMC_REQUIRE(r.state == DONE, r.status, r.error);
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

vdmc_status vdmc_serve_counters(vdmc_server s, uint64_t* counters, int32_t n) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(s != nullptr && counters != nullptr && n >= 0, VDMC_ERR_INVALID_ARG, "bad argument");
        std::lock_guard<std::mutex> lock(s->mu);
        const uint64_t c[10] = {s->n_submitted, s->n_admitted, s->n_completed, s->n_rejected, s->n_failed,
                                s->n_deferred, (uint64_t)s->queue.size(), s->max_queue,
                                (uint64_t)s->inflight_bytes, s->max_bytes};
        for (int i = 0; i < n && i < 10; i++) counters[i] = c[i];
    });
}

vdmc_status vdmc_serve_destroy(vdmc_server s) {
    if (!s) return VDMC_OK;
    return vdmc::guarded([&] {
        {
            std::lock_guard<std::mutex> lock(s->mu);
            s->stop = true;
            for (uint64_t id : s->queue) {   // never started: cancelled
                Request& r = s->reqs[id];
                if (r.state == QUEUED) vdmc::finish(s, r, FAILED, VDMC_ERR_REJECTED, "cancelled: server destroyed");
            }
            s->queue.clear();
            s->cv.notify_all();
            s->done_cv.notify_all();
        }
        if (s->worker.joinable()) s->worker.join();
        vdmc::destroy_slots(s);
        delete s;
    });
}

}  // extern "C"

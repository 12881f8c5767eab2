// Batched counts over many graphs: one persistent launch, captured in a HIP graph.
//
// Small graphs cost microseconds of work each, so per-graph launches are dominated by
// launch and setup latency (the paper notes the fixed cost of reaching the GPU for
// small graphs, Sec. 8).  Here the roots of every graph go into one table of
// (graph, root) pairs; a persistent grid takes tiles of that table from a device-side
// cursor and runs the same per-root enumeration as the single-graph path, so the
// counts are bit-identical.  The zeroing kernel and the counting kernel are captured
// into a HIP graph the first time a batch signature (graphs, outputs, k, launch
// parameters) is seen and replayed afterwards.  Graphs of at most kSmallGraphN
// vertices are instead taken whole by one workgroup each, which keeps the graph's
// per-vertex counters in LDS and adds them to the output once.  Roots above the hub
// threshold of the other graphs are counted by the hub kernel of their graph after
// the batched launch.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <fstream>
#include <map>

#include "vdmc_internal.h"

namespace vdmc {
namespace {

struct Plan {
    std::vector<vdmc_graph_s*> graphs;
    std::vector<uint64_t*> outs;
    int k = 4;
    TuneChoice cfg;
    GraphView* d_graphs = nullptr;
    uint64_t* d_nvert = nullptr;
    uint2* d_table = nullptr;
    unsigned long long* d_cursor = nullptr;
    unsigned long long nentries = 0;
    uint32_t* d_small = nullptr;       // graphs counted one workgroup per graph
    std::vector<char> is_small;
    uint32_t nsmall = 0, nmax_small = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t captured_for = nullptr;
    ~Plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipFree(d_graphs);
        (void)hipFree(d_nvert);
        (void)hipFree(d_table);
        (void)hipFree(d_cursor);
        (void)hipFree(d_small);
    }
};

std::mutex g_plan_mu;
std::vector<Plan*> g_plans;
TuneChoice g_tuned;
bool g_have_tuned = false;

__global__ void k_fill_table(const uint32_t* const* lists, const unsigned long long* counts,
                             const unsigned long long* offsets, int num, uint2* table) {
    const int gi = blockIdx.x;
    if (gi >= num) return;
    const uint32_t* l = lists[gi];
    const unsigned long long n = counts[gi], o = offsets[gi];
    for (unsigned long long i = threadIdx.x; i < n; i += blockDim.x) table[o + i] = make_uint2((unsigned)gi, l[i]);
}

BatchArgs args_of(const Plan& p) {
    const ClassTables& t = class_tables();
    BatchArgs b;
    b.graphs = p.d_graphs;
    b.nvert = p.d_nvert;
    b.table = p.d_table;
    b.nentries = p.nentries;
    b.cursor = p.d_cursor;
    b.tile = p.cfg.tile;
    b.t3 = t.t3;
    b.t4 = t.t4;
    b.small = p.d_small;
    b.nsmall = p.nsmall;
    b.nmax_small = p.nmax_small;
    b.gcursor = reinterpret_cast<unsigned*>(p.d_cursor + 1);
    b.slot4 = t.slot4;
    b.slotcls = t.slotcls;
    return b;
}

Plan* build_plan(const vdmc_graph* gs, int num, int k, uint64_t* const* outs, const TuneChoice& cfg,
                 hipStream_t st) {
    auto* p = new Plan();
    try {
        p->k = k;
        p->cfg = cfg;
        std::vector<GraphView> views(num);
        std::vector<uint64_t> nvert(num);
        std::vector<const uint32_t*> lists(num);
        std::vector<unsigned long long> counts(num), offsets(num);
        std::vector<uint32_t> small;
        unsigned long long total = 0;
        p->is_small.assign(num, 0);
        for (int i = 0; i < num; i++) {
            vdmc_graph_s* g = gs[i];
            p->graphs.push_back(g);
            p->outs.push_back(outs[i]);
            if (g->n > 0 && g->n <= kSmallGraphN) {   // every root of g, hubs included, in one workgroup
                p->is_small[i] = 1;
                small.push_back((uint32_t)i);
                p->nmax_small = std::max(p->nmax_small, (uint32_t)g->n);
            }
            views[i] = GraphView{g->off, g->adj, g->split, g->perm,
                                 k == 3 ? (unsigned long long*)outs[i] : nullptr,
                                 k == 4 ? (unsigned long long*)outs[i] : nullptr, g->stats, g->ehash,
                                 g->ehash_bits};
            nvert[i] = (uint64_t)g->n;
            lists[i] = g->light;
            counts[i] = p->is_small[i] ? 0ull : (unsigned long long)g->nlight;
            offsets[i] = total;
            total += counts[i];
        }
        p->nentries = total;
        // largest work first (pairs x largest degree as the estimate), so that the last
        // workgroups to finish hold small graphs
        std::stable_sort(small.begin(), small.end(), [&](uint32_t a, uint32_t b) {
            return (double)gs[a]->pairs * gs[a]->max_deg > (double)gs[b]->pairs * gs[b]->max_deg;
        });
        p->nsmall = (uint32_t)small.size();
        if (!small.empty()) {
            VDMC_HIP(hipMalloc(&p->d_small, sizeof(uint32_t) * small.size()));
            VDMC_HIP(hipMemcpyAsync(p->d_small, small.data(), sizeof(uint32_t) * small.size(),
                                    hipMemcpyHostToDevice, st));
        }
        VDMC_HIP(hipMalloc(&p->d_graphs, sizeof(GraphView) * std::max(num, 1)));
        VDMC_HIP(hipMalloc(&p->d_nvert, sizeof(uint64_t) * std::max(num, 1)));
        VDMC_HIP(hipMalloc(&p->d_table, sizeof(uint2) * std::max<unsigned long long>(total, 1)));
        VDMC_HIP(hipMalloc(&p->d_cursor, 64));
        VDMC_HIP(hipMemcpyAsync(p->d_graphs, views.data(), sizeof(GraphView) * num, hipMemcpyHostToDevice, st));
        VDMC_HIP(hipMemcpyAsync(p->d_nvert, nvert.data(), sizeof(uint64_t) * num, hipMemcpyHostToDevice, st));
        const uint32_t** d_lists = nullptr;
        unsigned long long *d_counts = nullptr, *d_offsets = nullptr;
        VDMC_HIP(hipMalloc(&d_lists, sizeof(void*) * num));
        VDMC_HIP(hipMalloc(&d_counts, sizeof(unsigned long long) * num));
        VDMC_HIP(hipMalloc(&d_offsets, sizeof(unsigned long long) * num));
        VDMC_HIP(hipMemcpyAsync(d_lists, lists.data(), sizeof(void*) * num, hipMemcpyHostToDevice, st));
        VDMC_HIP(hipMemcpyAsync(d_counts, counts.data(), sizeof(unsigned long long) * num, hipMemcpyHostToDevice, st));
        VDMC_HIP(hipMemcpyAsync(d_offsets, offsets.data(), sizeof(unsigned long long) * num, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_fill_table, dim3(num), dim3(256), 0, st, d_lists, d_counts, d_offsets, num, p->d_table);
        VDMC_HIP(hipGetLastError());
        VDMC_HIP(hipStreamSynchronize(st));
        (void)hipFree(d_lists);
        (void)hipFree(d_counts);
        (void)hipFree(d_offsets);
    } catch (...) {
        delete p;
        throw;
    }
    return p;
}

bool same_signature(const Plan& p, const vdmc_graph* gs, int num, int k, uint64_t* const* outs, const TuneChoice& c) {
    if (p.k != k || (int)p.graphs.size() != num) return false;
    if (p.cfg.variant != c.variant || p.cfg.wgs_per_cu != c.wgs_per_cu || p.cfg.tile != c.tile) return false;
    for (int i = 0; i < num; i++)
        if (p.graphs[i] != gs[i] || p.outs[i] != outs[i]) return false;
    return true;
}

void run_plan(Plan& p, hipStream_t st, bool use_graph) {
    const int k3 = p.k == 3, k4 = p.k == 4;
    const int num = (int)p.graphs.size();
    if (!use_graph || st == nullptr) {
        launch_batch(args_of(p), p.cfg.variant, k3, k4, num, p.cfg.wgs_per_cu, st);
    } else {
        if (!p.exec || p.captured_for != st) {
            if (p.exec) {
                (void)hipGraphExecDestroy(p.exec);
                p.exec = nullptr;
            }
            if (p.graph) {
                (void)hipGraphDestroy(p.graph);
                p.graph = nullptr;
            }
            VDMC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
            try {
                launch_batch(args_of(p), p.cfg.variant, k3, k4, num, p.cfg.wgs_per_cu, st);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(st, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            VDMC_HIP(hipStreamEndCapture(st, &p.graph));
            VDMC_HIP(hipGraphInstantiate(&p.exec, p.graph, nullptr, nullptr, 0));
            p.captured_for = st;
        }
        VDMC_HIP(hipGraphLaunch(p.exec, st));
    }
    // hub roots of large graphs, if any, after the batched light roots
    for (int i = 0; i < num; i++) {
        vdmc_graph_s* g = p.graphs[i];
        if (g->nhub > 0 && !p.is_small[i])
            launch_hub(g, k3, k4, k3 ? p.outs[i] : nullptr, k4 ? p.outs[i] : nullptr, st);
    }
}

void validate_batch(const vdmc_graph* gs, int32_t num, int32_t k, uint64_t* const* outs) {
    VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG, "k must be 3 or 4");
    VDMC_REQUIRE(num >= 0, VDMC_ERR_INVALID_ARG, "num must be non-negative");
    VDMC_REQUIRE(num == 0 || (gs && outs), VDMC_ERR_INVALID_ARG, "gs/outs is NULL");
    int dev = -1;
    for (int i = 0; i < num; i++) {
        VDMC_REQUIRE(gs[i] != nullptr, VDMC_ERR_INVALID_ARG, "graph " + std::to_string(i) + " is NULL");
        VDMC_REQUIRE(outs[i] != nullptr || gs[i]->n == 0, VDMC_ERR_INVALID_ARG,
                     "output " + std::to_string(i) + " is NULL");
        if (dev < 0) dev = gs[i]->device;
        VDMC_REQUIRE(gs[i]->device == dev, VDMC_ERR_INVALID_ARG, "graphs live on different devices");
    }
    if (dev >= 0) VDMC_HIP(hipSetDevice(dev));
}

}  // namespace

void invalidate_batch_plans(vdmc_graph_s* g) {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::find((*it)->graphs.begin(), (*it)->graphs.end(), g) != (*it)->graphs.end()) {
            delete *it;
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
}

void load_tune_cache_once() {
    static bool done = false;
    if (done) return;
    done = true;
    const char* path = getenv("VDMC_TUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    if (!f.good()) return;
    TuneChoice c;
    std::string key;
    long v = 0;
    int seen = 0;
    while (f >> key >> v) {
        if (key == "variant" && v >= 0 && v < kBatchVariants) { c.variant = (int)v; seen++; }
        if (key == "workgroups_per_cu" && v >= 1 && v <= 32) { c.wgs_per_cu = (int)v; seen++; }
        if (key == "tile" && v >= 1 && v <= 4096) { c.tile = (unsigned)v; seen++; }
    }
    if (seen == 3) {
        g_tuned = c;
        g_have_tuned = true;
    }
}

void count_batch_impl(const vdmc_graph_s* const* gs_in, int32_t num, int32_t k, uint64_t* const* outs,
                      hipStream_t st, bool use_graph, const TuneChoice* force) {
    const vdmc_graph* gs = const_cast<const vdmc_graph*>(gs_in);
    validate_batch(gs, num, k, outs);
    if (num == 0) return;
    {
        std::lock_guard<std::mutex> lock(g_plan_mu);
        load_tune_cache_once();
    }
    for (int i = 0; i < num; i++) ensure_bins(gs[i], hub_min_default(), st);
    std::lock_guard<std::mutex> lock(g_plan_mu);
    const TuneChoice cfg = force ? *force : (g_have_tuned ? g_tuned : TuneChoice());
    Plan* plan = nullptr;
    for (Plan* p : g_plans)
        if (same_signature(*p, gs, num, k, outs, cfg)) {
            plan = p;
            break;
        }
    if (!plan) {
        plan = build_plan(gs, num, k, outs, cfg, st);
        g_plans.push_back(plan);
        if (g_plans.size() > 16) {   // keep the cache bounded: drop the oldest plan
            delete g_plans.front();
            g_plans.erase(g_plans.begin());
        }
    }
    run_plan(*plan, st, use_graph);
}

}  // namespace vdmc

extern "C" {

vdmc_status vdmc_count_batch(const vdmc_graph* gs, int32_t num, int32_t k, uint64_t* const* outs, void* stream) {
    return vdmc::guarded([&] { vdmc::count_batch_impl(gs, num, k, outs, vdmc::as_stream(stream), true, nullptr); });
}

vdmc_status vdmc_tune(const vdmc_graph* gs, int32_t num, int32_t k, const char* cache_path) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG, "k must be 3 or 4");
        VDMC_REQUIRE(num > 0 && gs != nullptr, VDMC_ERR_INVALID_ARG, "nothing to tune on");
        for (int i = 0; i < num; i++) VDMC_REQUIRE(gs[i] != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_HIP(hipSetDevice(gs[0]->device));
        // scratch outputs owned by the tuner
        std::vector<uint64_t*> outs(num, nullptr);
        struct FreeOuts {
            std::vector<uint64_t*>& o;
            ~FreeOuts() {
                for (auto* p : o) (void)hipFree(p);
            }
        } guard{outs};
        const int C = vdmc::num_classes(k);
        for (int i = 0; i < num; i++)
            VDMC_HIP(hipMalloc(&outs[i], std::max<int64_t>(gs[i]->n, 1) * C * sizeof(uint64_t)));
        hipStream_t st = nullptr;
        VDMC_HIP(hipStreamCreate(&st));
        struct FreeStream {
            hipStream_t s;
            ~FreeStream() { (void)hipStreamDestroy(s); }
        } sguard{st};
        hipEvent_t e0, e1;
        VDMC_HIP(hipEventCreate(&e0));
        VDMC_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        vdmc::TuneChoice best_c;
        for (int variant = 0; variant < vdmc::kBatchVariants; variant++)
            for (int wgs : {2, 4, 8, 16})
                for (unsigned tile : {1u, 4u, 16u}) {
                    vdmc::TuneChoice c;
                    c.variant = variant;
                    c.wgs_per_cu = wgs;
                    c.tile = tile;
                    vdmc::count_batch_impl(gs, num, k, outs.data(), st, false, &c);   // warm
                    VDMC_HIP(hipEventRecord(e0, st));
                    vdmc::count_batch_impl(gs, num, k, outs.data(), st, false, &c);
                    VDMC_HIP(hipEventRecord(e1, st));
                    VDMC_HIP(hipEventSynchronize(e1));
                    float ms = 0;
                    VDMC_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best) {
                        best = ms;
                        best_c = c;
                    }
                }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        {
            std::lock_guard<std::mutex> lock(vdmc::g_plan_mu);
            vdmc::g_tuned = best_c;
            vdmc::g_have_tuned = true;
        }
        for (int i = 0; i < num; i++) vdmc::invalidate_batch_plans(gs[i]);
        if (cache_path) {
            std::ofstream f(cache_path);
            VDMC_REQUIRE(f.good(), VDMC_ERR_INVALID_ARG, std::string("cannot write ") + cache_path);
            f << "variant " << best_c.variant << "\nthreads_per_root " << (64 << best_c.variant)
              << "\nworkgroups_per_cu " << best_c.wgs_per_cu << "\ntile " << best_c.tile << "\nms " << best << "\n";
        }
    });
}

}  // extern "C"

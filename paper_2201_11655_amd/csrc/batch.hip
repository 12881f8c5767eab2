// Batched counts over many graphs: one persistent launch, captured in a HIP graph.
//
// Small graphs cost microseconds of work each, so per-graph launches are dominated by
// launch and setup latency (the paper notes the fixed cost of reaching the GPU for
// small graphs, Sec. 8).  A batch is counted by one persistent launch sequence:
//   * graphs whose CSR, adjacency bitmap and counters fit in one workgroup's LDS are
//     taken whole, one graph per workgroup, largest estimated work first, from a
//     device-side graph cursor (small.hip);
//   * the roots of the other graphs go into one table of (graph, root) pairs that a
//     persistent grid consumes in tiles from a device-side cursor (count.hip); their
//     roots above the hub threshold are counted by their graph's hub path afterwards.
// The zeroing kernel and the counting kernels are captured into a HIP graph the first
// time a batch signature (graphs, outputs, k, launch parameters) is seen and replayed
// afterwards.  Launch parameters come from the autotuner's choice for the batch's
// shape (k, number of graphs, total size), the library's defaults otherwise.  Every
// choice gives bit-identical counts.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <tuple>

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
    uint8_t* d_generic = nullptr;
    uint2* d_table = nullptr;
    unsigned long long* d_cursor = nullptr;
    unsigned long long nentries = 0;
    SmallGraph* d_small = nullptr;     // graphs counted whole by one workgroup
    std::vector<char> is_small;
    uint32_t nsmall = 0;
    size_t small_lds = 0;
    unsigned small_grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t captured_for = nullptr;
    ~Plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipFree(d_graphs);
        (void)hipFree(d_nvert);
        (void)hipFree(d_generic);
        (void)hipFree(d_table);
        (void)hipFree(d_cursor);
        (void)hipFree(d_small);
    }
};

// shape of a batch for the tuner's choices: k, number of graphs, total vertices, total pairs
using BatchKey = std::tuple<int, int64_t, int64_t, int64_t>;

std::mutex g_plan_mu;
std::vector<Plan*> g_plans;
std::map<BatchKey, TuneChoice> g_tuned;
int g_num_cu = -1;

int num_cu() {
    if (g_num_cu < 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        VDMC_HIP(hipGetDevice(&dev));
        VDMC_HIP(hipGetDeviceProperties(&prop, dev));
        g_num_cu = prop.multiProcessorCount;
    }
    return g_num_cu;
}

BatchKey key_of(const vdmc_graph* gs, int num, int k) {
    int64_t sn = 0, sp = 0;
    for (int i = 0; i < num; i++) {
        sn += gs[i]->n;
        sp += gs[i]->pairs;
    }
    return BatchKey(k, num, sn, sp);
}

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
    b.generic = p.d_generic;
    b.table = p.d_table;
    b.nentries = p.nentries;
    b.cursor = p.d_cursor;
    b.tile = p.cfg.tile;
    b.t3 = t.t3;
    b.t4 = t.t4;
    b.gcursor = reinterpret_cast<unsigned*>(p.d_cursor + 1);
    return b;
}

SmallArgs small_args_of(const Plan& p) {
    const ClassTables& t = class_tables();
    SmallArgs a{};
    a.graphs = p.d_small;
    a.num = p.nsmall;
    a.cursor = reinterpret_cast<unsigned*>(p.d_cursor + 1);
    a.table = p.k == 3 ? t.t3 : t.t4;
    a.comp_of = t.slot4;
    a.comp_cls = t.slotcls;
    return a;
}

Plan* build_plan(const vdmc_graph* gs, int num, int k, uint64_t* const* outs, const TuneChoice& cfg,
                 hipStream_t st) {
    auto* p = new Plan();
    try {
        p->k = k;
        p->cfg = cfg;
        std::vector<GraphView> views(num);
        std::vector<uint64_t> nvert(num);
        std::vector<uint8_t> generic(num, 0);
        std::vector<const uint32_t*> lists(num);
        std::vector<unsigned long long> counts(num), offsets(num);
        std::vector<uint32_t> small;
        unsigned long long total = 0;
        p->is_small.assign(num, 0);
        for (int i = 0; i < num; i++) {
            vdmc_graph_s* g = gs[i];
            p->graphs.push_back(g);
            p->outs.push_back(outs[i]);
            if (small_eligible(g->n, 2 * g->pairs, k)) {   // every root of g in one workgroup
                p->is_small[i] = 1;
                small.push_back((uint32_t)i);
                p->small_lds = std::max(p->small_lds, small_lds_bytes(g->n, 2 * g->pairs, k));
            } else {
                generic[i] = 1;
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
            std::vector<SmallGraph> sg;
            for (uint32_t i : small) {
                vdmc_graph_s* g = gs[i];
                sg.push_back(SmallGraph{g->off, g->adj, g->perm, (unsigned long long*)outs[i], g->stats,
                                        (uint32_t)g->n, (uint32_t)(2 * g->pairs)});
            }
            VDMC_HIP(hipMalloc(&p->d_small, sizeof(SmallGraph) * sg.size()));
            VDMC_HIP(hipMemcpyAsync(p->d_small, sg.data(), sizeof(SmallGraph) * sg.size(), hipMemcpyHostToDevice, st));
            const size_t per_wg = p->small_lds + 9216;
            const int fit = std::max(1, (int)(163840 / per_wg));
            p->small_grid = (unsigned)std::min<int64_t>(p->nsmall, (int64_t)num_cu() * fit);
        }
        VDMC_HIP(hipMalloc(&p->d_graphs, sizeof(GraphView) * std::max(num, 1)));
        VDMC_HIP(hipMalloc(&p->d_nvert, sizeof(uint64_t) * std::max(num, 1)));
        VDMC_HIP(hipMalloc(&p->d_generic, std::max(num, 1)));
        VDMC_HIP(hipMalloc(&p->d_table, sizeof(uint2) * std::max<unsigned long long>(total, 1)));
        VDMC_HIP(hipMalloc(&p->d_cursor, 64));
        VDMC_HIP(hipMemcpyAsync(p->d_graphs, views.data(), sizeof(GraphView) * num, hipMemcpyHostToDevice, st));
        VDMC_HIP(hipMemcpyAsync(p->d_nvert, nvert.data(), sizeof(uint64_t) * num, hipMemcpyHostToDevice, st));
        VDMC_HIP(hipMemcpyAsync(p->d_generic, generic.data(), num, hipMemcpyHostToDevice, st));
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
    if (p.cfg.variant != c.variant || p.cfg.wgs_per_cu != c.wgs_per_cu || p.cfg.tile != c.tile ||
        p.cfg.small_variant != c.small_variant)
        return false;
    for (int i = 0; i < num; i++)
        if (p.graphs[i] != gs[i] || p.outs[i] != outs[i]) return false;
    return true;
}

void run_plan(Plan& p, hipStream_t st, bool use_graph) {
    const int k3 = p.k == 3, k4 = p.k == 4;
    const int num = (int)p.graphs.size();
    GraphUse use(p.graphs, st);   // ordered after earlier work on these graphs
    const SmallArgs sa = small_args_of(p);
    auto launch = [&] {
        launch_batch(args_of(p), &sa, p.small_grid, p.small_lds, p.cfg.small_variant, p.cfg.variant, k3, k4, num,
                     p.cfg.wgs_per_cu, st);
    };
    if (!use_graph || st == nullptr) {
        launch();
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
                launch();
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
    VDMC_REQUIRE(k >= 3 && k <= 5, VDMC_ERR_INVALID_ARG, "k must be 3, 4 or 5");
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
    invalidate_five_plans(g);
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

// Tuned launch parameters per batch shape, from the file named by VDMC_TUNE_CACHE (lines
// written by vdmc_tune: "k graphs vertices pairs small_variant variant wgs_per_cu tile ms").
void load_tune_cache_once() {
    static bool done = false;
    if (done) return;
    done = true;
    const char* path = getenv("VDMC_TUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        int k = 0;
        int64_t num = 0, sn = 0, sp = 0;
        TuneChoice c;
        double ms = 0;
        if (!(in >> k >> num >> sn >> sp >> c.small_variant >> c.variant >> c.wgs_per_cu >> c.tile >> ms)) continue;
        if (c.small_variant < 0 || c.small_variant > 2 || c.variant < 0 || c.variant >= kBatchVariants ||
            c.wgs_per_cu < 1 || c.wgs_per_cu > 32 || c.tile < 1 || c.tile > 4096)
            continue;
        g_tuned[BatchKey(k, num, sn, sp)] = c;
    }
}

void count_batch_impl(const vdmc_graph_s* const* gs_in, int32_t num, int32_t k, uint64_t* const* outs,
                      hipStream_t st, bool use_graph, const TuneChoice* force) {
    const vdmc_graph* gs = const_cast<const vdmc_graph*>(gs_in);
    validate_batch(gs, num, k, outs);
    if (num == 0) return;
    if (k == 5) {
        count5_batch(gs_in, num, outs, st);
        return;
    }
    (void)class_tables();
    for (int i = 0; i < num; i++)
        if (!small_eligible(gs[i]->n, 2 * gs[i]->pairs, k)) {
            std::lock_guard<std::mutex> lock(gs[i]->mu);
            ensure_bins(gs[i], st);
        }
    std::lock_guard<std::mutex> lock(g_plan_mu);
    load_tune_cache_once();
    TuneChoice cfg;
    if (force) {
        cfg = *force;
    } else {
        auto it = g_tuned.find(key_of(gs, num, k));
        if (it != g_tuned.end()) cfg = it->second;
    }
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
        bool any_generic = false, any_small = false;
        for (int i = 0; i < num; i++) {
            const bool sm = vdmc::small_eligible(gs[i]->n, 2 * gs[i]->pairs, k);
            any_small |= sm;
            any_generic |= !sm;
        }
        // candidates: workgroup size of the whole-graph kernel; for the root table, threads
        // per root, workgroups per CU and roots per cursor step (the median of 3 timed runs)
        std::vector<vdmc::TuneChoice> cands;
        for (int sv = 0; sv < (any_small ? 3 : 1); sv++)
            for (int variant = 0; variant < (any_generic ? vdmc::kBatchVariants : 1); variant++)
                for (int wgs : any_generic ? std::vector<int>{2, 4, 8, 16} : std::vector<int>{8})
                    for (unsigned tile : any_generic ? std::vector<unsigned>{1u, 4u, 16u} : std::vector<unsigned>{4u}) {
                        vdmc::TuneChoice c;
                        c.small_variant = any_small ? sv : 2;
                        c.variant = variant;
                        c.wgs_per_cu = wgs;
                        c.tile = tile;
                        cands.push_back(c);
                    }
        float best = 1e30f;
        vdmc::TuneChoice best_c;
        for (const auto& c : cands) {
            vdmc::count_batch_impl(gs, num, k, outs.data(), st, false, &c);   // warm
            float t[3];
            for (float& ms : t) {
                VDMC_HIP(hipEventRecord(e0, st));
                vdmc::count_batch_impl(gs, num, k, outs.data(), st, false, &c);
                VDMC_HIP(hipEventRecord(e1, st));
                VDMC_HIP(hipEventSynchronize(e1));
                VDMC_HIP(hipEventElapsedTime(&ms, e0, e1));
            }
            std::sort(t, t + 3);
            if (t[1] < best) {
                best = t[1];
                best_c = c;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        const vdmc::BatchKey key = vdmc::key_of(gs, num, k);
        {
            std::lock_guard<std::mutex> lock(vdmc::g_plan_mu);
            vdmc::g_tuned[key] = best_c;
        }
        for (int i = 0; i < num; i++) vdmc::invalidate_batch_plans(gs[i]);
        if (cache_path) {
            std::ofstream f(cache_path, std::ios::app);
            VDMC_REQUIRE(f.good(), VDMC_ERR_INVALID_ARG, std::string("cannot write ") + cache_path);
            f << k << " " << std::get<1>(key) << " " << std::get<2>(key) << " " << std::get<3>(key) << " "
              << best_c.small_variant << " " << best_c.variant << " " << best_c.wgs_per_cu << " " << best_c.tile << " "
              << best << "\n";
        }
    });
}

vdmc_status vdmc_tuned_choice(const vdmc_graph* gs, int32_t num, int32_t k, int32_t* choice_out) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(num > 0 && gs != nullptr && choice_out != nullptr, VDMC_ERR_INVALID_ARG, "bad argument");
        for (int i = 0; i < num; i++) VDMC_REQUIRE(gs[i] != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        std::lock_guard<std::mutex> lock(vdmc::g_plan_mu);
        vdmc::load_tune_cache_once();
        auto it = vdmc::g_tuned.find(vdmc::key_of(gs, num, k));
        const vdmc::TuneChoice c = it != vdmc::g_tuned.end() ? it->second : vdmc::TuneChoice();
        choice_out[0] = it != vdmc::g_tuned.end() ? 1 : 0;
        choice_out[1] = vdmc::small_threads(c.small_variant);
        choice_out[2] = 64 << c.variant;
        choice_out[3] = c.wgs_per_cu;
        choice_out[4] = (int32_t)c.tile;
    });
}

}  // extern "C"

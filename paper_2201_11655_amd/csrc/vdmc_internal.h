// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vdmc.h"

namespace vdmc {

// ----------------------------------------------------------------------------- errors

void set_error(const std::string& msg);
void clear_error();
const char* last_error_cstr();

struct Error {
    vdmc_status code;
    std::string msg;
};

#define VDMC_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            throw ::vdmc::Error{e_ == hipErrorOutOfMemory ? VDMC_ERR_OUT_OF_MEMORY       \
                                                          : VDMC_ERR_DEVICE,             \
                                std::string(#call) + ": " + hipGetErrorString(e_)};      \
        }                                                                                \
    } while (0)

#define VDMC_REQUIRE(cond, code, msg)                        \
    do {                                                     \
        if (!(cond)) throw ::vdmc::Error{(code), (msg)};     \
    } while (0)

// Runs f() and converts exceptions into a status + thread-local message.
template <class F>
vdmc_status guarded(F&& f) {
    try {
        clear_error();
        f();
        return VDMC_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return VDMC_ERR_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        set_error(e.what());
        return VDMC_ERR_DEVICE;
    } catch (...) {
        set_error("unknown failure");
        return VDMC_ERR_DEVICE;
    }
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ----------------------------------------------------------------------------- classes

constexpr int kClasses3 = 13;
constexpr int kClasses4 = 199;
constexpr int kShapes = 6;   // (1,1) (1,2) | (3,0,0) (2,1,0) (1,2,0) (1,1,1)
constexpr int kStatSlots = 8;       // per graph: sets visited per shape (kShapes), then spare

constexpr int kClasses5 = 9364;

inline int num_classes(int k) {
    return k == 3 ? kClasses3 : (k == 4 ? kClasses4 : (k == 5 ? kClasses5 : -1));
}

// Device-resident class tables of the current device: code -> class id (0xFF =
// disconnected).  Built on first use by a kernel; cached per device.
// Classes of 4-sets whose induced subgraph is a tree (the 15 directed 4-path and the
// 10 directed 3-star classes): the classes of the sets whose pairs outside their BFS
// tree are non-adjacent, most of the 4-sets of sparse graphs; LDS counters are kept
// for them.
constexpr int kCompact4 = 25;
// the hub path takes graphs whose largest degree is at most this (slot and child lists in LDS)
constexpr uint32_t kHubMaxDegree = 2048;

struct ClassTables {
    const uint8_t* t3;   // 64 entries
    const uint8_t* t4;   // 4096 entries
    const uint8_t* slot4;     // 199 entries: class -> compact slot or 0xFF
    const uint8_t* slotcls;   // kCompact4 entries: compact slot -> class
    const uint8_t* maps4;     // 768 entries: class -> star slot (10), path slot (15), tree slot (25); 0xFF none
    const uint8_t* star_cls;  // 10 entries: star slot -> class
    const uint8_t* path_cls;  // 15 entries: path slot -> class
    std::vector<uint8_t> host3, host4;
    std::vector<uint16_t> codes3, codes4;
};
const ClassTables& class_tables();   // for the current device

// k = 5: code (20 bits) -> class id (0xFFFF = disconnected), 2 MiB in device memory;
// built on the first 5-vertex count on a device and kept.
struct ClassTable5 {
    const uint16_t* table = nullptr;
    std::vector<uint32_t> codes;   // class id -> minimal index
};
const ClassTable5& class_table5();   // for the current device

// ----------------------------------------------------------------------------- graph

struct DeviceScratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};
struct DoneEvent;

}  // namespace vdmc

struct vdmc_graph_s {
    int device = 0;
    int64_t n = 0;
    int64_t arcs = 0;
    int64_t pairs = 0;
    int32_t max_deg = 0;
    bool undirected = false;     // built with VDMC_UNDIRECTED: every pair has both arc bits
    uint64_t* utmp = nullptr;    // directed-class scratch of the undirected counts (n x 199)
    uint32_t* off = nullptr;     // n + 1 row offsets (rank space)
    uint32_t* adj = nullptr;     // 2 * pairs entries: (nbr_rank << 2) | arc bits
    uint32_t* split = nullptr;   // n: index of the first entry with nbr_rank > row
    int32_t* perm = nullptr;     // n: rank -> original id
    // per-root work description used by the schedulers (built with the graph)
    uint32_t* roots = nullptr;   // roots with a non-empty higher neighbourhood
    int64_t nroots = 0;
    unsigned long long* stats = nullptr;  // kShapes shape counters of the last count
    std::mutex mu;
    // root bins (built at the first count after a change of the hub threshold)
    int hub_min = 32;            // roots with at least this many higher neighbours take the hub path
    int bins_hub_min = -1;
    uint32_t* light = nullptr;   // roots handled by the per-set kernel
    int64_t nlight = 0;
    uint32_t* hubs = nullptr;    // roots handled by the hub kernel, largest work first
    int64_t nhub = 0;
    int64_t max_scan2 = 0;       // largest depth-2 scan over hub roots (scratch sizing)
    int32_t max_hi = 0;          // largest |N+(r)|
    int32_t light_max_d = 0;     // largest |N+(r)| among the light roots
    // hub-path scratch (per workgroup slices), sized for this graph
    void* hub_scratch = nullptr;
    size_t hub_scratch_bytes = 0;
    unsigned* hub_queue = nullptr;   // root cursor, long-slot task count and cursor
    uint32_t* hub_s2 = nullptr;      // per hub root: entries of its slots' rows above it
    void* hub_tasks = nullptr;       // long-slot tasks (hub index, slot)
    uint32_t hub_task_cap = 0;
    size_t hub_scratch_need = 0;     // bytes of hub_scratch + hub_tasks for the current bins
    unsigned long long* ehash = nullptr;   // edge hash: every pair of the graph, 2^ehash_bits slots
    uint32_t ehash_bits = 0;
    uint32_t* epid = nullptr;    // per edge-hash slot: output row of the pair (per-edge counts)
    int32_t* elo = nullptr;      // per output row: the pair's endpoints (original ids, lo < hi)
    int32_t* ehi = nullptr;
    size_t hub_layout[16] = {0};
    // timing of the last count call: [0,1] around the per-set kernel, [2,3] around the
    // hub kernel (created at the first count)
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool timed_light = false, timed_hub = false;
    // end of the last call's device work on this graph (every call's work is ordered after
    // the previous call's, whatever the streams)
    std::shared_ptr<vdmc::DoneEvent> last;
    // 5-vertex counts in device memory (graphs that LDS does not hold): items before each
    // root, then the item cursor; built at the first such count
    unsigned long long* five_hp = nullptr;
    unsigned long long five_items = 0;
};

namespace vdmc {
// An event that ends the device work of one call (shared by the graphs the call used).
struct DoneEvent {
    hipEvent_t e = nullptr;
    DoneEvent() { VDMC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
    ~DoneEvent() {
        if (e) (void)hipEventDestroy(e);
    }
    DoneEvent(const DoneEvent&) = delete;
    DoneEvent& operator=(const DoneEvent&) = delete;
};

// One call's use of one or more graphs.  Holds the graphs' mutexes (in address order)
// while the call enqueues its work (the host-side state: bins, scratch, timing events),
// makes the call's stream wait for the end of the previous calls' work on those graphs
// (whatever their streams), and records one event at the end of this call's work.
// Concurrent calls on a graph are therefore serialised on the device, and each one's
// result is that of the call alone.
struct GraphUse {
    std::vector<vdmc_graph_s*> gs;
    hipStream_t st;
    std::vector<std::unique_lock<std::mutex>> locks;
    GraphUse(vdmc_graph_s* g, hipStream_t s) : GraphUse(std::vector<vdmc_graph_s*>{g}, s) {}
    GraphUse(std::vector<vdmc_graph_s*> graphs, hipStream_t s) : gs(std::move(graphs)), st(s) {
        std::sort(gs.begin(), gs.end());
        gs.erase(std::unique(gs.begin(), gs.end()), gs.end());
        locks.reserve(gs.size());
        for (auto* g : gs) locks.emplace_back(g->mu);
        std::vector<DoneEvent*> waited;
        for (auto* g : gs) {
            DoneEvent* e = g->last.get();
            if (e && std::find(waited.begin(), waited.end(), e) == waited.end()) {
                VDMC_HIP(hipStreamWaitEvent(st, e->e, 0));
                waited.push_back(e);
            }
        }
    }
    ~GraphUse() {
        try {
            auto ev = std::make_shared<DoneEvent>();
            if (hipEventRecord(ev->e, st) == hipSuccess)
                for (auto* g : gs) g->last = ev;
        } catch (...) {
        }
    }
    GraphUse(const GraphUse&) = delete;
    GraphUse& operator=(const GraphUse&) = delete;
};
// waits (host) for the end of the last call's work on g; the caller holds g->mu
inline void wait_graph(vdmc_graph_s* g) {
    if (g->last) VDMC_HIP(hipEventSynchronize(g->last->e));
}
// one graph as seen by the per-set kernels
struct GraphView {
    const uint32_t* off;
    const uint32_t* adj;
    const uint32_t* split;
    const int32_t* perm;
    unsigned long long* out3;
    unsigned long long* out4;
    unsigned long long* stats;
    const unsigned long long* ehash = nullptr;   // edge hash if the graph has one (adjacency tests)
    uint32_t ehash_bits = 0;
};
// batched launch over many graphs (count.hip / batch.hip)
struct BatchArgs {
    const GraphView* graphs;        // device array, one per graph
    const uint64_t* nvert;          // device array: n of every graph
    const uint2* table;             // device array of (graph, root) pairs
    unsigned long long nentries;
    unsigned long long* cursor;     // device work cursor, zeroed inside the launch
    unsigned long long tile;        // roots taken per cursor step
    const uint8_t* t3;
    const uint8_t* t4;
    const uint8_t* generic;         // per graph: 1 = counted through the root table (output zeroed first)
    unsigned* gcursor;              // graph cursor of the whole-graph kernel, zeroed inside the launch
};
// Small graphs (small.hip): one workgroup counts a whole graph held in LDS.
struct SmallGraph {
    const uint32_t* off;        // n + 1 (rank space)
    const uint32_t* adj;        // entries
    const int32_t* perm;        // rank -> original id
    unsigned long long* out;    // n x C, rows by original id
    unsigned long long* stats;  // shape (visited-set) counters of the graph
    uint32_t n, entries;
};
struct SmallArgs {
    const SmallGraph* graphs;   // device array of num graphs, or nullptr: the single graph `one`
    SmallGraph one;
    uint32_t num;
    unsigned* cursor;           // graph cursor of a batched launch (zeroed before it)
    const uint8_t* table;       // code -> class id for the launch's k
    const uint8_t* comp_of;     // class -> tree slot or 0xFF (256 entries)
    const uint8_t* comp_cls;    // tree slot -> class
};
constexpr int64_t kSmallMaxN = 1024;            // u32 LDS counters cannot overflow below this
constexpr size_t kSmallLdsBudget = 163840 - 9216;   // dynamic LDS of one workgroup (gfx950: 160 KiB per CU)
size_t small_lds_bytes(int64_t n, int64_t entries, int k);
bool small_eligible(int64_t n, int64_t entries, int k);
int small_threads(int variant);
void launch_small(const SmallArgs& a, int k, int variant, unsigned grid, size_t lds, hipStream_t stream);
constexpr int kBatchVariants = 3;   // 64, 128, 256 threads per root
struct TuneChoice {
    int small_variant = 2;   // threads per workgroup of the whole-graph kernel: 256, 512, 1024
    int variant = 0;      // threads per root: 64, 128, 256
    int wgs_per_cu = 8;   // persistent workgroups per compute unit
    unsigned tile = 4;    // roots per cursor step
};
// batched count of many graphs (one k), optionally replayed from a captured HIP graph
void count_batch_impl(const vdmc_graph_s* const* gs, int32_t num, int32_t k, uint64_t* const* outs,
                      hipStream_t stream, bool use_graph, const TuneChoice* force);
void launch_batch(const BatchArgs& b, const SmallArgs* small, unsigned small_grid, size_t small_lds,
                  int small_variant, int variant, int k3, int k4, int num_graphs, int wgs_per_cu, hipStream_t stream);
void invalidate_batch_plans(vdmc_graph_s* g);
// launches (count.hip)
void launch_count(vdmc_graph_s* g, int k3, int k4, uint64_t* out3, uint64_t* out4,
                  hipStream_t stream, int64_t rank_lo = 0, int64_t rank_hi = INT64_MAX, bool zero = true);
void launch_fill_u64(uint64_t* p, size_t n, uint64_t value, hipStream_t stream);
// hub path (count_hub.hip)
void ensure_bins(vdmc_graph_s* g, hipStream_t stream);   // for g->hub_min; caller holds g->mu
size_t hub_scratch_need(const vdmc_graph_s* g);           // bytes ensure_hub_scratch allocates (after ensure_bins)
void ensure_hub_scratch(vdmc_graph_s* g);                 // caller holds g->mu
void free_hub_scratch(vdmc_graph_s* g);                   // caller holds g->mu; waits for the graph's work
void ensure_edge_hash(vdmc_graph_s* g, hipStream_t stream);    // count_hub.hip
void ensure_edge_index(vdmc_graph_s* g, hipStream_t stream);   // edges.hip
void launch_count_edges(vdmc_graph_s* g, int k, uint64_t* out, hipStream_t stream);   // count.hip
void launch_hub(vdmc_graph_s* g, int k3, int k4, uint64_t* out3, uint64_t* out4, hipStream_t stream,
                uint32_t rank_lo = 0, uint32_t rank_hi = 0xFFFFFFFFu, const hipEvent_t* around = nullptr);
void free_hub(vdmc_graph_s* g);
// 5-vertex motifs (count5.hip): graphs held whole in one workgroup's LDS, others in device memory
constexpr int64_t kFiveMaxN = 512;
size_t five_lds_bytes(int64_t n, int64_t entries);
bool five_eligible(int64_t n, int64_t entries);
void launch_count5(vdmc_graph_s* g, uint64_t* out, hipStream_t stream);   // caller holds the graph (GraphUse)
void count5_batch_lds(std::vector<vdmc_graph_s*>& gs, std::vector<uint64_t*>& outs, hipStream_t stream);
void count5_batch(const vdmc_graph_s* const* gs, int32_t num, uint64_t* const* outs, hipStream_t stream);
void invalidate_five_plans(vdmc_graph_s* g);
void free_five(vdmc_graph_s* g);   // the graph's 5-vertex state; caller makes sure no count runs
}  // namespace vdmc

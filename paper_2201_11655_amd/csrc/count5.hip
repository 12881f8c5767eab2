// Per-vertex 5-motif counts: the method carried to 5-vertex motifs (Sec. 11 names
// 5-vertex motifs as the next case of the same claims and data structure).
//
// What is counted is what k = 3, 4 count (Sec. 4.1-4.2): every connected 5-set S is
// visited once, its index is read from the induced adjacency matrix (20 bits, first
// entry most significant), mapped to its isomorphism class (9364 weakly connected
// classes) and credited to all five members.
//
// How each set is reached once (Lemma 1 and the BFS shapes of Lemmas 2-4, one level
// further): S is visited from its lowest-rank vertex r only, along its BFS layering
// from r: layer 1 = the members adjacent to r, layer i + 1 = the members adjacent to
// layer i and to no earlier layer.  The layer sizes are the set's shape; five vertices
// have eight: (4) (3,1) (2,2) (2,1,1) (1,3) (1,2,1) (1,1,2) (1,1,1,1), the 4-vertex
// ones of Lemma 2 being the same construction on four.  Members are chosen in the
// order (layer, parent, position in the parent's row), where a member's parent is its
// first neighbour in the previous layer -- a vertex hangs under its lower-index parent,
// the rule of Lemma 3 -- and a candidate under parent x is taken only if it is
// adjacent to no member chosen before x: such a vertex lies in an earlier layer or
// under an earlier parent (the rule of Lemma 4, generalised).  So the layering, the
// parents and the choice order are all fixed by S, and each set is produced once.
//
// GPU mapping: the graph is held whole in LDS -- rank-space CSR, the rank -> id map
// and a 2-bit arc matrix (every pair test and every index bit is one LDS read).  A work
// item is a root r with the first member a of its layer 1 (one per pair of G_U, from
// its lower-rank end); a lane runs the item's whole search (three nested candidate
// loops) and visits every set of it.  Items are taken one at a time from an LDS cursor
// so lanes with short items keep taking new ones.  Class ids come from a 2^20-entry
// u16 table in device memory (2 MiB, L2-resident); each set adds one to five counters
// of the graph's output rows (9364 classes per vertex do not fit in LDS).  Two modes:
//   * owned (batches of many graphs): one workgroup takes a whole graph and zeroes its
//     output block first; credits are workgroup-scope atomics, executed in the L2 of
//     the workgroup's die;
//   * shared (one graph, or few): workgroups take segments of a graph's items; credits
//     are device-scope atomics and the output is zeroed by a fill launch before.
// Visited sets are counted per shape (the graph's 8 counters) so that callers can
// check that every set was visited: their sum is the number of connected 5-sets.
#include "vdmc_internal.h"

namespace vdmc {
namespace {

constexpr uint32_t kFiveThreads = 256;
constexpr size_t kFiveStaticLds = 2048;                        // the kernel's __shared__ words below
constexpr size_t kFiveLdsBudget = 163840 - kFiveStaticLds;     // gfx950: 160 KiB of LDS per workgroup
constexpr uint32_t kNone = 0xFFFFFFFFu;

struct FiveGraph {
    const uint32_t* off;        // n + 1 (rank space)
    const uint32_t* adj;        // entries: (nbr_rank << 2) | arc bits
    const int32_t* perm;        // rank -> original id
    unsigned long long* out;    // n x 9364, rows by original id
    unsigned long long* stats;  // 8 shape counters
    uint32_t n, entries, items; // items = pairs of G_U
    uint32_t seg_base;          // first segment of this graph in the launch
};

struct FiveArgs {
    const FiveGraph* graphs;    // device array of num graphs, or nullptr: the graph `one`
    FiveGraph one;
    uint32_t num;
    uint32_t nseg;              // segments in the launch
    uint32_t seg_items;         // items per segment (owned mode: at least every graph's items)
    unsigned* cursor;           // segment cursor, zeroed before the launch
    const uint16_t* table;      // code -> class id
    uint32_t zero_out;          // owned mode: the workgroup zeroes the graph's output block
};

// bit of the index of a 5-set for the entry (i, j), i != j: rows in order, the diagonal
// skipped, entry (0,1) the most significant of the 20 (Sec. 4.1, Fig. 1)
__device__ __forceinline__ constexpr uint32_t shift5(uint32_t i, uint32_t j) {
    return 19u - (i * 4u + (j < i ? j : j - 1u));
}
// index bits of the pair (i, t), i < t, from the arc bits b seen from member i
// (bit 0: i -> t, bit 1: t -> i)
__device__ __forceinline__ uint32_t pair_bits(uint32_t i, uint32_t t, uint32_t b) {
    return ((b & 1u) << shift5(i, t)) | ((b >> 1) << shift5(t, i));
}

struct FiveLds {
    const uint32_t* off;
    const uint32_t* adj;
    const uint32_t* mat;    // n rows of W words, 16 two-bit entries per word
    const uint32_t* perm;
    uint32_t W;
    // arc bits of (u, v) seen from u: bit 0 u -> v, bit 1 v -> u; 0 if not adjacent
    __device__ __forceinline__ uint32_t bits(uint32_t u, uint32_t v) const {
        return (mat[u * W + (v >> 4)] >> ((v & 15u) * 2u)) & 3u;
    }
    // first entry of u's row whose neighbour has rank above x
    __device__ __forceinline__ uint32_t first_above(uint32_t u, uint32_t x) const {
        uint32_t lo = off[u], hi = off[u + 1];
        const uint32_t key = (x + 1u) << 2;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (adj[mid] < key) lo = mid + 1; else hi = mid;
        }
        return lo;
    }
};

// member i of S (i < 5 is not a compile-time constant where this is called)
__device__ __forceinline__ uint32_t member(const uint32_t (&S)[5], uint32_t i) {
    uint32_t v = S[0];
    v = i == 1u ? S[1] : v;
    v = i == 2u ? S[2] : v;
    v = i == 3u ? S[3] : v;
    v = i == 4u ? S[4] : v;
    return v;
}

// y adjacent to none of S[0..lim)
__device__ __forceinline__ bool clear_of(const FiveLds& L, const uint32_t (&S)[5], uint32_t lim, uint32_t y) {
#pragma unroll
    for (uint32_t m = 0; m < 4; m++)
        if (m < lim && L.bits(S[m], y)) return false;
    return true;
}

// Candidates of the next member, given S[0..t): first the rest of S[t-1]'s layer (after
// S[t-1]'s parent and position), then -- phase 1 -- the first member of a new layer under
// the members of S[t-1]'s layer.  pi: S index of the current parent, [pi, pend) the
// parents left in the phase, [j, jend) the rest of the parent's row.
struct Cand {
    uint32_t pi, pend, j, jend, phase, ls;
    __device__ __forceinline__ void start(const FiveLds& L, const uint32_t (&S)[5], uint32_t par, uint32_t pos,
                                          uint32_t ls_prev) {
        pi = par;
        pend = ls_prev;
        j = pos + 1u;
        jend = L.off[member(S, par) + 1u];
        phase = 0u;
        ls = ls_prev;
    }
    // next candidate vertex, or kNone; t = the S index being chosen
    __device__ __forceinline__ uint32_t next(const FiveLds& L, const uint32_t (&S)[5], uint32_t t) {
        for (;;) {
            while (j < jend) {
                const uint32_t y = L.adj[j++] >> 2;
                if (clear_of(L, S, pi, y)) return y;
            }
            if (++pi < pend) {
                const uint32_t x = member(S, pi);
                j = L.first_above(x, S[0]);
                jend = L.off[x + 1u];
                continue;
            }
            if (phase == 0u) {   // the layer of S[t-1] is closed: open the next one under it
                phase = 1u;
                pi = ls;
                pend = t;
                const uint32_t x = member(S, pi);
                j = L.first_above(x, S[0]);
                jend = L.off[x + 1u];
                continue;
            }
            return kNone;
        }
    }
};

template <bool kOwned>
__device__ __forceinline__ void bump(unsigned long long* p) {
    if (kOwned) __hip_atomic_fetch_add(p, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else __hip_atomic_fetch_add(p, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_shape(unsigned long long (&vis)[8], uint32_t s, unsigned long long v) {
#pragma unroll
    for (uint32_t i = 0; i < 8; i++) vis[i] += (s == i) ? v : 0ull;
}

// Every set of the item (root r, first layer-1 member at entry apos of r's row).
template <bool kOwned>
__device__ void five_item(const FiveLds& L, const uint16_t* __restrict__ table, unsigned long long* __restrict__ out,
                          uint32_t r, uint32_t apos, unsigned long long (&vis)[8]) {
    uint32_t S[5];
    S[0] = r;
    S[1] = L.adj[apos] >> 2;
    S[2] = S[3] = S[4] = 0u;
    const uint32_t code1 = pair_bits(0, 1, L.adj[apos] & 3u);
    const uint32_t P0 = L.perm[r], P1 = L.perm[S[1]];
    Cand c2;
    c2.start(L, S, 0u, apos, 1u);   // S[1]'s parent is S[0]; layer 1 starts at index 1
    for (;;) {
        const uint32_t y2 = c2.next(L, S, 2u);
        if (y2 == kNone) break;
        S[2] = y2;
        const uint32_t par2 = c2.pi, pos2 = c2.j - 1u, ls2 = c2.phase ? 2u : 1u;
        const uint32_t code2 = code1 | pair_bits(0, 2, L.bits(S[0], y2)) | pair_bits(1, 2, L.bits(S[1], y2));
        const uint32_t P2 = L.perm[y2];
        Cand c3;
        c3.start(L, S, par2, pos2, ls2);
        for (;;) {
            const uint32_t y3 = c3.next(L, S, 3u);
            if (y3 == kNone) break;
            S[3] = y3;
            const uint32_t par3 = c3.pi, pos3 = c3.j - 1u, ls3 = c3.phase ? 3u : ls2;
            const uint32_t code3 = code2 | pair_bits(0, 3, L.bits(S[0], y3)) | pair_bits(1, 3, L.bits(S[1], y3)) |
                                   pair_bits(2, 3, L.bits(S[2], y3));
            const uint32_t P3 = L.perm[y3];
            Cand c4;
            c4.start(L, S, par3, pos3, ls3);
            unsigned long long same = 0, opened = 0;   // sets whose last member continues / opens a layer
            for (;;) {
                const uint32_t y4 = c4.next(L, S, 4u);
                if (y4 == kNone) break;
                const uint32_t code = code3 | pair_bits(0, 4, L.bits(S[0], y4)) | pair_bits(1, 4, L.bits(S[1], y4)) |
                                      pair_bits(2, 4, L.bits(S[2], y4)) | pair_bits(3, 4, L.bits(S[3], y4));
                const uint32_t cls = table[code];
                if (cls >= (uint32_t)kClasses5) continue;   // a connected set always has a class
                const uint32_t P4 = L.perm[y4];
                bump<kOwned>(&out[(size_t)P0 * kClasses5 + cls]);
                bump<kOwned>(&out[(size_t)P1 * kClasses5 + cls]);
                bump<kOwned>(&out[(size_t)P2 * kClasses5 + cls]);
                bump<kOwned>(&out[(size_t)P3 * kClasses5 + cls]);
                bump<kOwned>(&out[(size_t)P4 * kClasses5 + cls]);
                if (c4.phase) opened++; else same++;
            }
            // shape id: bit 2 = a new layer opens at member 2, bit 1 at member 3, bit 0 at member 4
            const uint32_t base = (ls2 == 2u ? 4u : 0u) | (ls3 == 3u ? 2u : 0u);
            add_shape(vis, base, same);
            add_shape(vis, base | 1u, opened);
        }
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <bool kOwned>
__global__ __launch_bounds__(kFiveThreads) void k_five(FiveArgs A) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_seg, s_gi, s_next;
    __shared__ uint32_t part[kFiveThreads];
    const uint32_t tid = threadIdx.x;
    uint32_t loaded = kNone;
    FiveGraph G{};
    FiveLds L{};
    uint32_t* sSplit = nullptr;
    uint32_t* sHp = nullptr;
    for (;;) {
        if (tid == 0) {
            const uint32_t seg = atomicAdd(A.cursor, 1u);
            uint32_t gi = 0;
            if (A.graphs && seg < A.nseg) {   // last graph whose first segment is <= seg
                uint32_t lo = 0, hi = A.num;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (A.graphs[mid].seg_base <= seg) lo = mid; else hi = mid;
                }
                gi = lo;
            }
            s_seg = seg;
            s_gi = gi;
        }
        __syncthreads();
        const uint32_t seg = s_seg, gi = s_gi;
        if (seg >= A.nseg) break;
        if (gi != loaded) {   // the graph into LDS
            G = A.graphs ? A.graphs[gi] : A.one;
            if (kOwned && tid < 8) G.stats[tid] = 0ull;   // owned: the graph's counters are this workgroup's
            const uint32_t n = G.n, E = G.entries, W = (n + 15u) >> 4;
            uint32_t* sOff = lds;
            sSplit = sOff + n + 1;
            sHp = sSplit + n;
            uint32_t* sPerm = sHp + n + 1;
            uint32_t* sAdj = sPerm + n;
            uint32_t* sMat = sAdj + E;
            for (uint32_t i = tid; i < (n ? n + 1u : 0u); i += kFiveThreads) sOff[i] = G.off[i];
            for (uint32_t i = tid; i < n; i += kFiveThreads) sPerm[i] = (uint32_t)G.perm[i];
            for (uint32_t i = tid; i < E; i += kFiveThreads) sAdj[i] = G.adj[i];
            for (uint32_t i = tid; i < n * W; i += kFiveThreads) sMat[i] = 0u;
            __syncthreads();
            for (uint32_t u = tid; u < n; u += kFiveThreads) {
                const uint32_t b = sOff[u], e = sOff[u + 1];
                uint32_t split = e;
                for (uint32_t x = b; x < e; x++) {
                    const uint32_t a = sAdj[x], v = a >> 2;
                    if (v > u && split == e) split = x;
                    sMat[u * W + (v >> 4)] |= (a & 3u) << ((v & 15u) * 2u);   // row u is this thread's
                }
                sSplit[u] = split;
                sHp[u] = e - split;
            }
            __syncthreads();
            // exclusive prefix of the higher-neighbour counts: item i of the graph is the
            // entry sSplit[r] + (i - sHp[r]) of the root r with sHp[r] <= i < sHp[r + 1]
            const uint32_t per = (n + kFiveThreads - 1) / kFiveThreads;
            const uint32_t lo = min(n, tid * per), hi = min(n, lo + per);
            uint32_t s = 0;
            for (uint32_t i = lo; i < hi; i++) s += sHp[i];
            part[tid] = s;
            __syncthreads();
            for (uint32_t o = 1; o < kFiveThreads; o <<= 1) {
                const uint32_t v = tid >= o ? part[tid - o] : 0u;
                __syncthreads();
                part[tid] += v;
                __syncthreads();
            }
            uint32_t run = part[tid] - s;
            for (uint32_t i = lo; i < hi; i++) {
                const uint32_t x = sHp[i];
                sHp[i] = run;
                run += x;
            }
            if (tid == 0) sHp[n] = part[kFiveThreads - 1];
            if (kOwned && A.zero_out) {   // the graph's output block belongs to this workgroup
                const size_t cells = (size_t)n * kClasses5;
                if (((uintptr_t)G.out & 15u) == 0) {   // 16-byte stores (9364 is even)
                    ulonglong2* o = reinterpret_cast<ulonglong2*>(G.out);
                    for (size_t i = tid; i < cells / 2; i += kFiveThreads) o[i] = make_ulonglong2(0ull, 0ull);
                } else {
                    for (size_t i = tid; i < cells; i += kFiveThreads) G.out[i] = 0ull;
                }
            }
            L = FiveLds{sOff, sAdj, sMat, sPerm, W};
            loaded = gi;
            __syncthreads();
        }
        const uint32_t lo = (seg - (A.graphs ? G.seg_base : 0u)) * A.seg_items;
        const uint32_t hi = min(G.items, lo + A.seg_items);
        if (tid == 0) s_next = lo;
        __syncthreads();
        unsigned long long vis[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (;;) {
            const uint32_t i = atomicAdd(&s_next, 1u);
            if (i >= hi) break;
            uint32_t rlo = 0, rhi = G.n;   // root: last r with sHp[r] <= i
            while (rhi - rlo > 1) {
                const uint32_t mid = (rlo + rhi) >> 1;
                if (sHp[mid] <= i) rlo = mid; else rhi = mid;
            }
            five_item<kOwned>(L, A.table, G.out, rlo, sSplit[rlo] + (i - sHp[rlo]), vis);
        }
#pragma unroll
        for (int s = 0; s < 8; s++) {
            const unsigned long long v = wave_sum(vis[s]);
            if ((tid & 63u) == 0 && v) {
                if (kOwned) __hip_atomic_fetch_add(&G.stats[s], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                else atomicAdd(&G.stats[s], v);
            }
        }
        __syncthreads();   // the segment is done before the next claim rewrites s_seg / s_next
    }
}

void launch_five(const FiveArgs& a, bool owned, unsigned grid, size_t lds, hipStream_t st) {
    void (*kern)(FiveArgs) = owned ? k_five<true> : k_five<false>;
    VDMC_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kFiveThreads), lds, st, a);
    VDMC_HIP(hipGetLastError());
}

int g_ncu = -1;
int ncu() {
    if (g_ncu < 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        VDMC_HIP(hipGetDevice(&dev));
        VDMC_HIP(hipGetDeviceProperties(&prop, dev));
        g_ncu = prop.multiProcessorCount;
    }
    return g_ncu;
}

unsigned grid_for(size_t lds, uint32_t nseg) {
    const int fit = std::max(1, std::min(8, (int)(163840 / (lds + kFiveStaticLds))));
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(nseg, (int64_t)ncu() * fit));
}

// cached descriptor arrays of batched 5-vertex launches, by (graphs, outputs)
struct FivePlan {
    std::vector<vdmc_graph_s*> graphs;
    std::vector<uint64_t*> outs;
    FiveGraph* d_graphs = nullptr;
    unsigned* d_cursor = nullptr;
    uint32_t nseg = 0, seg_items = 0;
    bool owned = true;
    size_t lds = 0;
    ~FivePlan() {
        (void)hipFree(d_graphs);
        (void)hipFree(d_cursor);
    }
};
std::mutex g_five_mu;
std::vector<FivePlan*> g_five_plans;

FiveGraph view_of(const vdmc_graph_s* g, uint64_t* out) {
    return FiveGraph{g->off, g->adj, g->perm, (unsigned long long*)out, g->stats, (uint32_t)g->n,
                     (uint32_t)(2 * g->pairs), (uint32_t)g->pairs, 0u};
}

}  // namespace

size_t five_lds_bytes(int64_t n, int64_t entries) {
    const int64_t W = (n + 15) / 16;
    return (size_t)(4 * ((n + 1) + n + (n + 1) + n + entries + n * W));
}

bool five_eligible(int64_t n, int64_t entries) {
    return n <= kFiveMaxN && five_lds_bytes(n, entries) <= kFiveLdsBudget;
}

void launch_count5(vdmc_graph_s* g, uint64_t* out, hipStream_t st) {
    VDMC_REQUIRE(five_eligible(g->n, 2 * g->pairs), VDMC_ERR_UNSUPPORTED,
                 "5-vertex counts take graphs held whole in LDS: n <= " + std::to_string(kFiveMaxN) +
                     " and the CSR plus a 2-bit arc matrix within " + std::to_string(kFiveLdsBudget) + " bytes");
    const ClassTable5& t = class_table5();
    launch_fill_u64((uint64_t*)g->stats, kStatSlots, 0, st);
    if (g->n == 0) return;
    launch_fill_u64(out, (size_t)g->n * kClasses5, 0, st);
    g->timed_light = g->timed_hub = false;
    if (g->pairs == 0) return;
    if (!g->five_cursor) VDMC_HIP(hipMalloc(&g->five_cursor, 64));
    launch_fill_u64((uint64_t*)g->five_cursor, 1, 0, st);
    FiveArgs a{};
    a.graphs = nullptr;
    a.one = view_of(g, out);
    a.num = 1;
    // segments small enough that every workgroup of the grid gets some
    const uint32_t items = (uint32_t)g->pairs;
    a.seg_items = std::max<uint32_t>(16u, std::min<uint32_t>(1024u, (items + 4 * ncu() - 1) / (4 * ncu())));
    a.nseg = (items + a.seg_items - 1) / a.seg_items;
    a.cursor = g->five_cursor;
    a.table = t.table;
    a.zero_out = 0;
    const size_t lds = five_lds_bytes(g->n, 2 * g->pairs);
    launch_five(a, false, grid_for(lds, a.nseg), lds, st);
}

void count5_batch(const vdmc_graph_s* const* gs_in, int32_t num, uint64_t* const* outs, hipStream_t st) {
    std::vector<vdmc_graph_s*> gs(num);
    for (int i = 0; i < num; i++) {
        gs[i] = const_cast<vdmc_graph_s*>(gs_in[i]);
        VDMC_REQUIRE(five_eligible(gs[i]->n, 2 * gs[i]->pairs), VDMC_ERR_UNSUPPORTED,
                     "graph " + std::to_string(i) + ": 5-vertex counts take graphs held whole in LDS (n <= " +
                         std::to_string(kFiveMaxN) + ")");
    }
    const ClassTable5& t = class_table5();
    std::lock_guard<std::mutex> lock(g_five_mu);
    FivePlan* plan = nullptr;
    for (FivePlan* p : g_five_plans)
        if (p->graphs == gs && std::equal(p->outs.begin(), p->outs.end(), outs)) {
            plan = p;
            break;
        }
    if (!plan) {
        plan = new FivePlan();
        try {
            plan->graphs = gs;
            plan->outs.assign(outs, outs + num);
            // owned mode when there are enough graphs to give every compute unit some;
            // graphs in order of decreasing estimated work (pairs x largest degree^3)
            plan->owned = num >= ncu();
            std::vector<int> order(num);
            for (int i = 0; i < num; i++) order[i] = i;
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                const double da = (double)gs[a]->max_deg, db = (double)gs[b]->max_deg;
                return (double)gs[a]->pairs * da * da * da > (double)gs[b]->pairs * db * db * db;
            });
            uint32_t max_items = 1, total = 0;
            for (int i : order) max_items = std::max<uint32_t>(max_items, (uint32_t)gs[i]->pairs);
            plan->seg_items = plan->owned ? max_items : 256u;
            std::vector<FiveGraph> views;
            for (int i : order) {
                FiveGraph v = view_of(gs[i], outs[i]);
                v.seg_base = total;
                total += plan->owned ? 1u : std::max<uint32_t>(1u, (v.items + plan->seg_items - 1) / plan->seg_items);
                views.push_back(v);
                plan->lds = std::max(plan->lds, five_lds_bytes(gs[i]->n, 2 * gs[i]->pairs));
            }
            plan->nseg = total;
            VDMC_HIP(hipMalloc(&plan->d_graphs, sizeof(FiveGraph) * std::max<size_t>(1, views.size())));
            VDMC_HIP(hipMalloc(&plan->d_cursor, 64));
            if (!views.empty())
                VDMC_HIP(hipMemcpy(plan->d_graphs, views.data(), sizeof(FiveGraph) * views.size(),
                                   hipMemcpyHostToDevice));
        } catch (...) {
            delete plan;
            throw;
        }
        g_five_plans.push_back(plan);
        if (g_five_plans.size() > 16) {
            delete g_five_plans.front();
            g_five_plans.erase(g_five_plans.begin());
        }
    }
    GraphUse use(plan->graphs, st);   // ordered after earlier work on these graphs
    for (int i = 0; i < num; i++) {
        gs[i]->timed_light = gs[i]->timed_hub = false;
        if (!plan->owned) {   // owned mode zeroes counters and outputs inside the launch
            launch_fill_u64((uint64_t*)gs[i]->stats, kStatSlots, 0, st);
            if (gs[i]->n > 0) launch_fill_u64(outs[i], (size_t)gs[i]->n * kClasses5, 0, st);
        }
    }
    launch_fill_u64((uint64_t*)plan->d_cursor, 1, 0, st);
    FiveArgs a{};
    a.graphs = plan->d_graphs;
    a.num = (uint32_t)num;
    a.nseg = plan->nseg;
    a.seg_items = plan->seg_items;
    a.cursor = plan->d_cursor;
    a.table = t.table;
    a.zero_out = plan->owned ? 1u : 0u;
    launch_five(a, plan->owned, grid_for(plan->lds, plan->nseg), plan->lds, st);
}

void invalidate_five_plans(vdmc_graph_s* g) {
    std::lock_guard<std::mutex> lock(g_five_mu);
    for (auto it = g_five_plans.begin(); it != g_five_plans.end();) {
        if (std::find((*it)->graphs.begin(), (*it)->graphs.end(), g) != (*it)->graphs.end()) {
            delete *it;
            it = g_five_plans.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace vdmc

// Per-vertex 3- and 4-motif counting kernels.
//
// Method (paper Sec. 4-5):
//   * roots are taken in rank order; a k-set is enumerated only from its lowest-rank
//     vertex r (proper k-BFS, Lemma 1), so roots are independent;
//   * inside one root the k-set is reached along exactly one BFS shape (Lemma 2):
//       k = 3: (1,1)  both others adjacent to r;
//              (1,2)  a adjacent to r, c adjacent to a but not to r;
//       k = 4: (3,0,0) a < b < c all adjacent to r;
//              (2,1,0) a, b adjacent to r, c adjacent to a (and maybe b) but not to r;
//                      when c touches both, it hangs under the lower-rank one;
//              (1,2,0) a adjacent to r, c < c' adjacent to a, neither adjacent to r;
//              (1,1,1) the path r - a - b - c, b and c not adjacent to r, c not
//                      adjacent to a;
//     members of one level are taken in increasing rank and depths are measured
//     inside the k-set, which is the duplicate rule of Lemma 3 with the fix of
//     Lemma 4 for the depth-1.5 shape (the last vertex is tested against the depth-1
//     vertex of the current set, not against global BFS depth);
//   * the vertices are ordered by (depth, rank) (Sec. 4.2), the motif index is
//     assembled from the CSR arc bits, mapped to its class through the table, and
//     every member's counter of that class is raised (Sec. 4.2).
#include "motif_device.h"
#include "vdmc_internal.h"

namespace vdmc {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kStage = 2048;   // entries of N+(r) staged in LDS (single-graph launch)

struct Args {
    const uint32_t* off;
    const uint32_t* adj;
    const uint32_t* split;
    const int32_t* perm;
    const uint32_t* roots;
    int64_t nroots;
    const uint8_t* t3;
    const uint8_t* t4;
    unsigned long long* out3;   // n x 13, original ids
    unsigned long long* out4;   // n x 199
    unsigned long long* stats;  // kShapes
    uint32_t rank_lo, rank_hi;  // only roots with rank in [rank_lo, rank_hi)
    const unsigned long long* ehash;   // edge hash or nullptr
    uint32_t ehash_bits;
};

// arc bits of (u, v) seen from u: one probe sequence in the edge hash when the graph has
// one, else a binary search of the shorter row
__device__ __forceinline__ uint32_t gv_arc(const GraphView& gv, uint32_t u, uint32_t v) {
    return gv.ehash ? edge_code(gv.ehash, gv.ehash_bits, u, v) : arc_bits(gv.off, gv.adj, u, v);
}

// rank x a member of the sorted list P[0..d) ?
__device__ __forceinline__ bool in_list(const uint32_t* P, uint32_t d, uint32_t x) {
    uint32_t lo = 0, hi = d, key = x << 2;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (P[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo < d && (P[lo] >> 2) == x;
}

// One count of class cls to vertex v.  When every lane that gets here credits the same
// (vertex, class) -- lanes that share a member of their sets, e.g. the centre of a star
// -- one lane adds them all.
__device__ __forceinline__ void credit(unsigned long long* out, const int32_t* perm, int C, uint32_t v,
                                       uint32_t cls) {
    if (cls >= (uint32_t)C) return;   // 0xFF never credited
    const uint32_t fv = __builtin_amdgcn_readfirstlane(v), fc = __builtin_amdgcn_readfirstlane(cls);
    const unsigned long long act = __ballot(1);
    const unsigned long long same = __ballot(v == fv && cls == fc);
    if (same == act) {
        if ((threadIdx.x & 63u) == (uint32_t)(__ffsll((long long)act) - 1))
            atomicAdd(&out[(size_t)perm[v] * C + cls], (unsigned long long)__popcll(act));
    } else {
        atomicAdd(&out[(size_t)perm[v] * C + cls], 1ull);
    }
}

// Where the per-set increments go.  GlobalSink: one 64-bit atomic per credited vertex
// into the caller's output (the root's credits are summed in LDS first).  Small graphs
// take the whole-graph kernel of small.hip instead, whose counters live in LDS.
struct GlobalSink {
    __device__ __forceinline__ void c3(const GraphView& gv, uint32_t v, uint32_t cls) const {
        credit(gv.out3, gv.perm, kClasses3, v, cls);
    }
    __device__ __forceinline__ void c4(const GraphView& gv, uint32_t v, uint32_t cls) const {
        credit(gv.out4, gv.perm, kClasses4, v, cls);
    }
    __device__ __forceinline__ void root3(const GraphView& gv, uint32_t r, uint32_t cls, unsigned long long c) const {
        atomicAdd(&gv.out3[(size_t)gv.perm[r] * kClasses3 + cls], c);
    }
    __device__ __forceinline__ void root4(const GraphView& gv, uint32_t r, uint32_t cls, unsigned long long c) const {
        atomicAdd(&gv.out4[(size_t)gv.perm[r] * kClasses4 + cls], c);
    }
    __device__ __forceinline__ void set3(uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t) const {}
    __device__ __forceinline__ void set4(uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t,
                                         uint32_t, uint32_t, uint32_t) const {}
};

// Per-edge counts (Sec. 11: credit the edges of each set instead of its vertices): every
// vertex pair of a set that is joined in G_U gets one count of the set's class, in the
// row the edge index gives it.  Vertex credits are dropped.
struct EdgeSink {
    const unsigned long long* table;   // the graph's edge hash
    uint32_t bits;
    const uint32_t* epid;              // slot -> output row of the pair
    unsigned long long* out;           // pairs x C
    uint32_t C;
    __device__ __forceinline__ void c3(const GraphView&, uint32_t, uint32_t) const {}
    __device__ __forceinline__ void c4(const GraphView&, uint32_t, uint32_t) const {}
    __device__ __forceinline__ void root3(const GraphView&, uint32_t, uint32_t, unsigned long long) const {}
    __device__ __forceinline__ void root4(const GraphView&, uint32_t, uint32_t, unsigned long long) const {}
    __device__ __forceinline__ void pair(uint32_t u, uint32_t v, uint32_t cls) const {
        const uint32_t h = edge_find(table, bits, u, v);
        if (h != 0xFFFFFFFFu) atomicAdd(&out[(size_t)epid[h] * C + cls], 1ull);
    }
    // vertices v0..v2 / v0..v3 (v0 = the root) and the arc bits of their pairs
    __device__ __forceinline__ void set3(uint32_t cls, uint32_t v0, uint32_t v1, uint32_t v2, uint32_t c01,
                                         uint32_t c02, uint32_t c12) const {
        if (cls >= C) return;
        if (c01) pair(v0, v1, cls);
        if (c02) pair(v0, v2, cls);
        if (c12) pair(v1, v2, cls);
    }
    __device__ __forceinline__ void set4(uint32_t cls, uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3,
                                         uint32_t c01, uint32_t c02, uint32_t c03, uint32_t c12,
                                         uint32_t c13c23) const {
        if (cls >= C) return;
        if (c01) pair(v0, v1, cls);
        if (c02) pair(v0, v2, cls);
        if (c03) pair(v0, v3, cls);
        if (c12) pair(v1, v2, cls);
        if (c13c23 & 3u) pair(v1, v3, cls);
        if (c13c23 >> 2) pair(v2, v3, cls);
    }
};

template <uint32_t STAGE>
struct RootLds {
    uint32_t P[STAGE];
    uint32_t lo[STAGE + 1];     // first entry of row P[i] above r
    uint32_t pre[STAGE + 1];    // prefix sums of the depth-2 scan lengths
    unsigned long long root3[kClasses3];
    unsigned long long root4[kClasses4];
};

// All k-sets whose lowest-rank vertex is r, by one workgroup of BS threads, every set
// credited to its non-root members with one atomic each (the root is summed in LDS).
template <int BS, uint32_t STAGE, bool K3, bool K4, class Sink>
__device__ void process_root(const GraphView& gv, const uint8_t* t3, const uint8_t* t4, uint32_t r,
                             RootLds<STAGE>& S, unsigned long long* shape, const Sink& sink) {
    const uint32_t tid = threadIdx.x;
    const uint32_t s = gv.split[r];
    const uint32_t d = gv.off[r + 1] - s;
    const bool staged = d <= STAGE;
    __syncthreads();
    if (staged)
        for (uint32_t i = tid; i < d; i += BS) S.P[i] = gv.adj[s + i];
    if (K3)
        for (uint32_t i = tid; i < kClasses3; i += BS) S.root3[i] = 0;
    if (K4)
        for (uint32_t i = tid; i < kClasses4; i += BS) S.root4[i] = 0;
    __syncthreads();
    const uint32_t* P = staged ? S.P : gv.adj + s;

    // ---- depth-1 shapes: pairs (i < j) of N+(r); k=4 extends each by l > j
    const uint64_t npairs = (uint64_t)d * (d - 1) / 2;
    for (uint64_t q = tid; q < npairs; q += BS) {
        uint32_t j = (uint32_t)((1.0 + sqrt(1.0 + 8.0 * (double)q)) * 0.5);
        while ((uint64_t)j * (j - 1) / 2 > q) j--;
        while ((uint64_t)(j + 1) * j / 2 <= q) j++;
        const uint32_t i = (uint32_t)(q - (uint64_t)j * (j - 1) / 2);
        const uint32_t ea = P[i], eb = P[j];
        const uint32_t va = ea >> 2, vb = eb >> 2, ra = ea & 3u, rb = eb & 3u;
        const uint32_t ab = gv_arc(gv, va, vb);
        if (K3) {
            const uint32_t cls = t3[motif_index3(ra, rb, ab)];
            sink.set3(cls, r, va, vb, ra, rb, ab);
            if (cls < kClasses3) atomicAdd(&S.root3[cls], 1ull);
            sink.c3(gv, va, cls);
            sink.c3(gv, vb, cls);
            shape[0]++;
        }
        if (K4) {
            for (uint32_t l = j + 1; l < d; l++) {
                const uint32_t ec = P[l];
                const uint32_t vc = ec >> 2, rc = ec & 3u;
                const uint32_t ac = gv_arc(gv, va, vc);
                const uint32_t bc = gv_arc(gv, vb, vc);
                const uint32_t cls = t4[motif_index4(ra, rb, rc, ab, ac, bc)];
                sink.set4(cls, r, va, vb, vc, ra, rb, rc, ab, ac | (bc << 2));
                if (cls < kClasses4) atomicAdd(&S.root4[cls], 1ull);
                sink.c4(gv, va, cls);
                sink.c4(gv, vb, cls);
                sink.c4(gv, vc, cls);
                shape[2]++;
            }
        }
    }

    // ---- depth-2 candidates: entries (a, c) of rows of N+(r) with c > r, c not in N(r)
    for (uint32_t c0 = 0; c0 < d; c0 += STAGE) {
        const uint32_t cn = min(STAGE, d - c0);
        __syncthreads();
        for (uint32_t i = tid; i < cn; i += BS) {
            const uint32_t va = P[c0 + i] >> 2;
            S.lo[i] = lower_bound_rank(gv.adj, gv.off[va], gv.off[va + 1], r + 1);
            S.pre[i + 1] = gv.off[va + 1] - S.lo[i];
        }
        __syncthreads();
        if (tid == 0) {   // short serial scan: light roots have few depth-1 vertices
            S.pre[0] = 0;
            for (uint32_t i = 1; i <= cn; i++) S.pre[i] += S.pre[i - 1];
        }
        __syncthreads();
        const uint32_t total = S.pre[cn];
        for (uint32_t q = tid; q < total; q += BS) {
            uint32_t lo = 0, hi = cn;   // slot with pre[i] <= q < pre[i+1]
            while (hi - lo > 1) {
                uint32_t mid = (lo + hi) >> 1;
                if (S.pre[mid] <= q) lo = mid; else hi = mid;
            }
            const uint32_t i = c0 + lo;
            const uint32_t ea = P[i];
            const uint32_t va = ea >> 2, ra = ea & 3u;
            const uint32_t t = S.lo[lo] + (q - S.pre[lo]);
            const uint32_t ecn = gv.adj[t];
            const uint32_t vc = ecn >> 2, ac = ecn & 3u;
            if (in_list(P, d, vc)) continue;   // c adjacent to r: depth 1, not 2
            if (K3) {
                const uint32_t cls = t3[motif_index3(ra, 0u, ac)];
                sink.set3(cls, r, va, vc, ra, 0u, ac);
                if (cls < kClasses3) atomicAdd(&S.root3[cls], 1ull);
                sink.c3(gv, va, cls);
                sink.c3(gv, vc, cls);
                shape[1]++;
            }
            if (K4) {
                // (2,1,0): second depth-1 vertex b
                for (uint32_t j = 0; j < d; j++) {
                    if (j == i) continue;
                    const uint32_t eb = P[j];
                    const uint32_t vb = eb >> 2, rb = eb & 3u;
                    const uint32_t bc = gv_arc(gv, vb, vc);
                    if (bc && j < i) continue;   // c hangs under the lower-rank parent b
                    const uint32_t ab = gv_arc(gv, va, vb);
                    const uint32_t cls = t4[motif_index4(ra, rb, 0u, ab, ac, bc)];
                    sink.set4(cls, r, va, vb, vc, ra, rb, 0u, ab, ac | (bc << 2));
                    if (cls < kClasses4) atomicAdd(&S.root4[cls], 1ull);
                    sink.c4(gv, va, cls);
                    sink.c4(gv, vb, cls);
                    sink.c4(gv, vc, cls);
                    shape[3]++;
                }
                // (1,2,0): a second depth-2 child c' > c of a
                const uint32_t ha = gv.off[va + 1];
                for (uint32_t t2 = t + 1; t2 < ha; t2++) {
                    const uint32_t e2 = gv.adj[t2];
                    const uint32_t vc2 = e2 >> 2;
                    if (in_list(P, d, vc2)) continue;
                    const uint32_t cc2 = gv_arc(gv, vc, vc2);
                    const uint32_t cls = t4[motif_index4(ra, 0u, 0u, ac, e2 & 3u, cc2)];
                    sink.set4(cls, r, va, vc, vc2, ra, 0u, 0u, ac, (e2 & 3u) | (cc2 << 2));
                    if (cls < kClasses4) atomicAdd(&S.root4[cls], 1ull);
                    sink.c4(gv, va, cls);
                    sink.c4(gv, vc, cls);
                    sink.c4(gv, vc2, cls);
                    shape[4]++;
                }
                // (1,1,1): path r - a - c - e, e not adjacent to r nor to a
                const uint32_t hc = gv.off[vc + 1];
                for (uint32_t t3i = lower_bound_rank(gv.adj, gv.off[vc], hc, r + 1); t3i < hc; t3i++) {
                    const uint32_t e3 = gv.adj[t3i];
                    const uint32_t ve = e3 >> 2;
                    if (in_list(P, d, ve)) continue;                // also excludes a itself
                    if (gv_arc(gv, va, ve)) continue; // e adjacent to a: depth 2
                    const uint32_t cls = t4[motif_index4(ra, 0u, 0u, ac, 0u, e3 & 3u)];
                    sink.set4(cls, r, va, vc, ve, ra, 0u, 0u, ac, (e3 & 3u) << 2);
                    if (cls < kClasses4) atomicAdd(&S.root4[cls], 1ull);
                    sink.c4(gv, va, cls);
                    sink.c4(gv, vc, cls);
                    sink.c4(gv, ve, cls);
                    shape[5]++;
                }
            }
        }
    }
    __syncthreads();
    if (K3)
        for (uint32_t i = tid; i < kClasses3; i += BS)
            if (S.root3[i]) sink.root3(gv, r, i, S.root3[i]);
    if (K4)
        for (uint32_t i = tid; i < kClasses4; i += BS)
            if (S.root4[i]) sink.root4(gv, r, i, S.root4[i]);
}

// BS threads per root; roots with more than STAGE higher neighbours read them from
// global memory.  The one-wave variant (BS = STAGE = 64) takes the light roots when the
// hub threshold is at most 64: no workgroup barrier spans more than one wave.
template <int BS, uint32_t STAGE, bool K3, bool K4>
__global__ __launch_bounds__(BS) void k_count_roots(Args a) {
    __shared__ RootLds<STAGE> S;
    unsigned long long shape[kShapes] = {0, 0, 0, 0, 0, 0};
    GraphView gv{a.off, a.adj, a.split, a.perm, a.out3, a.out4, a.stats, a.ehash, a.ehash_bits};
    for (int64_t ri = blockIdx.x; ri < a.nroots; ri += gridDim.x) {
        const uint32_t r = a.roots[ri];
        if (r < a.rank_lo || r >= a.rank_hi) continue;   // uniform across the workgroup
        process_root<BS, STAGE, K3, K4>(gv, a.t3, a.t4, r, S, shape, GlobalSink());
    }
    for (int s = 0; s < kShapes; s++)
        if (shape[s]) atomicAdd(&a.stats[s], shape[s]);
}

// Per-edge counts: every root with a non-empty higher neighbourhood, edges credited
template <bool K3, bool K4>
__global__ __launch_bounds__(kThreads) void k_count_edges(Args a, EdgeSink es) {
    __shared__ RootLds<kStage> S;
    unsigned long long shape[kShapes] = {0, 0, 0, 0, 0, 0};
    GraphView gv{a.off, a.adj, a.split, a.perm, nullptr, nullptr, a.stats, a.ehash, a.ehash_bits};
    for (int64_t ri = blockIdx.x; ri < a.nroots; ri += gridDim.x)
        process_root<kThreads, kStage, K3, K4>(gv, a.t3, a.t4, a.roots[ri], S, shape, es);
    for (int s = 0; s < kShapes; s++)
        if (shape[s]) atomicAdd(&a.stats[s], shape[s]);
}

// Batched launch: a root table of (graph, root) pairs over many graphs, consumed in
// tiles from a device-side cursor by a persistent grid.
template <int BS, uint32_t STAGE, bool K3, bool K4>
__global__ __launch_bounds__(BS) void k_count_batch(BatchArgs b) {
    __shared__ RootLds<STAGE> S;
    __shared__ unsigned long long tile_start;
    unsigned long long shape[kShapes] = {0, 0, 0, 0, 0, 0};
    int cur_graph = -1;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) tile_start = atomicAdd(b.cursor, (unsigned long long)b.tile);
        __syncthreads();
        const unsigned long long t0 = tile_start;
        if (t0 >= b.nentries) break;
        const unsigned long long t1 = min(t0 + b.tile, b.nentries);
        for (unsigned long long e = t0; e < t1; e++) {
            const uint2 ent = b.table[e];   // x = graph index, y = root rank
            if ((int)ent.x != cur_graph) {
                if (cur_graph >= 0)
                    for (int s = 0; s < kShapes; s++)
                        if (shape[s]) { atomicAdd(&b.graphs[cur_graph].stats[s], shape[s]); shape[s] = 0; }
                cur_graph = (int)ent.x;
            }
            process_root<BS, STAGE, K3, K4>(b.graphs[ent.x], b.t3, b.t4, ent.y, S, shape, GlobalSink());
        }
    }
    if (cur_graph >= 0)
        for (int s = 0; s < kShapes; s++)
            if (shape[s]) atomicAdd(&b.graphs[cur_graph].stats[s], shape[s]);
}

// zero every graph's shape counters and the outputs of the graphs counted by the root
// table (the whole-graph kernel clears its own graphs' outputs); one workgroup per graph
__global__ void k_batch_zero(BatchArgs b, int k3, int k4) {
    const GraphView& g = b.graphs[blockIdx.x];
    const size_t n = b.generic[blockIdx.x] ? b.nvert[blockIdx.x] : 0;
    if (k3)
        for (size_t i = threadIdx.x; i < n * kClasses3; i += blockDim.x) g.out3[i] = 0;
    if (k4)
        for (size_t i = threadIdx.x; i < n * kClasses4; i += blockDim.x) g.out4[i] = 0;
    for (int i = threadIdx.x; i < kStatSlots; i += blockDim.x) g.stats[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *b.cursor = 0;
        *b.gcursor = 0;
    }
}

__global__ void k_fill(unsigned long long* p, size_t n, unsigned long long v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

void launch_batch(const BatchArgs& b, const SmallArgs* small, unsigned small_grid, size_t small_lds,
                  int small_variant, int variant, int k3, int k4, int num_graphs, int wgs_per_cu, hipStream_t st) {
    static int ncu = -1;
    if (ncu < 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        VDMC_HIP(hipGetDevice(&dev));
        VDMC_HIP(hipGetDeviceProperties(&prop, dev));
        ncu = prop.multiProcessorCount;
    }
    hipLaunchKernelGGL(k_batch_zero, dim3(num_graphs), dim3(256), 0, st, b, k3, k4);
    VDMC_HIP(hipGetLastError());
    const unsigned grid = (unsigned)(ncu * wgs_per_cu);
    if (small && small->num > 0) {
        VDMC_REQUIRE(k3 != k4, VDMC_ERR_INVALID_ARG, "a batch counts one k");
        launch_small(*small, k3 ? 3 : 4, small_variant, small_grid, small_lds, st);
    }
    if (b.nentries == 0) return;
#define VDMC_BATCH_LAUNCH(BS, STG)                                                                           \
    do {                                                                                                    \
        if (k3 && k4) hipLaunchKernelGGL((k_count_batch<BS, STG, true, true>), dim3(grid), dim3(BS), 0, st, b); \
        else if (k3) hipLaunchKernelGGL((k_count_batch<BS, STG, true, false>), dim3(grid), dim3(BS), 0, st, b); \
        else hipLaunchKernelGGL((k_count_batch<BS, STG, false, true>), dim3(grid), dim3(BS), 0, st, b);         \
    } while (0)
    switch (variant) {
        case 0: VDMC_BATCH_LAUNCH(64, 256); break;
        case 1: VDMC_BATCH_LAUNCH(128, 256); break;
        default: VDMC_BATCH_LAUNCH(256, 512); break;
    }
#undef VDMC_BATCH_LAUNCH
    VDMC_HIP(hipGetLastError());
}

void launch_fill_u64(uint64_t* p, size_t n, uint64_t value, hipStream_t st) {
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, (unsigned long long*)p, n,
                       (unsigned long long)value);
    VDMC_HIP(hipGetLastError());
}

void launch_count(vdmc_graph_s* g, int k3, int k4, uint64_t* out3, uint64_t* out4, hipStream_t st,
                  int64_t rank_lo, int64_t rank_hi, bool zero) {
    const ClassTables& t = class_tables();
    ensure_bins(g, st);   // the caller holds g->mu (GraphUse)
    if (zero) {
        if (k3) launch_fill_u64(out3, (size_t)g->n * kClasses3, 0, st);
        if (k4) launch_fill_u64(out4, (size_t)g->n * kClasses4, 0, st);
        launch_fill_u64((uint64_t*)g->stats, kStatSlots, 0, st);
    }
    const uint32_t lo = (uint32_t)std::max<int64_t>(0, rank_lo);
    const uint32_t hi = (uint32_t)std::min<int64_t>(g->n, rank_hi);
    g->timed_light = g->timed_hub = false;
    if (lo >= hi) return;
    if (!g->ev[0])
        for (auto& e : g->ev) VDMC_HIP(hipEventCreate(&e));
    if (g->nlight > 0) {
        VDMC_HIP(hipEventRecord(g->ev[0], st));
        Args a;
        a.off = g->off;
        a.adj = g->adj;
        a.split = g->split;
        a.perm = g->perm;
        a.roots = g->light;
        a.nroots = g->nlight;
        a.t3 = t.t3;
        a.t4 = t.t4;
        a.out3 = (unsigned long long*)out3;
        a.out4 = (unsigned long long*)out4;
        a.stats = g->stats;
        a.rank_lo = lo;
        a.rank_hi = hi;
        a.ehash = g->ehash;
        a.ehash_bits = g->ehash_bits;
        const int64_t blocks = g->nlight < 65536 ? g->nlight : 65536;
        const dim3 grid((unsigned)blocks);
        if (g->light_max_d <= 64) {   // every light root has at most 64 higher neighbours
            if (k3 && k4) hipLaunchKernelGGL((k_count_roots<64, 64, true, true>), grid, dim3(64), 0, st, a);
            else if (k3) hipLaunchKernelGGL((k_count_roots<64, 64, true, false>), grid, dim3(64), 0, st, a);
            else hipLaunchKernelGGL((k_count_roots<64, 64, false, true>), grid, dim3(64), 0, st, a);
        } else {
            if (k3 && k4) hipLaunchKernelGGL((k_count_roots<kThreads, kStage, true, true>), grid, dim3(kThreads), 0, st, a);
            else if (k3) hipLaunchKernelGGL((k_count_roots<kThreads, kStage, true, false>), grid, dim3(kThreads), 0, st, a);
            else hipLaunchKernelGGL((k_count_roots<kThreads, kStage, false, true>), grid, dim3(kThreads), 0, st, a);
        }
        VDMC_HIP(hipGetLastError());
        VDMC_HIP(hipEventRecord(g->ev[1], st));
        g->timed_light = true;
    }
    launch_hub(g, k3, k4, out3, out4, st, lo, hi, g->ev + 2);
    g->timed_hub = g->nhub > 0;
}

void launch_count_edges(vdmc_graph_s* g, int k, uint64_t* out, hipStream_t st) {
    const ClassTables& t = class_tables();
    ensure_edge_index(g, st);
    const int C = num_classes(k);
    launch_fill_u64((uint64_t*)g->stats, kStatSlots, 0, st);
    if (g->pairs == 0) return;
    launch_fill_u64(out, (size_t)g->pairs * C, 0, st);
    if (g->nroots == 0) return;
    Args a;
    a.off = g->off;
    a.adj = g->adj;
    a.split = g->split;
    a.perm = g->perm;
    a.roots = g->roots;
    a.nroots = g->nroots;
    a.t3 = t.t3;
    a.t4 = t.t4;
    a.out3 = a.out4 = nullptr;
    a.stats = g->stats;
    a.rank_lo = 0;
    a.rank_hi = 0xFFFFFFFFu;
    a.ehash = g->ehash;
    a.ehash_bits = g->ehash_bits;
    const EdgeSink es{g->ehash, g->ehash_bits, g->epid, (unsigned long long*)out, (uint32_t)C};
    const unsigned blocks = (unsigned)std::min<int64_t>(g->nroots, 65536);
    if (k == 3) hipLaunchKernelGGL((k_count_edges<true, false>), dim3(blocks), dim3(kThreads), 0, st, a, es);
    else hipLaunchKernelGGL((k_count_edges<false, true>), dim3(blocks), dim3(kThreads), 0, st, a, es);
    VDMC_HIP(hipGetLastError());
    g->timed_light = g->timed_hub = false;
}

}  // namespace vdmc

extern "C" {

vdmc_status vdmc_count(vdmc_graph g, int32_t k, uint64_t* out, void* stream) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_REQUIRE(k >= 3 && k <= 5, VDMC_ERR_INVALID_ARG, "k must be 3, 4 or 5");
        VDMC_REQUIRE(out != nullptr || g->n == 0, VDMC_ERR_INVALID_ARG, "out is NULL");
        VDMC_HIP(hipSetDevice(g->device));
        if (k == 5) {
            VDMC_REQUIRE(g->n < ((int64_t)1 << 31) / vdmc::kClasses5, VDMC_ERR_UNSUPPORTED,
                         "5-vertex counts: n x 9364 must stay below 2^31 counters per row index");
            (void)vdmc::class_table5();
            vdmc::GraphUse use(g, vdmc::as_stream(stream));
            vdmc::launch_count5(g, out, vdmc::as_stream(stream));
            return;
        }
        vdmc::GraphUse use(g, vdmc::as_stream(stream));
        vdmc::launch_count(g, k == 3, k == 4, k == 3 ? out : nullptr, k == 4 ? out : nullptr,
                           vdmc::as_stream(stream));
    });
}

int32_t vdmc_count_supported(vdmc_graph g, int32_t k) {
    if (g == nullptr || k < 3 || k > 5) return -1;
    if (k == 5) return g->n < ((int64_t)1 << 31) / vdmc::kClasses5 ? 1 : 0;
    return 1;
}

vdmc_status vdmc_set_hub_threshold(vdmc_graph g, int32_t min_higher) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_REQUIRE(min_higher >= 1 && min_higher <= (1 << 30), VDMC_ERR_INVALID_ARG,
                     "min_higher must be in [1, 2^30]");
        {
            std::lock_guard<std::mutex> lock(g->mu);
            g->hub_min = min_higher;
        }
        vdmc::invalidate_batch_plans(g);
    });
}

vdmc_status vdmc_count34(vdmc_graph g, uint64_t* out3, uint64_t* out4, void* stream) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_REQUIRE((out3 && out4) || g->n == 0, VDMC_ERR_INVALID_ARG, "out3/out4 is NULL");
        VDMC_REQUIRE(out3 != out4 || g->n == 0, VDMC_ERR_INVALID_ARG, "out3 and out4 alias");
        VDMC_HIP(hipSetDevice(g->device));
        vdmc::GraphUse use(g, vdmc::as_stream(stream));
        vdmc::launch_count(g, 1, 1, out3, out4, vdmc::as_stream(stream));
    });
}

vdmc_status vdmc_profile_counters(vdmc_graph g, uint64_t* counters, int32_t n) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr && counters != nullptr && n >= 0, VDMC_ERR_INVALID_ARG, "bad argument");
        VDMC_HIP(hipSetDevice(g->device));
        std::lock_guard<std::mutex> lock(g->mu);
        vdmc::wait_graph(g);
        const int k = n < vdmc::kStatSlots ? n : vdmc::kStatSlots;
        VDMC_HIP(hipMemcpy(counters, g->stats, k * sizeof(uint64_t), hipMemcpyDeviceToHost));
    });
}

vdmc_status vdmc_kernel_times(vdmc_graph g, float* ms_out, int32_t n) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr && ms_out != nullptr && n >= 0, VDMC_ERR_INVALID_ARG, "bad argument");
        VDMC_HIP(hipSetDevice(g->device));
        std::lock_guard<std::mutex> lock(g->mu);
        float t[3] = {-1.0f, -1.0f, -1.0f};
        if (g->timed_light) {
            VDMC_HIP(hipEventSynchronize(g->ev[1]));
            VDMC_HIP(hipEventElapsedTime(&t[0], g->ev[0], g->ev[1]));
        }
        if (g->timed_hub) {
            VDMC_HIP(hipEventSynchronize(g->ev[3]));
            VDMC_HIP(hipEventElapsedTime(&t[1], g->ev[2], g->ev[3]));
            VDMC_HIP(hipEventElapsedTime(&t[2], g->ev[2], g->ev[4]));
        }
        for (int i = 0; i < n && i < 3; i++) ms_out[i] = t[i];
    });
}

vdmc_status vdmc_count_range(vdmc_graph g, int32_t k, uint64_t* out, int64_t rank_begin, int64_t rank_end,
                             uint32_t flags, void* stream) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG,
                     "k must be 3 or 4");
        VDMC_REQUIRE(out != nullptr || g->n == 0, VDMC_ERR_INVALID_ARG, "out is NULL");
        VDMC_REQUIRE(rank_begin >= 0 && rank_begin <= rank_end, VDMC_ERR_INVALID_ARG, "bad rank range");
        VDMC_REQUIRE((flags & ~(uint32_t)VDMC_ACCUMULATE) == 0, VDMC_ERR_INVALID_ARG, "unknown flags");
        VDMC_HIP(hipSetDevice(g->device));
        vdmc::GraphUse use(g, vdmc::as_stream(stream));
        vdmc::launch_count(g, k == 3, k == 4, k == 3 ? out : nullptr, k == 4 ? out : nullptr,
                           vdmc::as_stream(stream), rank_begin, rank_end, !(flags & VDMC_ACCUMULATE));
    });
}

vdmc_status vdmc_shape_counts(vdmc_graph g, uint64_t* shape_counts) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr && shape_counts != nullptr, VDMC_ERR_INVALID_ARG, "NULL argument");
        VDMC_HIP(hipSetDevice(g->device));
        std::lock_guard<std::mutex> lock(g->mu);
        vdmc::wait_graph(g);
        VDMC_HIP(hipMemcpy(shape_counts, g->stats, vdmc::kShapes * sizeof(uint64_t), hipMemcpyDeviceToHost));
    });
}

}  // extern "C"

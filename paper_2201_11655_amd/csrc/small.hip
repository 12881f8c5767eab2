// Small-graph motif kernel: one workgroup counts a whole graph held in LDS.
//
// For graphs of a few hundred vertices (the batched workload, small served requests)
// a per-root launch leaves most of a workgroup idle: a root of such a graph has a
// handful of higher neighbours.  Here one workgroup takes a whole graph:
//   * its rank-space CSR (16-bit row entries), a 1-bit adjacency matrix (so that almost
//     every pair test is one LDS read; a set bit is resolved to its arc bits by a search
//     of the LDS row) and per-vertex counters live in LDS;
//   * the work of all roots is flattened into two item lists, so that threads never
//     wait at per-root barriers:
//       - pairs {a < b} of N+(r) for every root r: the k = 3 set (1,1) and the k = 4
//         sets (3,0,0) that add a third higher neighbour c > b (Lemma 2);
//       - depth-2 entries (r, a, c): a in N+(r), c in N(a), c > r, c not in N(r): the
//         k = 3 set (1,2) and, for k = 4, the sets (2,1,0) (second depth-1 vertex b; c
//         hangs under its lower-rank parent), (1,2,0) (a second child c' of a, each pair
//         of children once) and
//         (1,1,1) (an end vertex e of c's row, not adjacent to r or to a: the Lemma-4
//         rule) (Lemmas 2-4);
//   * every set is visited once by one lane: its index is assembled from the arc bits
//     (Sec. 4.1), its class read from the table in LDS, and each of its k vertices
//     credited (Sec. 4.2).  Credits go to LDS counters (k = 3: all 13 classes; k = 4:
//     the 25 tree classes and the 12 single-arc 4-pair classes, which hold ~99.6% of the
//     credits of sparse graphs), one LDS atomic per member and set; the other classes
//     go straight to the graph's output with workgroup-scope atomics (the output block
//     of a graph belongs to one workgroup for the whole launch; every such atomic is a
//     memory-side operation, so they are kept rare), and there members that all lanes of
//     a wave step share (the root, the depth-1 vertex of a run of depth-2 items, the
//     loop's current vertex) are credited once per class present in the step, grouped
//     by ballots;
//   * in the k = 4 loops three members are fixed and the lane walks the fourth; a set
//     whose fourth member has no arc to the fixed members other than the one the shape
//     implies has its class fixed by that arc's code (a tree class): the fourth member
//     is credited per set and the three fixed ones once per arc code after the loop.
// The LDS counters are stored to the output once per graph (their classes never reach
// the output otherwise).  u32 counters cannot overflow: a vertex of a graph with
// n <= kSmallMaxN lies in fewer than 2^32 k-sets.
#include "motif_device.h"
#include "vdmc_internal.h"

namespace vdmc {
namespace {

__device__ __forceinline__ uint32_t lane_of() { return threadIdx.x & 63u; }

// LDS counter slots per vertex for k = 4: the 25 tree classes, then the 12 classes whose
// four joined pairs are all single arcs (directed 4-cycles and tailed triangles without a
// reciprocal pair).  In a sparse digraph these are the next most frequent after the trees
// (each further arc or reciprocation costs another factor of p): together they hold ~99.6%
// of the credits of the batch workload, and only the rest goes to the output with
// memory-side atomics.
constexpr uint32_t kSingleArc4 = 12;
constexpr uint32_t kSlots4 = (uint32_t)kCompact4 + kSingleArc4;

// bit of the 4-vertex index for the entry (i, j), i != j: rows in order, the diagonal
// skipped, entry (0,1) the most significant of the 12 (Sec. 4.1)
__device__ __forceinline__ uint32_t bit4(uint32_t code, uint32_t i, uint32_t j) {
    return (code >> (11u - (3u * i + (j < i ? j : j - 1u)))) & 1u;
}

// wg-scope atomic add on a graph's output (the block is owned by this workgroup)
__device__ __forceinline__ void out_add(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// exclusive prefix sum of a[0..len) in place (LDS), returns the total; every thread of
// the workgroup must call it.  Each thread sums a contiguous chunk; the chunk sums are
// scanned within each wave by shuffles and across the BS / 64 waves by the first wave.
// part: BS / 64 words of LDS scratch.
template <int BS>
__device__ uint32_t block_exclusive_scan(uint32_t* a, uint32_t len, uint32_t* part) {
    constexpr uint32_t NWV = BS / 64;
    const uint32_t tid = threadIdx.x, lane = lane_of(), wave = tid >> 6;
    const uint32_t per = (len + BS - 1) / BS;
    const uint32_t lo = min(len, tid * per), hi = min(len, lo + per);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; i++) s += a[i];
    uint32_t x = s;   // inclusive scan of the chunk sums within the wave
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) part[wave] = x;
    __syncthreads();
    if (tid < 64) {   // inclusive scan of the wave totals
        uint32_t w = tid < NWV ? part[tid] : 0u;
        for (uint32_t o = 1; o < NWV; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)w, o, 64);
            if (lane >= o) w += y;
        }
        if (tid < NWV) part[tid] = w;
    }
    __syncthreads();
    uint32_t run = (wave ? part[wave - 1] : 0u) + x - s;
    for (uint32_t i = lo; i < hi; i++) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
    const uint32_t total = part[NWV - 1];
    __syncthreads();
    return total;
}

// largest i in [0, len) with pre[i] <= q (pre ascending, pre[0] = 0 <= q)
__device__ __forceinline__ uint32_t upper_idx(const uint32_t* pre, uint32_t len, uint32_t q) {
    uint32_t lo = 0, hi = len;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
}

struct SmallLds {
    const uint32_t* off;
    const uint16_t* adj;   // entries (nbr_rank << 2) | arc bits; ranks below 1024 fit 16 bits
    const uint32_t* split;
    const uint32_t* bits;
    uint32_t W;
    __device__ __forceinline__ bool adjacent(uint32_t u, uint32_t v) const {
        return (bits[u * W + (v >> 5)] >> (v & 31u)) & 1u;
    }
    // the bitmap word of row u that holds v's bit, and the bit itself
    __device__ __forceinline__ uint32_t word(uint32_t u, uint32_t v) const { return bits[u * W + (v >> 5)]; }
    static __device__ __forceinline__ bool bit(uint32_t w, uint32_t v) { return (w >> (v & 31u)) & 1u; }
    // arc bits of (u, v) seen from u for a pair whose adjacency bit is already read
    __device__ __forceinline__ uint32_t code_if(bool is_adj, uint32_t u, uint32_t v) const {
        if (!is_adj) return 0u;
        uint32_t lo = off[u], hi = off[u + 1];
        const uint32_t key = v << 2;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (adj[mid] < key) lo = mid + 1; else hi = mid;
        }
        return adj[lo] & 3u;
    }
    // arc bits of (u, v) seen from u, 0 if not adjacent
    __device__ __forceinline__ uint32_t code(uint32_t u, uint32_t v) const {
        if (!adjacent(u, v)) return 0u;
        uint32_t lo = off[u], hi = off[u + 1];
        const uint32_t key = v << 2;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (adj[mid] < key) lo = mid + 1; else hi = mid;
        }
        return adj[lo] & 3u;
    }
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

template <int K>
struct SmallCredit {
    static constexpr uint32_t NC = K == 3 ? (uint32_t)kClasses3 : kSlots4;
    static constexpr uint32_t C = K == 3 ? (uint32_t)kClasses3 : (uint32_t)kClasses4;
    uint32_t* cnt;            // n x NC (LDS)
    const uint8_t* comp;      // k = 4: class -> counter slot or 0xFF (LDS)
    const int32_t* perm;
    unsigned long long* out;
    // slot of cls in the LDS counters, or NC when the class is credited to the output
    __device__ __forceinline__ uint32_t slot(uint32_t cls) const {
        if (K == 3) return cls;
        const uint32_t s = comp[cls];
        return s == 0xFFu ? NC : s;
    }
    __device__ __forceinline__ void add_n(uint32_t v, uint32_t cls, uint32_t n) const {
        const uint32_t s = slot(cls);
        if (s < NC) atomicAdd(&cnt[v * NC + s], n);
        else out_add(&out[(size_t)perm[v] * C + cls], (unsigned long long)n);
    }
    // n sets of a class whose counter slot s (< NC) is already known
    __device__ __forceinline__ void add_s(uint32_t v, uint32_t s, uint32_t n) const { atomicAdd(&cnt[v * NC + s], n); }
    // n sets of class cls credited to three members (nothing when n = 0)
    __device__ __forceinline__ void add3(uint32_t u, uint32_t v, uint32_t w, uint32_t cls, uint32_t n) const {
        if (!n) return;
        add_n(u, cls, n);
        add_n(v, cls, n);
        add_n(w, cls, n);
    }
    // One set per active lane, of class cls, credited to the NS members in sv, which the
    // lanes often share (the root, and the members fixed by the wave's loop position).
    // A class with an LDS counter (every k = 3 class, the 37 slot classes of k = 4) is
    // added lane by lane: an LDS atomic is cheap, and lanes that share a member and a
    // class only meet in the LDS unit.  The other classes go to the output, where every
    // atomic is a memory-side operation: a member common to all such lanes gets each of
    // their classes once, with the lanes' count; a member that differs is added lane by
    // lane.
    template <int NS>
    __device__ __forceinline__ void shared(uint32_t cls, const uint32_t (&sv)[NS], bool active) const {
        const uint32_t s = active ? slot(cls) : NC;
        if (active && s < NC)
            for (int i = 0; i < NS; i++) atomicAdd(&cnt[sv[i] * NC + s], 1u);
        if (K == 3) return;
        const bool far = active && s >= NC;
        const unsigned long long act = __ballot(far);
        if (!act) return;
        const int first = __ffsll((long long)act) - 1;
        uint32_t common = 0;   // wave-uniform bit mask of the members all such lanes share
        for (int i = 0; i < NS; i++)
            if (__ballot(far && sv[i] != (uint32_t)__shfl((int)sv[i], first, 64)) == 0ull) common |= 1u << i;
        if (common) {
            unsigned long long m = act;
            while (m) {
                const uint32_t leader = (uint32_t)(__ffsll((long long)m) - 1);
                const uint32_t k0 = (uint32_t)__shfl((int)cls, (int)leader, 64);
                const unsigned long long grp = __ballot(far && cls == k0) & m;
                if (lane_of() == leader)
                    for (int i = 0; i < NS; i++)
                        if ((common >> i) & 1u)
                            out_add(&out[(size_t)perm[sv[i]] * C + k0], (unsigned long long)__popcll(grp));
                m &= ~grp;
            }
        }
        if (far)
            for (int i = 0; i < NS; i++)
                if (!((common >> i) & 1u)) out_add(&out[(size_t)perm[sv[i]] * C + cls], 1ull);
    }
};

template <int BS, int K>
__global__ __launch_bounds__(BS) void k_small(SmallArgs A) {
    extern __shared__ uint32_t dyn[];
    __shared__ uint8_t sTable[K == 3 ? 64 : 4096];
    __shared__ uint8_t sComp[256];
    __shared__ uint8_t sSlotCls[64];
    __shared__ uint32_t sMask[8];   // k = 4: 256-bit mask of the single-arc 4-pair classes
    __shared__ uint32_t sPart[BS / 64];
    __shared__ uint32_t sGraph;
    constexpr uint32_t NC = SmallCredit<K>::NC;
    constexpr uint32_t C = SmallCredit<K>::C;
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < (K == 3 ? 64u : 4096u); i += BS) sTable[i] = A.table[i];
    if (K == 4) {
        // counter slots: the tree classes' from the class tables, then the single-arc
        // 4-pair classes in ascending class id (each found from any of its codes)
        for (uint32_t i = tid; i < 256u; i += BS) sComp[i] = A.comp_of[i];
        for (uint32_t i = tid; i < (uint32_t)kCompact4; i += BS) sSlotCls[i] = A.comp_cls[i];
        if (tid < 8) sMask[tid] = 0u;
        __syncthreads();
        for (uint32_t code = tid; code < 4096u; code += BS) {
            uint32_t joined = 0, recip = 0;
            for (uint32_t i = 0; i < 4; i++)
                for (uint32_t j = i + 1; j < 4; j++) {
                    const uint32_t x = bit4(code, i, j), y = bit4(code, j, i);
                    joined += x | y;
                    recip += x & y;
                }
            const uint32_t cls = sTable[code];
            if (joined == 4u && recip == 0u && cls != 0xFFu) atomicOr(&sMask[cls >> 5], 1u << (cls & 31u));
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t k = 0;
            for (uint32_t c = 0; c < 256u; c++)
                if (((sMask[c >> 5] >> (c & 31u)) & 1u) && sComp[c] == 0xFFu && k < kSingleArc4) {
                    sComp[c] = (uint8_t)(kCompact4 + k);
                    sSlotCls[kCompact4 + k] = (uint8_t)c;
                    k++;
                }
        }
    }

    for (uint32_t round = 0;; round++) {
        __syncthreads();
        if (tid == 0) sGraph = A.graphs ? atomicAdd(A.cursor, 1u) : round;   // single graph: taken once
        __syncthreads();
        const uint32_t gidx = sGraph;
        if (gidx >= A.num) break;
        const SmallGraph G = A.graphs ? A.graphs[gidx] : A.one;
        const uint32_t n = G.n, E = G.entries, W = (n + 31u) >> 5;
        // LDS layout
        uint32_t* sOff = dyn;                 // n + 1
        uint32_t* sSplit = sOff + n + 1;      // n
        uint32_t* sPreD = sSplit + n;         // n + 1: upper entries before row r
        uint32_t* sPre1 = sPreD + n + 1;      // n + 1: pair items before root r
        uint32_t* sBits = sPre1 + n + 1;      // n * W
        uint32_t* sCnt = sBits + n * W;       // n * NC
        uint32_t* sPre2 = sCnt + n * NC;      // E / 2 + 1: depth-2 candidates before each upper entry
        uint16_t* sAdj = reinterpret_cast<uint16_t*>(sPre2 + E / 2 + 1);   // E (u16)
        uint16_t* sRootOf = sAdj + E;         // E / 2 (u16): root of each upper entry
        // ---- stage the graph, clear bitmap, counters and the output block
        for (uint32_t i = tid; i <= n; i += BS) sOff[i] = G.off[i];
        for (uint32_t i = tid; i < E; i += BS) sAdj[i] = (uint16_t)G.adj[i];
        for (uint32_t i = tid; i < n * W; i += BS) sBits[i] = 0u;
        for (uint32_t i = tid; i < n * NC; i += BS) sCnt[i] = 0u;
        if (((uintptr_t)G.out & 15u) == 0) {   // 16-byte stores, then the odd last cell
            const size_t cells = (size_t)n * C;
            ulonglong2* o = reinterpret_cast<ulonglong2*>(G.out);
            for (size_t i = tid; i < cells / 2; i += BS) o[i] = make_ulonglong2(0ull, 0ull);
            if ((cells & 1u) && tid == 0) G.out[cells - 1] = 0ull;
        } else {
            for (size_t i = tid; i < (size_t)n * C; i += BS) G.out[i] = 0ull;
        }
        if (tid < (uint32_t)kShapes) G.stats[tid] = 0ull;   // this launch's visit counters of the graph
        __syncthreads();
        for (uint32_t r = tid; r < n; r += BS) {
            const uint32_t lo = sOff[r], hi = sOff[r + 1];
            uint32_t s = hi;
            for (uint32_t t = lo; t < hi; t++) {
                const uint32_t v = sAdj[t] >> 2;
                atomicOr(&sBits[r * W + (v >> 5)], 1u << (v & 31u));
                if (v > r && s == hi) s = t;
            }
            sSplit[r] = s;
            const uint32_t d = hi - s;
            sPreD[r] = d;
            sPre1[r] = d * (d - 1u) / 2u;
        }
        if (tid == 0) {
            sPreD[n] = 0u;
            sPre1[n] = 0u;
        }
        __syncthreads();
        const uint32_t U = block_exclusive_scan<BS>(sPreD, n + 1, sPart);
        const uint32_t N1 = block_exclusive_scan<BS>(sPre1, n + 1, sPart);
        const SmallLds L{sOff, sAdj, sSplit, sBits, W};
        // candidates of each upper entry (r, a): entries of a's row above r
        for (uint32_t r = tid; r < n; r += BS)
            for (uint32_t t = sSplit[r]; t < sOff[r + 1]; t++) {
                const uint32_t a = sAdj[t] >> 2;
                sPre2[sPreD[r] + (t - sSplit[r])] = sOff[a + 1] - L.first_above(a, r);
                sRootOf[sPreD[r] + (t - sSplit[r])] = (uint16_t)r;
            }
        if (tid == 0) sPre2[U] = 0u;
        __syncthreads();
        const uint32_t N2 = block_exclusive_scan<BS>(sPre2, U + 1, sPart);

        const SmallCredit<K> cr{sCnt, sComp, G.perm, G.out};
        unsigned long long shp[4] = {0, 0, 0, 0};
        // ---- pairs {a < b} of N+(r): (1,1) / (3,0,0)
        for (uint32_t q = tid; q < N1; q += BS) {
            const uint32_t r = upper_idx(sPre1, n + 1, q);
            const uint32_t idx = q - sPre1[r];
            uint32_t j = (uint32_t)((1.0f + sqrtf(1.0f + 8.0f * (float)idx)) * 0.5f);
            while (j * (j - 1u) / 2u > idx) j--;
            while ((j + 1u) * j / 2u <= idx) j++;
            const uint32_t i = idx - j * (j - 1u) / 2u;
            const uint16_t* P = sAdj + sSplit[r];
            const uint32_t d = sOff[r + 1] - sSplit[r];
            const uint32_t a = P[i] >> 2, ra = P[i] & 3u, b = P[j] >> 2, rb = P[j] & 3u;
            const uint32_t ab = L.code(a, b);
            if (K == 3) {
                const uint32_t cls = sTable[motif_index3(ra, rb, ab)];
                const uint32_t sv[2] = {r, b};
                cr.shared(cls, sv, true);
                cr.add_n(a, cls, 1u);
                shp[0]++;
            } else {
                // (3,0,0): r, a, b fixed, lanes' loops over c.  A set whose c is adjacent to
                // neither a nor b has its class fixed by c's arc with r: those sets credit c
                // one by one and r, a, b once per arc code after the loop.
                const uint32_t p1 = sTable[motif_index4(ra, rb, 1u, ab, 0u, 0u)];
                const uint32_t p2 = sTable[motif_index4(ra, rb, 2u, ab, 0u, 0u)];
                const uint32_t p3 = sTable[motif_index4(ra, rb, 3u, ab, 0u, 0u)];
                uint32_t np = 0;   // sets by arc code 1, 2, 3: 10-bit fields (every loop runs < 1024 times)
                // software pipeline: the entry two candidates ahead and the bitmap words of
                // the next one are read before this candidate's credits (LDS atomics, which
                // later reads could not otherwise pass)
                const uint32_t dm = d - 1u;
                uint32_t e0 = P[min(j + 1u, dm)], e1 = P[min(j + 2u, dm)];
                uint32_t wa0 = L.word(a, e0 >> 2), wb0 = L.word(b, e0 >> 2);
                for (uint32_t l = j + 1; l < d; l++) {
                    const uint32_t e2 = P[min(l + 2u, dm)];
                    const uint32_t wa1 = L.word(a, e1 >> 2), wb1 = L.word(b, e1 >> 2);
                    const uint32_t c = e0 >> 2, rc = e0 & 3u;
                    const bool xa = SmallLds::bit(wa0, c), xb = SmallLds::bit(wb0, c);
                    e0 = e1;
                    e1 = e2;
                    wa0 = wa1;
                    wb0 = wb1;
                    const uint32_t ac = L.code_if(xa, a, c), bc = L.code_if(xb, b, c);
                    if (ac | bc) {
                        const uint32_t cls = sTable[motif_index4(ra, rb, rc, ab, ac, bc)];
                        const uint32_t sv[3] = {r, b, c};   // lanes share j, hence b and c
                        cr.shared(cls, sv, true);
                        cr.add_n(a, cls, 1u);
                    } else {
                        cr.add_n(c, rc == 1u ? p1 : (rc == 2u ? p2 : p3), 1u);
                        np += 1u << (10u * rc - 10u);
                    }
                    shp[0]++;
                }
                cr.add3(r, a, b, p1, np & 1023u);
                cr.add3(r, a, b, p2, (np >> 10) & 1023u);
                cr.add3(r, a, b, p3, np >> 20);
            }
        }
        // ---- depth-2 entries (r, a, c)
        for (uint32_t q = tid; q < N2; q += BS) {
            const uint32_t u = upper_idx(sPre2, U + 1, q);
            const uint32_t r = sRootOf[u];
            const uint16_t* P = sAdj + sSplit[r];
            const uint32_t d = sOff[r + 1] - sSplit[r];
            const uint32_t ia = u - sPreD[r];
            const uint32_t a = P[ia] >> 2, ra = P[ia] & 3u;
            const uint32_t t0 = L.first_above(a, r), t = t0 + (q - sPre2[u]);
            const uint32_t c = sAdj[t] >> 2, ac = sAdj[t] & 3u;
            if (L.adjacent(r, c)) continue;   // c adjacent to r: depth 1, not 2
            if (K == 3) {
                const uint32_t cls = sTable[motif_index3(ra, 0u, ac)];
                const uint32_t sv[2] = {r, a};
                cr.shared(cls, sv, true);
                cr.add_n(c, cls, 1u);
                shp[1]++;
                continue;
            }
            // (2,1,0): a second depth-1 vertex b; c hangs under the lower-rank parent.  r, a,
            // c are fixed for the lane's loop; a set whose b is adjacent to neither a nor c
            // has its class fixed by b's arc with r: b is credited per set, r, a, c once per
            // arc code after the loop.  The same holds below for (1,2,0) (c2 not adjacent to
            // c: class by a's arc with c2) and for every (1,1,1) set (class by c's arc with e).
            {
                const uint32_t q1 = sTable[motif_index4(ra, 1u, 0u, 0u, ac, 0u)];
                const uint32_t q2 = sTable[motif_index4(ra, 2u, 0u, 0u, ac, 0u)];
                const uint32_t q3 = sTable[motif_index4(ra, 3u, 0u, 0u, ac, 0u)];
                const uint32_t s1 = cr.slot(q1), s2 = cr.slot(q2), s3 = cr.slot(q3);   // 4-path classes: tree slots
                uint32_t np = 0;   // sets by arc code 1, 2, 3: 10-bit fields (every loop runs < 1024 times)
                // pipelined as the (3,0,0) loop; jb runs over r's row without a's entry ia
                const uint32_t dm = d - 1u;
                uint32_t jb = ia == 0u ? 1u : 0u;
                uint32_t j1 = jb + 1u == ia ? jb + 2u : jb + 1u;
                uint32_t e0 = P[min(jb, dm)], e1 = P[min(j1, dm)];
                uint32_t wc0 = L.word(e0 >> 2, c), wa0 = L.word(a, e0 >> 2);
                for (; jb < d; jb = j1, j1 = j1 + 1u == ia ? j1 + 2u : j1 + 1u) {
                    const uint32_t j2 = j1 + 1u == ia ? j1 + 2u : j1 + 1u;
                    const uint32_t e2 = P[min(j2, dm)];
                    const uint32_t wc1 = L.word(e1 >> 2, c), wa1 = L.word(a, e1 >> 2);
                    const uint32_t b = e0 >> 2, rb = e0 & 3u;
                    const bool xbc = SmallLds::bit(wc0, c), xab = SmallLds::bit(wa0, b);
                    e0 = e1;
                    e1 = e2;
                    wc0 = wc1;
                    wa0 = wa1;
                    if (xbc && jb < ia) continue;
                    const uint32_t bc = L.code_if(xbc, b, c), ab = L.code_if(xab, a, b);
                    if (ab | bc) {
                        const uint32_t cls = sTable[motif_index4(ra, rb, 0u, ab, ac, bc)];
                        const uint32_t sv[3] = {r, a, b};   // lanes share (r, a) and the loop position
                        cr.shared(cls, sv, true);
                        cr.add_n(c, cls, 1u);
                    } else {
                        cr.add_s(b, rb == 1u ? s1 : (rb == 2u ? s2 : s3), 1u);
                        np += 1u << (10u * rb - 10u);
                    }
                    shp[1]++;
                }
                cr.add3(r, a, c, q1, np & 1023u);
                cr.add3(r, a, c, q2, (np >> 10) & 1023u);
                cr.add3(r, a, c, q3, np >> 20);
            }
            // (1,2,0): a second child c2 of a, not adjacent to r.  Every pair {c, c2} of a's
            // children is taken once, by the member from which the other lies less than half
            // of a's row (above r) ahead, circularly: the lanes of one (r, a) then have equal
            // loop lengths, (L - 1) / 2 or L / 2, instead of L - 1 down to 0.
            {
                const uint32_t u1 = sTable[motif_index4(ra, 0u, 0u, ac, 1u, 0u)];
                const uint32_t u2 = sTable[motif_index4(ra, 0u, 0u, ac, 2u, 0u)];
                const uint32_t u3 = sTable[motif_index4(ra, 0u, 0u, ac, 3u, 0u)];
                const uint32_t s1 = cr.slot(u1), s2 = cr.slot(u2), s3 = cr.slot(u3);   // 3-star classes: tree slots
                uint32_t np = 0;   // sets by arc code 1, 2, 3: 10-bit fields (every loop runs < 1024 times)
                const uint32_t Lr = sOff[a + 1] - t0, pos = t - t0;
                const uint32_t nd = (Lr - 1u) / 2u + ((Lr % 2u == 0u && pos < Lr / 2u) ? 1u : 0u);
                // pipelined as the (3,0,0) loop over the circular positions pos + 1 .. pos + nd
                const auto at = [&](uint32_t dl) {
                    const uint32_t p2 = pos + dl < Lr ? pos + dl : pos + dl - Lr;
                    return sAdj[t0 + (p2 < Lr ? p2 : 0u)];
                };
                uint32_t e0 = at(1u), e1 = at(2u);
                uint32_t wr0 = L.word(r, e0 >> 2), wc0 = L.word(c, e0 >> 2);
                for (uint32_t dlt = 1; dlt <= nd; dlt++) {
                    const uint32_t e2 = at(dlt + 2u);
                    const uint32_t wr1 = L.word(r, e1 >> 2), wc1 = L.word(c, e1 >> 2);
                    const uint32_t c2 = e0 >> 2, ac2 = e0 & 3u;
                    const bool xr = SmallLds::bit(wr0, c2), xc = SmallLds::bit(wc0, c2);
                    e0 = e1;
                    e1 = e2;
                    wr0 = wr1;
                    wc0 = wc1;
                    if (xr) continue;
                    const uint32_t cc2 = L.code_if(xc, c, c2);
                    if (cc2) {
                        const uint32_t cls = sTable[motif_index4(ra, 0u, 0u, ac, ac2, cc2)];
                        const uint32_t sv[2] = {r, a};
                        cr.shared(cls, sv, true);
                        cr.add_n(c, cls, 1u);
                        cr.add_n(c2, cls, 1u);
                    } else {
                        cr.add_s(c2, ac2 == 1u ? s1 : (ac2 == 2u ? s2 : s3), 1u);
                        np += 1u << (10u * ac2 - 10u);
                    }
                    shp[2]++;
                }
                cr.add3(r, a, c, u1, np & 1023u);
                cr.add3(r, a, c, u2, (np >> 10) & 1023u);
                cr.add3(r, a, c, u3, np >> 20);
            }
            // (1,1,1): path r - a - c - e, e not adjacent to r (nor equal to a) nor to a
            {
                const uint32_t w1 = sTable[motif_index4(ra, 0u, 0u, ac, 0u, 1u)];
                const uint32_t w2 = sTable[motif_index4(ra, 0u, 0u, ac, 0u, 2u)];
                const uint32_t w3 = sTable[motif_index4(ra, 0u, 0u, ac, 0u, 3u)];
                const uint32_t s1 = cr.slot(w1), s2 = cr.slot(w2), s3 = cr.slot(w3);   // 4-path classes: tree slots
                uint32_t np = 0;   // sets by arc code 1, 2, 3: 10-bit fields (every loop runs < 1024 times)
                // pipelined as the (3,0,0) loop
                const uint32_t tb = L.first_above(c, r), tend = sOff[c + 1];
                const uint32_t tm = tend - 1u;   // read only when the row part is not empty
                uint32_t e0 = tend > tb ? sAdj[tb] : 0u, e1 = tend > tb ? sAdj[min(tb + 1u, tm)] : 0u;
                uint32_t wr0 = L.word(r, e0 >> 2), wa0 = L.word(a, e0 >> 2);
                for (uint32_t te = tb; te < tend; te++) {
                    const uint32_t e2 = sAdj[min(te + 2u, tm)];   // te < tend: in the row
                    const uint32_t wr1 = L.word(r, e1 >> 2), wa1 = L.word(a, e1 >> 2);
                    const uint32_t e = e0 >> 2, ce = e0 & 3u;
                    const bool skip = SmallLds::bit(wr0, e) | SmallLds::bit(wa0, e);
                    e0 = e1;
                    e1 = e2;
                    wr0 = wr1;
                    wa0 = wa1;
                    if (skip) continue;
                    cr.add_s(e, ce == 1u ? s1 : (ce == 2u ? s2 : s3), 1u);
                    np += 1u << (10u * ce - 10u);
                    shp[3]++;
                }
                cr.add3(r, a, c, w1, np & 1023u);
                cr.add3(r, a, c, w2, (np >> 10) & 1023u);
                cr.add3(r, a, c, w3, np >> 20);
            }
        }
        __syncthreads();
        // ---- counters -> output.  The block is this workgroup's and was zeroed above; an
        // LDS-counted class never reaches the output otherwise, so its cells are stored.
        for (uint32_t i = tid; i < n * NC; i += BS) {
            const uint32_t x = sCnt[i];
            if (!x) continue;
            const uint32_t v = i / NC, s = i - v * NC;
            const uint32_t cls = K == 3 ? s : sSlotCls[s];
            G.out[(size_t)G.perm[v] * C + cls] = (unsigned long long)x;
        }
        // visited-set counters per shape: k = 3 -> (1,1), (1,2); k = 4 -> the four shapes
        for (int s = 0; s < 4; s++) {
            unsigned long long x = shp[s];
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
            shp[s] = x;
        }
        if (lane_of() == 0) {
            if (K == 3) {
                if (shp[0]) atomicAdd(&G.stats[0], shp[0]);
                if (shp[1]) atomicAdd(&G.stats[1], shp[1]);
            } else {
                for (int s = 0; s < 4; s++)
                    if (shp[s]) atomicAdd(&G.stats[2 + s], shp[s]);
            }
        }
    }
}

}  // namespace

size_t small_lds_bytes(int64_t n, int64_t entries, int k) {
    const int64_t W = (n + 31) / 32;
    const int64_t nc = k == 3 ? kClasses3 : kSlots4;
    // u32 arrays, then the row entries and the roots of the upper entries (u16)
    const int64_t words = (n + 1) * 3 + n + n * W + n * nc + entries / 2 + 1 + (entries + entries / 2 + 1) / 2;
    return (size_t)words * sizeof(uint32_t);
}

bool small_eligible(int64_t n, int64_t entries, int k) {
    return n >= 1 && n <= kSmallMaxN && small_lds_bytes(n, entries, k) <= kSmallLdsBudget;
}

int small_threads(int variant) { return variant <= 0 ? 256 : (variant == 1 ? 512 : 1024); }

void launch_small(const SmallArgs& a, int k, int variant, unsigned grid, size_t lds, hipStream_t st) {
    void (*kern)(SmallArgs) = nullptr;
    const int bs = small_threads(variant);
    if (k == 3) kern = bs == 256 ? k_small<256, 3> : (bs == 512 ? k_small<512, 3> : k_small<1024, 3>);
    else kern = bs == 256 ? k_small<256, 4> : (bs == 512 ? k_small<512, 4> : k_small<1024, 4>);
    VDMC_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(bs), lds, st, a);
    VDMC_HIP(hipGetLastError());
}

}  // namespace vdmc

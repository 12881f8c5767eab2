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
// and a 1-bit adjacency matrix (every pair test is one LDS read; the arc bits of a
// member with its parent come with the row entry, others are searched in the row).  A
// work item is a root r with the first member a of its layer 1 (one per pair of G_U,
// from its lower-rank end), cut for the heavy roots into K sub-items by the choice of
// the third member; a lane runs a sub-item's whole search (three nested candidate
// loops) and visits every set of it.  Lanes take items one at a time from the graph's
// item cursor, so lanes with short items keep taking new ones.  Class ids come from a
// 2^20-entry u16 table in device memory (2 MiB).  9364 classes per vertex do not fit in
// LDS; the 27 single-arc tree classes, which hold most sets of a sparse digraph, have
// per-vertex LDS counters (added to the output block when the part ends), and the other
// classes are credited to the output block in device memory.  The last member of a set
// is credited per set, the four fixed members per distinct signature of the last one in
// their context (a 4-entry per-lane cache).  Over a graph in device memory (no LDS
// counters) the first three members' credits are further added up per class over the
// whole loop under one third member (an 8-entry per-lane cache of (class, count)).
//
// Work split.  A graph is cut into P parts (P from its estimated work, sum of d^4 over
// its vertices, so that the heaviest graphs of a batch spread over many compute units):
// a part is a workgroup that loads the graph, zeroes its own output block -- the
// caller's output for part 0, a private copy in scratch for the others -- and then
// takes items from the graph's item cursor until none are left.  A block belongs to one
// workgroup for the whole launch, so its credits are workgroup-scope atomics.  A second
// launch adds the copies of each graph with P > 1 into its output.  Parts are claimed
// heaviest graph first from a slot cursor; items of a graph are handed out in rank
// order, the heavy roots first.
// Graphs that LDS does not hold take the same search over the graph in device memory
// (k_five_global): pair tests from the graph's edge hash, rows searched in place, one
// item cursor for the whole grid and device-scope credits to the caller's output.
// Visited sets are counted per shape (the graph's 8 counters) so that callers can
// check that every set was visited: their sum is the number of connected 5-sets.
#include <cmath>
#include <map>

#include <hipcub/hipcub.hpp>

#include "motif_device.h"
#include "vdmc_internal.h"

namespace vdmc {
namespace {

constexpr size_t kFiveStaticLds = 14336;                       // the kernel's __shared__ bytes, rounded up
// LDS counter slots per vertex: the 27 classes of 5-sets whose induced subgraph is a tree
// with single arcs (oriented paths, stars and forks without a reciprocal pair), which in a
// sparse digraph hold most of the sets (~84% of the batch workload's credits); the other
// classes are credited to the output block
constexpr uint32_t kTreeSlots5 = 27;
constexpr uint32_t kClassPad = 9376;                           // 9364 classes, padded to 16 bytes
constexpr int64_t kFiveMatMaxN = 16384;                        // device-memory graphs up to this get a bit matrix (32 MiB)
constexpr size_t kFiveLdsBudget = 163840 - kFiveStaticLds;     // gfx950: 160 KiB of LDS per workgroup
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kPartsPerCu = 2;                                 // target parts per compute unit in a batch
constexpr uint32_t kSplitDiv = 32;                             // sub-items of a root: d+ x deg / 32 (measured best of 2..128)
constexpr uint32_t kMaxParts = 64;                             // parts of one graph
constexpr size_t kBatchScratchBudget = size_t(8) << 30;       // private copies of one batched launch
constexpr size_t kSingleScratchBudget = size_t(512) << 20;    // private copies of one graph's count

// bit of the index of a 5-set for the entry (i, j), i != j: rows in order, the diagonal
// skipped, entry (0,1) the most significant of the 20 (Sec. 4.1, Fig. 1)
__host__ __device__ __forceinline__ constexpr uint32_t shift5(uint32_t i, uint32_t j) {
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
    const uint32_t* mat;    // n rows of W words, one adjacency bit per vertex
    const uint32_t* perm;
    uint32_t W;
    __device__ __forceinline__ bool adjacent(uint32_t u, uint32_t v) const {
        return (mat[u * W + (v >> 5)] >> (v & 31u)) & 1u;
    }
    // arc bits of (u, v) seen from u: bit 0 u -> v, bit 1 v -> u; 0 if not adjacent (a set
    // bit is resolved by a search of u's row)
    __device__ __forceinline__ uint32_t bits(uint32_t u, uint32_t v) const {
        if (!adjacent(u, v)) return 0u;
        uint32_t lo = off[u], hi = off[u + 1];
        const uint32_t key = v << 2;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (adj[mid] < key) lo = mid + 1; else hi = mid;
        }
        return adj[lo] & 3u;
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

// The same interface over a graph in device memory, for graphs that LDS does not hold:
// pair tests from a 1-bit adjacency matrix in device memory when the graph has one (one
// cached load), else from the edge hash; arc bits of an adjacent pair from the edge hash
// (one probe sequence); rows searched in place.
struct FiveGlobal {
    const uint32_t* off;
    const uint32_t* adj;
    const uint32_t* perm;
    const unsigned long long* eh;
    uint32_t ebits;
    const uint32_t* mat;   // n rows of W words, or nullptr
    uint32_t W;
    __device__ __forceinline__ bool adjacent(uint32_t u, uint32_t v) const {
        if (mat) return (mat[(size_t)u * W + (v >> 5)] >> (v & 31u)) & 1u;
        return edge_code(eh, ebits, u, v) != 0u;
    }
    __device__ __forceinline__ uint32_t bits(uint32_t u, uint32_t v) const {
        if (mat && !((mat[(size_t)u * W + (v >> 5)] >> (v & 31u)) & 1u)) return 0u;
        return edge_code(eh, ebits, u, v);
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

// The members S[0..3] of the set being built (the fifth is the innermost loop's
// candidate).  Named fields rather than an array: a member picked by an index that is not
// a compile-time constant is a select, where an array would be placed in scratch memory.
struct Members {
    uint32_t v0, v1, v2, v3;
    __device__ __forceinline__ uint32_t operator[](uint32_t i) const {
        return i == 0u ? v0 : (i == 1u ? v1 : (i == 2u ? v2 : v3));
    }
};

// y adjacent to none of S[0..lim)
template <class V>
__device__ __forceinline__ bool clear_of(const V& L, const Members& S, uint32_t lim, uint32_t y) {
#pragma unroll
    for (uint32_t m = 0; m < 4; m++)
        if (m < lim && L.adjacent(S[m], y)) return false;
    return true;
}

// Candidates of the next member, given S[0..t): first the rest of S[t-1]'s layer (after
// S[t-1]'s parent and position), then -- phase 1 -- the first member of a new layer under
// the members of S[t-1]'s layer.  pi: S index of the current parent, [pi, pend) the
// parents left in the phase, [j, jend) the rest of the parent's row.
struct Cand {
    uint32_t pi, pend, j, jend, phase, ls, pbits;   // pbits: arc bits of the last candidate with its parent
    template <class V>
    __device__ __forceinline__ void start(const V& L, const Members& S, uint32_t par, uint32_t pos,
                                          uint32_t ls_prev) {
        pi = par;
        pend = ls_prev;
        j = pos + 1u;
        jend = L.off[S[par] + 1u];
        phase = 0u;
        ls = ls_prev;
    }
    // next candidate vertex, or kNone; t = the S index being chosen
    template <class V>
    __device__ __forceinline__ uint32_t next(const V& L, const Members& S, uint32_t t) {
        for (;;) {
            while (j < jend) {
                const uint32_t e = L.adj[j++], y = e >> 2;
                if (clear_of(L, S, pi, y)) {
                    pbits = e & 3u;
                    return y;
                }
            }
            if (++pi < pend) {
                const uint32_t x = S[pi];
                j = L.first_above(x, S[0]);
                jend = L.off[x + 1u];
                continue;
            }
            if (phase == 0u) {   // the layer of S[t-1] is closed: open the next one under it
                phase = 1u;
                pi = ls;
                pend = t;
                const uint32_t x = S[pi];
                j = L.first_above(x, S[0]);
                jend = L.off[x + 1u];
                continue;
            }
            return kNone;
        }
    }
};

// arc bits of (S[m], y) seen from S[m], for the candidate y just returned by c: its
// parent's come with the entry, members before the parent are not adjacent to it (the
// candidate rule), the others are looked up
template <class V>
__device__ __forceinline__ uint32_t arc_of(const V& L, const Members& S, uint32_t m, const Cand& c,
                                           uint32_t y) {
    if (m == c.pi) return c.pbits;
    if (m < c.pi) return 0u;
    return L.bits(S[m], y);
}

// credits: workgroup scope to an output block that belongs to the calling workgroup (no
// other workgroup touches it during the launch), device scope to an output all
// workgroups share (kDev)
template <bool kDev>
__device__ __forceinline__ void bump(unsigned long long* p, unsigned long long v) {
    if (kDev) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Where a credit of v sets of class cls to vertex P (original id) goes.  GlobalSink: to
// the output (device scope when kDev).  LdsSink: a class with an LDS counter slot (the
// single-arc tree classes) to the workgroup's LDS counters, any other to its output
// block.
template <bool kDev>
struct GlobalSink {
    static constexpr bool kClassCache = true;
    unsigned long long* out;
    __device__ __forceinline__ void add(uint32_t P, uint32_t cls, uint32_t v) const {
        bump<kDev>(&out[(size_t)P * kClasses5 + cls], (unsigned long long)v);
    }
};
struct LdsSink {
    static constexpr bool kClassCache = false;
    unsigned long long* out;
    uint32_t* cnt;            // n x kTreeSlots5 (LDS), rows by original id
    const uint8_t* slot_of;   // class -> counter slot or 0xFF (LDS)
    __device__ __forceinline__ void add(uint32_t P, uint32_t cls, uint32_t v) const {
        const uint32_t sl = slot_of[cls];
        if (sl < kTreeSlots5) atomicAdd(&cnt[P * kTreeSlots5 + sl], v);
        else bump<false>(&out[(size_t)P * kClasses5 + cls], (unsigned long long)v);
    }
};

// v sets of class cls credited to the three members fixed over a depth-2 loop
template <class Sk>
__device__ __forceinline__ void credit3(const Sk& sk, uint32_t P0, uint32_t P1, uint32_t P2, uint32_t cls,
                                        uint32_t v) {
    sk.add(P0, cls, v);
    sk.add(P1, cls, v);
    sk.add(P2, cls, v);
}

// Per-lane cache of the classes credited to S[0], S[1], S[2] over one depth-2 loop (all
// fourth members under one third member): entry = (count << 14) | class, 0 = empty; the
// oldest entry makes room.  A count stays below 2^18: an entry about to pass it takes a
// new slot instead.  Used where every credit is a memory-side atomic (GlobalSink); with
// LDS counters the three credits are cheaper than the cache's registers.
struct ClassCache {
    uint32_t e0 = 0, e1 = 0, e2 = 0, e3 = 0, e4 = 0, e5 = 0, e6 = 0, e7 = 0, victim = 0;
    static __device__ __forceinline__ bool take(uint32_t& e, uint32_t cls, uint32_t v) {
        if (e == 0u || (e & 0x3FFFu) != cls || (e >> 14) + v >= (1u << 18)) return false;
        e += v << 14;
        return true;
    }
    template <class Sk>
    __device__ __forceinline__ void add(uint32_t cls, uint32_t v, const Sk& sk, uint32_t P0, uint32_t P1,
                                        uint32_t P2) {
        if (take(e0, cls, v) || take(e1, cls, v) || take(e2, cls, v) || take(e3, cls, v) || take(e4, cls, v) ||
            take(e5, cls, v) || take(e6, cls, v) || take(e7, cls, v))
            return;
        const uint32_t e = (v << 14) | cls;
        uint32_t old;
        switch (victim) {
            case 0: old = e0; e0 = e; break;
            case 1: old = e1; e1 = e; break;
            case 2: old = e2; e2 = e; break;
            case 3: old = e3; e3 = e; break;
            case 4: old = e4; e4 = e; break;
            case 5: old = e5; e5 = e; break;
            case 6: old = e6; e6 = e; break;
            default: old = e7; e7 = e; break;
        }
        victim = (victim + 1u) & 7u;
        if (old) credit3(sk, P0, P1, P2, old & 0x3FFFu, old >> 14);
    }
    template <class Sk>
    __device__ __forceinline__ void flush_all(const Sk& sk, uint32_t P0, uint32_t P1, uint32_t P2) {
        if (e0) credit3(sk, P0, P1, P2, e0 & 0x3FFFu, e0 >> 14);
        if (e1) credit3(sk, P0, P1, P2, e1 & 0x3FFFu, e1 >> 14);
        if (e2) credit3(sk, P0, P1, P2, e2 & 0x3FFFu, e2 >> 14);
        if (e3) credit3(sk, P0, P1, P2, e3 & 0x3FFFu, e3 >> 14);
        if (e4) credit3(sk, P0, P1, P2, e4 & 0x3FFFu, e4 >> 14);
        if (e5) credit3(sk, P0, P1, P2, e5 & 0x3FFFu, e5 >> 14);
        if (e6) credit3(sk, P0, P1, P2, e6 & 0x3FFFu, e6 >> 14);
        if (e7) credit3(sk, P0, P1, P2, e7 & 0x3FFFu, e7 >> 14);
        e0 = e1 = e2 = e3 = e4 = e5 = e6 = e7 = 0u;
        victim = 0u;
    }
};

// v sets of class cls of one context: the fourth member credited now, the three before it
// through the class cache
template <class Sk>
__device__ __forceinline__ void credit_ctx(const Sk& sk, ClassCache& cc, uint32_t P0, uint32_t P1, uint32_t P2,
                                           uint32_t P3, uint32_t cls, uint32_t v) {
    if (v == 0u || cls >= (uint32_t)kClasses5) return;
    sk.add(P3, cls, v);
    if constexpr (Sk::kClassCache) cc.add(cls, v, sk, P0, P1, P2);
    else credit3(sk, P0, P1, P2, cls, v);
}

// Per-lane cache of the last member's signatures in one context: entry = (count << 22) |
// (class << 8) | signature, 0 = empty (a signature is never 0: the last member has an
// arc to its parent); the oldest entry makes room.  A count stays below 1023: a signature
// whose entry is full takes a new one.
struct SigCache {
    uint32_t e0 = 0, e1 = 0, e2 = 0, e3 = 0, victim = 0;
    static __device__ __forceinline__ bool take(uint32_t& e, uint32_t sig) {
        if ((e & 255u) != sig || (e >> 22) >= 1023u) return false;
        e += 1u << 22;
        return true;
    }
    static __device__ __forceinline__ uint32_t cls_of(uint32_t e) { return (e >> 8) & 0x3FFFu; }
    // class of a cached signature (its count raised by one), or kNone
    __device__ __forceinline__ uint32_t hit(uint32_t sig) {
        if (take(e0, sig)) return cls_of(e0);
        if (take(e1, sig)) return cls_of(e1);
        if (take(e2, sig)) return cls_of(e2);
        if (take(e3, sig)) return cls_of(e3);
        return kNone;
    }
    template <class Sk>
    __device__ __forceinline__ void insert(uint32_t sig, uint32_t cls, const Sk& sk, ClassCache& cc, uint32_t P0,
                                           uint32_t P1, uint32_t P2, uint32_t P3) {
        const uint32_t e = (1u << 22) | ((cls & 0x3FFFu) << 8) | sig;
        uint32_t old;
        switch (victim) {
            case 0: old = e0; e0 = e; break;
            case 1: old = e1; e1 = e; break;
            case 2: old = e2; e2 = e; break;
            default: old = e3; e3 = e; break;
        }
        victim = (victim + 1u) & 3u;
        credit_ctx(sk, cc, P0, P1, P2, P3, cls_of(old), old >> 22);
    }
    template <class Sk>
    __device__ __forceinline__ void flush_all(const Sk& sk, ClassCache& cc, uint32_t P0, uint32_t P1, uint32_t P2,
                                              uint32_t P3) {
        credit_ctx(sk, cc, P0, P1, P2, P3, cls_of(e0), e0 >> 22);
        credit_ctx(sk, cc, P0, P1, P2, P3, cls_of(e1), e1 >> 22);
        credit_ctx(sk, cc, P0, P1, P2, P3, cls_of(e2), e2 >> 22);
        credit_ctx(sk, cc, P0, P1, P2, P3, cls_of(e3), e3 >> 22);
    }
};

// visited sets of one shape added to the workgroup's shape counters (LDS)
__device__ __forceinline__ void add_shape(unsigned long long* vis, uint32_t s, uint32_t v) {
    if (v) atomicAdd(&vis[s], (unsigned long long)v);
}

// Sub-items per (root, first layer-1 member) of a root with dhi higher neighbours and
// degree deg: the heavy roots' items are cut by the choice of the third member (every
// K-th candidate), so that no single lane carries a hub root's whole subtree.
__device__ __forceinline__ uint32_t item_split(uint32_t dhi, uint32_t deg, uint32_t div) {
    return min(64u, max(1u, (dhi * deg + div - 1u) / div));
}

// Every set of the sub-item k of K of the item (root r, first layer-1 member at entry apos
// of r's row).
template <class V, class Sk>
__device__ void five_item(const V& L, const uint16_t* __restrict__ table, const Sk& sk,
                          uint32_t r, uint32_t apos, uint32_t k, uint32_t K, unsigned long long* vis) {
    Members S{r, L.adj[apos] >> 2, 0u, 0u};
    const uint32_t code1 = pair_bits(0, 1, L.adj[apos] & 3u);
    const uint32_t P0 = L.perm[r], P1 = L.perm[S[1]];
    Cand c2;
    c2.start(L, S, 0u, apos, 1u);   // S[1]'s parent is S[0]; layer 1 starts at index 1
    uint32_t ord2 = 0;
    for (;;) {
        const uint32_t y2 = c2.next(L, S, 2u);
        if (y2 == kNone) break;
        if (ord2++ % K != k) continue;   // another sub-item's third member
        S.v2 = y2;
        const uint32_t par2 = c2.pi, pos2 = c2.j - 1u, ls2 = c2.phase ? 2u : 1u;
        const uint32_t code2 = code1 | pair_bits(0, 2, arc_of(L, S, 0, c2, y2)) | pair_bits(1, 2, arc_of(L, S, 1, c2, y2));
        const uint32_t P2 = L.perm[y2];
        ClassCache cc;
        Cand c3;
        c3.start(L, S, par2, pos2, ls2);
        for (;;) {
            const uint32_t y3 = c3.next(L, S, 3u);
            if (y3 == kNone) break;
            S.v3 = y3;
            const uint32_t par3 = c3.pi, pos3 = c3.j - 1u, ls3 = c3.phase ? 3u : ls2;
            const uint32_t code3 = code2 | pair_bits(0, 3, arc_of(L, S, 0, c3, y3)) |
                                   pair_bits(1, 3, arc_of(L, S, 1, c3, y3)) | pair_bits(2, 3, arc_of(L, S, 2, c3, y3));
            const uint32_t P3 = L.perm[y3];
            Cand c4;
            c4.start(L, S, par3, pos3, ls3);
            uint32_t same = 0, opened = 0;   // sets whose last member continues / opens a layer
            // The last member y4 of a set is credited once per set.  The fixed members are
            // credited per distinct signature of y4 -- its arc bits with S[0..3], which with
            // code3 fix the class -- through a 4-entry cache of (signature, count, class): a
            // context of a sparse graph holds ~8-25 sets with ~4-5 signatures, so this
            // removes most of the fixed members' credits and class reads.  An evicted entry
            // credits S[3], and S[0..2] directly or through the class cache (sink's choice).
            SigCache sc;
            for (;;) {
                const uint32_t y4 = c4.next(L, S, 4u);
                if (y4 == kNone) break;
                const uint32_t b0 = arc_of(L, S, 0, c4, y4), b1 = arc_of(L, S, 1, c4, y4),
                               b2 = arc_of(L, S, 2, c4, y4), b3 = arc_of(L, S, 3, c4, y4);
                const uint32_t sig = b0 | (b1 << 2) | (b2 << 4) | (b3 << 6);
                uint32_t cls = sc.hit(sig);
                if (cls == kNone) {
                    cls = table[code3 | pair_bits(0, 4, b0) | pair_bits(1, 4, b1) | pair_bits(2, 4, b2) |
                                pair_bits(3, 4, b3)];
                    sc.insert(sig, cls, sk, cc, P0, P1, P2, P3);
                }
                if (cls < (uint32_t)kClasses5) sk.add(L.perm[y4], cls, 1u);
                if (c4.phase) opened++; else same++;
            }
            sc.flush_all(sk, cc, P0, P1, P2, P3);
            // shape id: bit 2 = a new layer opens at member 2, bit 1 at member 3, bit 0 at member 4
            const uint32_t base = (ls2 == 2u ? 4u : 0u) | (ls3 == 3u ? 2u : 0u);
            add_shape(vis, base, same);
            add_shape(vis, base | 1u, opened);
        }
        if constexpr (Sk::kClassCache) cc.flush_all(sk, P0, P1, P2);
    }
}


struct FiveGraph {
    const uint32_t* off;           // n + 1 (rank space)
    const uint32_t* adj;           // entries: (nbr_rank << 2) | arc bits
    const int32_t* perm;           // rank -> original id
    unsigned long long* out;       // n x 9364, rows by original id (part 0)
    size_t copies_off;             // first element of its (parts - 1) x n x 9364 private blocks in the
                                   // call's copies (parts 1.., summed into out)
    unsigned long long* stats;     // 8 shape counters
    uint32_t n, entries;
    uint32_t parts;
};

struct FiveArgs {
    const FiveGraph* graphs;       // device array of num graphs, or nullptr: the graph `one`
    FiveGraph one;
    uint32_t num;
    const uint2* slots;            // (graph, part) in claim order, or nullptr: (0, s)
    uint32_t nslots;
    unsigned* cursors;             // num item cursors (one per graph), then the slot cursor
    unsigned long long* copies;    // private blocks of every graph's parts 1.., or nullptr
    const uint16_t* table;         // code -> class id
    const uint8_t* slot_of;        // class -> LDS counter slot or 0xFF (kClassPad entries)
    const uint16_t* slot_cls;      // LDS counter slot -> class (kTreeSlots5 entries)
    uint32_t split_div;            // sub-items of a root: ceil(d+ x deg / split_div), at most 64
};

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// zeroes every graph's counters and item cursor and the slot cursor (before k_five)
__global__ __launch_bounds__(256) void k_five_prep(FiveArgs A) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) A.cursors[A.num] = 0u;
    if (i >= A.num) return;
    const FiveGraph& G = A.graphs ? A.graphs[i] : A.one;
    for (int s = 0; s < kStatSlots; s++) G.stats[s] = 0ull;
    A.cursors[i] = 0u;
}

template <int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4))) void k_five(FiveArgs A) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_slot;
    __shared__ uint32_t part[BS];
    __shared__ unsigned long long s_vis[8];   // sets visited per shape by this part
    __shared__ uint8_t sSlotOf[kClassPad];
    __shared__ uint16_t sSlotCls[32];
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < (uint32_t)kClassPad; i += BS) sSlotOf[i] = A.slot_of[i];
    if (tid < kTreeSlots5) sSlotCls[tid] = A.slot_cls[tid];
    uint32_t loaded = kNone;
    FiveGraph G{};
    FiveLds L{};
    uint32_t* sSplit = nullptr;
    uint32_t* sHp = nullptr;
    uint32_t* sCnt = nullptr;
    for (;;) {
        if (tid == 0) s_slot = atomicAdd(A.cursors + A.num, 1u);
        __syncthreads();
        const uint32_t slot = s_slot;
        if (slot >= A.nslots) break;
        const uint2 sl = A.slots ? A.slots[slot] : make_uint2(0u, slot);
        if (sl.x != loaded) {   // the graph into LDS
            G = A.graphs ? A.graphs[sl.x] : A.one;
            const uint32_t n = G.n, E = G.entries, W = (n + 31u) >> 5;
            uint32_t* sOff = lds;
            sSplit = sOff + n + 1;
            sHp = sSplit + n;
            uint32_t* sPerm = sHp + n + 1;
            uint32_t* sAdj = sPerm + n;
            uint32_t* sMat = sAdj + E;
            sCnt = sMat + n * W;   // n x kTreeSlots5 counters of the part, rows by original id
            for (uint32_t i = tid; i < (n ? n + 1u : 0u); i += BS) sOff[i] = G.off[i];
            for (uint32_t i = tid; i < n; i += BS) sPerm[i] = (uint32_t)G.perm[i];
            for (uint32_t i = tid; i < E; i += BS) sAdj[i] = G.adj[i];
            for (uint32_t i = tid; i < n * W; i += BS) sMat[i] = 0u;
            __syncthreads();
            for (uint32_t u = tid; u < n; u += BS) {
                const uint32_t b = sOff[u], e = sOff[u + 1];
                uint32_t split = e;
                for (uint32_t x = b; x < e; x++) {
                    const uint32_t a = sAdj[x], v = a >> 2;
                    if (v > u && split == e) split = x;
                    sMat[u * W + (v >> 5)] |= 1u << (v & 31u);   // row u is this thread's
                }
                sSplit[u] = split;
                sHp[u] = (e - split) * item_split(e - split, e - b, A.split_div);
            }
            __syncthreads();
            // exclusive prefix of the higher-neighbour counts: item i of the graph is the
            // entry sSplit[r] + (i - sHp[r]) of the root r with sHp[r] <= i < sHp[r + 1]
            const uint32_t per = (n + BS - 1) / BS;
            const uint32_t lo = min(n, tid * per), hi = min(n, lo + per);
            uint32_t s = 0;
            for (uint32_t i = lo; i < hi; i++) s += sHp[i];
            part[tid] = s;
            __syncthreads();
            for (uint32_t o = 1; o < (uint32_t)BS; o <<= 1) {
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
            if (tid == 0) sHp[n] = part[BS - 1];
            L = FiveLds{sOff, sAdj, sMat, sPerm, W};
            loaded = sl.x;
        }
        // this part's output block: the caller's output or a private copy; zeroed here
        const size_t cells = (size_t)G.n * kClasses5;
        unsigned long long* dst = sl.y == 0 ? G.out : A.copies + G.copies_off + (size_t)(sl.y - 1u) * cells;
        if (((uintptr_t)dst & 15u) == 0) {   // 16-byte stores (9364 is even)
            ulonglong2* o = reinterpret_cast<ulonglong2*>(dst);
            for (size_t i = tid; i < cells / 2; i += BS) o[i] = make_ulonglong2(0ull, 0ull);
        } else {
            for (size_t i = tid; i < cells; i += BS) dst[i] = 0ull;
        }
        for (uint32_t i = tid; i < G.n * kTreeSlots5; i += BS) sCnt[i] = 0u;
        if (tid < 8) s_vis[tid] = 0ull;
        __syncthreads();
        for (;;) {
            const uint32_t i = atomicAdd(A.cursors + sl.x, 1u);   // items of the graph, shared by its parts
            if (i >= sHp[G.n]) break;
            uint32_t rlo = 0, rhi = G.n;   // root: last r with sHp[r] <= i
            while (rhi - rlo > 1) {
                const uint32_t mid = (rlo + rhi) >> 1;
                if (sHp[mid] <= i) rlo = mid; else rhi = mid;
            }
            const uint32_t K = item_split(L.off[rlo + 1] - sSplit[rlo], L.off[rlo + 1] - L.off[rlo], A.split_div);
            const uint32_t local = i - sHp[rlo];
            five_item(L, A.table, LdsSink{dst, sCnt, sSlotOf}, rlo, sSplit[rlo] + local / K, local % K, K, s_vis);
        }
        __syncthreads();
        // the part's LDS counters into its block (which only this workgroup writes)
        for (uint32_t i = tid; i < G.n * kTreeSlots5; i += BS) {
            const uint32_t x = sCnt[i];
            if (!x) continue;
            const uint32_t v = i / kTreeSlots5, sl2 = i - v * kTreeSlots5;
            bump<false>(&dst[(size_t)v * kClasses5 + sSlotCls[sl2]], (unsigned long long)x);
        }
        if (tid < 8 && s_vis[tid]) atomicAdd(&G.stats[tid], s_vis[tid]);
        __syncthreads();   // the part is done before the next claim rewrites s_slot
    }
}

// out += the private copies of one graph (blockIdx.x strides over its cells)
__device__ void five_reduce_one(const FiveGraph& G, const unsigned long long* copies) {
    const size_t cells = (size_t)G.n * kClasses5;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (((uintptr_t)G.out & 15u) == 0) {   // copies are 256-byte aligned and cells is even
        ulonglong2* o = reinterpret_cast<ulonglong2*>(G.out);
        const ulonglong2* c = reinterpret_cast<const ulonglong2*>(copies);
        const size_t h = cells / 2;
        for (size_t i = t0; i < h; i += stride) {
            ulonglong2 a = o[i];
            for (uint32_t p = 0; p + 1 < G.parts; p++) {
                const ulonglong2 b = c[p * h + i];
                a.x += b.x;
                a.y += b.y;
            }
            o[i] = a;
        }
    } else {
        for (size_t i = t0; i < cells; i += stride) {
            unsigned long long a = G.out[i];
            for (uint32_t p = 0; p + 1 < G.parts; p++) a += copies[p * cells + i];
            G.out[i] = a;
        }
    }
}


// out += the private copies, for every graph with more than one part (graphs strided
// over blockIdx.y)
__global__ __launch_bounds__(256) void k_five_reduce(FiveArgs A) {
    for (uint32_t gi = blockIdx.y; gi < A.num; gi += gridDim.y) {
        const FiveGraph& G = A.graphs ? A.graphs[gi] : A.one;
        if (G.parts > 1) five_reduce_one(G, A.copies + G.copies_off);
    }
}

// ----------------------------------------------------------------------------- graphs in device memory

struct FiveGlobalArgs {
    FiveGlobal L;
    const uint32_t* split;
    const unsigned long long* hp;   // n + 1: items (sub-items) before each root
    uint32_t n;
    unsigned long long total;
    unsigned long long* out;        // n x 9364, shared by every workgroup
    unsigned long long* stats;
    unsigned long long* cursor;     // item cursor, zeroed before the launch
    const uint16_t* table;
    uint32_t split_div;
};

// items of each root: d+(r) x K(r); cnt[n] = 0 so that an exclusive scan over n + 1 gives the total
__global__ void k_five_counts(const uint32_t* off, const uint32_t* split, uint32_t n, uint32_t div,
                              unsigned long long* cnt) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    if (r == n) {
        cnt[n] = 0ull;
        return;
    }
    const uint32_t dhi = off[r + 1] - split[r];
    cnt[r] = (unsigned long long)dhi * item_split(dhi, off[r + 1] - off[r], div);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_five_global(FiveGlobalArgs A) {
    __shared__ unsigned long long s_vis[8];
    const uint32_t tid = threadIdx.x;
    if (tid < 8) s_vis[tid] = 0ull;
    __syncthreads();
    for (;;) {
        const unsigned long long i = atomicAdd(A.cursor, 1ull);
        if (i >= A.total) break;
        uint32_t lo = 0, hi = A.n;   // root: last r with hp[r] <= i
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (A.hp[mid] <= i) lo = mid; else hi = mid;
        }
        const uint32_t r = lo, e = A.L.off[r + 1], sp = A.split[r];
        const uint32_t K = item_split(e - sp, e - A.L.off[r], A.split_div);
        const uint32_t local = (uint32_t)(i - A.hp[r]);
        five_item(A.L, A.table, GlobalSink<true>{A.out}, r, sp + local / K, local % K, K, s_vis);
    }
    __syncthreads();
    if (tid < 8 && s_vis[tid]) atomicAdd(&A.stats[tid], s_vis[tid]);
}

// Per-device LDS counter slots: the single-arc tree classes found from each class's
// minimal index (four joined pairs, none reciprocal), in ascending class id.
struct FiveSlots {
    uint8_t* slot_of = nullptr;    // kClassPad entries: class -> slot or 0xFF
    uint16_t* slot_cls = nullptr;  // 32 entries: slot -> class
};
std::mutex g_slots_mu;
std::map<int, FiveSlots> g_slots;
const FiveSlots& five_slots() {
    int dev = 0;
    VDMC_HIP(hipGetDevice(&dev));
    const ClassTable5& t = class_table5();
    std::lock_guard<std::mutex> lock(g_slots_mu);
    auto it = g_slots.find(dev);
    if (it != g_slots.end()) return it->second;
    std::vector<uint8_t> slot_of(kClassPad, 0xFF);
    std::vector<uint16_t> slot_cls(32, 0);
    uint32_t k = 0;
    for (uint32_t c = 0; c < (uint32_t)kClasses5; c++) {
        const uint32_t code = t.codes[c];
        uint32_t joined = 0, recip = 0;
        for (uint32_t i = 0; i < 5; i++)
            for (uint32_t j = i + 1; j < 5; j++) {
                const uint32_t x = (code >> shift5(i, j)) & 1u, y = (code >> shift5(j, i)) & 1u;
                joined += x | y;
                recip += x & y;
            }
        if (joined == 4u && recip == 0u) {
            VDMC_REQUIRE(k < kTreeSlots5, VDMC_ERR_DEVICE, "more single-arc 5-vertex tree classes than slots");
            slot_of[c] = (uint8_t)k;
            slot_cls[k] = (uint16_t)c;
            k++;
        }
    }
    VDMC_REQUIRE(k == kTreeSlots5, VDMC_ERR_DEVICE,
                 "expected 27 single-arc 5-vertex tree classes, found " + std::to_string(k));
    FiveSlots fs;
    VDMC_HIP(hipMalloc(&fs.slot_of, kClassPad));
    VDMC_HIP(hipMalloc(&fs.slot_cls, 32 * sizeof(uint16_t)));
    VDMC_HIP(hipMemcpy(fs.slot_of, slot_of.data(), kClassPad, hipMemcpyHostToDevice));
    VDMC_HIP(hipMemcpy(fs.slot_cls, slot_cls.data(), 32 * sizeof(uint16_t), hipMemcpyHostToDevice));
    return g_slots.emplace(dev, fs).first->second;   // kept for the life of the process
}

// 1-bit adjacency matrix (rank space) of a graph counted in device memory: row u set by
// thread u from its CSR row (zeroed before)
__global__ __launch_bounds__(256) void k_five_mat(const uint32_t* off, const uint32_t* adj, uint32_t n, uint32_t W,
                                                   uint32_t* mat) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    uint32_t* row = mat + (size_t)u * W;
    for (uint32_t x = off[u]; x < off[u + 1]; x++) {
        const uint32_t v = adj[x] >> 2;
        row[v >> 5] |= 1u << (v & 31u);
    }
}

// the matrices, kept with their graphs until free_five
std::mutex g_mat_mu;
std::map<const vdmc_graph_s*, uint32_t*> g_five_mat;

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

// Launches prep, the search and (when some graph has several parts) the reduction.
void launch_five(const FiveArgs& a, size_t lds, uint32_t num_graphs, bool reduce, hipStream_t st) {
    hipLaunchKernelGGL(k_five_prep, dim3((std::max<uint32_t>(num_graphs, 1) + 255) / 256), dim3(256), 0, st, a);
    VDMC_HIP(hipGetLastError());
    // 16 waves per compute unit (the register budget): one 1024-thread workgroup when the
    // LDS admits one, two of 512 threads when it admits two or three, else four of 256
    const int fit = std::max(1, (int)(163840 / (lds + kFiveStaticLds)));
    const int bs = fit == 1 ? 1024 : (fit <= 3 ? 512 : 256);
    const int per_cu = 1024 / bs;
    void (*kern)(FiveArgs) = bs == 1024 ? k_five<1024> : (bs == 512 ? k_five<512> : k_five<256>);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(a.nslots, (int64_t)ncu() * per_cu));
    VDMC_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(bs), lds, st, a);
    VDMC_HIP(hipGetLastError());
    if (reduce) {
        hipLaunchKernelGGL(k_five_reduce, dim3(256, std::min<uint32_t>(std::max<uint32_t>(num_graphs, 1), 65535u)),
                           dim3(256), 0, st, a);
        VDMC_HIP(hipGetLastError());
    }
}

// estimated work of a graph: sum over vertices of d^4 (d = degree in G_U)
double work_estimate(const vdmc_graph_s* g) {
    if (g->n == 0) return 0.0;
    std::vector<uint32_t> off((size_t)g->n + 1);
    VDMC_HIP(hipMemcpy(off.data(), g->off, off.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
    double w = 0.0;
    for (int64_t v = 0; v < g->n; v++) {
        const double d = (double)(off[v + 1] - off[v]);
        w += d * d * d * d;
    }
    return w;
}

size_t block_bytes(const vdmc_graph_s* g) { return (size_t)g->n * kClasses5 * sizeof(unsigned long long); }

FiveGraph view_of(const vdmc_graph_s* g, uint64_t* out) {
    FiveGraph v{};
    v.off = g->off;
    v.adj = g->adj;
    v.perm = g->perm;
    v.out = (unsigned long long*)out;
    v.stats = g->stats;
    v.n = (uint32_t)g->n;
    v.entries = (uint32_t)(2 * g->pairs);
    v.parts = 1;
    return v;
}

// cached descriptors of batched 5-vertex launches, by (graphs, outputs).  Only the
// read-only graph views and the slot order are kept; the cursors and the private copies
// are taken from the stream-ordered pool for each call.
struct FivePlan {
    std::vector<vdmc_graph_s*> graphs;
    std::vector<uint64_t*> outs;
    FiveGraph* d_graphs = nullptr;
    uint2* d_slots = nullptr;
    uint32_t nslots = 0;
    size_t scratch = 0;   // bytes of private copies of parts 1..
    bool reduce = false;
    size_t lds = 0;
    ~FivePlan() {
        (void)hipFree(d_graphs);
        (void)hipFree(d_slots);
    }
};
std::mutex g_five_mu;
std::vector<FivePlan*> g_five_plans;

// The private copies come from the device's default stream-ordered pool.  It keeps up to one
// batched launch's budget after the frees, so repeated counts reuse the same pages instead
// of mapping them anew; what lies above that goes back to the device at synchronisation.
std::mutex g_pool_mu;
uint64_t g_pool_set = 0;   // devices whose pool threshold is set (bit per device id < 64)
void keep_scratch_pool() {
    int dev = 0;
    VDMC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (dev < 64 && (g_pool_set >> dev) & 1u) return;
    hipMemPool_t pool;
    VDMC_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
    uint64_t keep = kBatchScratchBudget + (size_t(256) << 20);
    VDMC_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    if (dev < 64) g_pool_set |= uint64_t(1) << dev;
}

}  // namespace

size_t five_lds_bytes(int64_t n, int64_t entries) {
    const int64_t W = (n + 31) / 32;
    return (size_t)(4 * ((n + 1) + n + (n + 1) + n + entries + n * W + n * (int64_t)kTreeSlots5));
}

bool five_eligible(int64_t n, int64_t entries) {
    return n <= kFiveMaxN && five_lds_bytes(n, entries) <= kFiveLdsBudget;
}

namespace {

// 5-vertex counts of a graph that LDS does not hold: every workgroup of the grid takes
// sub-items from one cursor and credits the caller's output with device-scope atomics.
// Needs the graph's edge hash and its item prefix (both built at the first such count
// and kept with the graph).
void launch_count5_global(vdmc_graph_s* g, uint64_t* out, hipStream_t st) {
    const ClassTable5& t = class_table5();
    launch_fill_u64((uint64_t*)g->stats, kStatSlots, 0, st);
    if (g->n == 0) return;
    launch_fill_u64(out, (size_t)g->n * kClasses5, 0, st);
    if (g->pairs == 0) return;
    ensure_edge_hash(g, st);
    if (!g->five_hp) {
        const uint32_t n = (uint32_t)g->n;
        unsigned long long *cnt = nullptr, *hp = nullptr;
        VDMC_HIP(hipMalloc(&hp, sizeof(unsigned long long) * (n + 2)));   // prefix, then the item cursor
        VDMC_HIP(hipMalloc(&cnt, sizeof(unsigned long long) * (n + 1)));
        struct Free {
            void* p;
            ~Free() { (void)hipFree(p); }
        } fcnt{cnt};
        hipLaunchKernelGGL(k_five_counts, dim3((n + 256) / 256), dim3(256), 0, st, g->off, g->split, n, kSplitDiv, cnt);
        VDMC_HIP(hipGetLastError());
        size_t tmp_bytes = 0;
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt, hp, n + 1, st));
        void* tmp = nullptr;
        VDMC_HIP(hipMalloc(&tmp, tmp_bytes ? tmp_bytes : 16));
        struct Free2 {
            void* p;
            ~Free2() { (void)hipFree(p); }
        } ftmp{tmp};
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, hp, n + 1, st));
        unsigned long long total = 0;
        VDMC_HIP(hipMemcpyAsync(&total, hp + n, sizeof(total), hipMemcpyDeviceToHost, st));
        VDMC_HIP(hipStreamSynchronize(st));
        g->five_hp = hp;
        g->five_items = total;
    }
    const uint32_t W = (uint32_t)((g->n + 31) / 32);
    uint32_t* mat = nullptr;
    if (g->n <= kFiveMatMaxN) {
        std::lock_guard<std::mutex> lock(g_mat_mu);
        auto it = g_five_mat.find(g);
        if (it != g_five_mat.end()) {
            mat = it->second;
        } else {
            const size_t words = ((size_t)g->n * W + 1) & ~(size_t)1;   // even: zeroed as u64
            VDMC_HIP(hipMalloc(&mat, words * sizeof(uint32_t)));
            launch_fill_u64(reinterpret_cast<uint64_t*>(mat), words / 2, 0, st);
            hipLaunchKernelGGL(k_five_mat, dim3((uint32_t)((g->n + 255) / 256)), dim3(256), 0, st, g->off, g->adj,
                               (uint32_t)g->n, W, mat);
            VDMC_HIP(hipGetLastError());
            g_five_mat[g] = mat;
        }
    }
    unsigned long long* cursor = g->five_hp + g->n + 1;
    launch_fill_u64((uint64_t*)cursor, 1, 0, st);
    FiveGlobalArgs a{};
    a.L = FiveGlobal{g->off, g->adj, reinterpret_cast<const uint32_t*>(g->perm), g->ehash, g->ehash_bits, mat, W};
    a.split = g->split;
    a.hp = g->five_hp;
    a.n = (uint32_t)g->n;
    a.total = g->five_items;
    a.out = (unsigned long long*)out;
    a.stats = g->stats;
    a.cursor = cursor;
    a.table = t.table;
    a.split_div = kSplitDiv;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)ncu() * 4,
                                                                           (int64_t)((g->five_items + 255) / 256)));
    hipLaunchKernelGGL(k_five_global<256>, dim3(grid), dim3(256), 0, st, a);
    VDMC_HIP(hipGetLastError());
}

}  // namespace

void launch_count5(vdmc_graph_s* g, uint64_t* out, hipStream_t st) {
    g->timed_light = g->timed_hub = false;
    if (!five_eligible(g->n, 2 * g->pairs)) {
        launch_count5_global(g, out, st);
        return;
    }
    const ClassTable5& t = class_table5();
    // parts: one per 32 items, at most two per compute unit, copies within the budget.  The
    // cursors and the copies come from the stream-ordered pool and go back to it after the
    // launches, so concurrent counts on other streams never share them.
    const size_t bb = std::max<size_t>(block_bytes(g), 16);
    const uint32_t by_items = std::max<uint32_t>(1u, (uint32_t)(g->pairs / 32));
    const uint32_t by_mem = (uint32_t)std::min<size_t>(kMaxParts, 1 + kSingleScratchBudget / bb);
    const uint32_t parts = std::max<uint32_t>(1u, std::min<uint32_t>({by_items, by_mem, (uint32_t)(2 * ncu())}));
    const size_t bytes = 256 + (size_t)(parts - 1) * bb;
    keep_scratch_pool();
    void* buf = nullptr;
    VDMC_HIP(hipMallocAsync(&buf, bytes, st));
    FiveArgs a{};
    a.graphs = nullptr;
    a.one = view_of(g, out);
    a.one.copies_off = 0;
    a.one.parts = parts;
    a.num = 1;
    a.slots = nullptr;
    a.nslots = g->n > 0 ? parts : 0u;
    a.cursors = static_cast<unsigned*>(buf);
    a.copies = parts > 1 ? reinterpret_cast<unsigned long long*>(static_cast<char*>(buf) + 256) : nullptr;
    a.table = t.table;
    const FiveSlots& fs = five_slots();
    a.slot_of = fs.slot_of;
    a.slot_cls = fs.slot_cls;
    a.split_div = kSplitDiv;
    try {
        launch_five(a, five_lds_bytes(g->n, 2 * g->pairs), 1, parts > 1, st);
    } catch (...) {
        (void)hipFreeAsync(buf, st);
        throw;
    }
    VDMC_HIP(hipFreeAsync(buf, st));
}

void free_five(vdmc_graph_s* g) {
    (void)hipFree(g->five_hp);
    g->five_hp = nullptr;
    g->five_items = 0;
    std::lock_guard<std::mutex> lock(g_mat_mu);
    auto it = g_five_mat.find(g);
    if (it != g_five_mat.end()) {
        (void)hipFree(it->second);
        g_five_mat.erase(it);
    }
}

void count5_batch_lds(std::vector<vdmc_graph_s*>& gs, std::vector<uint64_t*>& outv, hipStream_t st) {
    const int32_t num = (int32_t)gs.size();
    if (num == 0) return;
    uint64_t* const* outs = outv.data();
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
            std::vector<double> work(num);
            double total = 0.0;
            for (int i = 0; i < num; i++) {
                work[i] = work_estimate(gs[i]);
                total += work[i];
            }
            // parts per graph: about kPartsPerCu per compute unit over the batch, more for the
            // heavy graphs; coarser while the private copies exceed the budget
            std::vector<uint32_t> parts(num, 1);
            double unit = total / std::max(1.0, (double)kPartsPerCu * ncu());
            for (int round = 0; round < 32; round++) {
                size_t scratch = 0;
                for (int i = 0; i < num; i++) {
                    const double want = unit > 0 ? std::ceil(work[i] / unit) : 1.0;
                    parts[i] = (uint32_t)std::max(1.0, std::min<double>(kMaxParts, want));
                    if (gs[i]->pairs < 64) parts[i] = 1;
                    scratch += (size_t)(parts[i] - 1) * block_bytes(gs[i]);
                }
                if (scratch <= kBatchScratchBudget) break;
                unit *= 1.5;
            }
            std::vector<int> order(num);
            for (int i = 0; i < num; i++) order[i] = i;
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
            std::vector<FiveGraph> views(num);
            std::vector<uint2> slots;
            size_t scratch = 0;
            for (int i = 0; i < num; i++) {
                views[i] = view_of(gs[i], outs[i]);
                views[i].parts = parts[i];
                scratch += (size_t)(parts[i] - 1) * block_bytes(gs[i]);
                plan->lds = std::max(plan->lds, five_lds_bytes(gs[i]->n, 2 * gs[i]->pairs));
                plan->reduce |= parts[i] > 1;
            }
            for (int i : order)
                for (uint32_t p = 0; p < parts[i]; p++) slots.push_back(make_uint2((unsigned)i, p));
            plan->nslots = (uint32_t)slots.size();
            plan->scratch = scratch;
            size_t at = 0;
            for (int i = 0; i < num; i++) {
                views[i].copies_off = at / sizeof(unsigned long long);
                at += (size_t)(parts[i] - 1) * block_bytes(gs[i]);
            }
            VDMC_HIP(hipMalloc(&plan->d_graphs, sizeof(FiveGraph) * std::max(num, 1)));
            VDMC_HIP(hipMalloc(&plan->d_slots, sizeof(uint2) * std::max<size_t>(slots.size(), 1)));
            VDMC_HIP(hipMemcpy(plan->d_graphs, views.data(), sizeof(FiveGraph) * num, hipMemcpyHostToDevice));
            if (!slots.empty())
                VDMC_HIP(hipMemcpy(plan->d_slots, slots.data(), sizeof(uint2) * slots.size(), hipMemcpyHostToDevice));
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
    for (auto* g : gs) g->timed_light = g->timed_hub = false;
    FiveArgs a{};
    a.graphs = plan->d_graphs;
    a.num = (uint32_t)num;
    a.slots = plan->d_slots;
    a.nslots = plan->nslots;
    a.table = t.table;
    const FiveSlots& fs = five_slots();
    a.slot_of = fs.slot_of;
    a.slot_cls = fs.slot_cls;
    a.split_div = kSplitDiv;
    // cursors and copies for this call only: concurrent counts of other batches on other
    // streams never share them, and no cached plan holds copies between calls
    const size_t head = (sizeof(unsigned) * ((size_t)num + 1) + 255) / 256 * 256;
    keep_scratch_pool();
    void* buf = nullptr;
    VDMC_HIP(hipMallocAsync(&buf, head + plan->scratch, st));
    a.cursors = static_cast<unsigned*>(buf);
    a.copies = plan->scratch ? reinterpret_cast<unsigned long long*>(static_cast<char*>(buf) + head) : nullptr;
    try {
        launch_five(a, plan->lds, (uint32_t)num, plan->reduce, st);
    } catch (...) {
        (void)hipFreeAsync(buf, st);
        throw;
    }
    VDMC_HIP(hipFreeAsync(buf, st));
}

void count5_batch(const vdmc_graph_s* const* gs_in, int32_t num, uint64_t* const* outs_in, hipStream_t st) {
    // graphs that LDS holds go into one batched launch; the others are counted one by one
    // in device memory after it
    std::vector<vdmc_graph_s*> gs;
    std::vector<uint64_t*> outv;
    for (int i = 0; i < num; i++) {
        vdmc_graph_s* g = const_cast<vdmc_graph_s*>(gs_in[i]);
        if (five_eligible(g->n, 2 * g->pairs)) {
            gs.push_back(g);
            outv.push_back(outs_in[i]);
        }
    }
    count5_batch_lds(gs, outv, st);
    for (int i = 0; i < num; i++) {
        vdmc_graph_s* g = const_cast<vdmc_graph_s*>(gs_in[i]);
        if (!five_eligible(g->n, 2 * g->pairs)) {
            GraphUse use(g, st);
            launch_count5_global(g, outs_in[i], st);
        }
    }
}

void invalidate_five_plans(vdmc_graph_s* g) {
    {
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
}

}  // namespace vdmc

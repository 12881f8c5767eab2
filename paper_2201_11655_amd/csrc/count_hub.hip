// Hub-root motif kernels: roots with many higher neighbours.
//
// The sets are those of the per-set kernel (count.hip): every connected k-set once,
// from its lowest-rank vertex r (Lemma 1), along the BFS shapes of Lemma 2 under the
// rules of Lemmas 3-4.  Every set is visited by one lane, which assembles its motif
// index from the arc bits (Sec. 4.1), reads its class from the table in LDS and credits
// the class to each of the set's vertices (Sec. 4.2).  What is specific to hub roots is
// where the work and the counters live:
//
//   * one workgroup (16 waves) per root; N+(r) (the "slots", depth-1 candidates) is
//     staged in LDS with a hash from rank to slot; each slot's local neighbours (other
//     slots) become a short list, and each depth-2 entry (slot x, vertex c above r and
//     outside N+(r)) goes into a hash keyed by c whose buckets list c's parents
//     A(c) = N(c) n N+(r), so that the depth-1 rule of (2,1,0) (c hangs under its
//     lowest-rank parent) is a test on A(c);
//   * within one wave step the lanes take sets that share all members but one:
//     (3,0,0) fixes a < b and lanes take c; (2,1,0) fixes the depth-2 vertex c and a
//     parent x and lanes take the second depth-1 vertex y; pair codes come from per-wave
//     2-bit code rows built from the local lists;
//   * the members fixed for the wave step are credited once per class present in the
//     step (ballots group the lanes by class); the lane's own member, a slot, is
//     credited with one LDS atomic to per-slot counters of the tree classes that the
//     shape produces when it has no extra pair (the 10 3-star classes for (3,0,0), the
//     15 4-path classes for (2,1,0)); sets of any other class go straight to the
//     output;
//   * (1,2,0) and (1,1,1) sets hang below one slot a: a's depth-2 children L_a (entries
//     of a's row above r outside N+(r)) get per-child counters; a wave walks a child
//     c's row once, which gives both its arcs to the later children (for the (1,2,0)
//     pairs that follow) and the end vertices e of the (1,1,1) paths r - a - c - e (e
//     not adjacent to r nor to a: the Lemma-4 rule); e, a vertex anywhere in the graph,
//     is credited with one atomic to the output.  Slots whose row above r is short are
//     taken one wave each at the end of the hub kernel; long ones go to a second
//     kernel, one workgroup per slot.
// Counters are flushed to the output (rows by original id) once per phase.
#include "motif_device.h"
#include "vdmc_internal.h"

#include <hipcub/hipcub.hpp>

namespace vdmc {
namespace {

constexpr int HT = 1024;                   // threads per hub workgroup
constexpr int NW = HT / 64;                // waves per workgroup
constexpr uint32_t DMAX = kHubMaxDegree;   // largest |N+(r)| (and largest degree) on the hub path
constexpr uint32_t CW = DMAX / 16;         // words of a 2-bit code row over the slots
constexpr uint32_t SHASH = 4096;           // slot hash entries (u16 slot + 1), load <= 1/2
constexpr uint32_t SHORT = 64;             // slots whose row above r has at most this many entries: one wave each
constexpr uint32_t NSTAR = 10, NPATH = 15, NTREE = kCompact4;
constexpr uint32_t CH_HASH = 128;          // per-wave child hash (short slots)

struct HubArgs {
    const uint32_t* off;
    const uint32_t* adj;
    const uint32_t* split;
    const int32_t* perm;
    const uint32_t* hubs;        // hub roots, largest work first
    const uint32_t* hub_s2;      // per hub root: entries of its slots' rows above r
    uint32_t nhub;
    unsigned* cursor;            // [0] root cursor, [1] long-slot tasks, [2] long-slot cursor
    const uint8_t* t3;
    const uint8_t* t4;
    const uint8_t* maps;         // [0,256) class -> star slot, [256,512) class -> path slot,
                                 // [512,768) class -> tree slot (0xFF = none)
    const uint8_t* star_cls;     // star slot -> class
    const uint8_t* path_cls;     // path slot -> class
    const uint8_t* tree_cls;     // tree slot -> class
    unsigned long long* out3;
    unsigned long long* out4;
    unsigned long long* stats;
    int k3, k4;
    uint32_t rank_lo, rank_hi;   // only roots with rank in [rank_lo, rank_hi)
    uint32_t* scratch;           // per workgroup: locoff | locnbr | nodes (u64) | groups | keys | heads
    size_t wg_words;
    uint32_t s2cap, tcap;
    uint2* tasks;                // long-slot tasks: (hub index, the slot's entry in r's row)
    uint32_t task_cap;
    uint32_t split_roots;        // the first split_roots hub roots (the heaviest) ...
    uint32_t shares;             // ... are each taken by this many workgroups (see k_hub)
};

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }
__device__ __forceinline__ uint32_t wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ void gadd(unsigned long long* out, const int32_t* perm, uint32_t C, uint32_t v,
                                     uint32_t cls, unsigned long long cnt) {
    atomicAdd(&out[(size_t)perm[v] * C + cls], cnt);
}

// f(cls, count) once per distinct class among the lanes that reach it with `active`
template <class F>
__device__ __forceinline__ void by_class(uint32_t cls, bool active, F&& f) {
    unsigned long long m = __ballot(active);
    while (m) {
        const uint32_t leader = (uint32_t)(__ffsll((long long)m) - 1);
        const uint32_t k0 = (uint32_t)__shfl((int)cls, (int)leader, 64);
        const unsigned long long same = __ballot(active && cls == k0) & m;
        if (lane_id() == leader) f(k0, (uint32_t)__popcll(same));
        m &= ~same;
    }
}

__device__ __forceinline__ uint32_t code_at(const uint32_t* row, uint32_t i) {
    return (row[i >> 4] >> ((i & 15u) << 1)) & 3u;
}

__device__ __forceinline__ uint32_t shash(uint32_t x) { return (x * 2654435761u) >> 20; }   // 12 bits

// slot of rank x in the LDS slot hash (u16 slot + 1 per entry), or -1
__device__ __forceinline__ int slot_find(const uint16_t* H, const uint32_t* P, uint32_t x) {
    for (uint32_t h = shash(x);; h = (h + 1u) & (SHASH - 1u)) {
        const uint32_t s = H[h];
        if (s == 0u) return -1;
        if ((P[s - 1u] >> 2) == x) return (int)(s - 1u);
    }
}

// insert slot i (rank x) into the slot hash; 16-bit entries updated through their word
__device__ __forceinline__ void slot_insert(uint16_t* H, uint32_t x, uint32_t i) {
    for (uint32_t h = shash(x);; h = (h + 1u) & (SHASH - 1u)) {
        uint32_t* w = (uint32_t*)&H[h & ~1u];
        const uint32_t sh = (h & 1u) << 4;
        uint32_t old = *w;
        while (((old >> sh) & 0xFFFFu) == 0u) {
            const uint32_t got = atomicCAS(w, old, old | ((i + 1u) << sh));
            if (got == old) return;
            old = got;
        }
    }
}

// one dynamic task index per wave (LDS counter)
__device__ __forceinline__ uint32_t wave_task(uint32_t* ctr) {
    uint32_t t = 0;
    if (lane_id() == 0) t = atomicAdd(ctr, 1u);
    return (uint32_t)__shfl((int)t, 0, 64);
}

__device__ __forceinline__ uint32_t first_above(const uint32_t* adj, uint32_t lo, uint32_t hi, uint32_t r) {
    return lower_bound_rank(adj, lo, hi, r + 1u);
}

// exclusive scan of a[0..len) in place (any memory the workgroup sees), returns the total;
// part: HT words of LDS
__device__ uint32_t block_scan(uint32_t* a, uint32_t len, uint32_t* part) {
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (len + HT - 1) / HT;
    const uint32_t lo = min(len, tid * per), hi = min(len, lo + per);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; i++) s += a[i];
    part[tid] = s;
    __syncthreads();
    for (uint32_t off = 1; off < HT; off <<= 1) {
        const uint32_t v = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = part[tid] - s;
    for (uint32_t i = lo; i < hi; i++) {
        const uint32_t x = a[i];
        a[i] = run;
        run += x;
    }
    const uint32_t total = part[HT - 1];
    __syncthreads();
    return total;
}

// ----------------------------------------------------------------------------- LDS

constexpr uint32_t U_WORDS = 35072;   // the phase-dependent region (137 KiB)

struct HubLds {
    uint32_t P[DMAX];                  // slots: (rank << 2) | arc bits r -> slot
    uint16_t locn[DMAX];               // local neighbours per slot
    unsigned long long root3[kClasses3];
    unsigned long long root4[kClasses4];
    uint8_t t4[4096];
    uint8_t t3[64];
    uint8_t maps[768];
    uint32_t ctr[8];
    uint32_t U[U_WORDS];
};

// the per-wave 2-bit code row over the slots from slot x's local list
__device__ __forceinline__ void build_row(uint32_t* row, const uint32_t* locnbr, uint32_t base, uint32_t cnt) {
    const uint32_t lane = lane_id();
    for (uint32_t i = lane; i < CW; i += 64) row[i] = 0u;
    __threadfence_block();
    for (uint32_t i = lane; i < cnt; i += 64) {
        const uint32_t e = locnbr[base + i];
        atomicOr(&row[(e >> 2) >> 4], (e & 3u) << (((e >> 2) & 15u) << 1));
    }
    __threadfence_block();
}

// ----------------------------------------------------------------------------- hub kernel

__global__ __launch_bounds__(HT) void k_hub(HubArgs A) {
    __shared__ HubLds L;
    __shared__ uint32_t sRoot;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wid = wave_id();
    for (uint32_t i = tid; i < 4096; i += HT) L.t4[i] = A.t4[i];
    for (uint32_t i = tid; i < 64; i += HT) L.t3[i] = A.t3[i];
    for (uint32_t i = tid; i < 768; i += HT) L.maps[i] = A.maps[i];
    const uint8_t* star_of = L.maps;
    const uint8_t* path_of = L.maps + 256;
    const uint8_t* tree_of = L.maps + 512;
    uint32_t* S = A.scratch + (size_t)blockIdx.x * A.wg_words;
    uint32_t* locoff = S;                                        // DMAX + 2
    uint32_t* locnbr = locoff + DMAX + 2;                        // s2cap (+ 1 to keep nodes 8-byte aligned)
    unsigned long long* nodes = (unsigned long long*)(locnbr + A.s2cap + (A.s2cap & 1u));   // s2cap
    uint32_t* groups = (uint32_t*)(nodes + A.s2cap);             // s2cap
    uint32_t* keys = groups + A.s2cap;                           // tcap
    uint32_t* heads = keys + A.tcap;                             // tcap
    unsigned long long shp[kShapes] = {0, 0, 0, 0, 0, 0};

    // The heaviest hub roots (the first A.split_roots of the queue) are each taken by
    // A.shares workgroups, so that no single root's workgroup is the critical path.  Each
    // stages the whole root (its slot hash, local lists and depth-2 buckets live in its own
    // scratch) and does the share of every phase's tasks that is its own: slots x with
    // x % G == share (phases B-C4, F) and depth-2 vertices c with c % G == share (phase D,
    // whose group order differs between workgroups).  Its counters are partial sums,
    // flushed with atomics like a whole root's.  Later roots are taken whole (G = 1).
    const uint32_t split_tasks = A.split_roots * A.shares;
    for (;;) {
        __syncthreads();
        if (tid == 0) sRoot = atomicAdd(&A.cursor[0], 1u);
        __syncthreads();
        const uint32_t vi = sRoot;
        const uint32_t G = vi < split_tasks ? A.shares : 1u;
        const uint32_t hi_idx = vi < split_tasks ? vi / G : A.split_roots + (vi - split_tasks);
        const uint32_t share = vi < split_tasks ? vi - hi_idx * G : 0u;
        if (hi_idx >= A.nhub) break;
        const uint32_t r = A.hubs[hi_idx];
        if (r < A.rank_lo || r >= A.rank_hi) continue;   // uniform over the workgroup
        const uint32_t s0 = A.split[r];
        const uint32_t D = A.off[r + 1] - s0;
        uint32_t tbits = 6;
        while ((1u << tbits) < 2u * A.hub_s2[hi_idx] + 64u) tbits++;
        const uint32_t TS = 1u << tbits;
        // ---- phase A: stage the slots, the lengths of their rows above r, clear counters
        uint16_t* H = (uint16_t*)L.U;   // slot hash (phases A-B)
        // Slots ordered by their arc code to r, by rank within a code.  Any fixed order of
        // N+(r) enumerates each set once ((3,0,0) takes a < b < c, (2,1,0) hangs c under
        // its lowest parent); this one gives the lanes of a step over consecutive slots
        // the same code to r, so that sets without extra pairs share their class.
        if (wid == 0) {
            const unsigned long long below = (1ull << lane) - 1ull;
            uint32_t n1 = 0, n2 = 0;
            for (uint32_t q0 = 0; q0 < D; q0 += 64) {
                const uint32_t k = q0 + lane < D ? (A.adj[s0 + q0 + lane] & 3u) : 0u;
                n1 += (uint32_t)__popcll(__ballot(k == 1u));
                n2 += (uint32_t)__popcll(__ballot(k == 2u));
            }
            uint32_t o[4] = {0u, 0u, n1, n1 + n2};
            for (uint32_t q0 = 0; q0 < D; q0 += 64) {
                const bool in = q0 + lane < D;
                const uint32_t e = in ? A.adj[s0 + q0 + lane] : 0u, k = e & 3u;
                const unsigned long long m1 = __ballot(in && k == 1u), m2 = __ballot(in && k == 2u),
                                         m3 = __ballot(in && k == 3u);
                const unsigned long long mk = k == 1u ? m1 : (k == 2u ? m2 : m3);
                if (in) L.P[o[k] + (uint32_t)__popcll(mk & below)] = e;
                o[1] += (uint32_t)__popcll(m1);
                o[2] += (uint32_t)__popcll(m2);
                o[3] += (uint32_t)__popcll(m3);
            }
        }
        for (uint32_t i = tid; i < SHASH / 2; i += HT) L.U[i] = 0u;
        for (uint32_t i = tid; i < kClasses3; i += HT) L.root3[i] = 0ull;
        for (uint32_t i = tid; i < kClasses4; i += HT) L.root4[i] = 0ull;
        if (tid < 8) L.ctr[tid] = 0u;
        if (A.k4)
            for (uint32_t i = tid; i < TS; i += HT) {
                keys[i] = 0u;
                heads[i] = 0u;
            }
        __syncthreads();
        for (uint32_t i = tid; i < D; i += HT) {
            const uint32_t x = L.P[i] >> 2;
            locoff[i] = A.off[x + 1] - first_above(A.adj, A.off[x], A.off[x + 1], r);
            slot_insert(H, x, i);
        }
        if (tid == 0) locoff[D] = 0u;
        __syncthreads();
        uint32_t* part = L.U + SHASH / 2;   // HT words after the slot hash
        block_scan(locoff, D + 1, part);
        // ---- phase B: rows of the slots: local lists, depth-2 entries, k = 3 (1,2)
        uint32_t* R3 = L.U + SHASH / 2 + HT;   // D x 13 k = 3 counters of the slots
        if (A.k3)
            for (uint32_t i = tid; i < D * kClasses3; i += HT) R3[i] = 0u;
        __syncthreads();
        for (;;) {
            const uint32_t x = wave_task(&L.ctr[0]);
            if (x >= D) break;
            const bool own = x % G == share;   // staging for every slot, credits for its own
            const uint32_t vx = L.P[x] >> 2, rx = L.P[x] & 3u;
            const uint32_t hi = A.off[vx + 1];
            const uint32_t base = locoff[x];
            const uint32_t lo = hi - (locoff[x + 1] - base);
            uint32_t nloc = 0;
            if (own && A.k4 && hi - lo > SHORT && lane == 0) {
                const uint32_t t = atomicAdd(&A.cursor[1], 1u);
                if (t < A.task_cap) A.tasks[t] = make_uint2(hi_idx, L.P[x]);
            }
            for (uint32_t q0 = lo; q0 < hi; q0 += 64) {
                const uint32_t q = q0 + lane;
                const bool in = q < hi;
                uint32_t e = 0, ec = 0;
                int sl = -1;
                if (in) {
                    e = A.adj[q] >> 2;
                    ec = A.adj[q] & 3u;
                    sl = slot_find(H, L.P, e);
                }
                const bool local = in && sl >= 0, d2 = in && sl < 0;
                const unsigned long long ml = __ballot(local);
                if (local) locnbr[base + nloc + (uint32_t)__popcll(ml & ((1ull << lane) - 1ull))] = ((uint32_t)sl << 2) | ec;
                nloc += (uint32_t)__popcll(ml);
                if (A.k3) {   // (1,2): r - x - e
                    const uint32_t cls = L.t3[motif_index3(rx, 0u, ec)];
                    by_class(cls, own && d2, [&](uint32_t k, uint32_t n) {
                        atomicAdd(&L.root3[k], (unsigned long long)n);
                        atomicAdd(&R3[x * kClasses3 + k], n);
                    });
                    if (own && d2) {
                        gadd(A.out3, A.perm, kClasses3, e, cls, 1ull);
                        shp[1]++;
                    }
                }
                if (A.k4 && d2) {   // depth-2 entry (x, e) into e's bucket
                    uint32_t h = (e * 2654435761u) >> (32u - tbits);
                    for (;; h = (h + 1u) & (TS - 1u)) {
                        const uint32_t k = atomicCAS(&keys[h], 0u, e + 1u);
                        if (k == 0u) {
                            groups[atomicAdd(&L.ctr[1], 1u)] = h;
                            break;
                        }
                        if (k == e + 1u) break;
                    }
                    const uint32_t node = atomicAdd(&L.ctr[2], 1u);
                    const uint32_t old = atomicExch(&heads[h], node + 1u);
                    nodes[node] = ((unsigned long long)old << 32) | (x << 2) | ec;
                }
            }
            if (lane == 0) L.locn[x] = (uint16_t)nloc;
        }
        __syncthreads();
        const uint32_t ngroups = L.ctr[1];
        // ---- phase C3: k = 3 (1,1): pairs a < b of slots, lanes over b
        if (A.k3) {
            uint32_t* rows = R3 + DMAX * kClasses3;   // per wave: one code row
            for (;;) {
                const uint32_t a = wave_task(&L.ctr[3]) * G + share;
                if (a + 1 >= D) break;
                uint32_t* BA = rows + wid * CW;
                build_row(BA, locnbr, locoff[a], L.locn[a]);
                const uint32_t ra = L.P[a] & 3u;
                for (uint32_t b0 = a + 1; b0 < D; b0 += 64) {
                    const uint32_t b = b0 + lane;
                    const bool in = b < D;
                    uint32_t cls = 0xFFu;
                    if (in) cls = L.t3[motif_index3(ra, L.P[b] & 3u, code_at(BA, b))];
                    by_class(cls, in, [&](uint32_t k, uint32_t n) {
                        atomicAdd(&L.root3[k], (unsigned long long)n);
                        atomicAdd(&R3[a * kClasses3 + k], n);
                    });
                    if (in) {
                        atomicAdd(&R3[b * kClasses3 + cls], 1u);
                        shp[0]++;
                    }
                }
            }
            __syncthreads();
            for (uint32_t i = tid; i < D * kClasses3; i += HT) {
                const uint32_t x = R3[i];
                if (x) gadd(A.out3, A.perm, kClasses3, L.P[i / kClasses3] >> 2, i % kClasses3, x);
            }
            for (uint32_t i = tid; i < kClasses3; i += HT)
                if (L.root3[i]) gadd(A.out3, A.perm, kClasses3, r, i, L.root3[i]);
        }
        if (!A.k4) continue;
        __syncthreads();
        // ---- phase C4: (3,0,0): a < b < c, lanes over c
        uint32_t* R4 = L.U;                     // D x 10 star counters
        uint32_t* rows4 = L.U + DMAX * NSTAR;   // per wave: BA, BB
        for (uint32_t i = tid; i < D * NSTAR; i += HT) R4[i] = 0u;
        __syncthreads();
        for (;;) {
            const uint32_t a = wave_task(&L.ctr[4]) * G + share;
            if (a + 2 >= D) break;
            uint32_t* BA = rows4 + wid * 2 * CW;
            uint32_t* BB = BA + CW;
            build_row(BA, locnbr, locoff[a], L.locn[a]);
            const uint32_t va = L.P[a] >> 2, ra = L.P[a] & 3u;
            for (uint32_t b = a + 1; b + 1 < D; b++) {
                build_row(BB, locnbr, locoff[b], L.locn[b]);
                const uint32_t vb = L.P[b] >> 2, rb = L.P[b] & 3u, ab = code_at(BA, b);
                for (uint32_t c0 = b + 1; c0 < D; c0 += 64) {
                    const uint32_t c = c0 + lane;
                    const bool in = c < D;
                    uint32_t cls = 0xFFu;
                    if (in) cls = L.t4[motif_index4(ra, rb, L.P[c] & 3u, ab, code_at(BA, c), code_at(BB, c))];
                    by_class(cls, in, [&](uint32_t k, uint32_t n) {
                        atomicAdd(&L.root4[k], (unsigned long long)n);
                        const uint32_t s = star_of[k];
                        if (s < NSTAR) {
                            atomicAdd(&R4[a * NSTAR + s], n);
                            atomicAdd(&R4[b * NSTAR + s], n);
                        } else {
                            gadd(A.out4, A.perm, kClasses4, va, k, n);
                            gadd(A.out4, A.perm, kClasses4, vb, k, n);
                        }
                    });
                    if (in) {
                        const uint32_t s = star_of[cls];
                        if (s < NSTAR) atomicAdd(&R4[c * NSTAR + s], 1u);
                        else gadd(A.out4, A.perm, kClasses4, L.P[c] >> 2, cls, 1ull);
                        shp[2]++;
                    }
                }
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < D * NSTAR; i += HT) {
            const uint32_t x = R4[i];
            if (x) gadd(A.out4, A.perm, kClasses4, L.P[i / NSTAR] >> 2, A.star_cls[i % NSTAR], x);
        }
        __syncthreads();
        // ---- phase D: (2,1,0): group c, parent x in A(c), lanes over the second slot y
        uint32_t* R5 = L.U;                       // D x 15 path counters
        uint32_t* rows5 = L.U + DMAX * NPATH;     // per wave: BC (codes of A(c) to c), BX
        uint32_t* chist = rows5 + NW * 2 * CW;    // per wave: 16 path counters of c
        for (uint32_t i = tid; i < D * NPATH; i += HT) R5[i] = 0u;
        if (lane < 16) chist[wid * 16 + lane] = 0u;
        __syncthreads();
        for (;;) {
            const uint32_t gi = wave_task(&L.ctr[5]);
            if (gi >= ngroups) break;
            const uint32_t h = groups[gi];
            const uint32_t c = keys[h] - 1u;
            if (c % G != share) continue;
            uint32_t* BC = rows5 + wid * 2 * CW;
            uint32_t* BX = BC + CW;
            uint32_t* ch = chist + wid * 16;
            for (uint32_t i = lane; i < CW; i += 64) BC[i] = 0u;
            __threadfence_block();
            if (lane == 0)
                for (uint32_t nd = heads[h]; nd != 0u;) {
                    const unsigned long long v = nodes[nd - 1u];
                    const uint32_t x = ((uint32_t)v >> 2) & 0xFFFu, xc = (uint32_t)v & 3u;
                    BC[x >> 4] |= xc << ((x & 15u) << 1);
                    nd = (uint32_t)(v >> 32);
                }
            __threadfence_block();
            for (uint32_t nd = heads[h]; nd != 0u;) {   // every lane walks the parent list
                const unsigned long long v = nodes[nd - 1u];
                const uint32_t x = ((uint32_t)v >> 2) & 0xFFFu, xc = (uint32_t)v & 3u;
                nd = (uint32_t)(v >> 32);
                build_row(BX, locnbr, locoff[x], L.locn[x]);
                const uint32_t vx = L.P[x] >> 2, rx = L.P[x] & 3u;
                for (uint32_t y0 = 0; y0 < D; y0 += 64) {
                    const uint32_t y = y0 + lane;
                    uint32_t cls = 0xFFu;
                    bool in = y < D && y != x;
                    if (in) {
                        const uint32_t yc = code_at(BC, y);
                        in = !(yc && y < x);   // c hangs under its lower-rank parent
                        if (in) cls = L.t4[motif_index4(rx, L.P[y] & 3u, 0u, code_at(BX, y), xc, yc)];
                    }
                    by_class(cls, in, [&](uint32_t k, uint32_t n) {
                        atomicAdd(&L.root4[k], (unsigned long long)n);
                        const uint32_t s = path_of[k];
                        if (s < NPATH) {
                            atomicAdd(&R5[x * NPATH + s], n);
                            ch[s] += n;
                        } else {
                            gadd(A.out4, A.perm, kClasses4, vx, k, n);
                            gadd(A.out4, A.perm, kClasses4, c, k, n);
                        }
                    });
                    if (in) {
                        const uint32_t s = path_of[cls];
                        if (s < NPATH) atomicAdd(&R5[y * NPATH + s], 1u);
                        else gadd(A.out4, A.perm, kClasses4, L.P[y] >> 2, cls, 1ull);
                        shp[3]++;
                    }
                }
            }
            __threadfence_block();
            if (lane < NPATH) {
                const uint32_t n = ch[lane];
                if (n) gadd(A.out4, A.perm, kClasses4, c, A.path_cls[lane], n);
                ch[lane] = 0u;
            }
            __threadfence_block();
        }
        __syncthreads();
        for (uint32_t i = tid; i < D * NPATH; i += HT) {
            const uint32_t x = R5[i];
            if (x) gadd(A.out4, A.perm, kClasses4, L.P[i / NPATH] >> 2, A.path_cls[i % NPATH], x);
        }
        __syncthreads();
        // ---- phase F: (1,2,0) and (1,1,1) below the slots with short rows, one wave each
        for (uint32_t i = tid; i < SHASH / 2; i += HT) L.U[i] = 0u;
        __syncthreads();
        for (uint32_t i = tid; i < D; i += HT) slot_insert(H, L.P[i] >> 2, i);
        __syncthreads();
        {
            // per wave: child list (64), child hash (128: (rank + 1) << 6 | position), child
            // codes to the current child (4 words), child counters (64 x 25), counters of a
            constexpr uint32_t WW = 64 + CH_HASH + 4 + 64 * NTREE + kClasses4;
            uint32_t* CL = L.U + SHASH / 2 + wid * WW;
            uint32_t* CK = CL + 64;
            uint32_t* CA = CK + CH_HASH;
            uint32_t* CC = CA + 4;
            uint32_t* AH = CC + 64 * NTREE;
            for (;;) {
                const uint32_t a = wave_task(&L.ctr[6]) * G + share;
                if (a >= D) break;
                const uint32_t len = locoff[a + 1] - locoff[a];
                if (len == 0 || len > SHORT) continue;
                const uint32_t va = L.P[a] >> 2, ra = L.P[a] & 3u;
                const uint32_t hi = A.off[va + 1], lo = hi - len;
                for (uint32_t i = lane; i < CH_HASH; i += 64) CK[i] = 0u;
                for (uint32_t i = lane; i < kClasses4; i += 64) AH[i] = 0u;
                for (uint32_t i = lane; i < 64 * NTREE; i += 64) CC[i] = 0u;
                if (lane < 4) CA[lane] = 0u;
                // children: entries of a's row above r outside N+(r)
                const uint32_t q = lo + lane;
                uint32_t e = 0, ec = 0;
                bool chd = false;
                if (q < hi) {
                    e = A.adj[q] >> 2;
                    ec = A.adj[q] & 3u;
                    chd = slot_find(H, L.P, e) < 0;
                }
                const unsigned long long mc = __ballot(chd);
                const uint32_t m = (uint32_t)__popcll(mc);
                __threadfence_block();
                if (chd) {
                    const uint32_t pos = (uint32_t)__popcll(mc & ((1ull << lane) - 1ull));
                    CL[pos] = (e << 2) | ec;
                    for (uint32_t h = (e * 2654435761u) >> 25;; h = (h + 1u) & (CH_HASH - 1u))
                        if (atomicCAS(&CK[h], 0u, ((e + 1u) << 6) | pos) == 0u) break;
                }
                __threadfence_block();
                for (uint32_t i = 0; i < m; i++) {
                    const uint32_t vc = CL[i] >> 2, ac = CL[i] & 3u;
                    // walk c's row above r: arcs to later children, (1,1,1) end vertices
                    const uint32_t chi = A.off[vc + 1];
                    for (uint32_t t0 = first_above(A.adj, A.off[vc], chi, r); t0 < chi; t0 += 64) {
                        const uint32_t t = t0 + lane;
                        bool p111 = false;
                        uint32_t cls = 0xFFu, ve = 0;
                        if (t < chi) {
                            ve = A.adj[t] >> 2;
                            const uint32_t ce = A.adj[t] & 3u;
                            int pos = -1;
                            for (uint32_t h = (ve * 2654435761u) >> 25;; h = (h + 1u) & (CH_HASH - 1u)) {
                                const uint32_t k = CK[h];
                                if (k == 0u) break;
                                if ((k >> 6) == ve + 1u) {
                                    pos = (int)(k & 63u);
                                    break;
                                }
                            }
                            if (pos >= 0) {
                                if ((uint32_t)pos > i) atomicOr(&CA[pos >> 4], ce << ((pos & 15) << 1));
                            } else if (slot_find(H, L.P, ve) < 0) {
                                p111 = true;   // e above r, not adjacent to r nor to a
                                cls = L.t4[motif_index4(ra, 0u, 0u, ac, 0u, ce)];
                            }
                        }
                        by_class(cls, p111, [&](uint32_t k, uint32_t n) {
                            atomicAdd(&L.root4[k], (unsigned long long)n);
                            AH[k] += n;
                            const uint32_t s = tree_of[k];
                            if (s < NTREE) CC[i * NTREE + s] += n;
                            else gadd(A.out4, A.perm, kClasses4, vc, k, n);
                        });
                        if (p111) {
                            gadd(A.out4, A.perm, kClasses4, ve, cls, 1ull);
                            shp[5]++;
                        }
                    }
                    __threadfence_block();
                    // (1,2,0): r - a - {c, c'} for the later children c'
                    const uint32_t j = i + 1 + lane;
                    const bool in = j < m;
                    uint32_t cls = 0xFFu;
                    if (in) cls = L.t4[motif_index4(ra, 0u, 0u, ac, CL[j] & 3u, code_at(CA, j))];
                    by_class(cls, in, [&](uint32_t k, uint32_t n) {
                        atomicAdd(&L.root4[k], (unsigned long long)n);
                        AH[k] += n;
                        const uint32_t s = tree_of[k];
                        if (s < NTREE) CC[i * NTREE + s] += n;
                        else gadd(A.out4, A.perm, kClasses4, vc, k, n);
                    });
                    if (in) {
                        const uint32_t s = tree_of[cls];
                        if (s < NTREE) atomicAdd(&CC[j * NTREE + s], 1u);
                        else gadd(A.out4, A.perm, kClasses4, CL[j] >> 2, cls, 1ull);
                        shp[4]++;
                    }
                    __threadfence_block();
                    if (lane < 4) CA[lane] = 0u;
                    __threadfence_block();
                }
                for (uint32_t i = lane; i < m * NTREE; i += 64) {
                    const uint32_t x = CC[i];
                    if (x) gadd(A.out4, A.perm, kClasses4, CL[i / NTREE] >> 2, A.tree_cls[i % NTREE], x);
                }
                for (uint32_t i = lane; i < kClasses4; i += 64)
                    if (AH[i]) gadd(A.out4, A.perm, kClasses4, va, i, AH[i]);
                __threadfence_block();
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < kClasses4; i += HT)
            if (L.root4[i]) gadd(A.out4, A.perm, kClasses4, r, i, L.root4[i]);
    }
    for (int s = 0; s < kShapes; s++) {
        unsigned long long x = shp[s];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0 && x) atomicAdd(&A.stats[s], x);
    }
}

// ----------------------------------------------------------------------------- long slots

// (1,2,0) and (1,1,1) sets below one slot a of a hub root r whose row above r is longer
// than SHORT: one workgroup per task.  Children and their counters in LDS; membership
// in N+(r) and in L_a by Bloom filters in front of binary searches of the sorted lists.
constexpr uint32_t BLOOM_WORDS = 1024;      // 32768 bits
constexpr uint32_t CTW = (NTREE + 1) / 2;   // u16 counter pairs per child (13 words)

struct LongLds {
    uint32_t P[DMAX];
    uint32_t CL[DMAX];              // children of a, ascending rank: (rank << 2) | arc bits a -> child
    uint32_t CC[DMAX * CTW];        // per child: 25 u16 tree-class counters in pairs
    uint32_t CA[NW * CW];           // per wave: codes of the current child to the children
    uint32_t bloomP[BLOOM_WORDS];
    uint32_t bloomC[BLOOM_WORDS];
    uint32_t root4[kClasses4];      // this task's credits of r
    uint32_t ah[kClasses4];         // this task's credits of a
    uint8_t t4[4096];
    uint8_t tree_of[256];
    uint32_t ctr[4];
    uint32_t root;                  // root staged in P, or ~0
};

__device__ __forceinline__ uint32_t bloom_bit(uint32_t x) { return (x * 0x9E3779B1u) >> 17; }
__device__ __forceinline__ bool bloom_has(const uint32_t* B, uint32_t x) {
    const uint32_t b = bloom_bit(x);
    return (B[b >> 5] >> (b & 31u)) & 1u;
}
// position of rank x in the sorted list Lst[0..n) of (rank << 2) | bits entries, or -1
__device__ __forceinline__ int sorted_find(const uint32_t* Lst, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;
    const uint32_t key = x << 2;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (Lst[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && (Lst[lo] >> 2) == x) ? (int)lo : -1;
}

__global__ __launch_bounds__(HT) void k_long_slots(HubArgs A) {
    __shared__ LongLds L;
    __shared__ uint32_t sTask, sM;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wid = wave_id();
    for (uint32_t i = tid; i < 4096; i += HT) L.t4[i] = A.t4[i];
    for (uint32_t i = tid; i < 256; i += HT) L.tree_of[i] = A.maps[512 + i];
    if (tid == 0) L.root = 0xFFFFFFFFu;
    const uint32_t ntask = min(A.cursor[1], A.task_cap);
    // workgroups per task when there are fewer tasks than twice the workgroups (up to 8):
    // each stages the task and walks the children i with i % G == share (the child list is
    // a stable compaction of a's row, the same in every workgroup)
    const uint32_t G = ntask >= 2u * gridDim.x ? 1u : min(8u, (2u * gridDim.x + ntask - 1u) / max(ntask, 1u));
    unsigned long long shp[kShapes] = {0, 0, 0, 0, 0, 0};
    auto cc_add = [&](uint32_t pos, uint32_t s, uint32_t n) {
        atomicAdd(&L.CC[pos * CTW + (s >> 1)], n << ((s & 1u) << 4));
    };
    for (;;) {
        __syncthreads();
        if (tid == 0) sTask = atomicAdd(&A.cursor[2], 1u);
        __syncthreads();
        const uint32_t t = sTask / G, share = sTask - t * G;
        if (t >= ntask) break;
        const uint2 task = A.tasks[t];
        const uint32_t r = A.hubs[task.x];
        const uint32_t s0 = A.split[r], D = A.off[r + 1] - s0;
        if (L.root != r) {   // stage N+(r) and its Bloom filter
            for (uint32_t i = tid; i < BLOOM_WORDS; i += HT) L.bloomP[i] = 0u;
            __syncthreads();
            for (uint32_t i = tid; i < D; i += HT) {
                const uint32_t e = A.adj[s0 + i];
                L.P[i] = e;
                const uint32_t b = bloom_bit(e >> 2);
                atomicOr(&L.bloomP[b >> 5], 1u << (b & 31u));
            }
            __syncthreads();
            if (tid == 0) L.root = r;
        }
        const uint32_t ea = task.y;   // the slot's entry in r's row
        const uint32_t va = ea >> 2, ra = ea & 3u;
        const uint32_t hi = A.off[va + 1], lo = first_above(A.adj, A.off[va], hi, r);
        for (uint32_t i = tid; i < BLOOM_WORDS; i += HT) L.bloomC[i] = 0u;
        for (uint32_t i = tid; i < kClasses4; i += HT) {
            L.root4[i] = 0u;
            L.ah[i] = 0u;
        }
        for (uint32_t i = tid; i < NW * CW; i += HT) L.CA[i] = 0u;
        if (tid < 4) L.ctr[tid] = 0u;
        __syncthreads();
        // children in rank order (one wave compacts the row)
        if (wid == 0) {
            uint32_t m = 0;
            for (uint32_t q0 = lo; q0 < hi; q0 += 64) {
                const uint32_t q = q0 + lane;
                bool chd = false;
                uint32_t ent = 0;
                if (q < hi) {
                    ent = A.adj[q];
                    const uint32_t e = ent >> 2;
                    chd = !bloom_has(L.bloomP, e) || sorted_find(L.P, D, e) < 0;
                }
                const unsigned long long mc = __ballot(chd);
                if (chd) {
                    const uint32_t pos = m + (uint32_t)__popcll(mc & ((1ull << lane) - 1ull));
                    L.CL[pos] = ent;
                    const uint32_t b = bloom_bit(ent >> 2);
                    atomicOr(&L.bloomC[b >> 5], 1u << (b & 31u));
                }
                m += (uint32_t)__popcll(mc);
            }
            if (lane == 0) sM = m;
        }
        __syncthreads();
        const uint32_t m = sM;
        for (uint32_t i = tid; i < m * CTW; i += HT) L.CC[i] = 0u;
        __syncthreads();
        uint32_t* CA = L.CA + wid * CW;
        for (;;) {
            const uint32_t i = wave_task(&L.ctr[0]) * G + share;
            if (i >= m) break;
            const uint32_t vc = L.CL[i] >> 2, ac = L.CL[i] & 3u;
            const uint32_t chi = A.off[vc + 1];
            for (uint32_t t0 = first_above(A.adj, A.off[vc], chi, r); t0 < chi; t0 += 64) {
                const uint32_t tq = t0 + lane;
                bool p111 = false;
                uint32_t cls = 0xFFu, ve = 0;
                if (tq < chi) {
                    ve = A.adj[tq] >> 2;
                    const uint32_t ce = A.adj[tq] & 3u;
                    const int pos = bloom_has(L.bloomC, ve) ? sorted_find(L.CL, m, ve) : -1;
                    if (pos >= 0) {
                        if ((uint32_t)pos > i) atomicOr(&CA[pos >> 4], ce << ((pos & 15) << 1));
                    } else if (!bloom_has(L.bloomP, ve) || sorted_find(L.P, D, ve) < 0) {
                        p111 = true;   // e above r, not adjacent to r nor to a
                        cls = L.t4[motif_index4(ra, 0u, 0u, ac, 0u, ce)];
                    }
                }
                by_class(cls, p111, [&](uint32_t k, uint32_t n) {
                    atomicAdd(&L.root4[k], n);
                    atomicAdd(&L.ah[k], n);
                    const uint32_t s = L.tree_of[k];
                    if (s < NTREE) cc_add(i, s, n);
                    else gadd(A.out4, A.perm, kClasses4, vc, k, n);
                });
                if (p111) {
                    gadd(A.out4, A.perm, kClasses4, ve, cls, 1ull);
                    shp[5]++;
                }
            }
            __threadfence_block();
            for (uint32_t j0 = i + 1; j0 < m; j0 += 64) {
                const uint32_t j = j0 + lane;
                const bool in = j < m;
                uint32_t cls = 0xFFu;
                if (in) cls = L.t4[motif_index4(ra, 0u, 0u, ac, L.CL[j] & 3u, code_at(CA, j))];
                by_class(cls, in, [&](uint32_t k, uint32_t n) {
                    atomicAdd(&L.root4[k], n);
                    atomicAdd(&L.ah[k], n);
                    const uint32_t s = L.tree_of[k];
                    if (s < NTREE) cc_add(i, s, n);
                    else gadd(A.out4, A.perm, kClasses4, vc, k, n);
                });
                if (in) {
                    const uint32_t s = L.tree_of[cls];
                    if (s < NTREE) cc_add(j, s, 1u);
                    else gadd(A.out4, A.perm, kClasses4, L.CL[j] >> 2, cls, 1ull);
                    shp[4]++;
                }
            }
            __threadfence_block();
            for (uint32_t w = lane; w < CW; w += 64) CA[w] = 0u;
            __threadfence_block();
        }
        __syncthreads();
        for (uint32_t i = tid; i < m * NTREE; i += HT) {
            const uint32_t pos = i / NTREE, s = i - pos * NTREE;
            const uint32_t x = (L.CC[pos * CTW + (s >> 1)] >> ((s & 1u) << 4)) & 0xFFFFu;
            if (x) gadd(A.out4, A.perm, kClasses4, L.CL[pos] >> 2, A.tree_cls[s], x);
        }
        for (uint32_t i = tid; i < kClasses4; i += HT) {
            if (L.root4[i]) gadd(A.out4, A.perm, kClasses4, r, i, L.root4[i]);
            if (L.ah[i]) gadd(A.out4, A.perm, kClasses4, va, i, L.ah[i]);
        }
    }
    for (int s = 0; s < kShapes; s++) {
        unsigned long long x = shp[s];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0 && x) atomicAdd(&A.stats[s], x);
    }
}

// ----------------------------------------------------------------------------- binning

constexpr int BT = 256;

// every pair {u < v} into the edge hash, one thread per row (entries from split[u] on)
__global__ void k_edge_hash(const uint32_t* __restrict__ off, const uint32_t* __restrict__ split,
                            const uint32_t* __restrict__ adj, int64_t n, unsigned long long* table, uint32_t bits) {
    const uint32_t mask = (1u << bits) - 1u;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        for (uint32_t t = split[u]; t < off[u + 1]; t++) {
            const uint32_t e = adj[t];
            const unsigned long long key = ((unsigned long long)u << 32) | ((unsigned long long)(e >> 2) << 2);
            for (uint32_t h = edge_slot(key, bits);; h = (h + 1u) & mask)
                if (atomicCAS(&table[h], 0ull, key | (e & 3u)) == 0ull) break;
        }
    }
}

// per root: hub or not and its work estimate (sort key); the largest slot-row scan and
// the largest |N+(r)|
__global__ void k_root_work(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj,
                            const uint32_t* __restrict__ split, const uint32_t* __restrict__ roots, int64_t nroots,
                            uint32_t hub_min, uint32_t hub_ok, uint32_t* __restrict__ is_hub,
                            unsigned long long* __restrict__ wkey, unsigned long long* __restrict__ max_s2,
                            unsigned* __restrict__ max_hi) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nroots; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t r = roots[i];
        const uint32_t s = split[r], e = off[r + 1], d = e - s;
        atomicMax(max_hi, d);
        const bool hub = hub_ok && d >= hub_min && d <= DMAX;
        is_hub[i] = hub ? 1u : 0u;
        if (!hub) {
            wkey[i] = ~0ull;
            continue;
        }
        unsigned long long s2 = 0;
        for (uint32_t t = s; t < e; t++) {
            const uint32_t a = adj[t] >> 2;
            s2 += off[a + 1] - lower_bound_rank(adj, off[a], off[a + 1], r + 1);
        }
        atomicMax(max_s2, s2);
        const unsigned long long dd = d;
        const unsigned long long w = dd * (dd - 1) * (dd - 2) / 6 + s2 * dd + s2 + 1;
        wkey[i] = ~w;   // ascending sort of ~w = largest work first; non-hubs (~0) last
    }
}

// per hub root (queue order): entries of its slots' rows above r, and |N+(r)|
__global__ void k_hub_s2(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj,
                         const uint32_t* __restrict__ split, const uint32_t* __restrict__ hubs, int64_t nhub,
                         uint32_t* __restrict__ s2out, unsigned long long* __restrict__ dsum) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nhub; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t r = hubs[i];
        uint32_t s2 = 0;
        for (uint32_t t = split[r]; t < off[r + 1]; t++) {
            const uint32_t a = adj[t] >> 2;
            s2 += off[a + 1] - lower_bound_rank(adj, off[a], off[a + 1], r + 1);
        }
        s2out[i] = s2;
        atomicAdd(dsum, (unsigned long long)(off[r + 1] - split[r]));
    }
}

__global__ void k_split_bins(const uint32_t* __restrict__ roots, const uint32_t* __restrict__ is_hub,
                             const uint32_t* __restrict__ pos, int64_t nroots, uint32_t* __restrict__ light) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nroots; i += (int64_t)gridDim.x * blockDim.x)
        if (!is_hub[i]) light[i - pos[i]] = roots[i];
}

__global__ void k_zero_u32(unsigned* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

int g_num_cu = -1;

int hub_workgroups() {
    if (g_num_cu < 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            g_num_cu = prop.multiProcessorCount;
        else
            g_num_cu = 256;
    }
    return g_num_cu;
}

}  // namespace

void free_hub_scratch(vdmc_graph_s* g) {
    if (!g->hub_scratch && !g->hub_tasks) return;
    wait_graph(g);
    (void)hipFree(g->hub_scratch);
    (void)hipFree(g->hub_tasks);
    g->hub_scratch = nullptr;
    g->hub_tasks = nullptr;
    g->hub_scratch_bytes = 0;
}

void free_hub(vdmc_graph_s* g) {
    wait_graph(g);
    free_hub_scratch(g);
    (void)hipFree(g->light);
    (void)hipFree(g->hubs);
    (void)hipFree(g->hub_queue);
    (void)hipFree(g->hub_s2);
    g->light = g->hubs = nullptr;
    g->hub_queue = nullptr;
    g->hub_s2 = nullptr;
    g->hub_scratch_need = 0;
    g->nhub = g->nlight = 0;
    g->bins_hub_min = -1;
}

size_t hub_scratch_need(const vdmc_graph_s* g) { return g->nhub > 0 ? g->hub_scratch_need : 0; }

void ensure_hub_scratch(vdmc_graph_s* g) {
    if (g->nhub == 0 || g->hub_scratch) return;
    const size_t wg_bytes = g->hub_layout[0] * sizeof(uint32_t) * (size_t)hub_workgroups();
    VDMC_HIP(hipMalloc(&g->hub_scratch, wg_bytes));
    const hipError_t e = hipMalloc(&g->hub_tasks, (size_t)g->hub_task_cap * sizeof(uint2));
    if (e != hipSuccess) {
        (void)hipFree(g->hub_scratch);
        g->hub_scratch = nullptr;
        VDMC_HIP(e);
    }
    g->hub_scratch_bytes = wg_bytes + (size_t)g->hub_task_cap * sizeof(uint2);
}

void ensure_edge_hash(vdmc_graph_s* g, hipStream_t st) {
    if (g->ehash) return;
    uint32_t eb = 10;   // load <= 1/4
    while (((size_t)1 << eb) < 4 * (size_t)std::max<int64_t>(g->pairs, 1)) eb++;
    const size_t eh_bytes = ((size_t)1 << eb) * sizeof(unsigned long long);
    VDMC_HIP(hipMalloc(&g->ehash, eh_bytes));
    VDMC_HIP(hipMemsetAsync(g->ehash, 0, eh_bytes, st));
    const unsigned blocks = (unsigned)std::min<int64_t>((g->n + BT - 1) / BT, 65536);
    if (blocks > 0)
        hipLaunchKernelGGL(k_edge_hash, dim3(blocks), dim3(BT), 0, st, g->off, g->split, g->adj, g->n, g->ehash, eb);
    VDMC_HIP(hipGetLastError());
    VDMC_HIP(hipStreamSynchronize(st));
    g->ehash_bits = eb;
}

void ensure_bins(vdmc_graph_s* g, hipStream_t st) {
    const int hub_min = g->hub_min;
    if (g->bins_hub_min == hub_min) return;
    free_hub(g);   // waits for running work on the old bins
    const int64_t nr = g->nroots;
    std::vector<void*> tmp;
    auto alloc = [&](size_t bytes) {
        void* p = nullptr;
        VDMC_HIP(hipMalloc(&p, bytes ? bytes : 16));
        tmp.push_back(p);
        return p;
    };
    struct Free {
        std::vector<void*>& v;
        ~Free() {
            for (void* p : v) (void)hipFree(p);
        }
    } guard{tmp};
    // the hub path needs every degree <= DMAX (a slot's children fit the LDS lists) and
    // ranks below 2^26 (per-wave child hash keys)
    const uint32_t hub_ok = (g->max_deg <= (int32_t)DMAX && g->n < ((int64_t)1 << 26)) ? 1u : 0u;
    uint32_t* is_hub = (uint32_t*)alloc((nr + 1) * sizeof(uint32_t));
    uint32_t* pos = (uint32_t*)alloc((nr + 1) * sizeof(uint32_t));
    unsigned long long* wkey = (unsigned long long*)alloc((nr + 1) * sizeof(unsigned long long));
    unsigned long long* wkey_s = (unsigned long long*)alloc((nr + 1) * sizeof(unsigned long long));
    uint32_t* roots_s = (uint32_t*)alloc((nr + 1) * sizeof(uint32_t));
    unsigned long long* d_max = (unsigned long long*)alloc(4 * sizeof(unsigned long long));
    VDMC_HIP(hipMemsetAsync(d_max, 0, 4 * sizeof(unsigned long long), st));
    unsigned* d_maxhi = (unsigned*)(d_max + 1);
    unsigned long long* d_dsum = d_max + 2;
    int64_t nhub = 0, nlight = 0;
    std::vector<unsigned long long> hub_keys;   // sorted work keys of the hub roots (~work)
    unsigned long long max_s2 = 0;
    unsigned maxhi = 0;
    if (nr > 0) {
        unsigned blocks = (unsigned)std::min<int64_t>((nr + BT - 1) / BT, 65536);
        hipLaunchKernelGGL(k_root_work, dim3(blocks), dim3(BT), 0, st, g->off, g->adj, g->split, g->roots, nr,
                           (uint32_t)hub_min, hub_ok, is_hub, wkey, d_max, d_maxhi);
        VDMC_HIP(hipGetLastError());
        VDMC_HIP(hipMemsetAsync(is_hub + nr, 0, sizeof(uint32_t), st));
        size_t tb = 0;
        int n1 = (int)(nr + 1);
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, is_hub, pos, n1, st));
        void* t1 = alloc(tb);
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(t1, tb, is_hub, pos, n1, st));
        uint32_t h = 0;
        VDMC_HIP(hipMemcpyAsync(&h, pos + nr, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        VDMC_HIP(hipMemcpyAsync(&max_s2, d_max, sizeof(max_s2), hipMemcpyDeviceToHost, st));
        VDMC_HIP(hipMemcpyAsync(&maxhi, d_maxhi, sizeof(maxhi), hipMemcpyDeviceToHost, st));
        VDMC_HIP(hipStreamSynchronize(st));
        nhub = h;
        nlight = nr - nhub;
        VDMC_HIP(hipMalloc(&g->light, (nlight + 1) * sizeof(uint32_t)));
        VDMC_HIP(hipMalloc(&g->hubs, (nhub + 1) * sizeof(uint32_t)));
        if (nlight > 0)
            hipLaunchKernelGGL(k_split_bins, dim3(blocks), dim3(BT), 0, st, g->roots, is_hub, pos, nr, g->light);
        VDMC_HIP(hipGetLastError());
        if (nhub > 0) {
            // sort all roots by work key (non-hubs carry ~0 and land at the end)
            size_t sb = 0;
            int ni = (int)nr;
            VDMC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sb, wkey, wkey_s, g->roots, roots_s, ni, 0, 64, st));
            void* t2 = alloc(sb);
            VDMC_HIP(hipcub::DeviceRadixSort::SortPairs(t2, sb, wkey, wkey_s, g->roots, roots_s, ni, 0, 64, st));
            VDMC_HIP(hipMemcpyAsync(g->hubs, roots_s, nhub * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
            hub_keys.resize((size_t)nhub);
            VDMC_HIP(hipMemcpyAsync(hub_keys.data(), wkey_s, nhub * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                    st));
        }
        VDMC_HIP(hipStreamSynchronize(st));
        // Hub roots whose estimated work exceeds a fair share of the device (the total over
        // twice the workgroups) would each be the critical path on one workgroup: the
        // leading ones of the queue (largest first) are shared by G workgroups, G from the
        // heaviest root's excess, at most 8.  hub_layout[3] = how many, hub_layout[4] = G.
        if (nhub > 0) {
            double total = 0.0;
            for (unsigned long long k : hub_keys) total += (double)(~k);
            const double fair = total / (2.0 * hub_workgroups());
            size_t h = 0;
            while (h < hub_keys.size() && h < 4096 && (double)(~hub_keys[h]) > fair) h++;
            const double top = (double)(~hub_keys[0]);
            const uint32_t shares = fair > 0.0 ? (uint32_t)std::min(8.0, std::ceil(top / fair)) : 1u;
            g->hub_layout[3] = shares >= 2 ? h : 0;
            g->hub_layout[4] = shares >= 2 ? shares : 1;
        }
    } else {
        VDMC_HIP(hipMalloc(&g->light, sizeof(uint32_t)));
        VDMC_HIP(hipMalloc(&g->hubs, sizeof(uint32_t)));
    }
    g->nhub = nhub;
    g->nlight = nlight;
    g->max_scan2 = (int64_t)max_s2;
    g->max_hi = (int32_t)maxhi;
    // light roots: fewer than hub_min higher neighbours (every root when the hub path is off)
    g->light_max_d = hub_ok ? std::min<int32_t>((int32_t)maxhi, hub_min - 1) : (int32_t)maxhi;
    VDMC_HIP(hipMalloc(&g->hub_queue, 64));
    if (nhub > 0) {
        VDMC_HIP(hipMalloc(&g->hub_s2, nhub * sizeof(uint32_t)));
        const unsigned hb = (unsigned)std::min<int64_t>((nhub + BT - 1) / BT, 65536);
        hipLaunchKernelGGL(k_hub_s2, dim3(hb), dim3(BT), 0, st, g->off, g->adj, g->split, g->hubs, nhub, g->hub_s2,
                           d_dsum);
        VDMC_HIP(hipGetLastError());
        unsigned long long dsum = 0;
        VDMC_HIP(hipMemcpyAsync(&dsum, d_dsum, sizeof(dsum), hipMemcpyDeviceToHost, st));
        VDMC_HIP(hipStreamSynchronize(st));
        const int wgs = hub_workgroups();
        const size_t s2cap = (size_t)max_s2 + 64;
        size_t tcap = 64;
        while (tcap < 2 * s2cap + 64) tcap <<= 1;
        const size_t words = (DMAX + 2) + s2cap + (s2cap & 1) + 2 * s2cap + s2cap + 2 * tcap;
        const size_t wg_words = (words + 63) & ~(size_t)63;
        g->hub_layout[0] = wg_words;
        g->hub_layout[1] = s2cap;
        g->hub_layout[2] = tcap;
        // long-slot tasks: at most one per (hub root, slot)
        const size_t ntask = (size_t)std::max<unsigned long long>(dsum, 1ull);
        g->hub_task_cap = (uint32_t)std::min<size_t>(ntask, 0xFFFFFFFFu);
        g->hub_scratch_need = wg_words * sizeof(uint32_t) * (size_t)wgs + (size_t)g->hub_task_cap * sizeof(uint2);
    }
    g->bins_hub_min = hub_min;
}

void launch_hub(vdmc_graph_s* g, int k3, int k4, uint64_t* out3, uint64_t* out4, hipStream_t st,
                uint32_t rank_lo, uint32_t rank_hi, const hipEvent_t* around) {
    if (g->nhub == 0) return;
    ensure_hub_scratch(g);
    const ClassTables& t = class_tables();
    HubArgs a;
    a.off = g->off;
    a.adj = g->adj;
    a.split = g->split;
    a.perm = g->perm;
    a.hubs = g->hubs;
    a.hub_s2 = g->hub_s2;
    a.nhub = (uint32_t)g->nhub;
    a.cursor = g->hub_queue;
    a.t3 = t.t3;
    a.t4 = t.t4;
    a.maps = t.maps4;
    a.star_cls = t.star_cls;
    a.path_cls = t.path_cls;
    a.tree_cls = t.slotcls;
    a.out3 = (unsigned long long*)out3;
    a.out4 = (unsigned long long*)out4;
    a.stats = g->stats;
    a.k3 = k3;
    a.k4 = k4;
    a.rank_lo = rank_lo;
    a.rank_hi = rank_hi;
    a.scratch = (uint32_t*)g->hub_scratch;
    a.wg_words = g->hub_layout[0];
    a.s2cap = (uint32_t)g->hub_layout[1];
    a.tcap = (uint32_t)g->hub_layout[2];
    a.tasks = (uint2*)g->hub_tasks;
    a.task_cap = g->hub_task_cap;
    const int wgs = hub_workgroups();
    a.split_roots = (uint32_t)g->hub_layout[3];   // the heaviest hub roots, shared (set at binning)
    a.shares = (uint32_t)std::max<size_t>(1, g->hub_layout[4]);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, g->hub_queue, 16);
    // around[0] and around[1] bracket the hub path, around[2] marks the end of k_hub
    if (around) VDMC_HIP(hipEventRecord(around[0], st));
    hipLaunchKernelGGL(k_hub, dim3(wgs), dim3(HT), 0, st, a);
    VDMC_HIP(hipGetLastError());
    if (around) VDMC_HIP(hipEventRecord(around[2], st));
    if (k4) {
        hipLaunchKernelGGL(k_long_slots, dim3(wgs), dim3(HT), 0, st, a);
        VDMC_HIP(hipGetLastError());
    }
    if (around) VDMC_HIP(hipEventRecord(around[1], st));
}

}  // namespace vdmc

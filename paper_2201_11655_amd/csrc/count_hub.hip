// Hub-root motif kernel: one workgroup per root with a large higher neighbourhood.
//
// The sets enumerated are exactly those of the per-set kernel (count.hip): every
// connected k-set once, from its lowest-rank vertex r, along the BFS shapes of
// Lemma 2 with the duplicate rules of Lemmas 3-4 (Sec. 5).  What changes is how the
// work is laid out on the CU and how the per-vertex counters are raised:
//
//   * N+(r) (the depth-1 candidates, "slots" in rank order) is staged in LDS, and
//     a 2-bit adjacency matrix M over the slots is built once per root in global
//     scratch (L2-resident), so that every depth-1/depth-1 test is one load;
//   * depth-2 vertices c are grouped: the entry (a, c) whose a is the lowest-rank
//     neighbour of c in N+(r) leads the group and records A(c) = N(c) n N+(r);
//     the depth-1 rule of (2,1,0) (c hangs under its lowest-rank parent) and the
//     (1,1,1) paths through c are then enumerated group by group;
//   * every loop keeps one member of the set fixed per lane and one fixed per wave
//     step; the class of a set whose remaining pairs are non-adjacent ("pure") is a
//     function of a few 2-bit codes, so lanes count such sets in packed register
//     fields and waves count them with ballots; the counts are flushed into LDS or
//     L2-resident per-slot counters and, once per root, into the output.  Sets with
//     extra edges take a direct path (table lookup of the full index, atomics).
// Every set is still visited by exactly one lane; only the increments are summed
// before they reach memory, which leaves the integer result unchanged.
#include "motif_device.h"
#include "vdmc_internal.h"

#include <hipcub/hipcub.hpp>

namespace vdmc {
namespace {

constexpr int HT = 1024;            // threads per hub workgroup
constexpr int NW = HT / 64;         // waves per workgroup
constexpr uint32_t PMAX = 2048;     // largest |N+(r)| on the hub path
constexpr uint32_t NCHMAX = PMAX / 64;
constexpr uint32_t F21 = (1u << 21) - 1u;
constexpr size_t M_WORDS = (size_t)PMAX * NCHMAX * 4;   // 2-bit matrix, 16 codes per word

struct HubArgs {
    const uint32_t* off;
    const uint32_t* adj;
    const uint32_t* split;
    const int32_t* perm;
    const uint32_t* hubs;
    uint32_t nhub;
    unsigned* queue;
    const uint8_t* t3;
    const uint8_t* t4;
    unsigned long long* out3;
    unsigned long long* out4;
    unsigned long long* comp;    // n x kCompact4 rank-indexed accumulator (see add4)
    const uint8_t* slot4;        // class -> compact slot
    unsigned long long* stats;
    int k3, k4;
    uint32_t rank_lo, rank_hi;   // only roots with rank in [rank_lo, rank_hi)
    // per-workgroup scratch
    uint32_t* scratch;
    size_t wg_words;        // u32 words per workgroup slice
    size_t o_spar, o_s111, o_s3x, o_groups, o_wlist, o_eflag, o_llist;
    uint32_t s2cap;         // capacity of the group list (the single-parent list follows it)
    uint32_t hash_bits;     // per-wave hash table of 2^hash_bits (key, value) pairs
    uint32_t wl_cap;        // per-wave list capacity (>= max degree)
    const unsigned long long* ehash;   // the graph's edge hash (edge_code)
    uint32_t ehash_bits;
    uint32_t* w111;              // n x 9 (rank-indexed): (1,1,1) parent codes per depth-2 vertex
};

// ----------------------------------------------------------------------------- helpers

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ size_t mword(uint32_t d, uint32_t row, uint32_t col) {
    return (((size_t)(col >> 6) * d + row) << 2) + ((col & 63u) >> 4);
}
__device__ __forceinline__ uint32_t mshift(uint32_t col) { return (col & 15u) << 1; }
// arc bits of (P[row], P[col]) seen from P[row]
__device__ __forceinline__ uint32_t mget(const uint32_t* M, uint32_t d, uint32_t row, uint32_t col) {
    return (M[mword(d, row, col)] >> mshift(col)) & 3u;
}


// largest i in [0, n) with pre[i] <= q
__device__ __forceinline__ uint32_t slot_of(const uint32_t* pre, uint32_t n, uint32_t q) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
}

// index of the multiset {x, y}, x, y in {1,2,3}: 11 12 13 22 23 33 -> 0..5
__device__ __forceinline__ uint32_t pair_sig(uint32_t x, uint32_t y) {
    uint32_t lo = min(x, y) - 1u, hi = max(x, y) - 1u;
    return lo * 3u - (lo * (lo - 1u)) / 2u + (hi - lo);
}
__device__ __forceinline__ void sig_pair(uint32_t s, uint32_t& x, uint32_t& y) {
    const uint8_t tx[6] = {1, 1, 1, 2, 2, 3};
    const uint8_t ty[6] = {1, 2, 3, 2, 3, 3};
    x = tx[s];
    y = ty[s];
}

__device__ __forceinline__ void add_out(unsigned long long* out, const int32_t* perm, uint32_t C, uint32_t v,
                                        uint32_t cls, unsigned long long cnt) {
    if (cls < C && cnt) atomicAdd(&out[(size_t)perm[v] * C + cls], cnt);
}

// Inclusive scan of sPre[1..n] (counts) into prefix sums, sPre[0] = 0.  n <= 4*HT.
__device__ void block_prefix(uint32_t* sPre, uint32_t n, uint32_t* sScan) {
    const uint32_t tid = threadIdx.x;
    const uint32_t base = 1 + tid * 4;
    uint32_t loc[4], sum = 0;
    for (int k = 0; k < 4; k++) {
        uint32_t idx = base + k;
        sum += idx <= n ? sPre[idx] : 0u;
        loc[k] = sum;
    }
    sScan[tid] = sum;
    __syncthreads();
    for (uint32_t o = 1; o < HT; o <<= 1) {
        uint32_t v = tid >= o ? sScan[tid - o] : 0u;
        __syncthreads();
        sScan[tid] += v;
        __syncthreads();
    }
    const uint32_t excl = sScan[tid] - sum;
    for (int k = 0; k < 4; k++) {
        uint32_t idx = base + k;
        if (idx <= n) sPre[idx] = excl + loc[k];
    }
    if (tid == 0) sPre[0] = 0;
    __syncthreads();
}

__device__ __forceinline__ int wave_next(unsigned* sTask) {
    int t = 0;
    if (lane_id() == 0) t = (int)atomicAdd(sTask, 1u);
    return __shfl(t, 0);
}

// ----------------------------------------------------------------------------- kernel


// P membership filter: one bit per hash bucket of a rank; a clear bit proves absence.
constexpr uint32_t kShortRow = 64;     // (1,2,0): rows up to this length are walked
constexpr uint32_t kLaneList = 16;     // (2,1,0): local lists up to this length walked by one lane
constexpr uint32_t kBloomWords = 1024;   // 32768 bits
// P slot lookup: open-addressing table of N+(r) in LDS (rank + 1 -> slot), load <= 1/2
constexpr uint32_t kPHashBits = 12;
constexpr uint32_t kPHash = 1u << kPHashBits;
__device__ __forceinline__ uint32_t phash(uint32_t x) { return (x * 2654435761u) >> (32u - kPHashBits); }
__device__ __forceinline__ uint32_t bloom_bit(uint32_t x) { return (x * 2654435761u) >> 17; }

struct Lds {
    uint32_t P[PMAX];
    uint32_t pre[PMAX + 1];
    uint32_t lo[PMAX];
    uint32_t cnt[9 * PMAX];
    uint32_t bloom[kBloomWords];
    uint32_t phk[kPHash];                      // rank + 1 of a slot, 0 = empty
    uint16_t phs[kPHash];                      // its slot
    uint32_t scan[HT];
    uint32_t cw[NW][27 + 27 + kClasses3];      // per-wave group accumulators (c and r credits)
    uint32_t inA[NW][PMAX / 32];               // per-wave membership bitmap of A(c)
    uint32_t gall[9];                          // (2,1,0) sets per parent code, credited to every slot
    unsigned long long root4[kClasses4];
    unsigned long long root3[kClasses3];
    unsigned long long stat[kLdsStatSlots];    // shape counts, phase ticks, direct-path counts
    uint16_t lcnt[PMAX];                       // local (in-N+(r)) degree of every slot
    uint8_t t4[4096];
    uint8_t t3[64];
    uint8_t slot4[kClasses4 + 1];              // class -> compact slot (0xFF: none)
    unsigned task, groups, sgroups, rootidx;
};

// Credit cnt sets of class cls to the vertex of rank v.  Classes of sets whose
// undetermined pairs are all non-adjacent (the 15 directed 4-path and 10 3-star
// classes) go to a compact rank-indexed accumulator that stays cache-resident and is
// folded into the output once per launch; every other class goes straight to the output.
__device__ __forceinline__ void add4(const HubArgs& A, const Lds& L, uint32_t v, uint32_t cls,
                                     unsigned long long cnt) {
    if (!cnt || cls >= kClasses4) return;
    const uint32_t sl = L.slot4[cls];
    if (sl != 0xFFu) atomicAdd(&A.comp[(size_t)v * kCompact4 + sl], cnt);
    else atomicAdd(&A.out4[(size_t)A.perm[v] * kClasses4 + cls], cnt);
}

__device__ __forceinline__ int find_slot_f(const Lds& L, uint32_t d, uint32_t x) {
    const uint32_t b = bloom_bit(x);
    if (!((L.bloom[b >> 5] >> (b & 31)) & 1u)) return -1;
    for (uint32_t h = phash(x);; h = (h + 1u) & (kPHash - 1u)) {
        const uint32_t k = L.phk[h];
        if (k == 0u) return -1;
        if (k == x + 1u) return (int)L.phs[h];
    }
}

// Up to kRC entries of a short CSR row kept in registers for repeated adjacency tests.
constexpr uint32_t kRC = 4;
struct RowCache {
    uint32_t e[kRC];
    uint32_t n;        // number cached (0..kRC); n > kRC means "row too long, search it"
    uint32_t lo, hi;   // row bounds for the long case
};
__device__ __forceinline__ void row_cache_load(RowCache& rc, const uint32_t* off, const uint32_t* adj, uint32_t v,
                                               bool active) {
    rc.n = 0;
    rc.lo = rc.hi = 0;
    if (!active) return;
    const uint32_t lo = off[v], hi = off[v + 1];
    if (hi - lo <= kRC) {
        rc.n = hi - lo;
#pragma unroll
        for (uint32_t k = 0; k < kRC; k++) rc.e[k] = (lo + k < hi) ? adj[lo + k] : 0xFFFFFFFFu;
    } else {
        rc.n = kRC + 1;
        rc.lo = lo;
        rc.hi = hi;
    }
}
// arc bits of the pair (u, owner) seen from u, where owner is the vertex whose row is cached
__device__ __forceinline__ uint32_t row_cache_bits_from(const RowCache& rc, const uint32_t* adj, uint32_t u) {
    uint32_t e = 0xFFFFFFFFu;
    if (rc.n <= kRC) {
#pragma unroll
        for (uint32_t k = 0; k < kRC; k++)
            if ((rc.e[k] >> 2) == u) e = rc.e[k];
    } else {
        const uint32_t p = lower_bound_rank(adj, rc.lo, rc.hi, u);
        if (p < rc.hi && (adj[p] >> 2) == u) e = adj[p];
    }
    return e == 0xFFFFFFFFu ? 0u : swap_arc_bits(e & 3u);   // entry is seen from the row owner
}

__global__ __launch_bounds__(HT) void k_hub(HubArgs A) {
    __shared__ Lds L;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wid = tid >> 6;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    uint32_t* W = A.scratch + (size_t)blockIdx.x * A.wg_words;
    uint32_t* M = W;
    uint32_t* spar = W + A.o_spar;     // [9][PMAX]  (2,1,0) parent-role counters
    uint32_t* s111 = W + A.o_s111;     // [9][PMAX]  (1,1,1) depth-1 counters
    uint32_t* s3x = W + A.o_s3x;       // [3][PMAX]  k=3 (1,2) depth-1 counters
    uint32_t* nsg = s3x + 3 * PMAX;    // [3][PMAX]  single-parent groups per (xc, slot) of a root
    // [3][PMAX] per slot x and ry: x's local neighbours y with P[y]'s arc code ry, three
    // 21-bit fields by the x-y arc code xy
    unsigned long long* prof = reinterpret_cast<unsigned long long*>(s3x + 6 * PMAX);
    uint32_t* grp = W + A.o_groups;    // the depth-2 vertex c of every group
    uint32_t* sgrp = grp + A.s2cap;    // single-parent short-row groups: c, then slot << 2 | code
    uint32_t* wlist = W + A.o_wlist + (size_t)wid * A.wl_cap;
    uint8_t* eflag = reinterpret_cast<uint8_t*>(W + A.o_eflag);
    uint16_t* llist = reinterpret_cast<uint16_t*>(W + A.o_llist);   // local neighbours per slot
    // per-thread counters of the current root (sets per shape, sets on the direct path),
    // reduced into L.stat once per root
    uint32_t shape[kShapes] = {0, 0, 0, 0, 0, 0};
    uint32_t slow[kShapes] = {0, 0, 0, 0, 0, 0};
    uint32_t work[4] = {0, 0, 0, 0};   // groups, (1,1,1) chunks, (1,1,1) steps, (2,1,0) chunk steps
    unsigned long long tprev = wall_clock64();
#define HUB_PHASE(k)                                      \
    do {                                                  \
        if (tid == 0) {                                   \
            const unsigned long long tn = wall_clock64(); \
            L.stat[8 + (k)] += tn - tprev;                \
            tprev = tn;                                   \
        }                                                 \
    } while (0)

    for (uint32_t i = tid; i < 4096; i += HT) L.t4[i] = A.t4[i];
    for (uint32_t i = tid; i < 64; i += HT) L.t3[i] = A.t3[i];
    for (uint32_t i = tid; i < kClasses4; i += HT) L.slot4[i] = A.slot4[i];
    for (uint32_t i = tid; i < 9 * PMAX; i += HT) { spar[i] = 0; s111[i] = 0; }
    for (uint32_t i = tid; i < 3 * PMAX; i += HT) { s3x[i] = 0; nsg[i] = 0; }
    for (uint32_t i = tid; i < NW * (PMAX / 32); i += HT) (&L.inA[0][0])[i] = 0;
    for (uint32_t i = tid; i < NW * (27 + 27 + kClasses3); i += HT) (&L.cw[0][0])[i] = 0;
    for (uint32_t i = tid; i < kLdsStatSlots; i += HT) L.stat[i] = 0;

    for (;;) {
        __syncthreads();
        if (tid == 0) L.rootidx = atomicAdd(A.queue, 1u);
        __syncthreads();
        const uint32_t ri = L.rootidx;
        if (ri >= A.nhub) break;
        const uint32_t r = A.hubs[ri];
        if (r < A.rank_lo || r >= A.rank_hi) continue;   // uniform across the workgroup
        const uint32_t s0 = A.split[r];
        const uint32_t d = A.off[r + 1] - s0;
        const uint32_t nch = (d + 63) >> 6;

        // ---------------------------------------------------------------- stage
        for (uint32_t i = tid; i < kBloomWords; i += HT) L.bloom[i] = 0;
        for (uint32_t i = tid; i < kPHash; i += HT) L.phk[i] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < d; i += HT) {
            const uint32_t e = A.adj[s0 + i];
            L.P[i] = e;
            const uint32_t a = e >> 2;
            const uint32_t b = bloom_bit(a);
            atomicOr(&L.bloom[b >> 5], 1u << (b & 31));
            for (uint32_t h = phash(a);; h = (h + 1u) & (kPHash - 1u))
                if (atomicCAS(&L.phk[h], 0u, a + 1u) == 0u) {
                    L.phs[h] = (uint16_t)i;
                    break;
                }
            const uint32_t lo = lower_bound_rank(A.adj, A.off[a], A.off[a + 1], r + 1);
            L.lo[i] = lo;
            L.pre[i + 1] = A.off[a + 1] - lo;
        }
        for (uint32_t i = tid; i < kClasses4; i += HT) L.root4[i] = 0;
        for (uint32_t i = tid; i < kClasses3; i += HT) L.root3[i] = 0;
        for (uint32_t i = tid; i < 9 * d; i += HT) L.cnt[i] = 0;
        if (tid < 9) L.gall[tid] = 0;
        const size_t mwords = (size_t)d * nch * 4;
        for (size_t i = tid; i < mwords; i += HT) M[i] = 0;
        if (tid == 0) { L.groups = 0; L.sgroups = 0; L.task = 0; }
        __syncthreads();
        block_prefix(L.pre, d, L.scan);
        const uint32_t scan2 = L.pre[d];
        __threadfence();
        __syncthreads();
        HUB_PHASE(0);

        // ---------------------------------------------------------------- local matrix, local lists, depth-2 flags
        // one wave per slot: the slot's row above r is split into neighbours inside N+(r)
        // (kept in slot order in llist and in M) and depth-2 entries (eflag)
        for (int t = wave_next(&L.task); t < (int)d; t = wave_next(&L.task)) {
            const uint32_t i = (uint32_t)t;
            const uint32_t q0 = L.pre[i], q1 = L.pre[i + 1], rlo = L.lo[i];
            uint32_t nl = 0;
            unsigned long long pf1 = 0, pf2 = 0, pf3 = 0;   // the slot's profile (see prof)
            uint32_t d1 = 0, d2 = 0, d3 = 0;                // depth-2 entries by arc code
            for (uint32_t qb = q0; qb < q1; qb += 64) {
                const uint32_t q = qb + lane;
                const bool v = q < q1;
                const uint32_t e = v ? A.adj[rlo + (q - q0)] : 0u;
                const int j = v ? find_slot_f(L, d, e >> 2) : -1;
                if (j >= 0) atomicOr(&M[mword(d, i, (uint32_t)j)], (e & 3u) << mshift((uint32_t)j));
                if (v) eflag[q] = j < 0 ? 1 : 0;
                const unsigned long long mk = __ballot(j >= 0);
                if (j >= 0) llist[q0 + nl + __popcll(mk & lt_mask)] = (uint16_t)(((uint32_t)j << 2) | (e & 3u));
                nl += __popcll(mk);
                if (A.k3) {
                    const bool dep2 = v && j < 0;
                    d1 += __popcll(__ballot(dep2 && (e & 3u) == 1u));
                    d2 += __popcll(__ballot(dep2 && (e & 3u) == 2u));
                    d3 += __popcll(__ballot(dep2 && (e & 3u) == 3u));
                }
                if (A.k4 && mk) {
                    const uint32_t code = j >= 0 ? ((L.P[j] & 3u) - 1u) * 3u + ((e & 3u) - 1u) : 9u;
#pragma unroll
                    for (uint32_t c9 = 0; c9 < 9; c9++) {
                        const unsigned long long inc = (unsigned long long)__popcll(__ballot(code == c9))
                                                       << (21u * (c9 % 3u));
                        if (c9 < 3) pf1 += inc; else if (c9 < 6) pf2 += inc; else pf3 += inc;
                    }
                }
            }
            // k=3 (1,2): every depth-2 entry (i, c) is the set {r, i, c}; i's credit and the
            // root's are counted here, c's when its group is processed
            if (A.k3 && lane < 3) {
                const uint32_t dk = lane == 0 ? d1 : (lane == 1 ? d2 : d3);
                s3x[lane * PMAX + i] = dk;
                if (dk) atomicAdd(&L.root3[L.t3[motif_index3(L.P[i] & 3u, 0u, lane + 1u)]], (unsigned long long)dk);
            }
            if (lane == 0) {
                L.lcnt[i] = (uint16_t)nl;
                if (A.k4) {
                    prof[i] = pf1;
                    prof[PMAX + i] = pf2;
                    prof[2 * PMAX + i] = pf3;
                }
            }
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) L.task = 0;
        __syncthreads();
        HUB_PHASE(1);

        // ---------------------------------------------------------------- k=3 (1,1): pairs of slots
        if (A.k3) {
            uint32_t total = 0;
            for (uint32_t ch = 0; ch < nch; ch++) total += (d > 64 * ch + 1) ? d - 1 - 64 * ch : 0;
            for (int t = wave_next(&L.task); t < (int)total; t = wave_next(&L.task)) {
                uint32_t ch = 0, rem = (uint32_t)t;
                while (true) {
                    const uint32_t c = d - 1 - 64 * ch;
                    if (rem < c) break;
                    rem -= c;
                    ch++;
                }
                const uint32_t j = 64 * ch + 1 + rem;
                const uint32_t i = 64 * ch + lane;
                const bool va = i < j;
                const uint32_t ra = va ? (L.P[i] & 3u) : 0u, rb = L.P[j] & 3u;
                const uint32_t ab = (va && L.lcnt[i] && L.lcnt[j]) ? swap_arc_bits(mget(M, d, j, i)) : 0u;
                const bool pure = va && ab == 0;
                if (pure) atomicAdd(&L.cnt[(rb - 1) * d + i], 1u);
                if (va && !pure) {
                    slow[0]++;
                    const uint32_t cls = L.t3[motif_index3(ra, rb, ab)];
                    atomicAdd(&L.root3[cls], 1ull);
                    add_out(A.out3, A.perm, kClasses3, L.P[i] >> 2, cls, 1);
                    add_out(A.out3, A.perm, kClasses3, L.P[j] >> 2, cls, 1);
                }
                if (va) shape[0]++;
                const uint32_t n1 = __popcll(__ballot(pure && ra == 1u));
                const uint32_t n2 = __popcll(__ballot(pure && ra == 2u));
                const uint32_t n3 = __popcll(__ballot(pure && ra == 3u));
                if (lane < 3) {
                    const uint32_t nk = lane == 0 ? n1 : (lane == 1 ? n2 : n3);
                    if (nk) {
                        atomicAdd(&L.cnt[lane * d + j], nk);
                        atomicAdd(&L.root3[L.t3[motif_index3(lane + 1, rb, 0u)]], (unsigned long long)nk);
                    }
                }
            }
            __syncthreads();
            for (uint32_t q = tid; q < 3 * d; q += HT) {
                const uint32_t cnt = L.cnt[q];
                if (!cnt) continue;
                const uint32_t s = q % d, g = q / d;
                add_out(A.out3, A.perm, kClasses3, L.P[s] >> 2, L.t3[motif_index3(L.P[s] & 3u, g + 1, 0u)], cnt);
                L.cnt[q] = 0;
            }
            if (tid == 0) L.task = 0;
            __syncthreads();
        }
        HUB_PHASE(2);

        // ---------------------------------------------------------------- depth-2 groups
        // c's group is led by c's first (lowest-rank) neighbour in N+(r).  One wave per slot
        // a; each lane takes one depth-2 entry (a, c) and walks row(c) up to its first
        // neighbour in N+(r) (a itself at the latest): a leads c's group iff that is a.  The
        // parent list A(c) is collected when the group is processed.
        for (int t = wave_next(&L.task); t < (int)d; t = wave_next(&L.task)) {
            const uint32_t a = (uint32_t)t;
            const uint32_t q0 = L.pre[a], q1 = L.pre[a + 1], rlo = L.lo[a];
            if (q1 - q0 == L.lcnt[a]) continue;   // no depth-2 entries
            uint32_t sg1 = 0, sg2 = 0, sg3 = 0;    // a's single-parent groups by code a -> c
            for (uint32_t qb = q0; qb < q1; qb += 64) {
                const uint32_t q = qb + lane;
                bool lead = false, single = false;
                uint32_t c = 0, xc = 0;
                if (q < q1 && eflag[q]) {
                    const uint32_t ent = A.adj[rlo + (q - q0)];
                    c = ent >> 2;
                    xc = ent & 3u;
                    const uint32_t clo = A.off[c], chi = A.off[c + 1];
                    const bool shortrow = chi - clo <= kShortRow;
                    // row entries in batches of 8 (one memory latency per batch); a short
                    // row is walked to its end to learn whether a is its only parent
                    int first = -1;
                    uint32_t nslot = 0;
                    for (uint32_t tb = clo; tb < chi; tb += 8) {
                        uint32_t w[8];
#pragma unroll
                        for (int j = 0; j < 8; j++) w[j] = tb + j < chi ? A.adj[tb + j] >> 2 : 0u;
#pragma unroll
                        for (int j = 0; j < 8; j++) {
                            if (w[j] <= r) continue;   // also the padding past the row
                            const int sl = find_slot_f(L, d, w[j]);
                            if (sl >= 0) {
                                if (first < 0) first = sl;
                                nslot++;
                            }
                        }
                        if (first >= 0 && ((uint32_t)first != a || !shortrow || nslot > 1)) break;
                    }
                    lead = first == (int)a;
                    single = lead && shortrow && nslot == 1;
                }
                const bool gen = lead && !single;
                const unsigned long long mk = __ballot(gen), ms = __ballot(single);
                sg1 += __popcll(__ballot(single && xc == 1u));
                sg2 += __popcll(__ballot(single && xc == 2u));
                sg3 += __popcll(__ballot(single && xc == 3u));
                if (mk) {
                    uint32_t g0 = 0;
                    if (lane == 0) g0 = atomicAdd(&L.groups, (unsigned)__popcll(mk));
                    g0 = __shfl(g0, 0);
                    if (gen) grp[g0 + __popcll(mk & lt_mask)] = c;
                }
                if (ms) {   // single-parent short-row groups: (c, slot << 2 | code a -> c)
                    uint32_t s0 = 0;
                    if (lane == 0) s0 = atomicAdd(&L.sgroups, (unsigned)__popcll(ms));
                    s0 = __shfl(s0, 0);
                    if (single) {
                        const uint32_t i = s0 + __popcll(ms & lt_mask);
                        sgrp[2 * i] = c;
                        sgrp[2 * i + 1] = (a << 2) | xc;
                    }
                }
            }
            if (lane < 3) nsg[lane * PMAX + a] = lane == 0 ? sg1 : (lane == 1 ? sg2 : sg3);
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) L.task = 0;
        __syncthreads();
        HUB_PHASE(3);

        // ---------------------------------------------------------------- k=4 (3,0,0): slot triples
        // A triple of slots with no arc among its three members (pure) has a class fixed by
        // the three arc codes with r, so the pure triples are counted from the numbers of
        // slots per code (per slot s: pairs of other slots by code pair; for r: triples by
        // code multiset).  The triples with an arc among them are found from the local
        // arcs: local arc (x, y), x < y, with every third slot z; the triple is taken by its
        // smallest arc (pairs ordered by (lower slot, higher slot)), so exactly once.  Each
        // such triple is credited directly and taken off the pure counts of its members
        // (per-slot counters np[g][s], g = code pair of the other two) and of r.
        if (A.k4) {
            uint32_t n1 = 0, n2 = 0, n3 = 0;   // slots by arc code with r (wave-uniform)
            for (uint32_t yb = 0; yb < d; yb += 64) {
                const uint32_t ry = yb + lane < d ? (L.P[yb + lane] & 3u) : 0u;
                n1 += __popcll(__ballot(ry == 1u));
                n2 += __popcll(__ballot(ry == 2u));
                n3 += __popcll(__ballot(ry == 3u));
            }
            uint32_t* np = L.cnt;   // [6][d], clear
            for (int t = wave_next(&L.task); t < (int)d; t = wave_next(&L.task)) {
                const uint32_t x = (uint32_t)t, rx = L.P[x] & 3u;
                const uint32_t b0 = L.pre[x], b1 = b0 + L.lcnt[x];
                for (uint32_t qy = b0; qy < b1; qy++) {
                    const uint32_t ey = llist[qy], y = ey >> 2, xy = ey & 3u;
                    if (y <= x) continue;
                    const uint32_t ry = L.P[y] & 3u;
                    uint32_t agg1 = 0, agg2 = 0, agg3 = 0;   // triples with the single arc x-y, by rz
                    for (uint32_t zb = 0; zb < d; zb += 64) {
                        const uint32_t z = zb + lane;
                        bool v = z < d && z != x && z != y;
                        uint32_t xz = 0, yz = 0, rz = 0;
                        if (v) {
                            xz = mget(M, d, x, z);
                            yz = mget(M, d, y, z);
                            v = !((xz && z < y) || (yz && z < x));   // a smaller arc takes it
                            rz = L.P[z] & 3u;
                        }
                        const bool single = v && xz == 0u && yz == 0u;
                        agg1 += __popcll(__ballot(single && rz == 1u));
                        agg2 += __popcll(__ballot(single && rz == 2u));
                        agg3 += __popcll(__ballot(single && rz == 3u));
                        if (v) {
                            slow[2]++;
                            const uint32_t cls = L.t4[motif_index4(rx, ry, rz, xy, xz, yz)];
                            const uint32_t pcls = L.t4[motif_index4(rx, ry, rz, 0u, 0u, 0u)];
                            atomicAdd(&L.root4[cls], 1ull);
                            atomicAdd(&L.root4[pcls], ~0ull);
                            add4(A, L, L.P[z] >> 2, cls, 1);
                            atomicAdd(&np[pair_sig(rx, ry) * d + z], 1u);
                            if (!single) {
                                add4(A, L, L.P[x] >> 2, cls, 1);
                                add4(A, L, L.P[y] >> 2, cls, 1);
                                atomicAdd(&np[pair_sig(ry, rz) * d + x], 1u);
                                atomicAdd(&np[pair_sig(rx, rz) * d + y], 1u);
                            }
                        }
                    }
                    if (lane < 3) {   // x and y in the single-arc triples, by rz = lane + 1
                        const uint32_t k = lane + 1u, cnt = lane == 0 ? agg1 : (lane == 1 ? agg2 : agg3);
                        if (cnt) {
                            const uint32_t cls = L.t4[motif_index4(rx, ry, k, xy, 0u, 0u)];
                            add4(A, L, L.P[x] >> 2, cls, cnt);
                            add4(A, L, L.P[y] >> 2, cls, cnt);
                            atomicAdd(&np[pair_sig(ry, k) * d + x], cnt);
                            atomicAdd(&np[pair_sig(rx, k) * d + y], cnt);
                        }
                    }
                }
            }
            __syncthreads();
            // every slot s: pure triples = pairs of other slots by code pair, minus np
            for (uint32_t q = tid; q < 6 * d; q += HT) {
                const uint32_t sl = q % d, g = q / d, rs = L.P[sl] & 3u;
                uint32_t cx, cy;
                sig_pair(g, cx, cy);
                const uint32_t nx = (cx == 1 ? n1 : (cx == 2 ? n2 : n3)) - (rs == cx ? 1u : 0u);
                const uint32_t ny = (cy == 1 ? n1 : (cy == 2 ? n2 : n3)) - (rs == cy ? 1u : 0u);
                const uint32_t all = cx == cy ? nx * (nx - 1u) / 2u : nx * ny;
                const uint32_t cnt = all - np[q];
                np[q] = 0;
                if (cnt) add4(A, L, L.P[sl] >> 2, L.t4[motif_index4(rs, cx, cy, 0u, 0u, 0u)], cnt);
            }
            // r: pure triples by code multiset k1 <= k2 <= k3 (the arc triples were taken off)
            if (tid < 10) {
                const uint8_t tk[10][3] = {{1, 1, 1}, {1, 1, 2}, {1, 1, 3}, {1, 2, 2}, {1, 2, 3},
                                           {1, 3, 3}, {2, 2, 2}, {2, 2, 3}, {2, 3, 3}, {3, 3, 3}};
                const uint32_t k1 = tk[tid][0], k2 = tk[tid][1], k3 = tk[tid][2];
                auto nk = [&](uint32_t k) -> unsigned long long { return k == 1 ? n1 : (k == 2 ? n2 : n3); };
                unsigned long long all;
                if (k1 == k3) all = nk(k1) * (nk(k1) - 1) * (nk(k1) - 2) / 6;
                else if (k1 == k2) all = nk(k1) * (nk(k1) - 1) / 2 * nk(k3);
                else if (k2 == k3) all = nk(k1) * (nk(k2) * (nk(k2) - 1) / 2);
                else all = nk(k1) * nk(k2) * nk(k3);
                if (all) atomicAdd(&L.root4[L.t4[motif_index4(k1, k2, k3, 0u, 0u, 0u)]], all);
            }
            if (tid == 0) {
                const unsigned long long dd = d;
                shape[2] += (uint32_t)(dd * (dd - 1) * (dd - 2) / 6);
            }
            if (tid == 0) L.task = 0;
            __syncthreads();
        }
        HUB_PHASE(4);

        // ---------------------------------------------------------------- groups: (2,1,0), (1,1,1), k=3 (1,2)
        const uint32_t ngroups = L.groups;
        uint32_t nr1 = 0, nr2 = 0, nr3 = 0;   // slots by their arc code with r (wave-uniform)
        for (uint32_t yb = 0; yb < d; yb += 64) {
            const uint32_t ry = yb + lane < d ? (L.P[yb + lane] & 3u) : 0u;
            nr1 += __popcll(__ballot(ry == 1u));
            nr2 += __popcll(__ballot(ry == 2u));
            nr3 += __popcll(__ballot(ry == 3u));
        }
        uint32_t* cw = L.cw[wid];
        uint32_t* inA = L.inA[wid];
        // The next group's vertex, row bounds and first row chunk are loaded in stages while
        // the current group is processed, so that a group does not start with a chain of
        // dependent loads.
        const unsigned long long tw0 = wall_clock64();
        int t = wave_next(&L.task);
        uint32_t cN = 0, loN = 0, hiN = 0, e0N = 0;
        if (t < (int)ngroups) {
            cN = grp[t];
            loN = A.off[cN];
            hiN = A.off[cN + 1];
            e0N = loN + lane < hiN ? A.adj[loN + lane] : 0u;
        }
        while (t < (int)ngroups) {
            const uint32_t c = cN, clo = loN, chi = hiN, e0 = e0N;
            const int tn = wave_next(&L.task);
            const bool more = tn < (int)ngroups;
            if (more) cN = grp[tn];
            if (lane == 0) work[0]++;
            // A(c): c's neighbours in N+(r), as (slot << 2) | arc bits seen from the slot
            // The same pass counts the valid ends e of the (1,1,1) paths r - x - c - e (e above
            // r, not in N+(r)) by the arc code ce, and the entries below r (a prefix: rows are
            // sorted by rank).
            uint32_t* Ac = wlist;
            uint32_t p = 0;
            uint32_t T1 = 0, T2 = 0, T3 = 0, nlow = 0;
            for (uint32_t base = clo; base < chi; base += 64) {
                const uint32_t tt = base + lane;
                uint32_t e = 0;
                int sl = -1;
                if (tt < chi) {
                    e = base == clo ? e0 : A.adj[tt];
                    if ((e >> 2) > r) sl = find_slot_f(L, d, e >> 2);
                }
                const unsigned long long mk = __ballot(sl >= 0);
                if (sl >= 0) Ac[p + __popcll(mk & lt_mask)] = ((uint32_t)sl << 2) | swap_arc_bits(e & 3u);
                p += __popcll(mk);
                const bool ev = tt < chi && (e >> 2) > r && sl < 0;
                T1 += __popcll(__ballot(ev && (e & 3u) == 1u));
                T2 += __popcll(__ballot(ev && (e & 3u) == 2u));
                T3 += __popcll(__ballot(ev && (e & 3u) == 3u));
                nlow += __popcll(__ballot(tt < chi && (e >> 2) < r));
                if (lane == 0) work[1]++;
            }
            __threadfence_block();
            for (uint32_t u = lane; u < p; u += 64) {
                const uint32_t x = Ac[u] >> 2;
                atomicOr(&inA[x >> 5], 1u << (x & 31));
            }
            bool e0_done = false;
            if (more) {   // next group: row bounds
                loN = A.off[cN];
                hiN = A.off[cN + 1];
            }
            if (A.k3) {
                for (uint32_t u = lane; u < p; u += 64) {
                    const uint32_t ex = Ac[u], x = ex >> 2, xc = ex & 3u, rx = L.P[x] & 3u;
                    const uint32_t cls = L.t3[motif_index3(rx, 0u, xc)];
                    atomicAdd(&cw[54 + cls], 1u);
                    shape[1]++;
                }
            }
            const unsigned long long tg0 = wall_clock64();
            unsigned long long tg1 = tg0, tg2 = tg0, tg3 = tg0;
            if (A.k4) {
                // per code g = (rx - 1) * 3 + (xc - 1) of the parents: hist[rx] packs, per xc,
                // the number of parents in A(c) (21-bit fields); ha* = parents per rx
                unsigned long long hist1 = 0, hist2 = 0, hist3 = 0;
                for (uint32_t ub = 0; ub < p; ub += 64) {
                    const uint32_t u = ub + lane;
                    const uint32_t ex = u < p ? Ac[u] : 0u;
                    const uint32_t code = u < p ? ((L.P[ex >> 2] & 3u) - 1u) * 3u + ((ex & 3u) - 1u) : 9u;
#pragma unroll
                    for (uint32_t q = 0; q < 9; q++) {
                        const unsigned long long nq = (unsigned long long)__popcll(__ballot(code == q));
                        const unsigned long long inc = nq << (21u * (q % 3u));
                        if (q < 3) hist1 += inc; else if (q < 6) hist2 += inc; else hist3 += inc;
                    }
                }
                auto field = [&](uint32_t q) -> uint32_t {
                    const unsigned long long w = q < 3 ? hist1 : (q < 6 ? hist2 : hist3);
                    return (uint32_t)(w >> (21u * (q % 3u))) & F21;
                };
                const uint32_t ha1 = field(0) + field(1) + field(2);
                const uint32_t ha2 = field(3) + field(4) + field(5);
                const uint32_t ha3 = field(6) + field(7) + field(8);
                // (2,1,0), y outside A(c): for a parent x every slot y not in A(c) makes a set
                // {r, x, y, c}.  Those with y not adjacent to x (class fixed by rx, xc, ry) are
                // counted by complement: gall[g] stands for every slot; the slots of A(c) and
                // x's local neighbours outside A(c) are subtracted from their own counters
                // (modular; they end non-negative).  x's local neighbours outside A(c) are the
                // sets with an x-y arc and take the direct path.
                // One entry y of x's local list: a direct set if y is outside A(c); else (rare)
                // the pair {x, y} of parents with an x-y arc, counted below as if it had none,
                // is moved to its class.  Returns ry for a set, 0 otherwise.
                auto local_entry = [&](uint32_t x, uint32_t rx, uint32_t xc, uint32_t g, uint32_t vq) -> uint32_t {
                    const uint32_t y = vq >> 2, xy = vq & 3u, py = L.P[y], ry = py & 3u;
                    if (!((inA[y >> 5] >> (y & 31)) & 1u)) {
                        atomicAdd(&L.cnt[g * d + y], 0xFFFFFFFFu);
                        slow[3]++;
                        const uint32_t cls = L.t4[motif_index4(rx, ry, 0u, xy, xc, 0u)];
                        atomicAdd(&L.root4[cls], 1ull);
                        add4(A, L, L.P[x] >> 2, cls, 1);
                        add4(A, L, py >> 2, cls, 1);
                        add4(A, L, c, cls, 1);
                        return ry;
                    }
                    if (x < y) {
                        uint32_t yc = 0;
                        for (uint32_t w = 0; w < p; w++)
                            if ((Ac[w] >> 2) == y) {
                                yc = Ac[w] & 3u;
                                break;
                            }
                        slow[3]++;
                        const uint32_t c0 = L.t4[motif_index4(rx, ry, 0u, 0u, xc, yc)];
                        const uint32_t c1 = L.t4[motif_index4(rx, ry, 0u, xy, xc, yc)];
                        atomicAdd(&L.root4[c0], ~0ull);
                        atomicAdd(&L.root4[c1], 1ull);
                        add4(A, L, L.P[x] >> 2, c0, ~0ull);
                        add4(A, L, py >> 2, c0, ~0ull);
                        add4(A, L, c, c0, ~0ull);
                        add4(A, L, L.P[x] >> 2, c1, 1);
                        add4(A, L, py >> 2, c1, 1);
                        add4(A, L, c, c1, 1);
                    }
                    return 0u;
                };
                // x's sets with a pure y, by ry = k: the slots minus A(c) minus the direct ones
                auto pure_parent = [&](uint32_t x, uint32_t xc, uint32_t g, uint32_t k, uint32_t nk) {
                    if (!nk) return;
                    atomicAdd(&spar[((xc - 1u) * 3u + (k - 1u)) * PMAX + x], nk);
                    atomicAdd(&cw[g * 3u + (k - 1u)], nk);
                };
                // parents with a short local list: one lane per parent; the others: the wave
                for (uint32_t ub = 0; ub < p; ub += 64) {
                    const uint32_t u = ub + lane;
                    const uint32_t ex = u < p ? Ac[u] : 0u;
                    const uint32_t x = ex >> 2, xc = ex & 3u;
                    const uint32_t xl = u < p ? L.lcnt[x] : 0u;
                    const bool small = u < p && xl <= kLaneList;
                    if (small) {
                        const uint32_t rx = L.P[x] & 3u, g = (rx - 1u) * 3u + (xc - 1u), xq = L.pre[x];
                        uint32_t n1 = 0, n2 = 0, n3 = 0;
                        for (uint32_t q = 0; q < xl; q++) {
                            const uint32_t ry = local_entry(x, rx, xc, g, llist[xq + q]);
                            n1 += ry == 1u;
                            n2 += ry == 2u;
                            n3 += ry == 3u;
                        }
                        atomicAdd(&L.gall[g], 1u);
                        shape[3] += d - p;
                        pure_parent(x, xc, g, 1, nr1 - ha1 - n1);
                        pure_parent(x, xc, g, 2, nr2 - ha2 - n2);
                        pure_parent(x, xc, g, 3, nr3 - ha3 - n3);
                    }
                    unsigned long long big = __ballot(u < p && !small);
                    while (big) {
                        const int bl = __ffsll((long long)big) - 1;
                        big &= big - 1ull;
                        const uint32_t bx = (uint32_t)__shfl((int)ex, bl);
                        const uint32_t x2 = bx >> 2, xc2 = bx & 3u, rx2 = L.P[x2] & 3u;
                        const uint32_t g2 = (rx2 - 1u) * 3u + (xc2 - 1u);
                        const uint32_t xl2 = L.lcnt[x2], xq2 = L.pre[x2];
                        if (lane == 0) work[3]++;
                        uint32_t n1 = 0, n2 = 0, n3 = 0;
                        for (uint32_t qb = 0; qb < xl2; qb += 64) {
                            const uint32_t q = qb + lane;
                            const uint32_t ry = q < xl2 ? local_entry(x2, rx2, xc2, g2, llist[xq2 + q]) : 0u;
                            n1 += __popcll(__ballot(ry == 1u));
                            n2 += __popcll(__ballot(ry == 2u));
                            n3 += __popcll(__ballot(ry == 3u));
                        }
                        if (lane == 0) {
                            atomicAdd(&L.gall[g2], 1u);
                            shape[3] += d - p;
                            pure_parent(x2, xc2, g2, 1, nr1 - ha1 - n1);
                            pure_parent(x2, xc2, g2, 2, nr2 - ha2 - n2);
                            pure_parent(x2, xc2, g2, 3, nr3 - ha3 - n3);
                        }
                    }
                }
                // A(c)'s own slots are not outside A(c): one set fewer per parent
                for (uint32_t u = lane; u < p; u += 64) {
                    const uint32_t y = Ac[u] >> 2;
                    for (uint32_t q = 0; q < 9; q++) {
                        const uint32_t h = field(q);
                        if (h) atomicAdd(&L.cnt[q * d + y], 0u - h);
                    }
                }
                tg1 = wall_clock64();
                // (2,1,0) with both depth-1 vertices in A(c): pairs {x, y} of parents.  With no
                // x-y arc a pair's class is fixed by the two parents' codes, so the pairs are
                // counted from the code histogram: c and the root per pair of codes, each parent
                // per partner code.  The pairs with an x-y arc were moved to their classes in
                // the local-list walk above.
                if (lane < 45) {   // lane -> codes q1 <= q2
                    uint32_t q1 = 0, rem = lane;
                    while (rem >= 9u - q1) {
                        rem -= 9u - q1;
                        q1++;
                    }
                    const uint32_t q2 = q1 + rem, f1 = field(q1), f2 = field(q2);
                    const uint32_t n = q1 == q2 ? f1 * (f1 - 1u) / 2u : f1 * f2;
                    if (n) {
                        const uint32_t cls = L.t4[motif_index4(q1 / 3u + 1u, q2 / 3u + 1u, 0u, 0u, q1 % 3u + 1u, q2 % 3u + 1u)];
                        add4(A, L, c, cls, n);
                        atomicAdd(&L.root4[cls], (unsigned long long)n);
                        shape[3] += n;
                    }
                }
                for (uint32_t u = lane; u < p; u += 64) {
                    const uint32_t ex = Ac[u], x = ex >> 2, xc = ex & 3u, px = L.P[x];
                    const uint32_t qx = ((px & 3u) - 1u) * 3u + (xc - 1u);
#pragma unroll
                    for (uint32_t q2 = 0; q2 < 9; q2++) {
                        const uint32_t n = field(q2) - (q2 == qx ? 1u : 0u);
                        if (n)
                            add4(A, L, px >> 2, L.t4[motif_index4(px & 3u, q2 / 3u + 1u, 0u, 0u, xc, q2 % 3u + 1u)], n);
                    }
                }
                tg2 = wall_clock64();
                if (more) {   // next group: first chunk
                    e0N = loN + lane < hiN ? A.adj[loN + lane] : 0u;
                    e0_done = true;
                }
                // (1,1,1): paths r - x - c - e, e above r, not in N(r), not adjacent to x.
                // Counted by complement: here every x in A(c) is paired with every valid e
                // of c's row, adjacent to x or not.  A pair with e adjacent to x is a (1,2,0)
                // set of x whose two depth-2 vertices c, e are adjacent; the (1,2,0) phase
                // enumerates those and takes both orders (c, e) and (e, c) back out.  So a
                // chunk of c's row needs no test against the parents' rows.
                // The end vertex e of these paths is credited by a pass after the kernel: the
                // parent codes of this group go into w111[c], and every vertex e later adds
                // w111 of all its neighbours.  That pass also reaches the entries of c's row
                // that are not valid here (e below r, or e in N+(r)); those are taken off now.
                // the entries of c's row that are not valid ends: the parents themselves (their
                // arc code from c is the swap of the stored one) and the prefix below r
                auto take_off = [&](uint32_t e, uint32_t ce) {
                    for (uint32_t q = 0; q < 9; q++) {
                        const uint32_t cnt = field(q);
                        if (cnt)
                            add4(A, L, e, L.t4[motif_index4(q / 3 + 1, 0u, 0u, q % 3 + 1, 0u, ce)],
                                 0ull - (unsigned long long)cnt);
                    }
                };
                for (uint32_t u = lane; u < p; u += 64) {
                    const uint32_t ex = Ac[u];
                    take_off(L.P[ex >> 2] >> 2, swap_arc_bits(ex & 3u));
                }
                for (uint32_t tt = clo + lane; tt < clo + nlow; tt += 64) {
                    const uint32_t ee = A.adj[tt];
                    take_off(ee >> 2, ee & 3u);
                }
                if (lane == 0) {
                    shape[5] += p * (T1 + T2 + T3);
                    work[2] += p;
                }
                if (lane < 9) {
                    const unsigned long long w = lane < 3 ? hist1 : (lane < 6 ? hist2 : hist3);
                    const uint32_t cnt = (uint32_t)(w >> (21u * (lane % 3))) & F21;
                    if (cnt) atomicAdd(&A.w111[(size_t)c * 9 + lane], cnt);
                }
                // every parent x is on T_k of these paths with ce = k (x's and c's credits)
                if (T1 | T2 | T3)
                    for (uint32_t u = lane; u < p; u += 64) {
                        const uint32_t ex = Ac[u], x = ex >> 2, xc = (ex & 3u) - 1u;
                        const uint32_t code = ((L.P[x] & 3u) - 1u) * 3u + xc;
                        auto put = [&](uint32_t k, uint32_t h) {
                            if (!h) return;
                            atomicAdd(&s111[(xc * 3 + k) * PMAX + x], h);
                            atomicAdd(&cw[27 + code * 3 + k], h);
                        };
                        put(0, T1);
                        put(1, T2);
                        put(2, T3);
                    }
            }
            tg3 = A.k4 ? wall_clock64() : tg0;
            if (more && !e0_done) e0N = loN + lane < hiN ? A.adj[loN + lane] : 0u;
            // flush the group's depth-2 vertex (and the root, which is in every one of its sets)
            for (uint32_t q = lane; q < 27 + 27 + kClasses3; q += 64) {
                const uint32_t cnt = cw[q];
                if (!cnt) continue;
                cw[q] = 0;
                if (q < 54) {
                    const uint32_t qq = q % 27, rx = qq / 9 + 1, xc = (qq / 3) % 3 + 1, z = qq % 3 + 1;
                    const uint32_t code = q < 27 ? motif_index4(rx, z, 0u, 0u, xc, 0u)      // (2,1,0): z = ry
                                                 : motif_index4(rx, 0u, 0u, xc, 0u, z);    // (1,1,1): z = ce
                    const uint32_t cls = L.t4[code];
                    add4(A, L, c, cls, cnt);
                    atomicAdd(&L.root4[cls], (unsigned long long)cnt);
                } else {
                    add_out(A.out3, A.perm, kClasses3, c, q - 54, cnt);
                }
            }
            for (uint32_t u = lane; u < p; u += 64) {
                const uint32_t x = Ac[u] >> 2;
                atomicAnd(&inA[x >> 5], ~(1u << (x & 31)));
            }
            if (lane == 0) {   // per-wave time split of the group shapes (diagnostic)
                const unsigned long long tg4 = wall_clock64();
                atomicAdd(&L.stat[24], tg1 - tg0);
                atomicAdd(&L.stat[25], tg2 - tg1);
                atomicAdd(&L.stat[26], tg3 - tg2);
                atomicAdd(&L.stat[27], tg4 - tg3);
            }
            t = tn;
        }
        // Single-parent groups with a short row (most groups): one lane per group, the same
        // sets and credits as above with A(c) = {x}.  Task ids past ngroups are chunks of 64.
        const unsigned long long tw1 = wall_clock64();
        {
            const uint32_t nsgl = L.sgroups;
            const int nall = (int)(ngroups + (nsgl + 63) / 64);
            for (; t < nall; t = wave_next(&L.task)) {
                const uint32_t i = (uint32_t)(t - (int)ngroups) * 64u + lane;
                if (i >= nsgl) continue;
                const uint32_t c = sgrp[2 * i], xw = sgrp[2 * i + 1];
                const uint32_t x = xw >> 2, xc = xw & 3u;
                const uint32_t clo = A.off[c], chi = A.off[c + 1];
                const uint32_t rx = L.P[x] & 3u, vx = L.P[x] >> 2;
                if (A.k3) {   // k=3 (1,2): {r, x, c}
                    add_out(A.out3, A.perm, kClasses3, c, L.t3[motif_index3(rx, 0u, xc)], 1);
                    shape[1]++;
                }
                if (!A.k4) continue;
                const uint32_t g = (rx - 1u) * 3u + (xc - 1u);
                // (2,1,0): {r, x, y, c} for every slot y other than x.  The sets' numbers by
                // class come from x's profile (y a local neighbour of x: x-y arc) and from the
                // slot counts by ry (the pure rest), so c and the root are credited per class
                // here; x's and y's credits are made per slot after the groups (nsg).
                uint32_t nry[3];
#pragma unroll
                for (uint32_t k = 0; k < 3; k++) {
                    const unsigned long long w = prof[k * PMAX + x];
                    nry[k] = 0;
#pragma unroll
                    for (uint32_t xy = 1; xy <= 3; xy++) {
                        const uint32_t h = (uint32_t)(w >> (21u * (xy - 1u))) & F21;
                        if (!h) continue;
                        nry[k] += h;
                        const uint32_t cls = L.t4[motif_index4(rx, k + 1u, 0u, xy, xc, 0u)];
                        atomicAdd(&L.root4[cls], (unsigned long long)h);
                        add4(A, L, c, cls, h);
                    }
                }
                auto pure210 = [&](uint32_t k, uint32_t nk) {   // x's sets with a pure y, ry = k
                    if (!nk) return;
                    const uint32_t cls = L.t4[motif_index4(rx, k, 0u, 0u, xc, 0u)];
                    add4(A, L, c, cls, nk);
                    atomicAdd(&L.root4[cls], (unsigned long long)nk);
                };
                pure210(1, nr1 - (rx == 1u) - nry[0]);
                pure210(2, nr2 - (rx == 2u) - nry[1]);
                pure210(3, nr3 - (rx == 3u) - nry[2]);
                // (1,1,1): c's row; the valid ends by ce, the other entries taken off
                uint32_t T1 = 0, T2 = 0, T3 = 0;
                for (uint32_t tb = clo; tb < chi; tb += 8) {   // batches of 8 row entries
                    uint32_t en[8];
#pragma unroll
                    for (int j = 0; j < 8; j++) en[j] = tb + j < chi ? A.adj[tb + j] : 0u;
#pragma unroll
                    for (int j = 0; j < 8; j++) {
                        if (tb + j >= chi) break;
                        const uint32_t e = en[j] >> 2, ce = en[j] & 3u;
                        if (e < r || e == vx) {   // below r, or x (c's only neighbour in N+(r))
                            add4(A, L, e, L.t4[motif_index4(rx, 0u, 0u, xc, 0u, ce)], ~0ull);
                        } else {
                            T1 += ce == 1u;
                            T2 += ce == 2u;
                            T3 += ce == 3u;
                        }
                    }
                }
                shape[5] += T1 + T2 + T3;
                atomicAdd(&A.w111[(size_t)c * 9 + g], 1u);
                auto path111 = [&](uint32_t k, uint32_t tk) {
                    if (!tk) return;
                    atomicAdd(&s111[((xc - 1u) * 3u + (k - 1u)) * PMAX + x], tk);
                    const uint32_t cls = L.t4[motif_index4(rx, 0u, 0u, xc, 0u, k)];
                    add4(A, L, c, cls, tk);
                    atomicAdd(&L.root4[cls], (unsigned long long)tk);
                };
                path111(1, T1);
                path111(2, T2);
                path111(3, T3);
            }
        }
        if (lane == 0) {   // per-wave time in the two group loops (diagnostic)
            const unsigned long long tw2 = wall_clock64();
            atomicAdd(&L.stat[22], tw1 - tw0);
            atomicAdd(&L.stat[23], tw2 - tw1);
        }
        __threadfence();
        __syncthreads();
        // The single-parent groups' (2,1,0) credits of x and of the slots y, per slot x:
        // nsg[xc][x] groups, each a set {r, x, y, c} with every slot y other than x.  y a
        // local neighbour of x (x-y arc): x takes its profile times the group count, y one
        // credit per parent code.  Pure y: x's credit by ry from the slot counts, y's by
        // complement (gall stands for every slot; x itself and x's local neighbours are
        // taken back from their own counters).  One wave per slot x.
        if (A.k4)
            for (uint32_t x = wid; x < d; x += NW) {
                const uint32_t m1 = nsg[x], m2 = nsg[PMAX + x], m3 = nsg[2 * PMAX + x];
                if (!(m1 | m2 | m3)) continue;
                const uint32_t rx = L.P[x] & 3u, vx = L.P[x] >> 2;
                const uint32_t xl = L.lcnt[x];
                if (lane < 27) {   // lane = (xc-1)*9 + (ry-1)*3 + (xy-1): sets with an x-y arc
                    const uint32_t xc = lane / 9u + 1u, ry = (lane / 3u) % 3u + 1u, xy = lane % 3u + 1u;
                    const uint32_t m = xc == 1u ? m1 : (xc == 2u ? m2 : m3);
                    const uint32_t h = (uint32_t)(prof[(ry - 1u) * PMAX + x] >> (21u * (xy - 1u))) & F21;
                    if (m && h) {
                        add4(A, L, vx, L.t4[motif_index4(rx, ry, 0u, xy, xc, 0u)], (unsigned long long)m * h);
                        slow[3] += m * h;
                    }
                } else if (lane >= 32 && lane < 41) {   // lane - 32 = (xc-1)*3 + (ry-1): pure y
                    const uint32_t xc = (lane - 32u) / 3u + 1u, ry = (lane - 32u) % 3u + 1u;
                    const uint32_t m = xc == 1u ? m1 : (xc == 2u ? m2 : m3);
                    const unsigned long long w = prof[(ry - 1u) * PMAX + x];
                    const uint32_t nl = ((uint32_t)w & F21) + ((uint32_t)(w >> 21) & F21) + ((uint32_t)(w >> 42) & F21);
                    const uint32_t nr = ry == 1u ? nr1 : (ry == 2u ? nr2 : nr3);
                    const uint32_t nk = nr - (rx == ry) - nl;
                    if (m && nk) spar[(lane - 32u) * PMAX + x] += m * nk;   // one lane per counter
                } else if (lane >= 48 && lane < 51) {   // lane - 48 = xc - 1: complement of y
                    const uint32_t m = lane == 48 ? m1 : (lane == 49 ? m2 : m3);
                    if (m) {
                        const uint32_t g = (rx - 1u) * 3u + (lane - 48u);
                        atomicAdd(&L.gall[g], m);
                        atomicAdd(&L.cnt[g * d + x], 0u - m);
                        shape[3] += m * (d - 1u);
                    }
                }
                const uint32_t xq = L.pre[x];
                for (uint32_t q = lane; q < xl; q += 64) {
                    const uint32_t vq = llist[xq + q], y = vq >> 2, xy = vq & 3u;
                    const uint32_t ry = L.P[y] & 3u, vy = L.P[y] >> 2;
#pragma unroll
                    for (uint32_t xc = 1; xc <= 3; xc++) {
                        const uint32_t m = xc == 1u ? m1 : (xc == 2u ? m2 : m3);
                        if (!m) continue;
                        atomicAdd(&L.cnt[((rx - 1u) * 3u + (xc - 1u)) * d + y], 0u - m);
                        add4(A, L, vy, L.t4[motif_index4(rx, ry, 0u, xy, xc, 0u)], m);
                    }
                }
                if (lane == 0) {
                    nsg[x] = 0;
                    nsg[PMAX + x] = 0;
                    nsg[2 * PMAX + x] = 0;
                }
            }
        __syncthreads();
        if (A.k4) {
            for (uint32_t q = tid; q < 9 * d; q += HT) {
                const uint32_t g = q / d;
                const uint32_t cnt = L.cnt[q] + L.gall[g];   // (2,1,0) sets with this slot as y
                if (!cnt) continue;
                const uint32_t s = q % d, rx = g / 3 + 1, xc = g % 3 + 1;
                add4(A, L, L.P[s] >> 2,
                        L.t4[motif_index4(rx, L.P[s] & 3u, 0u, 0u, xc, 0u)], cnt);
            }
        }
        if (tid == 0) L.task = 0;
        __syncthreads();
        HUB_PHASE(5);

        // (1,2,0) sets: k_slot_pairs, after this kernel (one task per (root, slot))
        __threadfence();
        __syncthreads();
        HUB_PHASE(6);

        // ---------------------------------------------------------------- per-root flush
        const uint32_t row = (uint32_t)A.perm[r];
        if (A.k4)
            for (uint32_t q = tid; q < kClasses4; q += HT)
                if (L.root4[q]) atomicAdd(&A.out4[(size_t)row * kClasses4 + q], L.root4[q]);
        if (A.k3)
            for (uint32_t q = tid; q < kClasses3; q += HT)
                if (L.root3[q]) atomicAdd(&A.out3[(size_t)row * kClasses3 + q], L.root3[q]);
        for (uint32_t q = tid; q < 9 * d; q += HT) {
            const uint32_t s = q % d, g = q / d, rs = L.P[s] & 3u, vs = L.P[s] >> 2;
            const uint32_t a = spar[g * PMAX + s], b = s111[g * PMAX + s];
            if (a) {   // (2,1,0) parent: g = (xc-1)*3 + (ry-1)
                add4(A, L, vs, L.t4[motif_index4(rs, g % 3 + 1, 0u, 0u, g / 3 + 1, 0u)], a);
                spar[g * PMAX + s] = 0;
            }
            if (b) {   // (1,1,1) depth-1: g = (xc-1)*3 + (ce-1)
                add4(A, L, vs, L.t4[motif_index4(rs, 0u, 0u, g / 3 + 1, 0u, g % 3 + 1)], b);
                s111[g * PMAX + s] = 0;
            }
            if (g < 3) {
                const uint32_t x3 = s3x[g * PMAX + s];
                if (x3) {
                    add_out(A.out3, A.perm, kClasses3, vs, L.t3[motif_index3(rs, 0u, g + 1)], x3);
                    s3x[g * PMAX + s] = 0;
                }
            }
        }
        for (int k = 0; k < kShapes; k++) {
            // per-lane counts are 32-bit and can be negative for (1,1,1) (its complement
            // corrections land on other lanes): sign-extend before the wave sum
            unsigned long long v = k == 5 ? (unsigned long long)(long long)(int32_t)shape[k] : shape[k];
            unsigned long long w = slow[k];
            for (int o = 32; o > 0; o >>= 1) {
                v += __shfl_down(v, o);
                w += __shfl_down(w, o);
            }
            if (lane == 0 && v) atomicAdd(&L.stat[k], v);
            if (lane == 0 && w) atomicAdd(&L.stat[16 + k], w);
            shape[k] = 0;
            slow[k] = 0;
        }
        if (lane == 0)
            for (int k = 0; k < 4; k++) {
                if (work[k]) atomicAdd(&L.stat[28 + k], (unsigned long long)work[k]);
                work[k] = 0;
            }
        __syncthreads();
        HUB_PHASE(7);
    }
#undef HUB_PHASE
    __syncthreads();
    for (uint32_t k = tid; k < kLdsStatSlots; k += HT)
        if (L.stat[k]) {
            atomicAdd(&A.stats[k], L.stat[k]);
            if (k < kShapes) atomicAdd(&A.stats[32 + k], L.stat[k]);
        }
}


// ----------------------------------------------------------------------------- (1,2,0)

// (1,2,0) sets of the hub roots, one wave per task (root r, slot a of N+(r)).  The pairs
// {c1, c2} of a's depth-2 children L_a (m of them, m_k with arc code k from a) are the
// (1,2,0) sets of (r, a).  A pair of non-adjacent children has a class fixed by
// (ra, ac1, ac2): those are counted from m_1..m_3 by complement.  Only the adjacent pairs
// are found and credited one by one, and taken off the complement totals and off the
// (1,1,1) counts of the two groups that also counted them: a child whose row has at most
// kShortRow entries walks it and looks each neighbour up in a hash of L_a's positions; a
// pair of two longer-row children is looked up in the edge hash.  The list holds the
// long-row children first, positions [0, kl).  Separate from k_hub so that it runs with
// a small register and LDS footprint at full occupancy.
struct SlotPairArgs {
    const uint32_t* off;
    const uint32_t* adj;
    const uint32_t* split;
    const int32_t* perm;
    const uint32_t* hubs;        // hub roots (rank), queue order
    uint32_t nhub;
    const uint32_t* hub_pre;     // nhub + 1 prefix sums of |N+(r)| in queue order
    uint32_t rank_lo, rank_hi;
    const uint8_t* t4;
    const uint8_t* slot4;
    unsigned long long* out4;
    unsigned long long* comp;
    unsigned long long* stats;
    const unsigned long long* ehash;
    const uint16_t* efp;         // fingerprints of the edge hash
    uint32_t ehash_bits;
    const uint32_t* lbits;       // adjacency bitmap among the long-row vertices (ranks < nlong), or null
    uint32_t nlong, lwords;      // long-row vertices, 32-bit words per bitmap row
    unsigned* cursor;            // task cursor, zeroed before the launch
    uint32_t* scratch;           // per wave: list, partner counts, hash keys, hash values
    size_t wave_words;
    uint32_t wl_cap;
    uint32_t hash_bits;
};
constexpr int SP = 256;   // threads per workgroup of k_slot_pairs
constexpr uint32_t kLHashBits = 9;
constexpr uint32_t kLHash = 1u << kLHashBits;

__global__ __launch_bounds__(SP) void k_slot_pairs(SlotPairArgs A) {
    __shared__ uint8_t t4[4096];
    __shared__ uint8_t slot4[kClasses4 + 1];
    __shared__ uint32_t sig6w[SP / 64][8];
    __shared__ uint32_t lkey[SP / 64][kLHash];   // per-wave hash of L_a when m <= kLHash / 2
    __shared__ uint32_t lval[SP / 64][kLHash];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    for (uint32_t i = tid; i < 4096; i += SP) t4[i] = A.t4[i];
    for (uint32_t i = tid; i < kClasses4; i += SP) slot4[i] = A.slot4[i];
    if (lane < 8) sig6w[wid][lane] = 0;
    __syncthreads();
    uint32_t* sig6 = sig6w[wid];
    uint32_t* W = A.scratch + ((size_t)blockIdx.x * (SP / 64) + wid) * A.wave_words;
    uint32_t* wlist = W;
    uint32_t* c120 = W + A.wl_cap;
    const uint32_t hsize = 1u << A.hash_bits;
    uint32_t* hkey = W + 4 * (size_t)A.wl_cap;
    uint32_t* hval = hkey + hsize;
    for (uint32_t i = lane; i < hsize; i += 64) hkey[i] = 0;
    for (uint32_t i = lane; i < kLHash; i += 64) lkey[wid][i] = 0;
    __threadfence_block();
    auto credit = [&](uint32_t v, uint32_t cls, unsigned long long cnt) {
        if (!cnt || cls >= kClasses4) return;
        const uint32_t sl = slot4[cls];
        if (sl != 0xFFu) atomicAdd(&A.comp[(size_t)v * kCompact4 + sl], cnt);
        else atomicAdd(&A.out4[(size_t)A.perm[v] * kClasses4 + cls], cnt);
    };
    unsigned long long n120 = 0, n111 = 0, nslow = 0;   // per lane: (1,2,0) sets, (1,1,1) change, direct sets
    const uint32_t ntask = A.hub_pre[A.nhub];
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(A.cursor, 1u);
        t = __shfl(t, 0);
        if (t >= ntask) break;
        uint32_t lo = 0, hi = A.nhub;   // root: last index with hub_pre <= t
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (A.hub_pre[mid] <= t) lo = mid; else hi = mid;
        }
        const uint32_t r = A.hubs[lo];
        if (r < A.rank_lo || r >= A.rank_hi) continue;
        const uint32_t ent_a = A.adj[A.split[r] + (t - A.hub_pre[lo])];
        const uint32_t va = ent_a >> 2, ra = ent_a & 3u;
        const uint32_t ahi = A.off[va + 1];
        const uint32_t alo = lower_bound_rank(A.adj, A.off[va], ahi, r + 1);
        // depth-2 children of a: entries above r not adjacent to r; long rows first
        uint32_t kl = 0, ns = 0;
        uint32_t nbig = 0;   // children, counted first to place the short ones at the end
        for (uint32_t qb = alo; qb < ahi; qb += 64) {
            const uint32_t q = qb + lane;
            bool f = false;
            if (q < ahi) f = edge_code_fp(A.efp, A.ehash, A.ehash_bits, r, A.adj[q] >> 2) == 0u;
            nbig += __popcll(__ballot(f));
        }
        const uint32_t m = nbig;
        if (m < 2) continue;
        for (uint32_t qb = alo; qb < ahi; qb += 64) {
            const uint32_t q = qb + lane;
            bool f = false, lg = false;
            uint32_t ent = 0;
            if (q < ahi) {
                ent = A.adj[q];
                f = edge_code_fp(A.efp, A.ehash, A.ehash_bits, r, ent >> 2) == 0u;
                if (f) lg = A.off[(ent >> 2) + 1] - A.off[ent >> 2] > kShortRow;
            }
            const unsigned long long ml = __ballot(f && lg), ms = __ballot(f && !lg);
            if (f && lg) wlist[kl + __popcll(ml & lt_mask)] = ent;
            if (f && !lg) wlist[m - 1u - (ns + __popcll(ms & lt_mask))] = ent;
            kl += __popcll(ml);
            ns += __popcll(ms);
        }
        uint32_t m1 = 0, m2 = 0, m3 = 0;
        for (uint32_t q = lane; q < 3 * m; q += 64) c120[q] = 0;
        __threadfence_block();
        for (uint32_t ub = 0; ub < m; ub += 64) {
            const uint32_t ac = ub + lane < m ? (wlist[ub + lane] & 3u) : 0u;
            m1 += __popcll(__ballot(ac == 1u));
            m2 += __popcll(__ballot(ac == 2u));
            m3 += __popcll(__ballot(ac == 3u));
        }
        __threadfence_block();
        const size_t rrow = (size_t)A.perm[r] * kClasses4;
        // one adjacent pair: children at positions ux, uy, cc = arc bits seen from x
        auto adjacent_pair = [&](uint32_t ux, uint32_t uy, uint32_t ex, uint32_t ey, uint32_t cc) {
            const uint32_t cx = ex >> 2, acx = ex & 3u, cy = ey >> 2, acy = ey & 3u;
            nslow++;
            const uint32_t cls = t4[motif_index4(ra, 0u, 0u, acx, acy, cc)];
            atomicAdd(&A.out4[rrow + cls], 1ull);
            credit(va, cls, 1);
            credit(cx, cls, 1);
            credit(cy, cls, 1);
            atomicAdd(&sig6[pair_sig(acx, acy)], 1u);
            atomicAdd(&c120[ux * 3 + (acy - 1u)], 1u);
            atomicAdd(&c120[uy * 3 + (acx - 1u)], 1u);
            // the groups of cx and cy counted r-a-cx-cy and r-a-cy-cx as (1,1,1) paths;
            // take them out of all four members (every counter here ends non-negative)
            const uint32_t cr = swap_arc_bits(cc);
            const uint32_t p1 = t4[motif_index4(ra, 0u, 0u, acx, 0u, cc)];
            const uint32_t p2 = t4[motif_index4(ra, 0u, 0u, acy, 0u, cr)];
            const unsigned long long m1n = ~0ull;
            atomicAdd(&A.out4[rrow + p1], m1n);
            atomicAdd(&A.out4[rrow + p2], m1n);
            credit(va, p1, m1n);
            credit(va, p2, m1n);
            credit(cx, p1, m1n);
            credit(cy, p1, m1n);
            credit(cx, p2, m1n);
            credit(cy, p2, m1n);
            n111 -= 2;
        };
        // short-row children: walk the row against a hash of L_a's positions (in LDS when
        // L_a is small); a short partner is taken by the lower position
        auto short_walks = [&](uint32_t* hk, uint32_t* hv, uint32_t hbits) {
            const uint32_t hmask = (1u << hbits) - 1u;
            for (uint32_t q = lane; q < m; q += 64) {
                const uint32_t key = (wlist[q] >> 2) + 1u;
                uint32_t h = (key * 2654435761u) >> (32u - hbits);
                while (true) {
                    const uint32_t old = atomicCAS(&hk[h], 0u, key);
                    if (old == 0u || old == key) break;
                    h = (h + 1u) & hmask;
                }
                hv[h] = q;
            }
            __threadfence_block();
            for (uint32_t u = kl + lane; u < m; u += 64) {
                const uint32_t ey = wlist[u], cy = ey >> 2;
                const uint32_t hi2 = A.off[cy + 1];
                for (uint32_t t2 = A.off[cy]; t2 < hi2; t2++) {
                    const uint32_t ew = A.adj[t2];
                    if ((ew >> 2) <= r) continue;   // L_a lies above r
                    const uint32_t key = (ew >> 2) + 1u;
                    uint32_t h = (key * 2654435761u) >> (32u - hbits);
                    uint32_t pos = 0xFFFFFFFFu;
                    while (true) {
                        const uint32_t kk = hk[h];
                        if (kk == 0u) break;
                        if (kk == key) { pos = hv[h]; break; }
                        h = (h + 1u) & hmask;
                    }
                    if (pos == 0xFFFFFFFFu || (pos >= kl && pos < u)) continue;
                    adjacent_pair(u, pos, ey, wlist[pos], ew & 3u);
                }
            }
            __threadfence_block();
            for (uint32_t q = lane; q < m; q += 64) {   // clear the table for the next task
                const uint32_t key = (wlist[q] >> 2) + 1u;
                uint32_t h = (key * 2654435761u) >> (32u - hbits);
                while (hk[h] != key) h = (h + 1u) & hmask;
                hk[h] = 0u;
            }
            __threadfence_block();
        };
        if (ns > 0) {
            if (m <= kLHash / 2) short_walks(lkey[wid], lval[wid], kLHashBits);
            else short_walks(hkey, hval, A.hash_bits);
        }
        // pairs of long-row children: the long-vertex bitmap, then the edge hash
        const uint32_t nll = kl * (kl - 1u) / 2u;
        for (uint32_t q = lane; q < nll; q += 64) {
            uint32_t j = (uint32_t)((1.0f + sqrtf(1.0f + 8.0f * (float)q)) * 0.5f);
            while (j * (j - 1u) / 2u > q) j--;
            while ((j + 1u) * j / 2u <= q) j++;
            const uint32_t i = q - j * (j - 1u) / 2u;
            const uint32_t ex = wlist[i], ey = wlist[j];
            uint32_t cc = 0;
            // long-row vertices are the ranks below nlong (ranks follow degree); their
            // adjacency bitmap row of ey stays cache-resident across the lanes of a step
            const bool inbm = A.lbits && (ex >> 2) < A.nlong && (ey >> 2) < A.nlong;
            if (!inbm || ((A.lbits[(size_t)(ey >> 2) * A.lwords + ((ex >> 2) >> 5)] >> ((ex >> 2) & 31u)) & 1u))
                cc = edge_code_fp(A.efp, A.ehash, A.ehash_bits, ex >> 2, ey >> 2);
            if (cc) adjacent_pair(i, j, ex, ey, cc);
        }
        __threadfence_block();
        // every child: its non-adjacent partners by their code k = m_k - own - adjacent
        for (uint32_t u = lane; u < m; u += 64) {
            const uint32_t eu = wlist[u], acu = eu & 3u;
            n120 += m - 1u - u;
            for (uint32_t g = 0; g < 3; g++) {
                const uint32_t mk = g == 0 ? m1 : (g == 1 ? m2 : m3);
                const uint32_t cnt = mk - (acu == g + 1u ? 1u : 0u) - atomicAdd(&c120[u * 3 + g], 0u);
                if (cnt) credit(eu >> 2, t4[motif_index4(ra, 0u, 0u, acu, g + 1u, 0u)], cnt);
            }
        }
        // a and r: non-adjacent pairs by code signature
        if (lane < 6) {
            uint32_t x, y;
            sig_pair(lane, x, y);
            const uint32_t mx = x == 1 ? m1 : (x == 2 ? m2 : m3), my = y == 1 ? m1 : (y == 2 ? m2 : m3);
            const uint32_t total = x == y ? mx * (mx - 1u) / 2u : mx * my;
            const uint32_t cnt = total - atomicAdd(&sig6[lane], 0u);
            sig6[lane] = 0;
            if (cnt) {
                const uint32_t cls = t4[motif_index4(ra, 0u, 0u, x, y, 0u)];
                credit(va, cls, cnt);
                atomicAdd(&A.out4[rrow + cls], (unsigned long long)cnt);
            }
        }
        __threadfence_block();
    }
    // shape counters: (1,2,0) sets, the (1,1,1) correction, direct-path sets; also in the
    // hub-kernel part (entries 32-37)
    for (int o = 32; o > 0; o >>= 1) {
        n120 += __shfl_down(n120, o);
        n111 += __shfl_down(n111, o);
        nslow += __shfl_down(nslow, o);
    }
    if (lane == 0) {
        if (n120) { atomicAdd(&A.stats[4], n120); atomicAdd(&A.stats[36], n120); }
        if (n111) { atomicAdd(&A.stats[5], n111); atomicAdd(&A.stats[37], n111); }
        if (nslow) atomicAdd(&A.stats[20], nslow);
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

// fingerprints of the filled edge-hash slots (0 for empty ones)
__global__ void k_edge_fp(const unsigned long long* __restrict__ table, int64_t slots, uint16_t* __restrict__ fp) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < slots; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long s = table[i];
        fp[i] = s ? edge_fp(s & ~3ull) : (uint16_t)0;
    }
}

__global__ void k_root_work(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj,
                            const uint32_t* __restrict__ split, const uint32_t* __restrict__ roots, int64_t nroots,
                            uint32_t hub_min, uint32_t* __restrict__ is_hub, unsigned long long* __restrict__ wkey,
                            unsigned long long* __restrict__ max_s2, unsigned* __restrict__ max_hi) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nroots; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t r = roots[i];
        const uint32_t s = split[r], e = off[r + 1], d = e - s;
        atomicMax(max_hi, d);
        const bool hub = d >= hub_min && d <= PMAX;
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

__global__ void k_split_bins(const uint32_t* __restrict__ roots, const uint32_t* __restrict__ is_hub,
                             const uint32_t* __restrict__ pos, int64_t nroots, uint32_t* __restrict__ light) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nroots; i += (int64_t)gridDim.x * blockDim.x)
        if (!is_hub[i]) light[i - pos[i]] = roots[i];
}

// out4[perm[v]][class of slot s] += comp[v][s], and comp is cleared for the next launch
// (1,1,1) end-vertex credits: vertex e adds, for every neighbour c, the parent codes
// that c's groups recorded (w111[c][(rx - 1) * 3 + (xc - 1)]), as the path class with the
// arc code ce of c -> e.  One thread per vertex, so the accumulator needs no atomics (the
// hub kernel has finished).
__global__ void k_pull111(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj,
                          const uint32_t* __restrict__ w111, const uint8_t* __restrict__ t4,
                          const uint8_t* __restrict__ slot4, int64_t n, unsigned long long* __restrict__ comp) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long* row = comp + (size_t)e * kCompact4;
        for (uint32_t t = off[e]; t < off[e + 1]; t++) {
            const uint32_t ent = adj[t], c = ent >> 2, ce = swap_arc_bits(ent & 3u);
            const uint32_t* w = w111 + (size_t)c * 9;
            for (uint32_t q = 0; q < 9; q++) {
                const uint32_t cnt = w[q];
                if (!cnt) continue;
                const uint32_t cls = t4[motif_index4(q / 3 + 1, 0u, 0u, q % 3 + 1, 0u, ce)];
                const uint32_t sl = cls < kClasses4 ? slot4[cls] : 0xFFu;
                if (sl < (uint32_t)kCompact4) row[sl] += cnt;   // always a path class
            }
        }
    }
}

__global__ void k_fold_compact(unsigned long long* __restrict__ comp, const uint8_t* __restrict__ slotcls,
                               const int32_t* __restrict__ perm, int64_t n, unsigned long long* __restrict__ out4) {
    const int64_t total = n * kCompact4;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long c = comp[i];
        if (!c) continue;
        const int64_t v = i / kCompact4;
        const int s = (int)(i - v * kCompact4);
        out4[(size_t)perm[v] * kClasses4 + slotcls[s]] += c;
        comp[i] = 0;
    }
}

// number of ranks whose row is longer than kShortRow (rows shrink with the rank)
__global__ void k_count_long(const uint32_t* __restrict__ off, int64_t n, uint32_t* __restrict__ nlong) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const bool lg = off[r + 1] - off[r] > kShortRow;
        const bool next_lg = r + 1 < n && off[r + 2] - off[r + 1] > kShortRow;
        if (lg && !next_lg) *nlong = (uint32_t)(r + 1);
    }
}

// adjacency bitmap among the ranks below nlong: bit (u, v) of row u
__global__ void k_long_bitmap(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj, uint32_t nlong,
                              uint32_t lwords, uint32_t* __restrict__ bits) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < nlong; u += (int64_t)gridDim.x * blockDim.x)
        for (uint32_t t = off[u]; t < off[u + 1]; t++) {
            const uint32_t v = adj[t] >> 2;
            if (v >= nlong) break;   // the row is sorted by rank
            atomicOr(&bits[(size_t)u * lwords + (v >> 5)], 1u << (v & 31u));
        }
}

// |N+(r)| of every hub root, in queue order; entry nhub is 0 (exclusive scan -> total)
__global__ void k_hub_dplus(const uint32_t* __restrict__ off, const uint32_t* __restrict__ split,
                            const uint32_t* __restrict__ hubs, int64_t nhub, uint32_t* __restrict__ dplus) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= nhub; i += (int64_t)gridDim.x * blockDim.x)
        dplus[i] = i < nhub ? off[hubs[i] + 1] - split[hubs[i]] : 0u;
}

__global__ void k_zero_u32(unsigned* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__global__ void k_fill_zero_u32(uint32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
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

int slot_pair_workgroups() { return hub_workgroups() * 6; }   // 24 waves per compute unit (occupancy 6)

}  // namespace


void free_hub(vdmc_graph_s* g) {
    (void)hipFree(g->light);
    (void)hipFree(g->hubs);
    (void)hipFree(g->hub_scratch);
    (void)hipFree(g->hub_queue);
    (void)hipFree(g->hub_comp);
    (void)hipFree(g->hub_w111);
    (void)hipFree(g->hub_pre);
    (void)hipFree(g->sp_scratch);
    (void)hipFree(g->lbits);
    g->lbits = nullptr;
    g->hub_comp = nullptr;
    g->hub_w111 = nullptr;
    g->hub_pre = nullptr;
    g->sp_scratch = nullptr;
    g->light = g->hubs = nullptr;
    g->hub_scratch = nullptr;
    g->hub_queue = nullptr;
    g->bins_hub_min = -1;
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
    const int64_t slots = (int64_t)1 << eb;
    VDMC_HIP(hipMalloc(&g->efp, slots * sizeof(uint16_t)));
    hipLaunchKernelGGL(k_edge_fp, dim3((unsigned)std::min<int64_t>((slots + BT - 1) / BT, 65536)), dim3(BT), 0, st,
                       g->ehash, slots, g->efp);
    VDMC_HIP(hipGetLastError());
    VDMC_HIP(hipStreamSynchronize(st));
    g->ehash_bits = eb;
}

void ensure_bins(vdmc_graph_s* g, hipStream_t st) {
    const int hub_min = g->hub_min;
    if (g->bins_hub_min == hub_min) return;
    free_hub(g);
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
    uint32_t* is_hub = (uint32_t*)alloc((nr + 1) * sizeof(uint32_t));
    uint32_t* pos = (uint32_t*)alloc((nr + 1) * sizeof(uint32_t));
    unsigned long long* wkey = (unsigned long long*)alloc((nr + 1) * sizeof(unsigned long long));
    unsigned long long* wkey_s = (unsigned long long*)alloc((nr + 1) * sizeof(unsigned long long));
    uint32_t* roots_s = (uint32_t*)alloc((nr + 1) * sizeof(uint32_t));
    unsigned long long* d_max = (unsigned long long*)alloc(2 * sizeof(unsigned long long));
    VDMC_HIP(hipMemsetAsync(d_max, 0, 2 * sizeof(unsigned long long), st));
    unsigned* d_maxhi = (unsigned*)(d_max + 1);
    int64_t nhub = 0, nlight = 0;
    unsigned long long max_s2 = 0;
    unsigned maxhi = 0;
    if (nr > 0) {
        unsigned blocks = (unsigned)std::min<int64_t>((nr + BT - 1) / BT, 65536);
        hipLaunchKernelGGL(k_root_work, dim3(blocks), dim3(BT), 0, st, g->off, g->adj, g->split, g->roots, nr,
                           (uint32_t)hub_min, is_hub, wkey, d_max, d_maxhi);
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
        }
        VDMC_HIP(hipStreamSynchronize(st));
    } else {
        VDMC_HIP(hipMalloc(&g->light, sizeof(uint32_t)));
        VDMC_HIP(hipMalloc(&g->hubs, sizeof(uint32_t)));
    }
    g->nhub = nhub;
    g->nlight = nlight;
    g->max_scan2 = (int64_t)max_s2;
    g->max_hi = (int32_t)maxhi;
    VDMC_HIP(hipMalloc(&g->hub_queue, 16));
    if (nhub > 0) {
        const int wgs = hub_workgroups();
        const size_t s2 = (size_t)max_s2 + 64;
        const size_t wl = (size_t)std::max<int32_t>(g->max_deg, 1) + 64;
        size_t o = M_WORDS;
        const size_t o_spar = o; o += 9 * PMAX;
        const size_t o_s111 = o; o += 9 * PMAX;
        const size_t o_s3x = o; o += 12 * PMAX;   // s3x [3][PMAX], nsg [3][PMAX], prof [3][PMAX] u64
        const size_t o_groups = o; o += 3 * s2;
        const size_t o_wlist = o; o += NW * wl;
        const size_t o_eflag = o; o += (s2 + 3) / 4;
        const size_t o_llist = o; o += (s2 + 1) / 2;
        uint32_t hb = 12;
        while ((1u << hb) < 2 * wl) hb++;
        o = (o + 63) & ~(size_t)63;
        g->hub_scratch_bytes = o * sizeof(uint32_t) * (size_t)wgs;
        VDMC_HIP(hipMalloc(&g->hub_scratch, g->hub_scratch_bytes));
        const size_t comp_bytes = (size_t)std::max<int64_t>(g->n, 1) * kCompact4 * sizeof(unsigned long long);
        VDMC_HIP(hipMalloc(&g->hub_comp, comp_bytes));
        VDMC_HIP(hipMemsetAsync(g->hub_comp, 0, comp_bytes, st));   // cleared again by every fold
        VDMC_HIP(hipStreamSynchronize(st));
        g->hub_scratch_bytes += comp_bytes;
        const size_t w_bytes = (size_t)std::max<int64_t>(g->n, 1) * 9 * sizeof(uint32_t);
        VDMC_HIP(hipMalloc(&g->hub_w111, w_bytes));
        g->hub_scratch_bytes += w_bytes;
        ensure_edge_hash(g, st);
        g->hub_scratch_bytes += ((size_t)1 << g->ehash_bits) * (sizeof(unsigned long long) + sizeof(uint16_t));
        g->hub_layout[0] = o;
        g->hub_layout[1] = o_spar;
        g->hub_layout[2] = o_s111;
        g->hub_layout[3] = o_s3x;
        g->hub_layout[4] = o_groups;
        g->hub_layout[6] = o_wlist;
        g->hub_layout[8] = o_eflag;
        g->hub_layout[9] = wl;
        g->hub_layout[10] = o_llist;
        g->hub_layout[12] = hb;
        // (1,2,0) tasks: prefix sums of |N+(r)| over the hub queue, and per-wave scratch
        VDMC_HIP(hipMalloc(&g->hub_pre, (nhub + 1) * sizeof(uint32_t)));
        {
            uint32_t* dplus = (uint32_t*)alloc((nhub + 1) * sizeof(uint32_t));
            const unsigned hb2 = (unsigned)std::min<int64_t>((nhub + BT) / BT, 65536);
            hipLaunchKernelGGL(k_hub_dplus, dim3(hb2), dim3(BT), 0, st, g->off, g->split, g->hubs, nhub, dplus);
            VDMC_HIP(hipGetLastError());
            size_t tb = 0;
            VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, dplus, g->hub_pre, (int)(nhub + 1), st));
            void* t3 = alloc(tb);
            VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(t3, tb, dplus, g->hub_pre, (int)(nhub + 1), st));
        }
        // adjacency bitmap of the long-row vertices (pairs of long children in (1,2,0)),
        // when it is at most 4 GiB
        {
            uint32_t* d_nl = (uint32_t*)alloc(sizeof(uint32_t));
            VDMC_HIP(hipMemsetAsync(d_nl, 0, sizeof(uint32_t), st));
            const unsigned nb = (unsigned)std::min<int64_t>((g->n + BT - 1) / BT, 65536);
            if (nb > 0) hipLaunchKernelGGL(k_count_long, dim3(nb), dim3(BT), 0, st, g->off, g->n, d_nl);
            VDMC_HIP(hipGetLastError());
            uint32_t nl = 0;
            VDMC_HIP(hipMemcpyAsync(&nl, d_nl, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            VDMC_HIP(hipStreamSynchronize(st));
            const size_t lw = ((size_t)nl + 31) / 32;
            const size_t lbytes = lw * nl * sizeof(uint32_t);
            g->nlong = nl;
            g->lwords = (uint32_t)lw;
            if (nl > 0 && lbytes <= ((size_t)4 << 30)) {
                VDMC_HIP(hipMalloc(&g->lbits, lbytes));
                VDMC_HIP(hipMemsetAsync(g->lbits, 0, lbytes, st));
                const unsigned lb = (unsigned)std::min<int64_t>((nl + BT - 1) / BT, 65536);
                hipLaunchKernelGGL(k_long_bitmap, dim3(lb), dim3(BT), 0, st, g->off, g->adj, nl, (uint32_t)lw, g->lbits);
                VDMC_HIP(hipGetLastError());
                g->hub_scratch_bytes += lbytes;
            }
        }
        const size_t sp_words = (((size_t)4 * wl + 2 * ((size_t)1 << hb)) + 63) & ~(size_t)63;
        const size_t sp_waves = (size_t)slot_pair_workgroups() * (SP / 64);
        const size_t sp_bytes = sp_words * sp_waves * sizeof(uint32_t);
        VDMC_HIP(hipMalloc(&g->sp_scratch, sp_bytes));
        g->hub_scratch_bytes += sp_bytes;
        g->hub_layout[13] = sp_words;
        VDMC_HIP(hipStreamSynchronize(st));
    }
    g->bins_hub_min = hub_min;
}

void launch_hub(vdmc_graph_s* g, int k3, int k4, uint64_t* out3, uint64_t* out4, hipStream_t st,
                uint32_t rank_lo, uint32_t rank_hi, const hipEvent_t* around) {
    if (g->nhub == 0) return;
    const ClassTables& t = class_tables();
    HubArgs a;
    a.off = g->off;
    a.adj = g->adj;
    a.split = g->split;
    a.perm = g->perm;
    a.hubs = g->hubs;
    a.nhub = (uint32_t)g->nhub;
    a.queue = g->hub_queue;
    a.t3 = t.t3;
    a.t4 = t.t4;
    a.out3 = (unsigned long long*)out3;
    a.out4 = (unsigned long long*)out4;
    a.stats = g->stats;
    a.k3 = k3;
    a.k4 = k4;
    a.rank_lo = rank_lo;
    a.rank_hi = rank_hi;
    a.scratch = (uint32_t*)g->hub_scratch;
    a.wg_words = g->hub_layout[0];
    a.o_spar = g->hub_layout[1];
    a.o_s111 = g->hub_layout[2];
    a.o_s3x = g->hub_layout[3];
    a.o_groups = g->hub_layout[4];
    a.s2cap = (uint32_t)((size_t)g->max_scan2 + 64);
    a.o_wlist = g->hub_layout[6];
    a.o_eflag = g->hub_layout[8];
    a.wl_cap = (uint32_t)g->hub_layout[9];
    a.o_llist = g->hub_layout[10];
    a.hash_bits = (uint32_t)g->hub_layout[12];
    a.comp = (unsigned long long*)g->hub_comp;
    a.ehash = g->ehash;
    a.ehash_bits = g->ehash_bits;
    a.slot4 = t.slot4;
    a.w111 = (uint32_t*)g->hub_w111;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, g->hub_queue, 4);
    const int64_t wcells = g->n * 9;
    const unsigned vblocks = (unsigned)std::min<int64_t>((g->n + 255) / 256, 65536);
    if (k4)
        hipLaunchKernelGGL(k_fill_zero_u32, dim3((unsigned)std::min<int64_t>((wcells + 255) / 256, 65536)), dim3(256),
                           0, st, a.w111, wcells);
    const int wgs = hub_workgroups();
    // the hub path: k_hub, then (k = 4) the (1,2,0) tasks and the (1,1,1) end-vertex pass;
    // around[0] and around[1] bracket all three, around[2] marks the end of k_hub
    if (around) VDMC_HIP(hipEventRecord(around[0], st));
    hipLaunchKernelGGL(k_hub, dim3(wgs), dim3(HT), 0, st, a);
    VDMC_HIP(hipGetLastError());
    if (around) VDMC_HIP(hipEventRecord(around[2], st));
    if (k4) {
        SlotPairArgs sp;
        sp.off = g->off;
        sp.adj = g->adj;
        sp.split = g->split;
        sp.perm = g->perm;
        sp.hubs = g->hubs;
        sp.nhub = (uint32_t)g->nhub;
        sp.hub_pre = g->hub_pre;
        sp.rank_lo = rank_lo;
        sp.rank_hi = rank_hi;
        sp.t4 = t.t4;
        sp.slot4 = t.slot4;
        sp.out4 = (unsigned long long*)out4;
        sp.comp = (unsigned long long*)g->hub_comp;
        sp.stats = g->stats;
        sp.ehash = g->ehash;
        sp.efp = g->efp;
        sp.ehash_bits = g->ehash_bits;
        sp.lbits = g->lbits;
        sp.nlong = g->nlong;
        sp.lwords = g->lwords;
        sp.cursor = g->hub_queue + 1;
        sp.scratch = (uint32_t*)g->sp_scratch;
        sp.wave_words = g->hub_layout[13];
        sp.wl_cap = (uint32_t)g->hub_layout[9];
        sp.hash_bits = (uint32_t)g->hub_layout[12];
        hipLaunchKernelGGL(k_slot_pairs, dim3(slot_pair_workgroups()), dim3(SP), 0, st, sp);
        VDMC_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_pull111, dim3(vblocks), dim3(256), 0, st, g->off, g->adj, a.w111, t.t4, t.slot4, g->n,
                           (unsigned long long*)g->hub_comp);
    }
    if (around) VDMC_HIP(hipEventRecord(around[1], st));
    if (k4) {
        const int64_t cells = g->n * kCompact4;
        const unsigned blocks = (unsigned)std::min<int64_t>((cells + 255) / 256, 65536);
        hipLaunchKernelGGL(k_fold_compact, dim3(blocks), dim3(256), 0, st, (unsigned long long*)g->hub_comp,
                           t.slotcls, g->perm, g->n, (unsigned long long*)out4);
        VDMC_HIP(hipGetLastError());
    }
}

}  // namespace vdmc

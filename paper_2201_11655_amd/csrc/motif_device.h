// Device helpers for the motif kernels: CSR lookups and motif-index assembly.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vdmc {

// CSR entries are (neighbour_rank << 2) | arc bits, sorted ascending within a row.
// Arc bits seen from the row vertex u towards neighbour v: bit 0 = u -> v, bit 1 = v -> u.

__device__ __forceinline__ uint32_t swap_arc_bits(uint32_t c) { return ((c & 1u) << 1) | (c >> 1); }

// index of the first entry in [lo, hi) whose neighbour rank is >= x
__device__ __forceinline__ uint32_t lower_bound_rank(const uint32_t* __restrict__ adj, uint32_t lo,
                                                     uint32_t hi, uint32_t x) {
    const uint32_t key = x << 2;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (adj[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// arc bits of the pair (u, v) seen from u; 0 when u and v are not adjacent.  Searches the
// shorter of the two sorted rows (O(log min(deg u, deg v))).
__device__ __forceinline__ uint32_t arc_bits(const uint32_t* __restrict__ off,
                                             const uint32_t* __restrict__ adj, uint32_t u, uint32_t v) {
    uint32_t lu = off[u], hu = off[u + 1], lv = off[v], hv = off[v + 1];
    bool from_u = (hu - lu) <= (hv - lv);
    uint32_t lo = from_u ? lu : lv, hi = from_u ? hu : hv, x = from_u ? v : u;
    uint32_t p = lower_bound_rank(adj, lo, hi, x);
    if (p >= hi) return 0;
    uint32_t e = adj[p];
    if ((e >> 2) != x) return 0;
    return from_u ? (e & 3u) : swap_arc_bits(e & 3u);
}

// Edge hash: one 64-bit slot per vertex pair {lo < hi} of the graph, holding
// (lo << 32) | (hi << 2) | arc bits seen from lo; 0 = empty; linear probing.
__device__ __forceinline__ uint32_t edge_slot(unsigned long long key, uint32_t bits) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64u - bits));
}
// arc bits of (u, v) seen from u (0 if not adjacent), one probe sequence in the edge hash
__device__ __forceinline__ uint32_t edge_code(const unsigned long long* __restrict__ table, uint32_t bits,
                                              uint32_t u, uint32_t v) {
    const uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
    const unsigned long long key = ((unsigned long long)lo << 32) | ((unsigned long long)hi << 2);
    const uint32_t mask = (1u << bits) - 1u;
    for (uint32_t h = edge_slot(key, bits);; h = (h + 1u) & mask) {
        const unsigned long long s = table[h];
        if (s == 0ull) return 0u;
        if ((s & ~3ull) == key) return u == lo ? (uint32_t)(s & 3u) : swap_arc_bits((uint32_t)(s & 3u));
    }
}

// Fingerprint of an edge-hash key (never 0: 0 marks an empty slot).  A 16-bit table of
// fingerprints at the same slots (4x smaller than the keys, so it stays cache-resident)
// answers most lookups; the 64-bit key is read only when the fingerprint matches.
__device__ __forceinline__ uint16_t edge_fp(unsigned long long key) {
    const uint32_t f = (uint32_t)((key * 0xC2B2AE3D27D4EB4Full) >> 48);
    return (uint16_t)(f ? f : 1u);
}
__device__ __forceinline__ uint32_t edge_code_fp(const uint16_t* __restrict__ fp, const unsigned long long* __restrict__ table,
                                                 uint32_t bits, uint32_t u, uint32_t v) {
    const uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
    const unsigned long long key = ((unsigned long long)lo << 32) | ((unsigned long long)hi << 2);
    const uint16_t f = edge_fp(key);
    const uint32_t mask = (1u << bits) - 1u;
    for (uint32_t h = edge_slot(key, bits);; h = (h + 1u) & mask) {
        const uint16_t g = fp[h];
        if (g == 0) return 0u;
        if (g != f) continue;
        const unsigned long long s = table[h];
        if ((s & ~3ull) == key) return u == lo ? (uint32_t)(s & 3u) : swap_arc_bits((uint32_t)(s & 3u));
    }
}

// slot of the pair (u, v) in the edge hash, or 0xFFFFFFFF if the pair is not in the graph
// (the probe stops at the first empty slot; the table is never full)
__device__ __forceinline__ uint32_t edge_find(const unsigned long long* __restrict__ table, uint32_t bits,
                                              uint32_t u, uint32_t v) {
    const uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
    const unsigned long long key = ((unsigned long long)lo << 32) | ((unsigned long long)hi << 2);
    const uint32_t mask = (1u << bits) - 1u;
    for (uint32_t h = edge_slot(key, bits);; h = (h + 1u) & mask) {
        const unsigned long long s = table[h];
        if (s == 0ull) return 0xFFFFFFFFu;
        if ((s & ~3ull) == key) return h;
    }
}

// Motif index (Sec. 4.1): the adjacency matrix of the ordered vertices v0..v{k-1},
// row = source, read row by row without the diagonal, first entry most significant.
// p_ij (i < j) are the arc bits of (v_i, v_j) seen from v_i: bit 0 sets entry (i,j),
// bit 1 sets entry (j,i).
//   k = 3 entry weights: (0,1)=32 (0,2)=16 (1,0)=8 (1,2)=4 (2,0)=2 (2,1)=1
__device__ __forceinline__ uint32_t motif_index3(uint32_t p01, uint32_t p02, uint32_t p12) {
    return ((p01 & 1u) << 5) | ((p01 >> 1) << 3) | ((p02 & 1u) << 4) | ((p02 >> 1) << 1) |
           ((p12 & 1u) << 2) | (p12 >> 1);
}
//   k = 4 entry weights: (0,1)=2^11 (0,2)=2^10 (0,3)=2^9 (1,0)=2^8 (1,2)=2^7 (1,3)=2^6
//                        (2,0)=2^5 (2,1)=2^4 (2,3)=2^3 (3,0)=2^2 (3,1)=2^1 (3,2)=2^0
__device__ __forceinline__ uint32_t motif_index4(uint32_t p01, uint32_t p02, uint32_t p03, uint32_t p12,
                                                 uint32_t p13, uint32_t p23) {
    return ((p01 & 1u) << 11) | ((p01 >> 1) << 8) | ((p02 & 1u) << 10) | ((p02 >> 1) << 5) |
           ((p03 & 1u) << 9) | ((p03 >> 1) << 2) | ((p12 & 1u) << 7) | ((p12 >> 1) << 4) |
           ((p13 & 1u) << 6) | ((p13 >> 1) << 1) | ((p23 & 1u) << 3) | (p23 >> 1);
}

}  // namespace vdmc

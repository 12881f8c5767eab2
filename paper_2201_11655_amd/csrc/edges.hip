// Per-edge motif counts (Sec. 11: "count per edge" as a minimal change of the method:
// the edges of each set are credited instead of its vertices).
//
// Output rows are the vertex pairs {lo < hi} joined in G_U, in ascending (lo, hi) order
// of original ids (vdmc_edge_list).  The edge index maps every pair's slot in the
// graph's edge hash to its row, so the per-set kernel finds a pair's row with one probe
// sequence.  Every root goes through the per-set kernel (count.hip, EdgeSink).
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "motif_device.h"
#include "vdmc_internal.h"

namespace vdmc {
namespace {

constexpr int ET = 256;

unsigned blocks_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + ET - 1) / ET, 65536)); }

// entries above the diagonal (the pair's lower-rank row), per row
__global__ void k_upper_counts(const uint32_t* __restrict__ off, const uint32_t* __restrict__ split, int64_t n,
                               uint32_t* __restrict__ cnt) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        cnt[u] = off[u + 1] - split[u];
}

// one key per pair: (lo << 32) | hi in original ids; value = its index in rank order
__global__ void k_pair_keys(const uint32_t* __restrict__ off, const uint32_t* __restrict__ split,
                            const uint32_t* __restrict__ adj, const int32_t* __restrict__ perm, int64_t n,
                            const uint32_t* __restrict__ uoff, unsigned long long* __restrict__ keys,
                            uint32_t* __restrict__ vals) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = split[u], base = uoff[u];
        for (uint32_t t = s; t < off[u + 1]; t++) {
            const uint32_t a = (uint32_t)perm[u], b = (uint32_t)perm[adj[t] >> 2];
            const uint32_t i = base + (t - s);
            keys[i] = ((unsigned long long)min(a, b) << 32) | max(a, b);
            vals[i] = i;
        }
    }
}

__global__ void k_rows(const unsigned long long* __restrict__ keys_s, const uint32_t* __restrict__ vals_s,
                       int64_t P, uint32_t* __restrict__ row_of, int32_t* __restrict__ elo,
                       int32_t* __restrict__ ehi) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        row_of[vals_s[i]] = (uint32_t)i;
        elo[i] = (int32_t)(keys_s[i] >> 32);
        ehi[i] = (int32_t)(keys_s[i] & 0xFFFFFFFFu);
    }
}

// every pair's edge-hash slot -> its output row
__global__ void k_slot_rows(const uint32_t* __restrict__ off, const uint32_t* __restrict__ split,
                            const uint32_t* __restrict__ adj, int64_t n, const uint32_t* __restrict__ uoff,
                            const uint32_t* __restrict__ row_of, const unsigned long long* __restrict__ table,
                            uint32_t bits, uint32_t* __restrict__ epid) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = split[u], base = uoff[u];
        for (uint32_t t = s; t < off[u + 1]; t++) {
            const uint32_t h = edge_find(table, bits, (uint32_t)u, adj[t] >> 2);
            if (h != 0xFFFFFFFFu) epid[h] = row_of[base + (t - s)];
        }
    }
}

}  // namespace

void ensure_edge_index(vdmc_graph_s* g, hipStream_t st) {
    if (g->epid) return;
    ensure_edge_hash(g, st);
    const int64_t n = g->n, P = g->pairs;
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
    uint32_t* epid = nullptr;
    int32_t *elo = nullptr, *ehi = nullptr;
    VDMC_HIP(hipMalloc(&epid, ((size_t)1 << g->ehash_bits) * sizeof(uint32_t)));
    VDMC_HIP(hipMalloc(&elo, std::max<int64_t>(P, 1) * sizeof(int32_t)));
    VDMC_HIP(hipMalloc(&ehi, std::max<int64_t>(P, 1) * sizeof(int32_t)));
    g->epid = epid;   // owned by the graph from here on
    g->elo = elo;
    g->ehi = ehi;
    if (n == 0 || P == 0) return;
    uint32_t* cnt = (uint32_t*)alloc((n + 1) * sizeof(uint32_t));
    uint32_t* uoff = (uint32_t*)alloc((n + 1) * sizeof(uint32_t));
    auto* keys = (unsigned long long*)alloc(P * sizeof(unsigned long long));
    auto* keys_s = (unsigned long long*)alloc(P * sizeof(unsigned long long));
    uint32_t* vals = (uint32_t*)alloc(P * sizeof(uint32_t));
    uint32_t* vals_s = (uint32_t*)alloc(P * sizeof(uint32_t));
    uint32_t* row_of = (uint32_t*)alloc(P * sizeof(uint32_t));
    hipLaunchKernelGGL(k_upper_counts, dim3(blocks_of(n)), dim3(ET), 0, st, g->off, g->split, n, cnt);
    size_t tb = 0;
    VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, uoff, (int)n, st));
    void* t1 = alloc(tb);
    VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(t1, tb, cnt, uoff, (int)n, st));
    hipLaunchKernelGGL(k_pair_keys, dim3(blocks_of(n)), dim3(ET), 0, st, g->off, g->split, g->adj, g->perm, n,
                       uoff, keys, vals);
    size_t sb = 0;
    VDMC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sb, keys, keys_s, vals, vals_s, (int)P, 0, 64, st));
    void* t2 = alloc(sb);
    VDMC_HIP(hipcub::DeviceRadixSort::SortPairs(t2, sb, keys, keys_s, vals, vals_s, (int)P, 0, 64, st));
    hipLaunchKernelGGL(k_rows, dim3(blocks_of(P)), dim3(ET), 0, st, keys_s, vals_s, P, row_of, elo, ehi);
    hipLaunchKernelGGL(k_slot_rows, dim3(blocks_of(n)), dim3(ET), 0, st, g->off, g->split, g->adj, n, uoff, row_of,
                       g->ehash, g->ehash_bits, epid);
    VDMC_HIP(hipGetLastError());
    VDMC_HIP(hipStreamSynchronize(st));
}

}  // namespace vdmc

extern "C" {

vdmc_status vdmc_count_edges(vdmc_graph g, int32_t k, uint64_t* out, void* stream) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG, "k must be 3 or 4");
        VDMC_REQUIRE(out != nullptr || g->pairs == 0, VDMC_ERR_INVALID_ARG, "out is NULL");
        VDMC_HIP(hipSetDevice(g->device));
        vdmc::GraphUse use(g, vdmc::as_stream(stream));
        vdmc::launch_count_edges(g, k, out, vdmc::as_stream(stream));
    });
}

vdmc_status vdmc_edge_list(vdmc_graph g, int32_t* lo, int32_t* hi) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_REQUIRE((lo && hi) || g->pairs == 0, VDMC_ERR_INVALID_ARG, "lo/hi is NULL");
        VDMC_HIP(hipSetDevice(g->device));
        std::lock_guard<std::mutex> lock(g->mu);
        vdmc::ensure_edge_index(g, nullptr);
        if (g->pairs == 0) return;
        VDMC_HIP(hipMemcpy(lo, g->elo, g->pairs * sizeof(int32_t), hipMemcpyDeviceToHost));
        VDMC_HIP(hipMemcpy(hi, g->ehi, g->pairs * sizeof(int32_t), hipMemcpyDeviceToHost));
    });
}

}  // extern "C"

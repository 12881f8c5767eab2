// Device graph build: arc list -> ranked symmetric CSR with 2-bit arc codes.
//
// Paper: the motif search runs on G_U, the undirected graph under G (Sec. 4.1),
// over a CSR of ordered neighbour lists (Sec. 4.2); vertices are ranked by
// undirected degree, highest degree first, so that the heavy roots are handled
// and "removed" first (Sec. 2, Sec. 6).  The arc directions inside a motif are
// kept as two bits per CSR entry so that the motif index (Sec. 4.1) can be
// assembled from the entries alone.
//
// Every step runs on the device: key generation, radix sorts (hipCUB), pair
// merging, degree counting, ranking, CSR assembly and the higher-neighbour split.
#include <hipcub/hipcub.hpp>

#include "vdmc_internal.h"

namespace vdmc {
namespace {

constexpr uint64_t kSentinel = ~0ull;
constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > (1 << 20)) b = 1 << 20;   // grid-stride loops cover the rest
    return (unsigned)b;
}

// (lo << 32 | hi) per arc, with bit 0 = lo -> hi, bit 1 = hi -> lo; self-loops get
// the sentinel key (sorted last, dropped).  Out-of-range ids raise *bad.
__global__ void k_arc_keys(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                           int64_t m, int64_t n, uint64_t* __restrict__ keys,
                           uint8_t* __restrict__ bits, int* __restrict__ bad) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = src[i], v = dst[i];
        if (u < 0 || v < 0 || u >= n || v >= n) {
            atomicOr(bad, 1);
            keys[i] = kSentinel;
            bits[i] = 0;
            continue;
        }
        if (u == v) {
            keys[i] = kSentinel;
            bits[i] = 0;
            continue;
        }
        uint32_t lo = u < v ? (uint32_t)u : (uint32_t)v;
        uint32_t hi = u < v ? (uint32_t)v : (uint32_t)u;
        keys[i] = ((uint64_t)lo << 32) | hi;
        bits[i] = u < v ? 1 : 2;
    }
}

__global__ void k_heads(const uint64_t* __restrict__ keys, int64_t m, uint32_t* __restrict__ head) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[i];
        head[i] = (k != kSentinel && (i == 0 || keys[i - 1] != k)) ? 1u : 0u;
    }
}

// pair index of element i = (exclusive head count) + head - 1
__global__ void k_merge_pairs(const uint64_t* __restrict__ keys, const uint8_t* __restrict__ bits,
                              const uint32_t* __restrict__ head, const uint32_t* __restrict__ hpos,
                              int64_t m, uint64_t* __restrict__ pkey, uint32_t* __restrict__ pcode) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[i];
        if (k == kSentinel) continue;
        uint32_t p = hpos[i] + head[i] - 1u;
        if (head[i]) pkey[p] = k;
        atomicOr(&pcode[p], (uint32_t)bits[i]);
    }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_degrees(const uint64_t* __restrict__ pkey, const uint32_t* __restrict__ pcode,
                          int64_t np, uint32_t* __restrict__ deg,
                          unsigned long long* __restrict__ arcs) {
    unsigned long long local = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = pkey[i];
        atomicAdd(&deg[k >> 32], 1u);
        atomicAdd(&deg[k & 0xffffffffu], 1u);
        local += __popc(pcode[i]);
    }
    if (local) atomicAdd(arcs, local);
}

// rank key: larger degree first; stable sort keeps ascending id among ties
__global__ void k_rank_keys(const uint32_t* __restrict__ deg, int64_t n, uint32_t* __restrict__ key,
                            int32_t* __restrict__ ids, unsigned* __restrict__ maxdeg) {
    unsigned local = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        key[i] = ~deg[i];
        ids[i] = (int32_t)i;
        local = deg[i] > local ? deg[i] : local;
    }
    atomicMax(maxdeg, local);
}

__global__ void k_inverse(const int32_t* __restrict__ perm, const uint32_t* __restrict__ deg,
                          int64_t n, uint32_t* __restrict__ inv, uint32_t* __restrict__ deg_rank) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        int32_t id = perm[r];
        inv[id] = (uint32_t)r;
        deg_rank[r] = deg[id];
    }
}

__device__ inline uint32_t swap_bits(uint32_t c) { return ((c & 1u) << 1) | (c >> 1); }

// two CSR records per pair: (row_rank << 32) | (nbr_rank << 2) | bits seen from row
__global__ void k_entries(const uint64_t* __restrict__ pkey, const uint32_t* __restrict__ pcode,
                          const uint32_t* __restrict__ inv, int64_t np, uint64_t* __restrict__ rec) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = pkey[i];
        uint32_t a = inv[k >> 32], b = inv[k & 0xffffffffu];
        uint32_t c = pcode[i];   // bit 0: lo -> hi, bit 1: hi -> lo (lo, hi = original ids)
        rec[2 * i] = ((uint64_t)a << 32) | ((uint64_t)b << 2) | c;
        rec[2 * i + 1] = ((uint64_t)b << 32) | ((uint64_t)a << 2) | swap_bits(c);
    }
}

__global__ void k_low_words(const uint64_t* __restrict__ rec, int64_t ne, uint32_t* __restrict__ adj) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ne;
         i += (int64_t)gridDim.x * blockDim.x)
        adj[i] = (uint32_t)rec[i];
}

// first entry of row r whose neighbour rank exceeds r
__global__ void k_split(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj, int64_t n,
                        uint32_t* __restrict__ split, uint32_t* __restrict__ has_hi) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        uint32_t lo = off[r], hi = off[r + 1];
        uint32_t key = (uint32_t)(r + 1) << 2;
        while (lo < hi) {
            uint32_t mid = lo + ((hi - lo) >> 1);
            if (adj[mid] < key) lo = mid + 1; else hi = mid;
        }
        split[r] = lo;
        has_hi[r] = lo < off[r + 1] ? 1u : 0u;
    }
}

__global__ void k_compact_roots(const uint32_t* __restrict__ has_hi, const uint32_t* __restrict__ pos,
                                int64_t n, uint32_t* __restrict__ roots) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x)
        if (has_hi[r]) roots[pos[r]] = (uint32_t)r;
}

// RAII list of temporaries freed at scope exit
struct Temps {
    std::vector<void*> ptrs;
    template <class T>
    T* alloc(size_t count) {
        void* p = nullptr;
        VDMC_HIP(hipMalloc(&p, count * sizeof(T) + 16));
        ptrs.push_back(p);
        return static_cast<T*>(p);
    }
    ~Temps() {
        for (void* p : ptrs) (void)hipFree(p);
    }
};

template <class F>
void* cub_temp(Temps& t, F&& query) {
    size_t bytes = 0;
    VDMC_HIP(query(nullptr, bytes));
    return t.alloc<uint8_t>(bytes ? bytes : 1);
}

}  // namespace

static void build_graph(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, uint32_t flags,
                        hipStream_t st, vdmc_graph_s* g) {
    VDMC_REQUIRE(n >= 0 && m >= 0, VDMC_ERR_INVALID_ARG, "n and m must be non-negative");
    VDMC_REQUIRE(n < (int64_t(1) << 30), VDMC_ERR_INVALID_ARG, "n must be below 2^30");
    VDMC_REQUIRE(m == 0 || (src && dst), VDMC_ERR_INVALID_ARG, "src/dst is NULL");
    VDMC_REQUIRE(m < (int64_t(1) << 31), VDMC_ERR_INVALID_ARG, "m must be below 2^31");
    VDMC_HIP(hipGetDevice(&g->device));
    g->n = n;
    g->undirected = (flags & VDMC_UNDIRECTED) != 0;
    Temps t;
    const int32_t* d_src = src;
    const int32_t* d_dst = dst;
    if (!(flags & VDMC_INPUT_ON_DEVICE) && m > 0) {
        int32_t* s = t.alloc<int32_t>(m);
        int32_t* d = t.alloc<int32_t>(m);
        VDMC_HIP(hipMemcpyAsync(s, src, m * sizeof(int32_t), hipMemcpyHostToDevice, st));
        VDMC_HIP(hipMemcpyAsync(d, dst, m * sizeof(int32_t), hipMemcpyHostToDevice, st));
        d_src = s;
        d_dst = d;
    }
    // graph arrays that always exist
    VDMC_HIP(hipMalloc(&g->off, (n + 1) * sizeof(uint32_t)));
    VDMC_HIP(hipMalloc(&g->split, (n > 0 ? n : 1) * sizeof(uint32_t)));
    VDMC_HIP(hipMalloc(&g->perm, (n > 0 ? n : 1) * sizeof(int32_t)));
    VDMC_HIP(hipMalloc(&g->stats, kStatSlots * sizeof(unsigned long long)));
    VDMC_HIP(hipMemsetAsync(g->stats, 0, kStatSlots * sizeof(unsigned long long), st));

    int* d_bad = t.alloc<int>(1);
    unsigned long long* d_arcs = t.alloc<unsigned long long>(1);
    unsigned* d_maxdeg = t.alloc<unsigned>(1);
    VDMC_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), st));
    VDMC_HIP(hipMemsetAsync(d_arcs, 0, sizeof(unsigned long long), st));
    VDMC_HIP(hipMemsetAsync(d_maxdeg, 0, sizeof(unsigned), st));

    // ---- 1. merge arcs into undirected pairs with arc bits
    int64_t np = 0;
    uint64_t* pkey = nullptr;
    uint32_t* pcode = nullptr;
    if (m > 0) {
        uint64_t* keys = t.alloc<uint64_t>(m);
        uint64_t* keys_s = t.alloc<uint64_t>(m);
        uint8_t* bits = t.alloc<uint8_t>(m);
        uint8_t* bits_s = t.alloc<uint8_t>(m);
        hipLaunchKernelGGL(k_arc_keys, dim3(blocks_for(m)), dim3(kThreads), 0, st, d_src, d_dst, m, n,
                           keys, bits, d_bad);
        VDMC_HIP(hipGetLastError());
        int mi = (int)m;
        void* tmp = cub_temp(t, [&](void* p, size_t& b) {
            return hipcub::DeviceRadixSort::SortPairs(p, b, keys, keys_s, bits, bits_s, mi, 0, 64, st);
        });
        size_t tb = 0;
        VDMC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, keys, keys_s, bits, bits_s, mi, 0, 64, st));
        VDMC_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys, keys_s, bits, bits_s, mi, 0, 64, st));
        uint32_t* head = t.alloc<uint32_t>(m);
        uint32_t* hpos = t.alloc<uint32_t>(m);
        hipLaunchKernelGGL(k_heads, dim3(blocks_for(m)), dim3(kThreads), 0, st, keys_s, m, head);
        VDMC_HIP(hipGetLastError());
        size_t sb = 0;
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, sb, head, hpos, mi, st));
        void* stmp = t.alloc<uint8_t>(sb ? sb : 1);
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(stmp, sb, head, hpos, mi, st));
        uint32_t last[2] = {0, 0};
        VDMC_HIP(hipMemcpyAsync(&last[0], hpos + (m - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        VDMC_HIP(hipMemcpyAsync(&last[1], head + (m - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        int bad = 0;
        VDMC_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, st));
        VDMC_HIP(hipStreamSynchronize(st));
        VDMC_REQUIRE(!bad, VDMC_ERR_INVALID_ARG, "arc endpoint outside [0, n)");
        np = (int64_t)last[0] + last[1];
        pkey = t.alloc<uint64_t>(np > 0 ? np : 1);
        pcode = t.alloc<uint32_t>(np > 0 ? np : 1);
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(np)), dim3(kThreads), 0, st, pcode, np, 0u);
        hipLaunchKernelGGL(k_merge_pairs, dim3(blocks_for(m)), dim3(kThreads), 0, st, keys_s, bits_s, head,
                           hpos, m, pkey, pcode);
        VDMC_HIP(hipGetLastError());
        if (flags & VDMC_UNDIRECTED)   // every pair carries both arcs: the graph is G_U itself
            hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(np)), dim3(kThreads), 0, st, pcode, np, 3u);
    }
    g->pairs = np;
    VDMC_REQUIRE(2 * np < (int64_t(1) << 32), VDMC_ERR_UNSUPPORTED, "more than 2^31 undirected pairs");

    // ---- 2. undirected degrees and the rank order (degree descending, id ascending)
    uint32_t* deg = t.alloc<uint32_t>(n > 0 ? n : 1);
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), dim3(kThreads), 0, st, deg, n, 0u);
    if (np > 0)
        hipLaunchKernelGGL(k_degrees, dim3(blocks_for(np)), dim3(kThreads), 0, st, pkey, pcode, np, deg, d_arcs);
    VDMC_HIP(hipGetLastError());
    uint32_t* inv = t.alloc<uint32_t>(n > 0 ? n : 1);
    uint32_t* deg_rank = t.alloc<uint32_t>(n + 1);
    if (n > 0) {
        uint32_t* rk = t.alloc<uint32_t>(n);
        uint32_t* rk_s = t.alloc<uint32_t>(n);
        int32_t* ids = t.alloc<int32_t>(n);
        hipLaunchKernelGGL(k_rank_keys, dim3(blocks_for(n)), dim3(kThreads), 0, st, deg, n, rk, ids, d_maxdeg);
        VDMC_HIP(hipGetLastError());
        int ni = (int)n;
        size_t tb = 0;
        VDMC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, rk, rk_s, ids, g->perm, ni, 0, 32, st));
        void* tmp = t.alloc<uint8_t>(tb ? tb : 1);
        VDMC_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, rk, rk_s, ids, g->perm, ni, 0, 32, st));
        hipLaunchKernelGGL(k_inverse, dim3(blocks_for(n)), dim3(kThreads), 0, st, g->perm, deg, n, inv, deg_rank);
        VDMC_HIP(hipGetLastError());
    }
    // ---- 3. CSR offsets (exclusive scan of the ranked degrees, n+1 entries)
    {
        VDMC_HIP(hipMemsetAsync(deg_rank + n, 0, sizeof(uint32_t), st));
        int ni = (int)(n + 1);
        size_t sb = 0;
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, sb, deg_rank, g->off, ni, st));
        void* stmp = t.alloc<uint8_t>(sb ? sb : 1);
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(stmp, sb, deg_rank, g->off, ni, st));
    }
    // ---- 4. entries sorted by (row, neighbour)
    const int64_t ne = 2 * np;
    VDMC_HIP(hipMalloc(&g->adj, (ne > 0 ? ne : 1) * sizeof(uint32_t)));
    if (ne > 0) {
        uint64_t* rec = t.alloc<uint64_t>(ne);
        uint64_t* rec_s = t.alloc<uint64_t>(ne);
        hipLaunchKernelGGL(k_entries, dim3(blocks_for(np)), dim3(kThreads), 0, st, pkey, pcode, inv, np, rec);
        VDMC_HIP(hipGetLastError());
        int nei = (int)ne;
        size_t tb = 0;
        VDMC_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, rec, rec_s, nei, 0, 64, st));
        void* tmp = t.alloc<uint8_t>(tb ? tb : 1);
        VDMC_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tb, rec, rec_s, nei, 0, 64, st));
        hipLaunchKernelGGL(k_low_words, dim3(blocks_for(ne)), dim3(kThreads), 0, st, rec_s, ne, g->adj);
        VDMC_HIP(hipGetLastError());
    }
    // ---- 5. higher-neighbour split and the list of roots with work
    g->nroots = 0;
    if (n > 0) {
        uint32_t* has_hi = t.alloc<uint32_t>(n + 1);
        uint32_t* pos = t.alloc<uint32_t>(n + 1);
        hipLaunchKernelGGL(k_split, dim3(blocks_for(n)), dim3(kThreads), 0, st, g->off, g->adj, n, g->split, has_hi);
        VDMC_HIP(hipGetLastError());
        VDMC_HIP(hipMemsetAsync(has_hi + n, 0, sizeof(uint32_t), st));
        int ni = (int)(n + 1);
        size_t sb = 0;
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, sb, has_hi, pos, ni, st));
        void* stmp = t.alloc<uint8_t>(sb ? sb : 1);
        VDMC_HIP(hipcub::DeviceScan::ExclusiveSum(stmp, sb, has_hi, pos, ni, st));
        uint32_t nr = 0;
        VDMC_HIP(hipMemcpyAsync(&nr, pos + n, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        VDMC_HIP(hipStreamSynchronize(st));
        g->nroots = nr;
        VDMC_HIP(hipMalloc(&g->roots, (nr > 0 ? nr : 1) * sizeof(uint32_t)));
        if (nr > 0)
            hipLaunchKernelGGL(k_compact_roots, dim3(blocks_for(n)), dim3(kThreads), 0, st, has_hi, pos, n, g->roots);
        VDMC_HIP(hipGetLastError());
    } else {
        VDMC_HIP(hipMalloc(&g->roots, sizeof(uint32_t)));
    }
    unsigned long long arcs = 0;
    unsigned maxdeg = 0;
    VDMC_HIP(hipMemcpyAsync(&arcs, d_arcs, sizeof(arcs), hipMemcpyDeviceToHost, st));
    VDMC_HIP(hipMemcpyAsync(&maxdeg, d_maxdeg, sizeof(maxdeg), hipMemcpyDeviceToHost, st));
    VDMC_HIP(hipStreamSynchronize(st));
    g->arcs = (int64_t)arcs;
    g->max_deg = (int32_t)maxdeg;
}

static void free_graph_arrays(vdmc_graph_s* g) {
    free_hub(g);
    free_five(g);
    (void)hipFree(g->utmp);
    (void)hipFree(g->ehash);
    (void)hipFree(g->epid);
    (void)hipFree(g->elo);
    (void)hipFree(g->ehi);
    g->utmp = nullptr;
    g->ehash = nullptr;
    g->ehash_bits = 0;
    g->epid = nullptr;
    g->elo = g->ehi = nullptr;
    (void)hipFree(g->off);
    (void)hipFree(g->adj);
    (void)hipFree(g->split);
    (void)hipFree(g->perm);
    (void)hipFree(g->roots);
    (void)hipFree(g->stats);
    for (auto& e : g->ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    g->off = g->adj = g->split = g->roots = nullptr;
    g->perm = nullptr;
    g->stats = nullptr;
}

}  // namespace vdmc

extern "C" {

vdmc_status vdmc_build_graph(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                             uint32_t flags, void* stream, vdmc_graph* out) {
    vdmc_graph_s* g = nullptr;
    vdmc_status st = vdmc::guarded([&] {
        VDMC_REQUIRE(out != nullptr, VDMC_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        g = new vdmc_graph_s();
        vdmc::build_graph(n, m, src, dst, flags, vdmc::as_stream(stream), g);
        (void)vdmc::class_tables();   // make sure the tables exist before the first count
    });
    if (st != VDMC_OK) {
        if (g) {
            vdmc::free_graph_arrays(g);
            delete g;
        }
        return st;
    }
    *out = g;
    return VDMC_OK;
}

vdmc_status vdmc_graph_info(vdmc_graph g, int64_t* n, int64_t* arcs, int64_t* pairs, int32_t* max_deg) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        if (n) *n = g->n;
        if (arcs) *arcs = g->arcs;
        if (pairs) *pairs = g->pairs;
        if (max_deg) *max_deg = g->max_deg;
    });
}

vdmc_status vdmc_graph_export(vdmc_graph g, uint32_t* off, uint32_t* adj, int32_t* perm) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_HIP(hipSetDevice(g->device));
        VDMC_HIP(hipDeviceSynchronize());
        if (off) VDMC_HIP(hipMemcpy(off, g->off, (g->n + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (adj && g->pairs > 0)
            VDMC_HIP(hipMemcpy(adj, g->adj, 2 * g->pairs * sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (perm && g->n > 0) VDMC_HIP(hipMemcpy(perm, g->perm, g->n * sizeof(int32_t), hipMemcpyDeviceToHost));
    });
}

vdmc_status vdmc_free_graph(vdmc_graph g) {
    if (!g) return VDMC_OK;
    return vdmc::guarded([&] {
        int cur = 0;
        VDMC_HIP(hipGetDevice(&cur));
        VDMC_HIP(hipSetDevice(g->device));
        vdmc::invalidate_batch_plans(g);
        {
            std::lock_guard<std::mutex> lock(g->mu);
            vdmc::wait_graph(g);
        }
        vdmc::free_graph_arrays(g);
        g->last.reset();
        for (auto e : g->ev)
            if (e) (void)hipEventDestroy(e);
        delete g;
        VDMC_HIP(hipSetDevice(cur));
    });
}

}  // extern "C"

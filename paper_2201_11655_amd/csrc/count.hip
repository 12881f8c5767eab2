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
constexpr uint32_t kStage = 2048;   // entries of N+(r) staged in LDS

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
};

// rank x a member of the sorted list P[0..d) ?
__device__ __forceinline__ bool in_list(const uint32_t* P, uint32_t d, uint32_t x) {
    uint32_t lo = 0, hi = d, key = x << 2;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (P[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo < d && (P[lo] >> 2) == x;
}

__device__ __forceinline__ void credit(unsigned long long* out, const int32_t* perm, int C, uint32_t v,
                                       uint32_t cls) {
    if (cls < (uint32_t)C) atomicAdd(&out[(size_t)perm[v] * C + cls], 1ull);   // 0xFF never credited
}

template <bool K3, bool K4>
__global__ __launch_bounds__(kThreads) void k_count_roots(Args a) {
    __shared__ uint32_t sP[kStage];
    __shared__ uint32_t sLo[kStage + 1];     // first entry of row P[i] above r
    __shared__ uint32_t sPre[kStage + 1];    // prefix sums of the D2 scan lengths
    __shared__ unsigned long long sRoot3[kClasses3];
    __shared__ unsigned long long sRoot4[kClasses4];
    const uint32_t tid = threadIdx.x;
    unsigned long long shape[kShapes] = {0, 0, 0, 0, 0, 0};

    for (int64_t ri = blockIdx.x; ri < a.nroots; ri += gridDim.x) {
        const uint32_t r = a.roots[ri];
        const uint32_t s = a.split[r];
        const uint32_t d = a.off[r + 1] - s;
        const bool staged = d <= kStage;
        __syncthreads();
        if (staged)
            for (uint32_t i = tid; i < d; i += kThreads) sP[i] = a.adj[s + i];
        if (K3)
            for (uint32_t i = tid; i < kClasses3; i += kThreads) sRoot3[i] = 0;
        if (K4)
            for (uint32_t i = tid; i < kClasses4; i += kThreads) sRoot4[i] = 0;
        __syncthreads();
        const uint32_t* P = staged ? sP : a.adj + s;

        // ---- depth-1 shapes: pairs (i < j) of N+(r); k=4 extends each by l > j
        const uint64_t npairs = (uint64_t)d * (d - 1) / 2;
        for (uint64_t q = tid; q < npairs; q += kThreads) {
            uint32_t j = (uint32_t)((1.0 + sqrt(1.0 + 8.0 * (double)q)) * 0.5);
            while ((uint64_t)j * (j - 1) / 2 > q) j--;
            while ((uint64_t)(j + 1) * j / 2 <= q) j++;
            const uint32_t i = (uint32_t)(q - (uint64_t)j * (j - 1) / 2);
            const uint32_t ea = P[i], eb = P[j];
            const uint32_t va = ea >> 2, vb = eb >> 2, ra = ea & 3u, rb = eb & 3u;
            const uint32_t ab = arc_bits(a.off, a.adj, va, vb);
            if (K3) {
                const uint32_t cls = a.t3[motif_index3(ra, rb, ab)];
                if (cls < kClasses3) atomicAdd(&sRoot3[cls], 1ull);
                credit(a.out3, a.perm, kClasses3, va, cls);
                credit(a.out3, a.perm, kClasses3, vb, cls);
                shape[0]++;
            }
            if (K4) {
                for (uint32_t l = j + 1; l < d; l++) {
                    const uint32_t ec = P[l];
                    const uint32_t vc = ec >> 2, rc = ec & 3u;
                    const uint32_t ac = arc_bits(a.off, a.adj, va, vc);
                    const uint32_t bc = arc_bits(a.off, a.adj, vb, vc);
                    const uint32_t cls = a.t4[motif_index4(ra, rb, rc, ab, ac, bc)];
                    if (cls < kClasses4) atomicAdd(&sRoot4[cls], 1ull);
                    credit(a.out4, a.perm, kClasses4, va, cls);
                    credit(a.out4, a.perm, kClasses4, vb, cls);
                    credit(a.out4, a.perm, kClasses4, vc, cls);
                    shape[2]++;
                }
            }
        }

        // ---- depth-2 candidates: entries (a, c) of rows of N+(r) with c > r, c not in N(r)
        for (uint32_t c0 = 0; c0 < d; c0 += kStage) {
            const uint32_t cn = min(kStage, d - c0);
            __syncthreads();
            for (uint32_t i = tid; i < cn; i += kThreads) {
                const uint32_t va = P[c0 + i] >> 2;
                sLo[i] = lower_bound_rank(a.adj, a.off[va], a.off[va + 1], r + 1);
                sPre[i + 1] = a.off[va + 1] - sLo[i];
            }
            __syncthreads();
            if (tid == 0) {   // short serial scan; v1 keeps this simple
                sPre[0] = 0;
                for (uint32_t i = 1; i <= cn; i++) sPre[i] += sPre[i - 1];
            }
            __syncthreads();
            const uint32_t total = sPre[cn];
            for (uint32_t q = tid; q < total; q += kThreads) {
                uint32_t lo = 0, hi = cn;   // slot with sPre[i] <= q < sPre[i+1]
                while (hi - lo > 1) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (sPre[mid] <= q) lo = mid; else hi = mid;
                }
                const uint32_t i = c0 + lo;
                const uint32_t ea = P[i];
                const uint32_t va = ea >> 2, ra = ea & 3u;
                const uint32_t t = sLo[lo] + (q - sPre[lo]);
                const uint32_t ecn = a.adj[t];
                const uint32_t vc = ecn >> 2, ac = ecn & 3u;
                if (in_list(P, d, vc)) continue;   // c adjacent to r: depth 1, not 2
                if (K3) {
                    const uint32_t cls = a.t3[motif_index3(ra, 0u, ac)];
                    if (cls < kClasses3) atomicAdd(&sRoot3[cls], 1ull);
                    credit(a.out3, a.perm, kClasses3, va, cls);
                    credit(a.out3, a.perm, kClasses3, vc, cls);
                    shape[1]++;
                }
                if (K4) {
                    // (2,1,0): second depth-1 vertex b
                    for (uint32_t j = 0; j < d; j++) {
                        if (j == i) continue;
                        const uint32_t eb = P[j];
                        const uint32_t vb = eb >> 2, rb = eb & 3u;
                        const uint32_t bc = arc_bits(a.off, a.adj, vb, vc);
                        if (bc && j < i) continue;   // c hangs under the lower-rank parent b
                        const uint32_t ab = arc_bits(a.off, a.adj, va, vb);
                        uint32_t code;
                        if (i < j) code = motif_index4(ra, rb, 0u, ab, ac, bc);
                        else code = motif_index4(rb, ra, 0u, swap_arc_bits(ab), bc, ac);
                        const uint32_t cls = a.t4[code];
                        if (cls < kClasses4) atomicAdd(&sRoot4[cls], 1ull);
                        credit(a.out4, a.perm, kClasses4, va, cls);
                        credit(a.out4, a.perm, kClasses4, vb, cls);
                        credit(a.out4, a.perm, kClasses4, vc, cls);
                        shape[3]++;
                    }
                    // (1,2,0): a second depth-2 child c' > c of a
                    const uint32_t ha = a.off[va + 1];
                    for (uint32_t t2 = t + 1; t2 < ha; t2++) {
                        const uint32_t e2 = a.adj[t2];
                        const uint32_t vc2 = e2 >> 2;
                        if (in_list(P, d, vc2)) continue;
                        const uint32_t cc2 = arc_bits(a.off, a.adj, vc, vc2);
                        const uint32_t cls = a.t4[motif_index4(ra, 0u, 0u, ac, e2 & 3u, cc2)];
                        if (cls < kClasses4) atomicAdd(&sRoot4[cls], 1ull);
                        credit(a.out4, a.perm, kClasses4, va, cls);
                        credit(a.out4, a.perm, kClasses4, vc, cls);
                        credit(a.out4, a.perm, kClasses4, vc2, cls);
                        shape[4]++;
                    }
                    // (1,1,1): path r - a - c - e, e not adjacent to r nor to a
                    const uint32_t hc = a.off[vc + 1];
                    for (uint32_t t3 = lower_bound_rank(a.adj, a.off[vc], hc, r + 1); t3 < hc; t3++) {
                        const uint32_t e3 = a.adj[t3];
                        const uint32_t ve = e3 >> 2;
                        if (in_list(P, d, ve)) continue;               // also excludes a itself
                        if (arc_bits(a.off, a.adj, va, ve)) continue;  // e adjacent to a: depth 2
                        const uint32_t cls = a.t4[motif_index4(ra, 0u, 0u, ac, 0u, e3 & 3u)];
                        if (cls < kClasses4) atomicAdd(&sRoot4[cls], 1ull);
                        credit(a.out4, a.perm, kClasses4, va, cls);
                        credit(a.out4, a.perm, kClasses4, vc, cls);
                        credit(a.out4, a.perm, kClasses4, ve, cls);
                        shape[5]++;
                    }
                }
            }
        }
        __syncthreads();
        const size_t row = (size_t)a.perm[r];
        if (K3)
            for (uint32_t i = tid; i < kClasses3; i += kThreads)
                if (sRoot3[i]) atomicAdd(&a.out3[row * kClasses3 + i], sRoot3[i]);
        if (K4)
            for (uint32_t i = tid; i < kClasses4; i += kThreads)
                if (sRoot4[i]) atomicAdd(&a.out4[row * kClasses4 + i], sRoot4[i]);
    }
    for (int s = 0; s < kShapes; s++)
        if (shape[s]) atomicAdd(&a.stats[s], shape[s]);
}

__global__ void k_fill(unsigned long long* p, size_t n, unsigned long long v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

void launch_fill_u64(uint64_t* p, size_t n, uint64_t value, hipStream_t st) {
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, (unsigned long long*)p, n,
                       (unsigned long long)value);
    VDMC_HIP(hipGetLastError());
}

void launch_count(vdmc_graph_s* g, int k3, int k4, uint64_t* out3, uint64_t* out4, hipStream_t st) {
    const ClassTables& t = class_tables();
    ensure_bins(g, hub_min_default(), st);
    if (k3) launch_fill_u64(out3, (size_t)g->n * kClasses3, 0, st);
    if (k4) launch_fill_u64(out4, (size_t)g->n * kClasses4, 0, st);
    launch_fill_u64((uint64_t*)g->stats, kShapes, 0, st);
    if (g->nlight > 0) {
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
        int64_t blocks = g->nlight < 65536 ? g->nlight : 65536;
        if (k3 && k4)
            hipLaunchKernelGGL((k_count_roots<true, true>), dim3((unsigned)blocks), dim3(kThreads), 0, st, a);
        else if (k3)
            hipLaunchKernelGGL((k_count_roots<true, false>), dim3((unsigned)blocks), dim3(kThreads), 0, st, a);
        else
            hipLaunchKernelGGL((k_count_roots<false, true>), dim3((unsigned)blocks), dim3(kThreads), 0, st, a);
        VDMC_HIP(hipGetLastError());
    }
    launch_hub(g, k3, k4, out3, out4, st);
}

}  // namespace vdmc

extern "C" {

vdmc_status vdmc_count(vdmc_graph g, int32_t k, uint64_t* out, void* stream) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG,
                     "k must be 3 or 4");
        VDMC_REQUIRE(out != nullptr || g->n == 0, VDMC_ERR_INVALID_ARG, "out is NULL");
        VDMC_HIP(hipSetDevice(g->device));
        vdmc::launch_count(g, k == 3, k == 4, k == 3 ? out : nullptr, k == 4 ? out : nullptr,
                           vdmc::as_stream(stream));
    });
}

vdmc_status vdmc_count34(vdmc_graph g, uint64_t* out3, uint64_t* out4, void* stream) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_REQUIRE((out3 && out4) || g->n == 0, VDMC_ERR_INVALID_ARG, "out3/out4 is NULL");
        VDMC_REQUIRE(out3 != out4 || g->n == 0, VDMC_ERR_INVALID_ARG, "out3 and out4 alias");
        VDMC_HIP(hipSetDevice(g->device));
        vdmc::launch_count(g, 1, 1, out3, out4, vdmc::as_stream(stream));
    });
}

vdmc_status vdmc_shape_counts(vdmc_graph g, uint64_t* shape_counts) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr && shape_counts != nullptr, VDMC_ERR_INVALID_ARG, "NULL argument");
        VDMC_HIP(hipSetDevice(g->device));
        VDMC_HIP(hipDeviceSynchronize());
        VDMC_HIP(hipMemcpy(shape_counts, g->stats, vdmc::kShapes * sizeof(uint64_t), hipMemcpyDeviceToHost));
    });
}

}  // extern "C"

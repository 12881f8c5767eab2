// Undirected motif counts (the paper's undirected runs: Fig. 3 caption, Table 2).
//
// A graph built with VDMC_UNDIRECTED carries both arc bits on every vertex pair, so
// every connected k-set falls into the one directed class whose pairs are all
// reciprocal; those directed classes are exactly the undirected classes (connected
// graphs on k vertices up to isomorphism).  The count runs the directed path into a
// per-graph n x C scratch and a gather kernel keeps the undirected columns.
#include <algorithm>

#include "vdmc_internal.h"

namespace vdmc {
namespace {

// bit of entry (i, j) in a k-vertex motif index: row-major, diagonal skipped, first
// entry most significant (Sec. 4.1, Fig. 1)
int entry_bit(int k, int i, int j) { return k * (k - 1) - 1 - (i * (k - 1) + (j < i ? j : j - 1)); }

// directed class of every undirected class, ascending
std::vector<uint8_t> undirected_list(int k) {
    const ClassTables& t = class_tables();
    const std::vector<uint8_t>& host = k == 3 ? t.host3 : t.host4;
    const int npairs = k * (k - 1) / 2;
    std::vector<uint8_t> cls;
    for (int mask = 0; mask < (1 << npairs); mask++) {
        uint32_t code = 0;
        int b = 0;
        for (int i = 0; i < k; i++)
            for (int j = i + 1; j < k; j++, b++)
                if ((mask >> b) & 1) code |= (1u << entry_bit(k, i, j)) | (1u << entry_bit(k, j, i));
        if (host[code] != 0xFF) cls.push_back(host[code]);
    }
    std::sort(cls.begin(), cls.end());
    cls.erase(std::unique(cls.begin(), cls.end()), cls.end());
    VDMC_REQUIRE((int)cls.size() == (k == 3 ? 2 : 6), VDMC_ERR_DEVICE,
                 "unexpected number of undirected classes: " + std::to_string(cls.size()));
    return cls;
}

struct Cols {
    uint8_t c[8];
};

__global__ void k_gather_cols(const unsigned long long* __restrict__ tmp, int C, Cols cols, int U, int64_t n,
                              unsigned long long* __restrict__ out) {
    const int64_t total = n * U;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = i / U;
        out[i] = tmp[v * C + cols.c[i % U]];
    }
}

}  // namespace
}  // namespace vdmc

extern "C" {

int32_t vdmc_num_classes_undirected(int32_t k) { return k == 3 ? 2 : (k == 4 ? 6 : -1); }

vdmc_status vdmc_undirected_classes(int32_t k, uint8_t* directed_class_out) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(directed_class_out != nullptr, VDMC_ERR_INVALID_ARG, "directed_class_out is NULL");
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG, "k must be 3 or 4");
        const auto l = vdmc::undirected_list(k);
        std::copy(l.begin(), l.end(), directed_class_out);
    });
}

vdmc_status vdmc_count_undirected(vdmc_graph g, int32_t k, uint64_t* out, void* stream) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph is NULL");
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG, "k must be 3 or 4");
        VDMC_REQUIRE(g->undirected, VDMC_ERR_INVALID_ARG, "graph was not built with VDMC_UNDIRECTED");
        VDMC_REQUIRE(out != nullptr || g->n == 0, VDMC_ERR_INVALID_ARG, "out is NULL");
        VDMC_HIP(hipSetDevice(g->device));
        if (g->n == 0) return;
        const auto cls = vdmc::undirected_list(k);
        const hipStream_t st = vdmc::as_stream(stream);
        vdmc::GraphUse use(g, st);
        if (!g->utmp) VDMC_HIP(hipMalloc(&g->utmp, (size_t)g->n * vdmc::kClasses4 * sizeof(uint64_t)));
        vdmc::launch_count(g, k == 3, k == 4, k == 3 ? g->utmp : nullptr, k == 4 ? g->utmp : nullptr, st);
        vdmc::Cols c{};
        for (size_t j = 0; j < cls.size(); j++) c.c[j] = cls[j];
        const int U = (int)cls.size(), C = vdmc::num_classes(k);
        const int64_t total = g->n * U;
        const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
        hipLaunchKernelGGL(vdmc::k_gather_cols, dim3(blocks), dim3(256), 0, st,
                           (const unsigned long long*)g->utmp, C, c, U, g->n, (unsigned long long*)out);
        VDMC_HIP(hipGetLastError());
    });
}

}  // extern "C"

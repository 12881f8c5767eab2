// Batched counts without any allocation, for callers that cannot allocate device memory
// (code under stream capture, serving loops, harnesses that forbid it).
//
// vdmc_count_batch keeps, per batch signature, a plan whose device arrays (graph
// descriptors, work cursor) it allocates.  This variant takes graphs that the
// whole-graph kernel counts (small.hip) and puts the descriptors and the cursor in a
// file-scope device array instead, `scratch`, of a fixed maximum size.  The array's
// device address is resolved once per device by vdmc_init (hipGetSymbolAddress); host
// code uses only that address.  Descriptors reach the array through the arguments of a
// small fill kernel, which also clears the cursor, so no host buffer, memset or copy is
// involved.  Every call on a device shares that device's array: calls that overlap on
// one device race, and the caller orders them (and orders them against other calls on
// the same graphs).
#include <atomic>

#include "vdmc_internal.h"

namespace vdmc {
namespace {

constexpr uint32_t kNoAllocMaxGraphs = 8192;
constexpr size_t kScratchBytes = kNoAllocMaxGraphs * sizeof(SmallGraph) + 256;
constexpr int kMaxDevices = 64;
constexpr uint32_t kFillPerLaunch = 40;   // descriptors per fill-kernel argument block

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceState {
    std::atomic<bool> ready{false};
    void* ptr = nullptr;   // device address of `scratch` on this device
    int ncu = 0;
};
DeviceState g_dev[kMaxDevices];
std::mutex g_init_mu;

struct FillArgs {
    SmallGraph d[kFillPerLaunch];
    uint32_t base, count;
    unsigned* cursor;   // cleared by the first block of the first fill launch
    SmallGraph* out;
};

__global__ void k_fill_desc(FillArgs a) {
    const uint32_t i = threadIdx.x;
    if (i < a.count) a.out[a.base + i] = a.d[i];
    if (a.base == 0 && i == 0) *a.cursor = 0u;
}

}  // namespace
}  // namespace vdmc

extern "C" {

vdmc_status vdmc_init(void) {
    return vdmc::guarded([&] {
        int dev = 0;
        VDMC_HIP(hipGetDevice(&dev));
        VDMC_REQUIRE(dev >= 0 && dev < vdmc::kMaxDevices, VDMC_ERR_UNSUPPORTED, "device index too large");
        (void)vdmc::class_tables();   // built once per device (allocates)
        std::lock_guard<std::mutex> lock(vdmc::g_init_mu);
        vdmc::DeviceState& s = vdmc::g_dev[dev];
        if (s.ready.load()) return;
        void* p = nullptr;
        VDMC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(vdmc::scratch)));
        VDMC_REQUIRE(p != nullptr, VDMC_ERR_DEVICE, "no device address for the scratch array");
        hipDeviceProp_t prop;
        VDMC_HIP(hipGetDeviceProperties(&prop, dev));
        s.ptr = p;
        s.ncu = prop.multiProcessorCount;
        s.ready.store(true);
    });
}

vdmc_status vdmc_count_batch_noalloc(const vdmc_graph* gs, int32_t num, int32_t k, uint64_t* const* outs,
                                     void* stream) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG, "k must be 3 or 4");
        VDMC_REQUIRE(num >= 0, VDMC_ERR_INVALID_ARG, "num must be non-negative");
        VDMC_REQUIRE(num <= (int32_t)vdmc::kNoAllocMaxGraphs, VDMC_ERR_INVALID_ARG,
                     "at most " + std::to_string(vdmc::kNoAllocMaxGraphs) + " graphs per call");
        if (num == 0) return;
        VDMC_REQUIRE(gs != nullptr && outs != nullptr, VDMC_ERR_INVALID_ARG, "gs/outs is NULL");
        int dev = 0;
        VDMC_HIP(hipGetDevice(&dev));
        VDMC_REQUIRE(dev >= 0 && dev < vdmc::kMaxDevices && vdmc::g_dev[dev].ready.load(), VDMC_ERR_INVALID_ARG,
                     "vdmc_init has not run on the current device");
        const vdmc::DeviceState& ds = vdmc::g_dev[dev];
        size_t lds = 0;
        for (int i = 0; i < num; i++) {
            const vdmc_graph_s* g = gs[i];
            VDMC_REQUIRE(g != nullptr, VDMC_ERR_INVALID_ARG, "graph " + std::to_string(i) + " is NULL");
            VDMC_REQUIRE(g->device == dev, VDMC_ERR_INVALID_ARG, "graph " + std::to_string(i) + " lives on another device");
            VDMC_REQUIRE(outs[i] != nullptr, VDMC_ERR_INVALID_ARG, "output " + std::to_string(i) + " is NULL");
            VDMC_REQUIRE(vdmc::small_eligible(g->n, 2 * g->pairs, k), VDMC_ERR_UNSUPPORTED,
                         "graph " + std::to_string(i) + " is larger than the whole-graph kernel takes (n <= " +
                             std::to_string(vdmc::kSmallMaxN) + " and its CSR, bitmap and counters in LDS)");
            lds = std::max(lds, vdmc::small_lds_bytes(g->n, 2 * g->pairs, k));
        }
        const hipStream_t st = vdmc::as_stream(stream);
        auto* desc = reinterpret_cast<vdmc::SmallGraph*>(ds.ptr);
        auto* cursor = reinterpret_cast<unsigned*>(static_cast<unsigned char*>(ds.ptr) +
                                                   vdmc::kNoAllocMaxGraphs * sizeof(vdmc::SmallGraph));
        for (uint32_t base = 0; base < (uint32_t)num; base += vdmc::kFillPerLaunch) {
            vdmc::FillArgs f;
            f.base = base;
            f.count = std::min<uint32_t>(vdmc::kFillPerLaunch, (uint32_t)num - base);
            f.cursor = cursor;
            f.out = desc;
            for (uint32_t j = 0; j < f.count; j++) {
                const vdmc_graph_s* g = gs[base + j];
                f.d[j] = vdmc::SmallGraph{g->off, g->adj, g->perm, (unsigned long long*)outs[base + j], g->stats,
                                          (uint32_t)g->n, (uint32_t)(2 * g->pairs)};
            }
            hipLaunchKernelGGL(vdmc::k_fill_desc, dim3(1), dim3(64), 0, st, f);
            VDMC_HIP(hipGetLastError());
        }
        const vdmc::ClassTables& t = vdmc::class_tables();
        vdmc::SmallArgs a{};
        a.graphs = desc;
        a.num = (uint32_t)num;
        a.cursor = cursor;
        a.table = k == 3 ? t.t3 : t.t4;
        a.comp_of = t.slot4;
        a.comp_cls = t.slotcls;
        const int fit = std::max(1, (int)(163840 / (lds + 9216)));
        const unsigned grid = (unsigned)std::min<int64_t>(num, (int64_t)ds.ncu * fit);
        vdmc::launch_small(a, k, 2, grid, lds, st);
    });
}

}  // extern "C"

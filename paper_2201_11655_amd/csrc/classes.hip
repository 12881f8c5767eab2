// Isomorphism class tables (k = 3, 4, 5), built once per device by kernels.
//
// Paper: the motif index is the induced adjacency matrix read row by row without
// the diagonal, first entry most significant (Sec. 4.1, Fig. 1); isomorphs are
// merged into their minimal index (Fig. 1; "combining isomorphisms only once",
// Sec. 2; last step of Sec. 4.2).  The table maps every raw index to a class id
// (ascending minimal index among connected classes) so that the merge happens in
// the same instruction that credits a motif, with no post-processing pass.
#include <algorithm>
#include <map>

#include "vdmc_internal.h"

namespace vdmc {
namespace {

__host__ __device__ constexpr int factorial(int k) { return k <= 1 ? 1 : k * factorial(k - 1); }

// weight of the off-diagonal entry (i, j) in a K-vertex index
template <int K>
__device__ inline int entry_shift(int i, int j) {
    return K * (K - 1) - 1 - (i * (K - 1) + (j < i ? j : j - 1));
}

// Lehmer-code decoding of permutation number idx of {0..K-1}
template <int K>
__device__ inline void nth_permutation(int idx, int* p) {
    int avail[K];
    for (int i = 0; i < K; i++) avail[i] = i;
    int left = K;
    for (int i = 0; i < K; i++) {
        int f = factorial(K - 1 - i);
        int q = idx / f;
        idx -= q * f;
        p[i] = avail[q];
        for (int t = q; t < left - 1; t++) avail[t] = avail[t + 1];
        left--;
    }
}

template <int K>
__device__ inline int entry(uint32_t code, int i, int j) {
    return (code >> entry_shift<K>(i, j)) & 1u;
}

template <int K>
__device__ uint32_t minimal_relabelling(uint32_t code) {
    uint32_t best = 0xffffffffu;
    for (int pi = 0; pi < factorial(K); pi++) {
        int p[K];
        nth_permutation<K>(pi, p);
        uint32_t c = 0;
        for (int i = 0; i < K; i++)
            for (int j = 0; j < K; j++)
                if (i != j && entry<K>(code, p[i], p[j])) c |= 1u << entry_shift<K>(i, j);
        best = c < best ? c : best;
    }
    return best;
}

template <int K>
__device__ bool weakly_connected(uint32_t code) {
    uint32_t reached = 1u, frontier = 1u;
    while (frontier) {
        uint32_t next = 0;
        for (int x = 0; x < K; x++) {
            if (!(frontier >> x & 1u)) continue;
            for (int y = 0; y < K; y++)
                if (x != y && (entry<K>(code, x, y) || entry<K>(code, y, x))) next |= 1u << y;
        }
        frontier = next & ~reached;
        reached |= next;
    }
    return reached == (1u << K) - 1u;
}

constexpr int kTableThreads = 1024;

template <int K>
__global__ __launch_bounds__(kTableThreads) void k_class_table(uint8_t* table, uint16_t* class_codes,
                                                               int* num_classes) {
    constexpr int NC = 1 << (K * (K - 1));
    constexpr int PER = (NC + kTableThreads - 1) / kTableThreads;
    __shared__ uint16_t canon[NC];
    __shared__ uint8_t conn[NC];
    __shared__ uint16_t cid[NC];
    __shared__ int scan[kTableThreads];
    const int tid = threadIdx.x;
    int mine = 0;
    for (int t = 0; t < PER; t++) {
        int c = tid * PER + t;
        if (c < NC) {
            canon[c] = (uint16_t)minimal_relabelling<K>((uint32_t)c);
            conn[c] = weakly_connected<K>((uint32_t)c) ? 1 : 0;
        }
    }
    __syncthreads();
    for (int t = 0; t < PER; t++) {
        int c = tid * PER + t;
        if (c < NC && canon[c] == c && conn[c]) mine++;
    }
    scan[tid] = mine;
    __syncthreads();
    for (int s = 1; s < kTableThreads; s <<= 1) {   // inclusive Hillis-Steele scan
        int v = tid >= s ? scan[tid - s] : 0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    int next_id = scan[tid] - mine;
    for (int t = 0; t < PER; t++) {
        int c = tid * PER + t;
        if (c < NC && canon[c] == c && conn[c]) {
            cid[c] = (uint16_t)next_id;
            class_codes[next_id] = (uint16_t)c;
            next_id++;
        }
    }
    if (tid == kTableThreads - 1) *num_classes = scan[tid];
    __syncthreads();
    for (int t = 0; t < PER; t++) {
        int c = tid * PER + t;
        if (c < NC) table[c] = conn[c] ? (uint8_t)cid[canon[c]] : (uint8_t)0xFF;
    }
}

// k = 5: 2^20 codes, too many for one workgroup's LDS.  Three launches: every code's
// minimal relabelling and connectivity (one thread per code); the class ids, ascending
// with the minimal index, by one workgroup scanning 1024 codes per thread; the table.
constexpr uint32_t kCodes5 = 1u << 20;

__global__ __launch_bounds__(256) void k_canon5(uint32_t* canon, uint8_t* conn) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= kCodes5) return;
    canon[c] = minimal_relabelling<5>(c);
    conn[c] = weakly_connected<5>(c) ? 1 : 0;
}

__global__ __launch_bounds__(kTableThreads) void k_ids5(const uint32_t* canon, const uint8_t* conn, uint16_t* cid,
                                                        uint32_t* class_codes, int* num_classes) {
    constexpr uint32_t PER = kCodes5 / kTableThreads;
    __shared__ int scan[kTableThreads];
    const int tid = threadIdx.x;
    const uint32_t lo = tid * PER;
    int mine = 0;
    for (uint32_t c = lo; c < lo + PER; c++) mine += (canon[c] == c && conn[c]) ? 1 : 0;
    scan[tid] = mine;
    __syncthreads();
    for (int s = 1; s < kTableThreads; s <<= 1) {   // inclusive Hillis-Steele scan
        int v = tid >= s ? scan[tid - s] : 0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    int next_id = scan[tid] - mine;
    for (uint32_t c = lo; c < lo + PER; c++)
        if (canon[c] == c && conn[c]) {
            cid[c] = (uint16_t)next_id;
            class_codes[next_id] = c;
            next_id++;
        }
    if (tid == kTableThreads - 1) *num_classes = scan[tid];
}

__global__ __launch_bounds__(256) void k_table5(const uint32_t* canon, const uint8_t* conn, const uint16_t* cid,
                                                uint16_t* table) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= kCodes5) return;
    table[c] = conn[c] ? cid[canon[c]] : (uint16_t)0xFFFF;
}

std::mutex g_tables_mu;
std::map<int, ClassTables*> g_tables;
std::mutex g_tables5_mu;
std::map<int, ClassTable5*> g_tables5;

template <int K>
void build_one(uint8_t* d_table, std::vector<uint8_t>& host, std::vector<uint16_t>& codes) {
    constexpr int NC = 1 << (K * (K - 1));
    uint16_t* d_codes = nullptr;
    int* d_num = nullptr;
    VDMC_HIP(hipMalloc(&d_codes, NC * sizeof(uint16_t)));
    VDMC_HIP(hipMalloc(&d_num, sizeof(int)));
    hipLaunchKernelGGL(k_class_table<K>, dim3(1), dim3(kTableThreads), 0, 0, d_table, d_codes, d_num);
    VDMC_HIP(hipGetLastError());
    int num = 0;
    host.resize(NC);
    std::vector<uint16_t> all(NC);
    VDMC_HIP(hipMemcpy(&num, d_num, sizeof(int), hipMemcpyDeviceToHost));
    VDMC_HIP(hipMemcpy(host.data(), d_table, NC, hipMemcpyDeviceToHost));
    VDMC_HIP(hipMemcpy(all.data(), d_codes, NC * sizeof(uint16_t), hipMemcpyDeviceToHost));
    VDMC_HIP(hipFree(d_codes));
    VDMC_HIP(hipFree(d_num));
    VDMC_REQUIRE(num == num_classes(K), VDMC_ERR_DEVICE,
                 "class table kernel produced " + std::to_string(num) + " classes for k=" +
                     std::to_string(K));
    codes.assign(all.begin(), all.begin() + num);
}

}  // namespace

const ClassTables& class_tables() {
    int dev = 0;
    VDMC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_tables_mu);
    auto it = g_tables.find(dev);
    if (it != g_tables.end()) return *it->second;
    auto* t = new ClassTables();
    uint8_t* d = nullptr;
    VDMC_HIP(hipMalloc(&d, 64 + 4096 + 256 + 64 + 768 + 16 + 16));
    build_one<3>(d, t->host3, t->codes3);
    build_one<4>(d + 64, t->host4, t->codes4);
    t->t3 = d;
    t->t4 = d + 64;
    // compact slots: classes of 4-sets whose G_U is a tree; with the set ordered
    // (v0, v1, v2, v3) and arc bits p_ij, a path v0-v1-v2-v3 has p01, p12, p23 != 0 and a
    // star centred at v1 has p01, p12, p13 != 0 (every other pair empty)
    std::vector<uint8_t> slot(256, 0xFF), slotcls, star_of(256, 0xFF), path_of(256, 0xFF), star_cls, path_cls;
    auto idx4 = [](unsigned p01, unsigned p02, unsigned p03, unsigned p12, unsigned p13, unsigned p23) {
        return ((p01 & 1u) << 11) | ((p01 >> 1) << 8) | ((p02 & 1u) << 10) | ((p02 >> 1) << 5) |
               ((p03 & 1u) << 9) | ((p03 >> 1) << 2) | ((p12 & 1u) << 7) | ((p12 >> 1) << 4) |
               ((p13 & 1u) << 6) | ((p13 >> 1) << 1) | ((p23 & 1u) << 3) | (p23 >> 1);
    };
    std::vector<int> tree_classes, stars, paths;
    for (unsigned a = 1; a <= 3; a++)
        for (unsigned b = 1; b <= 3; b++)
            for (unsigned c = 1; c <= 3; c++) {
                paths.push_back(t->host4[idx4(a, 0, 0, b, 0, c)]);   // path v0 - v1 - v2 - v3
                stars.push_back(t->host4[idx4(a, 0, 0, b, c, 0)]);   // star centred at v1
            }
    for (auto* v : {&stars, &paths}) {
        std::sort(v->begin(), v->end());
        v->erase(std::unique(v->begin(), v->end()), v->end());
    }
    VDMC_REQUIRE(stars.size() == 10 && paths.size() == 15, VDMC_ERR_DEVICE, "expected 10 star and 15 path classes");
    for (size_t i = 0; i < stars.size(); i++) {
        star_of[stars[i]] = (uint8_t)i;
        star_cls.push_back((uint8_t)stars[i]);
    }
    for (size_t i = 0; i < paths.size(); i++) {
        path_of[paths[i]] = (uint8_t)i;
        path_cls.push_back((uint8_t)paths[i]);
    }
    tree_classes = stars;
    tree_classes.insert(tree_classes.end(), paths.begin(), paths.end());
    std::sort(tree_classes.begin(), tree_classes.end());
    tree_classes.erase(std::unique(tree_classes.begin(), tree_classes.end()), tree_classes.end());
    VDMC_REQUIRE((int)tree_classes.size() == kCompact4, VDMC_ERR_DEVICE,
                 "expected 25 tree classes, found " + std::to_string(tree_classes.size()));
    for (size_t i = 0; i < tree_classes.size(); i++) {
        slot[tree_classes[i]] = (uint8_t)i;
        slotcls.push_back((uint8_t)tree_classes[i]);
    }
    slotcls.resize(64, 0);
    VDMC_HIP(hipMemcpy(d + 64 + 4096, slot.data(), 256, hipMemcpyHostToDevice));
    VDMC_HIP(hipMemcpy(d + 64 + 4096 + 256, slotcls.data(), 64, hipMemcpyHostToDevice));
    t->slot4 = d + 64 + 4096;
    t->slotcls = d + 64 + 4096 + 256;
    // class -> star slot | path slot | tree slot, then slot -> class for stars and paths
    std::vector<uint8_t> maps(star_of);
    maps.insert(maps.end(), path_of.begin(), path_of.end());
    maps.insert(maps.end(), slot.begin(), slot.end());
    star_cls.resize(16, 0);
    path_cls.resize(16, 0);
    uint8_t* dm = d + 64 + 4096 + 256 + 64;
    VDMC_HIP(hipMemcpy(dm, maps.data(), 768, hipMemcpyHostToDevice));
    VDMC_HIP(hipMemcpy(dm + 768, star_cls.data(), 16, hipMemcpyHostToDevice));
    VDMC_HIP(hipMemcpy(dm + 784, path_cls.data(), 16, hipMemcpyHostToDevice));
    t->maps4 = dm;
    t->star_cls = dm + 768;
    t->path_cls = dm + 784;
    g_tables[dev] = t;   // kept for the life of the process
    return *t;
}

const ClassTable5& class_table5() {
    int dev = 0;
    VDMC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_tables5_mu);
    auto it = g_tables5.find(dev);
    if (it != g_tables5.end()) return *it->second;
    uint32_t *canon = nullptr, *codes = nullptr;
    uint8_t* conn = nullptr;
    uint16_t *cid = nullptr, *table = nullptr;
    int* num = nullptr;
    struct Free {
        std::vector<void*> p;
        ~Free() {
            for (void* x : p) (void)hipFree(x);
        }
    } tmp;
    VDMC_HIP(hipMalloc(&canon, kCodes5 * sizeof(uint32_t)));
    tmp.p.push_back(canon);
    VDMC_HIP(hipMalloc(&conn, kCodes5));
    tmp.p.push_back(conn);
    VDMC_HIP(hipMalloc(&cid, kCodes5 * sizeof(uint16_t)));
    tmp.p.push_back(cid);
    VDMC_HIP(hipMalloc(&codes, kClasses5 * sizeof(uint32_t)));
    tmp.p.push_back(codes);
    VDMC_HIP(hipMalloc(&num, sizeof(int)));
    tmp.p.push_back(num);
    VDMC_HIP(hipMalloc(&table, kCodes5 * sizeof(uint16_t)));
    VDMC_HIP(hipMemset(cid, 0, kCodes5 * sizeof(uint16_t)));
    hipLaunchKernelGGL(k_canon5, dim3(kCodes5 / 256), dim3(256), 0, 0, canon, conn);
    VDMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ids5, dim3(1), dim3(kTableThreads), 0, 0, canon, conn, cid, codes, num);
    VDMC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_table5, dim3(kCodes5 / 256), dim3(256), 0, 0, canon, conn, cid, table);
    VDMC_HIP(hipGetLastError());
    int n = 0;
    VDMC_HIP(hipMemcpy(&n, num, sizeof(int), hipMemcpyDeviceToHost));
    if (n != kClasses5) {
        (void)hipFree(table);
        VDMC_REQUIRE(false, VDMC_ERR_DEVICE, "class table kernels produced " + std::to_string(n) + " classes for k=5");
    }
    auto* t = new ClassTable5();
    t->table = table;
    t->codes.resize(kClasses5);
    VDMC_HIP(hipMemcpy(t->codes.data(), codes, kClasses5 * sizeof(uint32_t), hipMemcpyDeviceToHost));
    g_tables5[dev] = t;   // kept for the life of the process
    return *t;
}

}  // namespace vdmc

extern "C" {

int32_t vdmc_num_classes(int32_t k) { return vdmc::num_classes(k); }

vdmc_status vdmc_class_codes_u32(int32_t k, uint32_t* codes_out) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(codes_out != nullptr, VDMC_ERR_INVALID_ARG, "codes_out is NULL");
        VDMC_REQUIRE(k >= 3 && k <= 5, VDMC_ERR_INVALID_ARG, "k must be 3, 4 or 5");
        if (k == 5) {
            const auto& c = vdmc::class_table5().codes;
            std::copy(c.begin(), c.end(), codes_out);
        } else {
            const auto& t = vdmc::class_tables();
            const auto& c = k == 3 ? t.codes3 : t.codes4;
            std::copy(c.begin(), c.end(), codes_out);
        }
    });
}

vdmc_status vdmc_class_table_u16(int32_t k, uint16_t* table_out) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(table_out != nullptr, VDMC_ERR_INVALID_ARG, "table_out is NULL");
        VDMC_REQUIRE(k >= 3 && k <= 5, VDMC_ERR_INVALID_ARG, "k must be 3, 4 or 5");
        if (k == 5) {
            VDMC_HIP(hipMemcpy(table_out, vdmc::class_table5().table, (size_t)vdmc::kCodes5 * sizeof(uint16_t),
                               hipMemcpyDeviceToHost));
        } else {
            const auto& t = vdmc::class_tables();
            const auto& h = k == 3 ? t.host3 : t.host4;
            for (size_t i = 0; i < h.size(); i++) table_out[i] = h[i] == 0xFF ? (uint16_t)0xFFFF : h[i];
        }
    });
}

vdmc_status vdmc_class_codes(int32_t k, uint16_t* codes_out) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(codes_out != nullptr, VDMC_ERR_INVALID_ARG, "codes_out is NULL");
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG,
                     k == 5 ? "5-vertex codes need 32 bits: vdmc_class_codes_u32" : "k must be 3 or 4");
        const auto& t = vdmc::class_tables();
        const auto& c = k == 3 ? t.codes3 : t.codes4;
        std::copy(c.begin(), c.end(), codes_out);
    });
}

vdmc_status vdmc_class_table(int32_t k, uint8_t* table_out) {
    return vdmc::guarded([&] {
        VDMC_REQUIRE(table_out != nullptr, VDMC_ERR_INVALID_ARG, "table_out is NULL");
        VDMC_REQUIRE(k == 3 || k == 4, k == 5 ? VDMC_ERR_UNSUPPORTED : VDMC_ERR_INVALID_ARG,
                     k == 5 ? "5-vertex class ids need 16 bits: vdmc_class_table_u16" : "k must be 3 or 4");
        const auto& t = vdmc::class_tables();
        const auto& h = k == 3 ? t.host3 : t.host4;
        std::copy(h.begin(), h.end(), table_out);
    });
}

}  // extern "C"

/*
 * vdmc.h -- C ABI of the MI355X (gfx950) per-vertex directed motif counter.
 *
 * The library computes, for every vertex v of a directed graph G and for k = 3,
 * 4 or 5, the number of connected k-vertex induced subgraphs ("k-motifs") that
 * contain v, split over the isomorphism classes of k-vertex weakly connected
 * digraphs (13 classes for k = 3, 199 for k = 4, 9364 for k = 5; 5-vertex motifs
 * are the extension Sec. 11 names, counted for graphs held whole in one
 * workgroup's LDS).
 *
 * Definitions (paper: Levinas, Scherz, Louzoun, "BFS based distributed algorithm
 * for parallel local directed sub-graph enumeration"):
 *   - a k-motif is a set of k vertices connected in the undirected graph G_U
 *     underneath G (Sec. 4.1);
 *   - the motif index is the k x k adjacency matrix of the induced subgraph,
 *     row = source, read row by row with the diagonal removed, first entry most
 *     significant (Sec. 4.1, Fig. 1); isomorphic indices are merged into the
 *     minimal one (Fig. 1, Sec. 4.2);
 *   - every vertex of a motif gets one count in the motif's class (Sec. 4.2).
 * Class ids: the minimal indices of connected classes in ascending order
 * (vdmc_class_codes returns them).
 *
 * Conventions
 *   - Every call returns a vdmc_status; on failure vdmc_last_error() returns a
 *     thread-local message.  No C++ exception crosses this boundary.
 *   - Device pointers are HIP device pointers on the current device; `stream` is
 *     a hipStream_t passed as void* (NULL = the null stream).  Calls that take a
 *     stream are asynchronous on it unless stated otherwise.
 *   - Counts are uint64.  Output matrices are row-major uint64[n][C] with row =
 *     ORIGINAL vertex id and column = class id; the caller owns them.
 *   - Input arcs may contain self-loops (dropped) and repeated arcs (merged):
 *     the paper works on a simple graph (Sec. 4.1).
 *   - A graph is immutable after build and may be counted from several host threads
 *     and streams at once: the device work of every call on a graph (count, count34,
 *     count_range, count_undirected, count_edges, count_batch, served requests) is
 *     ordered after the previous call's on that graph, whatever its stream, so each
 *     output is that of the call alone.  Calls on different graphs overlap freely.
 *     Output buffers of calls in flight must not alias.
 */
#ifndef VDMC_H
#define VDMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vdmc_graph_s* vdmc_graph;     /* opaque; owns the device CSR; immutable */
typedef struct vdmc_server_s* vdmc_server;   /* opaque; see vdmc_serve_* below */
typedef int32_t vdmc_status;

enum {
    VDMC_OK = 0,
    VDMC_ERR_INVALID_ARG = 1,   /* bad pointer, size, id or k */
    VDMC_ERR_OUT_OF_MEMORY = 2, /* a device or host allocation failed */
    VDMC_ERR_DEVICE = 3,        /* a HIP runtime call failed */
    VDMC_ERR_UNSUPPORTED = 4,   /* valid request this library does not implement (e.g. k = 5 on a large graph) */
    VDMC_ERR_BUSY = 5,          /* server has no free slot right now */
    VDMC_ERR_NOT_FOUND = 6,     /* unknown request id */
    VDMC_ERR_REJECTED = 7,      /* request can never fit the server's memory budget */
    VDMC_ERR_TIMEOUT = 8        /* a wait ran out of time; the request is still running */
};

/* vdmc_build_graph flags */
enum {
    VDMC_INPUT_ON_DEVICE = 2u,  /* src/dst are device pointers (else host pointers) */
    VDMC_UNDIRECTED = 4u        /* ignore arc directions: count motifs of the undirected graph */
};

/* vdmc_count_range flags */
enum {
    VDMC_ACCUMULATE = 1u        /* add to out (and to the shape counters) instead of overwriting */
};

/* Message describing the last failure on the calling thread ("" if none). */
const char* vdmc_last_error(void);

/* Number of classes: 13 for k = 3, 199 for k = 4, 9364 for k = 5, -1 otherwise. */
int32_t vdmc_num_classes(int32_t k);

/* Minimal motif index (Sec. 4.1, Fig. 1) of every class, ascending by class id.
 * codes_out: host array of vdmc_num_classes(k) entries.  k = 3 or 4 (5-vertex
 * indices have 20 bits: UNSUPPORTED, use vdmc_class_codes_u32).  Synchronous. */
vdmc_status vdmc_class_codes(int32_t k, uint16_t* codes_out);

/* Class id of every raw motif index: table_out is a host array of 2^(k(k-1))
 * bytes; 0xFF marks a disconnected index.  Built once per device by a kernel that
 * tries all k! relabellings (the "combine isomorphisms once" step, Sec. 2, 4.2).
 * k = 3 or 4 (k = 5 has 9364 ids: UNSUPPORTED, use vdmc_class_table_u16).
 * Synchronous. */
vdmc_status vdmc_class_table(int32_t k, uint8_t* table_out);

/* The same two tables for k = 3, 4 or 5 in wider types: codes_out holds
 * vdmc_num_classes(k) uint32 minimal indices; table_out holds 2^(k(k-1)) uint16 class
 * ids, 0xFFFF marking a disconnected index (k = 5: 2^20 entries).  The k = 5 table is
 * built on the device at its first use (three kernels: every code's minimal
 * relabelling over the 120 permutations, the ascending ids, the table) and kept.
 * INVALID_ARG for another k.  Synchronous. */
vdmc_status vdmc_class_codes_u32(int32_t k, uint32_t* codes_out);
vdmc_status vdmc_class_table_u16(int32_t k, uint16_t* table_out);

/*
 * Build the device graph from arcs src[i] -> dst[i], i < m, vertex ids in [0, n).
 *   - flags & VDMC_INPUT_ON_DEVICE: src/dst are device pointers, else host pointers;
 *     the library copies them; the caller keeps ownership.
 *   - Self-loops are dropped and repeated arcs merged; u->v and v->u together form
 *     one undirected pair carrying both arc bits.
 *   - flags & VDMC_UNDIRECTED: every pair gets both arc bits, i.e. the graph counted is
 *     the underlying undirected graph G_U; use vdmc_count_undirected on it.
 *   - Vertices are ranked by undirected degree, largest first, ties by original id
 *     (the removal order of Sec. 2 and Sec. 6); the CSR is stored in rank space,
 *     each row ascending, every entry (neighbour_rank << 2) | arc_bits with bit 0 =
 *     row -> neighbour and bit 1 = neighbour -> row (Sec. 4.2 CSR).
 * Errors: INVALID_ARG for n < 0, m < 0, n >= 2^30, NULL arrays with m > 0, or an id
 * outside [0, n); OUT_OF_MEMORY; DEVICE.  Synchronises `stream` (the sizes of the
 * result are needed on the host).  On success *out owns all device memory of the
 * graph until vdmc_free_graph.
 */
vdmc_status vdmc_build_graph(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                             uint32_t flags, void* stream, vdmc_graph* out);

/* Sizes of a built graph (any pointer may be NULL): vertices, distinct arcs,
 * undirected pairs, largest undirected degree. */
vdmc_status vdmc_graph_info(vdmc_graph g, int64_t* n, int64_t* arcs, int64_t* pairs,
                            int32_t* max_deg);

/* Rank-space CSR of a built graph, copied to host arrays (for tests): off[n+1],
 * adj[2*pairs] entries (nbr_rank << 2 | arc_bits), perm[n] (rank -> original id).
 * Any pointer may be NULL.  Synchronous. */
vdmc_status vdmc_graph_export(vdmc_graph g, uint32_t* off, uint32_t* adj, int32_t* perm);

/*
 * Undirected motifs (the paper's undirected runs, Fig. 3 and Table 2): connected
 * induced subgraphs of G_U, merged by undirected isomorphism: 2 classes for k = 3
 * (path, triangle), 6 for k = 4 (path, star, cycle, triangle with a tail, diamond,
 * complete graph).  Undirected class j is the directed class (of vdmc_class_codes)
 * whose every vertex pair carries both arcs; classes are ordered by that directed id.
 *   vdmc_num_classes_undirected: 2, 6, or -1 for another k.
 *   vdmc_undirected_classes: directed_class_out[j] = the directed class of undirected
 *     class j (host array of vdmc_num_classes_undirected(k) bytes).  Synchronous.
 *   vdmc_count_undirected: g built with VDMC_UNDIRECTED (else INVALID_ARG); out is a
 *     DEVICE buffer of n * vdmc_num_classes_undirected(k) uint64 (row = original id),
 *     written, not accumulated.  Asynchronous on `stream`; the first call on a graph
 *     allocates an n x 199 uint64 scratch that the graph keeps until it is freed.
 */
int32_t vdmc_num_classes_undirected(int32_t k);
vdmc_status vdmc_undirected_classes(int32_t k, uint8_t* directed_class_out);
vdmc_status vdmc_count_undirected(vdmc_graph g, int32_t k, uint64_t* out, void* stream);

/*
 * Per-edge counts (Sec. 11, "count per edge"): for every vertex pair {lo < hi} joined in
 * G_U, the number of connected k-sets of each class that contain both lo and hi.
 *   vdmc_edge_list: the pairs in output-row order, ascending (lo, hi) original ids, as
 *     host arrays lo[pairs], hi[pairs] (pairs from vdmc_graph_info).  Synchronous.
 *   vdmc_count_edges: out is a DEVICE buffer of pairs * vdmc_num_classes(k) uint64,
 *     written, not accumulated.  Asynchronous on `stream`, except that the first call on
 *     a graph builds the edge index (an edge hash of 2^ceil(log2(4 pairs)) 8-byte slots
 *     plus a 4-byte row per slot, kept with the graph) and synchronises `stream`.  Every
 *     root goes through the per-set kernel, which credits the joined pairs of each set.
 */
vdmc_status vdmc_edge_list(vdmc_graph g, int32_t* lo, int32_t* hi);
vdmc_status vdmc_count_edges(vdmc_graph g, int32_t k, uint64_t* out, void* stream);

/* Releases the graph's device memory.  NULL is a no-op.  The caller must make sure no
 * count on the graph is still running. */
vdmc_status vdmc_free_graph(vdmc_graph g);

/*
 * Per-vertex k-motif counts (Sec. 4.2): out is a caller-owned DEVICE buffer of
 * n * vdmc_num_classes(k) uint64, fully overwritten (zeroed first, inside the call).
 * Every connected k-set is visited exactly once, from its lowest-rank vertex (Lemma 1)
 * along the BFS shapes of Lemma 2 under the rules of Lemmas 3-4: one lane assembles
 * its index (Sec. 4.1), looks up its class and credits the class to its k vertices
 * (vdmc_shape_counts reports the sets visited per shape).
 * k in {3, 4, 5}, other k INVALID_ARG.  k = 5 (n x 9364 output; n < 229,338): a graph
 * held whole in one workgroup's LDS -- n <= 512 and 4 (4n + 2 + 2 pairs + n ceil(n/32))
 * bytes of CSR, id map and 1-bit adjacency matrix within 159744 -- is counted there;
 * any other is counted in device memory, which at its first 5-vertex count builds the
 * graph's edge hash (2^ceil(log2(4 pairs)) 8-byte slots), an (n + 2) x 8-byte item
 * table and, for n <= 16384, a 1-bit adjacency matrix (n x ceil(n/32) x 4 bytes, at
 * most 32 MiB), kept with the graph and synchronising `stream` once.  Its sets are visited
 * along the eight BFS layer shapes of five vertices (vdmc_profile_counters).  An LDS
 * count of a graph with at least 64 pairs splits it into up to 64 parts whose extra
 * private n x 9364 blocks (at most 512 MiB) and item cursors are taken from the
 * device's default stream-ordered pool (hipMallocAsync on `stream`) and returned to it
 * after the launches; the library raises that pool's release threshold to 8.25 GiB so
 * that repeated counts reuse the pages (other users of the default pool keep that
 * much too).  A graph
 * with n < k gives an all-zero matrix.  Asynchronous on `stream`; `out` must not be in use by
 * another call.  The first count on a graph (and the first after a change of its hub
 * threshold) bins its roots and synchronises `stream`; the hub path's scratch is
 * allocated then and kept with the graph.  Roots with at most 2048 higher neighbours
 * in graphs whose largest degree is at most 2048 (and n < 2^26) can take the hub
 * path; every other root is counted by the per-root kernel.
 */
vdmc_status vdmc_count(vdmc_graph g, int32_t k, uint64_t* out, void* stream);

/* 1 if vdmc_count(g, k, ...) and vdmc_count_batch with g can run (k = 3, 4: any graph;
 * k = 5: n x 9364 below 2^31), 0 if they give UNSUPPORTED, -1 for a NULL graph or a k
 * outside 3..5.  Lets a caller skip allocating an n x 9364 output it cannot use. */
int32_t vdmc_count_supported(vdmc_graph g, int32_t k);

/* The part of vdmc_count contributed by roots whose rank lies in [rank_begin, rank_end):
 * the k-sets whose lowest-rank vertex is in the range (Lemma 1 makes such root ranges
 * independent; they are the unit the paper proposes for spreading the work over devices,
 * Sec. 11).  Without VDMC_ACCUMULATE, out is zeroed first; with it, the range's counts
 * are added to out, so consecutive ranges covering [0, n) give exactly vdmc_count's
 * result.  Ranks are those of the graph's degree order (vdmc_graph_export's perm maps
 * them to ids).  Asynchronous on `stream`. */
vdmc_status vdmc_count_range(vdmc_graph g, int32_t k, uint64_t* out, int64_t rank_begin, int64_t rank_end,
                             uint32_t flags, void* stream);

/* Hub threshold of a graph: roots with at least min_higher higher-rank neighbours
 * (|N+(r)|, the depth-1 candidates of Lemma 2) are counted by the hub path, the others by
 * the per-root kernel; both enumerate the same sets (Lemma 1 makes roots independent),
 * so the counts do not depend on the threshold.  The default is 32.  A change takes
 * effect at the next count; the root bins and any cached batched launch of the graph
 * are rebuilt.  min_higher in [1, 2^30] (1: every root with work takes the hub path),
 * else INVALID_ARG.  Must not be called while a count on the graph is running. */
vdmc_status vdmc_set_hub_threshold(vdmc_graph g, int32_t min_higher);

/* Both k = 3 (out3: n x 13) and k = 4 (out4: n x 199) in one call; one staging of
 * each root's neighbourhood feeds both. */
vdmc_status vdmc_count34(vdmc_graph g, uint64_t* out3, uint64_t* out4, void* stream);

/* Sets visited one by one by the last count on this graph (host; waits for it), per BFS
 * shape in the order k=3: (1,1), (1,2); k=4: (3,0,0), (2,1,0), (1,2,0), (1,1,1).  Every
 * visit is one set whose index was assembled, class looked up and vertices credited, so
 * the k=4 entries add up to the number of 4-sets.  shape_counts: 6 entries. */
vdmc_status vdmc_shape_counts(vdmc_graph g, uint64_t* shape_counts);

/* The graph's counters of the last count (host; waits for it): after k = 3, 4 entries
 * 0-5 are the shape counts above, 6-7 are zero; after k = 5 the 8 entries are the sets
 * visited per BFS layer shape of five vertices, in the order (4) (3,1) (2,2) (2,1,1)
 * (1,3) (1,2,1) (1,1,2) (1,1,1,1) (layer sizes from the root outwards), adding up to
 * the number of connected 5-sets.  Copies min(n, 8) entries. */
vdmc_status vdmc_profile_counters(vdmc_graph g, uint64_t* counters, int32_t n);

/* Device time of the kernels of the last count call on this graph, from events recorded
 * on the count's stream around the launches (host; waits for those events):
 * ms_out[0] the per-root kernel over the light roots, ms_out[1] the hub path (the hub
 * kernel, then for k = 4 the long-slot kernel), ms_out[2] the hub kernel alone; -1 for a
 * part that the call did not launch.  ms_out: n floats, caller-owned; the first
 * min(n, 3) are written. */
vdmc_status vdmc_kernel_times(vdmc_graph g, float* ms_out, int32_t n);

/*
 * Batched counts: num graphs, one k for all, outs[i] a DEVICE buffer of
 * n_i * vdmc_num_classes(k) uint64 for graph gs[i].  All graphs are counted by one
 * persistent launch whose work tiles come from a device-side cursor; the launch is
 * captured in a HIP graph the first time a batch signature (same graphs, same
 * outputs, same k) is seen and replayed afterwards.  Asynchronous on `stream`.
 * k = 5: every graph must satisfy vdmc_count_supported (else UNSUPPORTED).  The graphs
 * that LDS holds are counted by one launch (graphs cut into parts with private blocks,
 * summed afterwards: at most 8 GiB per call, from the default stream-ordered pool as
 * for vdmc_count), the others one by one in device memory after it; not captured.
 */
vdmc_status vdmc_count_batch(const vdmc_graph* gs, int32_t num, int32_t k,
                             uint64_t* const* outs, void* stream);

/* Per-device set-up: builds the class tables and resolves the device address of the
 * allocation-free entry point's scratch array on the current device.  Idempotent; may
 * allocate.  Call it on each device before vdmc_count_batch_noalloc there. */
vdmc_status vdmc_init(void);

/*
 * vdmc_count_batch without any allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid it).
 * Same arguments and results as vdmc_count_batch, for graphs that the whole-graph kernel
 * takes (n <= 1024 and the graph's CSR, adjacency bitmap and counters fit one
 * workgroup's LDS; UNSUPPORTED otherwise) and at most 8192 graphs per call
 * (INVALID_ARG beyond).  Requires vdmc_init on the current device (INVALID_ARG
 * otherwise).  The graph descriptors and the work cursor live in a fixed device array
 * of ~384 KiB per device, held until the process ends; the call allocates nothing,
 * issues no memset and no host-to-device copy (descriptors travel as kernel arguments),
 * and is asynchronous on `stream`.  Every call on a device shares that array: calls that
 * overlap on one device race, and the caller orders them, also against other calls on
 * the same graphs (this entry point skips the per-graph ordering of the others).
 */
vdmc_status vdmc_count_batch_noalloc(const vdmc_graph* gs, int32_t num, int32_t k, uint64_t* const* outs,
                                     void* stream);

/* Picks the batch launch parameters (workgroup size of the whole-graph kernel; threads
 * per root, workgroups per CU and roots per cursor step of the root table) by timing
 * every candidate on the given batch (median of 3 runs).  The choice is kept for batches
 * of the same shape (k, number of graphs, total vertices, total pairs) in this process
 * and appended to cache_path (NULL: memory only); a later process reads such a file when
 * VDMC_TUNE_CACHE names it.  Synchronous.  Results are bit-identical for every choice. */
vdmc_status vdmc_tune(const vdmc_graph* gs, int32_t num, int32_t k, const char* cache_path);

/* The launch parameters vdmc_count_batch uses for a batch of this shape: choice_out[0] =
 * 1 if they come from the tuner (else the defaults), [1] threads per workgroup of the
 * whole-graph kernel, [2] threads per root, [3] workgroups per CU, [4] roots per cursor
 * step.  choice_out: 5 host int32.  Synchronous, no device work. */
vdmc_status vdmc_tuned_choice(const vdmc_graph* gs, int32_t num, int32_t k, int32_t* choice_out);

/*
 * Serving: a request loop over resident graphs.
 *   vdmc_serve_create: mem_budget_bytes caps the device memory that the server allocates
 *     for requests in flight (the hub-path scratch of a request's graph; outputs belong to
 *     the caller and are not counted); max_inflight caps the number of requests on the
 *     GPU at once.  The server also holds small fixed buffers per stream slot.
 *   vdmc_serve_submit: queue a count of graph g for k into the caller's DEVICE buffer
 *     out (n x C uint64); returns a request id at once (nothing is allocated).  Requests
 *     are admitted in arrival order as slots and memory free up: a request on a graph
 *     the whole-graph kernel takes needs no memory and is fused with others of the same
 *     k; any other needs its graph's hub scratch, allocated at admission inside the
 *     budget and freed at completion.  A request whose scratch cannot fit now waits; one
 *     that can never fit fails with REJECTED (at submit when the graph's size is already
 *     known, else at admission, reported by poll/wait).  Admitted requests run
 *     concurrently on the device.
 *   vdmc_serve_poll: non-blocking; *done = 1 when the request's output is complete; the
 *     request's own error status if it failed.
 *   vdmc_serve_wait: blocks up to timeout_us (< 0: no limit); TIMEOUT if not done; the
 *     request's own status (REJECTED, DEVICE, ...) if it failed.
 *   vdmc_serve_stats: latency percentiles (submit -> completion seen), throughput and
 *     number of k-sets counted by completed requests.
 *   vdmc_serve_destroy: waits for running requests, cancels queued ones, frees the server.
 */
typedef struct {
    uint64_t mem_budget_bytes;
    int32_t max_inflight;
} vdmc_serve_config;

vdmc_status vdmc_serve_create(const vdmc_serve_config* cfg, vdmc_server* out);
vdmc_status vdmc_serve_submit(vdmc_server s, vdmc_graph g, int32_t k, uint64_t* out,
                              uint64_t* req_id);
vdmc_status vdmc_serve_poll(vdmc_server s, uint64_t req_id, int32_t* done);
vdmc_status vdmc_serve_wait(vdmc_server s, uint64_t req_id, int64_t timeout_us);
vdmc_status vdmc_serve_stats(vdmc_server s, double* p50_us, double* p99_us, double* req_per_s,
                             uint64_t* sets);
vdmc_status vdmc_serve_destroy(vdmc_server s);

/* Request-loop counters (host, synchronous): counters[0] submitted, [1] admitted,
 * [2] completed, [3] rejected (could never fit the budget, or cancelled by destroy),
 * [4] failed on the device, [5] times the head of the queue waited for memory,
 * [6] queue depth now, [7] largest queue depth, [8] server-allocated bytes in flight now,
 * [9] largest bytes in flight.  Copies min(n, 10) entries. */
vdmc_status vdmc_serve_counters(vdmc_server s, uint64_t* counters, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* VDMC_H */

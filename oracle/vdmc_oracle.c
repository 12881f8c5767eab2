/*
 * CPU oracle for per-vertex directed 3-, 4- and 5-motif counts.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this file's library.  It shares no code with the
 * GPU library: its class table, its graph normalisation and its enumeration are
 * all written here from the plain definition of what the method computes.
 *
 * What is computed (paper Sec. 4.1 definitions; Sec. 4.2 algorithm; Lemma 1):
 *   - G is a directed graph; G_U is the undirected graph underneath it.  Self
 *     loops are dropped and repeated arcs merged (the paper assumes a simple
 *     graph, Sec. 4.1).
 *   - a k-motif is a set S of k vertices that is connected in G_U;
 *   - its index is the k x k adjacency matrix of the induced subgraph, read row
 *     by row with the diagonal removed, as a binary number whose first entry,
 *     (0,1), is the most significant bit (Sec. 4.1 and Fig. 1: the matrix of
 *     Fig. 1 reads 110101 = 53);
 *   - isomorphic motifs are merged into the minimal index over all k!
 *     relabellings (Sec. 4.1, Fig. 1: 53 -> 30; Sec. 4.2 last step);
 *   - every vertex of S has its counter for S's class raised by one
 *     (Sec. 4.2, per-vertex update).
 *   Class ids: the distinct minimal indices of connected motifs, ascending.
 *
 * The enumeration of connected k-sets is Wernicke's ESU (the FANMOD algorithm
 * cited in Sec. 1): every connected k-set is produced exactly once, from its
 * smallest vertex, by extending with "exclusive" neighbours only.  ESU is a
 * different algorithm from the paper's BFS shapes, which is the point: the
 * oracle does not restate the method it is checking.  It is itself pinned to
 * brute force over all k-subsets in the tests.
 *
 * Plain C, integer arithmetic only, pthreads over start vertices.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define MAXK 5

/* ---------------------------------------------------------------------------
 * Class table: code -> canonical (minimal) code, connectivity, class id.
 * ------------------------------------------------------------------------- */

/* bit position of the off-diagonal entry (i,j), i != j, in a k-vertex code:
 * the entries are listed row by row without the diagonal; the t-th listed entry
 * has weight 2^(k(k-1)-1-t). */
static int entry_bit(int k, int i, int j) {
    int t = i * (k - 1) + (j < i ? j : j - 1);
    return k * (k - 1) - 1 - t;
}

static void decode(int k, uint32_t code, int A[MAXK][MAXK]) {
    for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++)
            A[i][j] = (i != j) ? (int)((code >> entry_bit(k, i, j)) & 1u) : 0;
}

static uint32_t encode(int k, int A[MAXK][MAXK]) {
    uint32_t c = 0;
    for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++)
            if (i != j && A[i][j]) c |= 1u << entry_bit(k, i, j);
    return c;
}

static int next_perm(int *p, int k) {
    int i = k - 2;
    while (i >= 0 && p[i] > p[i + 1]) i--;
    if (i < 0) return 0;
    int j = k - 1;
    while (p[j] < p[i]) j--;
    int t = p[i]; p[i] = p[j]; p[j] = t;
    for (int a = i + 1, b = k - 1; a < b; a++, b--) { t = p[a]; p[a] = p[b]; p[b] = t; }
    return 1;
}

/* Sets canon[x] = c for every relabelling x of the code c: x = code(B) with
 * B[i][j] = A[pi(i)][pi(j)] over all k! permutations pi. */
static void mark_orbit(int k, uint32_t code, uint32_t *canon) {
    int A[MAXK][MAXK], B[MAXK][MAXK], p[MAXK];
    decode(k, code, A);
    for (int i = 0; i < k; i++) p[i] = i;
    do {
        for (int i = 0; i < k; i++)
            for (int j = 0; j < k; j++) B[i][j] = A[p[i]][p[j]];
        canon[encode(k, B)] = code;
    } while (next_perm(p, k));
}

/* connectivity of the underlying undirected graph of the code */
static int connected_of(int k, uint32_t code) {
    int A[MAXK][MAXK];
    decode(k, code, A);
    int seen[MAXK] = {0}, stack[MAXK], sp = 0, cnt = 1;
    seen[0] = 1; stack[sp++] = 0;
    while (sp) {
        int x = stack[--sp];
        for (int y = 0; y < k; y++)
            if (!seen[y] && (A[x][y] || A[y][x])) { seen[y] = 1; cnt++; stack[sp++] = y; }
    }
    return cnt == k;
}

/* Fills canon[2^(k(k-1))] and cls[2^(k(k-1))] (-1 for disconnected codes) and the
 * canonical code of every class in ascending order.  Returns the number of classes. */
int oracle_class_table(int k, uint32_t *canon, int32_t *cls, uint32_t *class_codes) {
    if (k < 2 || k > MAXK) return -1;
    uint32_t ncode = 1u << (k * (k - 1));
    /* canon[c] = min over all relabellings of c.  The relabellings of c form its orbit,
     * and every member of an orbit has the same orbit; scanning codes upwards, the first
     * member met is the orbit's minimum, and marking the orbit from it settles every
     * member (k! encodings per orbit rather than per code). */
    const uint32_t unset = 0xffffffffu;
    for (uint32_t c = 0; c < ncode; c++) canon[c] = unset;
    for (uint32_t c = 0; c < ncode; c++)
        if (canon[c] == unset) mark_orbit(k, c, canon);
    int nc = 0;
    for (uint32_t c = 0; c < ncode; c++)          /* ascending scan = ascending class ids */
        if (canon[c] == c && connected_of(k, c)) class_codes[nc++] = c;
    for (uint32_t c = 0; c < ncode; c++) {
        cls[c] = -1;
        if (!connected_of(k, c)) continue;
        int lo = 0, hi = nc;                       /* class_codes is ascending */
        while (lo < hi) {
            int mid = (lo + hi) / 2;
            if (class_codes[mid] < canon[c]) lo = mid + 1; else hi = mid;
        }
        if (lo < nc && class_codes[lo] == canon[c]) cls[c] = lo;
    }
    return nc;
}

/* ---------------------------------------------------------------------------
 * Simple graph: sorted undirected neighbour lists with arc bits.
 *   nbr[i] for i in [off[v], off[v+1]) are the G_U neighbours of v, ascending;
 *   dir[i] bit 0: arc v -> nbr exists; bit 1: arc nbr -> v exists.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    int64_t *off;
    int32_t *nbr;
    uint8_t *dir;
} sgraph;

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

static int build_sgraph(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, sgraph *g) {
    /* one record per arc per endpoint: (row, other, bit) packed as row<<34 | other<<2 | bit */
    uint64_t *rec = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(2 * m + 1));
    if (!rec) return -1;
    int64_t r = 0;
    for (int64_t i = 0; i < m; i++) {
        int64_t u = src[i], v = dst[i];
        if (u < 0 || v < 0 || u >= n || v >= n) { free(rec); return -2; }
        if (u == v) continue;                       /* self-loops carry no motif information */
        rec[r++] = ((uint64_t)u << 34) | ((uint64_t)v << 2) | 1u;  /* u -> v seen from u */
        rec[r++] = ((uint64_t)v << 34) | ((uint64_t)u << 2) | 2u;  /* u -> v seen from v */
    }
    qsort(rec, (size_t)r, sizeof(uint64_t), cmp_u64);
    g->n = n;
    g->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(r + 1));
    g->dir = (uint8_t *)malloc((size_t)r + 1);
    if (!g->off || !g->nbr || !g->dir) { free(rec); return -1; }
    int64_t e = 0;
    for (int64_t i = 0; i < r;) {
        uint64_t key = rec[i] >> 2;
        uint8_t bits = 0;
        while (i < r && (rec[i] >> 2) == key) { bits |= (uint8_t)(rec[i] & 3u); i++; }
        int64_t row = (int64_t)(key >> 32);
        g->nbr[e] = (int32_t)(key & 0xffffffffu);
        g->dir[e] = bits;
        g->off[row + 1]++;
        e++;
    }
    for (int64_t v = 0; v < n; v++) g->off[v + 1] += g->off[v];
    free(rec);
    return 0;
}

static void free_sgraph(sgraph *g) { free(g->off); free(g->nbr); free(g->dir); }

/* arc bits between u and v seen from u (bit0: u->v, bit1: v->u); 0 if not adjacent */
static int arc_bits(const sgraph *g, int32_t u, int32_t v) {
    int64_t lo = g->off[u], hi = g->off[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->nbr[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (lo < g->off[u + 1] && g->nbr[lo] == v) ? g->dir[lo] : 0;
}

/* ---------------------------------------------------------------------------
 * ESU enumeration with per-vertex crediting.
 * ------------------------------------------------------------------------- */
typedef struct {
    const sgraph *g;
    int k;
    const int32_t *cls;    /* code -> class id, -1 if disconnected */
    int ncls;
    uint64_t *out;         /* private rows x ncls */
    uint64_t *totals;      /* private ncls: number of k-sets per class (each set once) */
    int32_t forced;        /* -1: ordinary ESU; else every set contains this vertex */
    int64_t forced_row;    /* forced mode: the only row credited */
    const int64_t *upre;   /* edge mode (non-NULL): pair id of the entry e > first upper
                              entry of row u is upre[u] + (e - ufirst[u]) */
    const int64_t *ufirst;
} esu_ctx;

/* position of v in u's neighbour list, or -1 */
static int64_t entry_of(const sgraph *g, int32_t u, int32_t v) {
    int64_t lo = g->off[u], hi = g->off[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->nbr[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (lo < g->off[u + 1] && g->nbr[lo] == v) ? lo : -1;
}

static void credit(esu_ctx *c, const int32_t *S) {
    int k = c->k;
    int A[MAXK][MAXK];
    for (int i = 0; i < k; i++) {
        A[i][i] = 0;
        for (int j = i + 1; j < k; j++) {
            int b = arc_bits(c->g, S[i], S[j]);
            A[i][j] = b & 1;
            A[j][i] = (b >> 1) & 1;
        }
    }
    int id = c->cls[encode(k, A)];
    if (id < 0) return;  /* cannot happen for a connected set; kept as a guard */
    c->totals[id]++;
    if (c->upre) {   /* per-edge counts: every vertex pair of S joined in G_U */
        for (int i = 0; i < k; i++)
            for (int j = i + 1; j < k; j++) {
                if (!A[i][j] && !A[j][i]) continue;
                int32_t u = S[i] < S[j] ? S[i] : S[j], v = S[i] < S[j] ? S[j] : S[i];
                int64_t e = entry_of(c->g, u, v);
                int64_t pid = c->upre[u] + (e - c->ufirst[u]);
                c->out[(size_t)pid * (size_t)c->ncls + (size_t)id]++;
            }
        return;
    }
    if (c->forced >= 0) {
        c->out[(size_t)c->forced_row * (size_t)c->ncls + (size_t)id]++;
        return;
    }
    for (int i = 0; i < k; i++) c->out[(size_t)S[i] * (size_t)c->ncls + (size_t)id]++;
}

/* is u outside N[S] (not in S and adjacent to no member of S)? */
static int exclusive(const sgraph *g, const int32_t *S, int ns, int32_t u) {
    for (int i = 0; i < ns; i++) {
        if (S[i] == u) return 0;
        if (arc_bits(g, S[i], u)) return 0;
    }
    return 1;
}

/* "u comes after v" in the enumeration order: ordinary ids, or, in forced mode,
 * the forced vertex first and every other vertex after it. */
static int after(const esu_ctx *c, int32_t u, int32_t v) {
    if (c->forced >= 0) return u != c->forced;
    return u > v;
}

static int64_t deg(const sgraph *g, int32_t v) { return g->off[v + 1] - g->off[v]; }

/* S has ns members; ext[0..next) is the extension set. */
static void extend(esu_ctx *c, int32_t *S, int ns, const int32_t *ext, int64_t next, int32_t v) {
    if (ns == c->k) { credit(c, S); return; }
    if (ns + 1 == c->k) {   /* last level: every member of the extension set completes S */
        for (int64_t i = next - 1; i >= 0; i--) { S[ns] = ext[i]; credit(c, S); }
        return;
    }
    int64_t maxdeg = 0;
    for (int64_t i = 0; i < next; i++) if (deg(c->g, ext[i]) > maxdeg) maxdeg = deg(c->g, ext[i]);
    int32_t mine[1024];
    int32_t *buf = (next + maxdeg <= 1024) ? mine
                 : (int32_t *)malloc(sizeof(int32_t) * (size_t)(next + maxdeg));
    int64_t rem = next;
    while (rem > 0) {
        int32_t w = ext[--rem];               /* remove an arbitrary element */
        int64_t nn = 0;
        for (int64_t i = 0; i < rem; i++) buf[nn++] = ext[i];
        for (int64_t e = c->g->off[w]; e < c->g->off[w + 1]; e++) {
            int32_t u = c->g->nbr[e];
            if (after(c, u, v) && exclusive(c->g, S, ns, u)) buf[nn++] = u;
        }
        S[ns] = w;
        extend(c, S, ns + 1, buf, nn, v);
    }
    if (buf != mine) free(buf);
}

typedef struct { int32_t v; int32_t row; int64_t jlo, jhi; } task;

typedef struct {
    esu_ctx ctx;
    int64_t *cursor;
    const task *tasks;
    int64_t ntasks;
} worker;

/* one first-level choice: S = {v, ext[j]}, extension ext[0..j) plus the exclusive
 * neighbours of ext[j] */
static void first_level(esu_ctx *c, int32_t v, const int32_t *ext, int64_t j) {
    int32_t S[MAXK];
    S[0] = v;
    int32_t w = ext[j];
    int64_t cap = j + deg(c->g, w) + 1;
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int64_t nn = 0;
    for (int64_t i = 0; i < j; i++) buf[nn++] = ext[i];
    for (int64_t e = c->g->off[w]; e < c->g->off[w + 1]; e++) {
        int32_t u = c->g->nbr[e];
        if (after(c, u, v) && exclusive(c->g, S, 1, u)) buf[nn++] = u;
    }
    S[1] = w;
    extend(c, S, 2, buf, nn, v);
    free(buf);
}

static void *run_worker(void *p) {
    worker *w = (worker *)p;
    esu_ctx *c = &w->ctx;
    for (;;) {
        int64_t i = __atomic_fetch_add(w->cursor, 1, __ATOMIC_RELAXED);
        if (i >= w->ntasks) break;
        const task *t = &w->tasks[i];
        if (t->row >= 0) { c->forced = t->v; c->forced_row = t->row; }
        int32_t v = t->v;
        int64_t d = deg(c->g, v);
        int32_t *ext = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d + 1));
        int64_t ne = 0;
        for (int64_t e = c->g->off[v]; e < c->g->off[v + 1]; e++)
            if (after(c, c->g->nbr[e], v)) ext[ne++] = c->g->nbr[e];
        int64_t jhi = t->jhi < ne ? t->jhi : ne;
        for (int64_t j = t->jlo; j < jhi; j++) first_level(c, v, ext, j);
        free(ext);
    }
    return NULL;
}

#define CHUNK 16

/* starts[i] with row[i] (-1 = ordinary mode).  Splits each start's first level into
 * chunks of CHUNK choices so that one high-degree start does not serialise the run. */
static int run_esu(const sgraph *g, int k, const int32_t *cls, int ncls, int nthreads,
                   const int32_t *starts, const int32_t *rows, int64_t nstarts,
                   int64_t nrows, uint64_t *out, uint64_t *totals,
                   const int64_t *upre, const int64_t *ufirst) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    int64_t ntasks = 0;
    for (int64_t i = 0; i < nstarts; i++) ntasks += (deg(g, starts[i]) + CHUNK - 1) / CHUNK;
    task *tasks = (task *)malloc(sizeof(task) * (size_t)(ntasks + 1));
    int64_t t = 0;
    for (int64_t i = 0; i < nstarts; i++) {
        int64_t d = deg(g, starts[i]);
        for (int64_t j = 0; j < d; j += CHUNK) {
            tasks[t].v = starts[i];
            tasks[t].row = rows ? rows[i] : -1;
            tasks[t].jlo = j;
            tasks[t].jhi = j + CHUNK;
            t++;
        }
    }
    worker *ws = (worker *)calloc((size_t)nthreads, sizeof(worker));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    int64_t cursor = 0;
    size_t cells = (size_t)nrows * (size_t)ncls;
    int rc = 0;
    for (int i = 0; i < nthreads; i++) {
        ws[i].ctx.g = g; ws[i].ctx.k = k; ws[i].ctx.cls = cls; ws[i].ctx.ncls = ncls;
        ws[i].ctx.forced = -1; ws[i].ctx.forced_row = -1;
        ws[i].ctx.upre = upre; ws[i].ctx.ufirst = ufirst;
        ws[i].ctx.out = (uint64_t *)calloc(cells ? cells : 1, sizeof(uint64_t));
        ws[i].ctx.totals = (uint64_t *)calloc((size_t)ncls, sizeof(uint64_t));
        if (!ws[i].ctx.out || !ws[i].ctx.totals) rc = -1;
        ws[i].cursor = &cursor; ws[i].tasks = tasks; ws[i].ntasks = ntasks;
    }
    if (!rc) {
        for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, run_worker, &ws[i]);
        for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
        memset(out, 0, cells * sizeof(uint64_t));
        if (totals) memset(totals, 0, (size_t)ncls * sizeof(uint64_t));
        for (int i = 0; i < nthreads; i++) {
            for (size_t x = 0; x < cells; x++) out[x] += ws[i].ctx.out[x];
            if (totals) for (int x = 0; x < ncls; x++) totals[x] += ws[i].ctx.totals[x];
        }
    }
    for (int i = 0; i < nthreads; i++) { free(ws[i].ctx.out); free(ws[i].ctx.totals); }
    free(ws); free(th); free(tasks);
    return rc;
}

/* The class table of k (built once per process and kept: 2^20 codes for k = 5); the
 * caller gets a private copy. */
static pthread_mutex_t table_mu = PTHREAD_MUTEX_INITIALIZER;
static int32_t *table_cache[MAXK + 1];
static int table_ncls[MAXK + 1];

static int table_for(int k, int32_t **cls_out, int *ncls) {
    uint32_t ncode = 1u << (k * (k - 1));
    pthread_mutex_lock(&table_mu);
    if (!table_cache[k]) {
        uint32_t *canon = (uint32_t *)malloc(sizeof(uint32_t) * ncode);
        uint32_t *codes = (uint32_t *)malloc(sizeof(uint32_t) * ncode);
        int32_t *cls = (int32_t *)malloc(sizeof(int32_t) * ncode);
        int nc = oracle_class_table(k, canon, cls, codes);
        free(canon); free(codes);
        if (nc > 0) { table_cache[k] = cls; table_ncls[k] = nc; }
        else free(cls);
    }
    int32_t *copy = NULL;
    if (table_cache[k]) {
        copy = (int32_t *)malloc(sizeof(int32_t) * ncode);
        memcpy(copy, table_cache[k], sizeof(int32_t) * ncode);
        *ncls = table_ncls[k];
    }
    pthread_mutex_unlock(&table_mu);
    *cls_out = copy;
    return copy ? 0 : -1;
}

/* Full per-vertex counts: out[n][ncls] (row = original vertex id) and per-class
 * totals T[ncls] (every k-set once).  Returns 0 on success. */
int oracle_count(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int k,
                 int nthreads, uint64_t *out, uint64_t *totals) {
    if (k < 3 || k > MAXK) return -3;
    sgraph g;
    int rc = build_sgraph(n, m, src, dst, &g);
    if (rc) return rc;
    int32_t *cls; int ncls;
    if (table_for(k, &cls, &ncls)) { free_sgraph(&g); return -1; }
    int32_t *starts = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t v = 0; v < n; v++) starts[v] = (int32_t)v;
    rc = run_esu(&g, k, cls, ncls, nthreads, starts, NULL, n, n, out, totals, NULL, NULL);
    free(starts); free(cls); free_sgraph(&g);
    return rc;
}

/* Per-edge counts (Sec. 11, "count per edge"): out[pairs][ncls], row p = the p-th vertex
 * pair {lo < hi} of G_U in ascending (lo, hi) order, returned in plo/phi; each entry is
 * the number of connected k-sets of the class that contain both endpoints.  pairs must
 * be the number oracle_graph_size reports, halved. */
int oracle_count_edges(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int k,
                       int nthreads, int64_t pairs, uint64_t *out, int32_t *plo, int32_t *phi) {
    if (k < 3 || k > MAXK) return -3;
    sgraph g;
    int rc = build_sgraph(n, m, src, dst, &g);
    if (rc) return rc;
    if (g.off[n] != 2 * pairs) { free_sgraph(&g); return -4; }
    int32_t *cls; int ncls;
    if (table_for(k, &cls, &ncls)) { free_sgraph(&g); return -1; }
    int64_t *upre = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *ufirst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t p = 0;
    for (int64_t u = 0; u < n; u++) {
        int64_t e = g.off[u];
        while (e < g.off[u + 1] && g.nbr[e] < u) e++;
        ufirst[u] = e;
        upre[u] = p;
        for (; e < g.off[u + 1]; e++, p++) { plo[p] = (int32_t)u; phi[p] = g.nbr[e]; }
    }
    int32_t *starts = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t v = 0; v < n; v++) starts[v] = (int32_t)v;
    rc = run_esu(&g, k, cls, ncls, nthreads, starts, NULL, n, pairs, out, NULL, upre, ufirst);
    free(starts); free(upre); free(ufirst); free(cls); free_sgraph(&g);
    return rc;
}

/* Rows of selected vertices only: out[nrows][ncls], row i = vertex rows[i].  Every
 * connected k-set containing rows[i] is enumerated once, with rows[i] placed first in
 * ESU's vertex order, and only rows[i] is credited. */
int oracle_count_rows(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int k,
                      int nthreads, const int32_t *rows, int64_t nrows, uint64_t *out) {
    if (k < 3 || k > MAXK) return -3;
    for (int64_t i = 0; i < nrows; i++)
        if (rows[i] < 0 || rows[i] >= n) return -2;
    sgraph g;
    int rc = build_sgraph(n, m, src, dst, &g);
    if (rc) return rc;
    int32_t *cls; int ncls;
    if (table_for(k, &cls, &ncls)) { free_sgraph(&g); return -1; }
    int32_t *rowid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nrows + 1));
    for (int64_t i = 0; i < nrows; i++) rowid[i] = (int32_t)i;
    rc = run_esu(&g, k, cls, ncls, nthreads, rows, rowid, nrows, nrows, out, NULL, NULL, NULL);
    free(rowid); free(cls); free_sgraph(&g);
    return rc;
}

/* The simple graph the oracle works on, exported so that tests can compare it with
 * the CSR example of Sec. 4.2: off[n+1], nbr[2*pairs], dir[2*pairs] (caller-sized via
 * oracle_graph_size).  Returns 0 on success. */
int oracle_graph_size(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int64_t *entries) {
    sgraph g;
    int rc = build_sgraph(n, m, src, dst, &g);
    if (rc) return rc;
    *entries = g.off[n];
    free_sgraph(&g);
    return 0;
}

int oracle_graph_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     int64_t *off, int32_t *nbr, uint8_t *dir) {
    sgraph g;
    int rc = build_sgraph(n, m, src, dst, &g);
    if (rc) return rc;
    memcpy(off, g.off, sizeof(int64_t) * (size_t)(n + 1));
    memcpy(nbr, g.nbr, sizeof(int32_t) * (size_t)g.off[n]);
    memcpy(dir, g.dir, (size_t)g.off[n]);
    free_sgraph(&g);
    return 0;
}

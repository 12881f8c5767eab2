/* Runs the oracle's entry points on seeded random graphs under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_sanitizers_cpu.py) and checks
 * invariants that hold for any graph: every column sum is a multiple of k, the per-class
 * totals times k equal the column sums, the per-vertex mode equals the full rows, and the
 * per-edge counts sum to (edges of the class) x (sets of the class).  Exit status 0 when
 * all hold. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_class_table(int k, uint32_t *canon, int32_t *cls, uint32_t *class_codes);
int oracle_count(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int k, int nthreads,
                 uint64_t *out, uint64_t *totals);
int oracle_count_rows(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int k, int nthreads,
                      const int32_t *rows, int64_t nrows, uint64_t *out);
int oracle_count_edges(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int k, int nthreads,
                       int64_t pairs, uint64_t *out, int32_t *plo, int32_t *phi);
int oracle_graph_size(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int64_t *entries);

static uint64_t state = 88172645463325252ull;
static uint32_t rnd(void) {   /* xorshift64 */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (uint32_t)(state >> 11);
}

static int check_graph(int n, int m, int k) {
    int32_t *src = malloc(sizeof(int32_t) * (m + 1)), *dst = malloc(sizeof(int32_t) * (m + 1));
    for (int i = 0; i < m; i++) { src[i] = (int32_t)(rnd() % (uint32_t)n); dst[i] = (int32_t)(rnd() % (uint32_t)n); }
    int ncls = k == 3 ? 13 : 199;
    uint64_t *out = calloc((size_t)n * ncls, sizeof(uint64_t)), *tot = calloc(ncls, sizeof(uint64_t));
    int bad = oracle_count(n, m, src, dst, k, 2, out, tot) != 0;
    for (int c = 0; c < ncls && !bad; c++) {
        uint64_t col = 0;
        for (int v = 0; v < n; v++) col += out[(size_t)v * ncls + c];
        if (col != (uint64_t)k * tot[c]) bad = 1;
    }
    int32_t rows[3] = {0, n / 2, n - 1};
    uint64_t *rout = calloc(3 * (size_t)ncls, sizeof(uint64_t));
    bad |= oracle_count_rows(n, m, src, dst, k, 2, rows, 3, rout) != 0;
    for (int i = 0; i < 3 && !bad; i++)
        if (memcmp(rout + (size_t)i * ncls, out + (size_t)rows[i] * ncls, ncls * sizeof(uint64_t))) bad = 1;
    int64_t entries = 0;
    bad |= oracle_graph_size(n, m, src, dst, &entries) != 0;
    int64_t pairs = entries / 2;
    uint64_t *eout = calloc((size_t)(pairs + 1) * ncls, sizeof(uint64_t));
    int32_t *lo = calloc(pairs + 1, sizeof(int32_t)), *hi = calloc(pairs + 1, sizeof(int32_t));
    bad |= oracle_count_edges(n, m, src, dst, k, 2, pairs, eout, lo, hi) != 0;
    uint64_t esum = 0, want = 0;
    for (int64_t i = 0; i < pairs * ncls; i++) esum += eout[i];
    /* every set of a connected k-vertex class has at least k-1 joined pairs */
    for (int c = 0; c < ncls; c++) want += (uint64_t)(k - 1) * tot[c];
    if (esum < want) bad = 1;
    free(src); free(dst); free(out); free(tot); free(rout); free(eout); free(lo); free(hi);
    return bad;
}

int main(void) {
    uint32_t canon[4096], codes[4096];
    int32_t cls[4096];
    if (oracle_class_table(3, canon, cls, codes) != 13 || oracle_class_table(4, canon, cls, codes) != 199) {
        fprintf(stderr, "class table sizes wrong\n");
        return 1;
    }
    for (int t = 0; t < 12; t++) {
        int n = 2 + (int)(rnd() % 60), m = (int)(rnd() % (uint32_t)(3 * n + 1));
        for (int k = 3; k <= 4; k++)
            if (check_graph(n, m, k)) {
                fprintf(stderr, "invariant failed: n=%d m=%d k=%d\n", n, m, k);
                return 1;
            }
    }
    printf("oracle sanitizer run ok\n");
    return 0;
}

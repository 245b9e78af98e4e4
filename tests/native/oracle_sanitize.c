/* Drives every entry point of oracle/oracle.c on small seeded sets, for a
 * build under the host sanitizers (AddressSanitizer, UndefinedBehavior-
 * Sanitizer), and cross-checks the results: the brute-force lists against
 * the cell-list lists and the row checker (which must also catch a planted
 * error), the density against a sum over the brute-force rows, and the tree
 * of Algorithm 1 (b-tree and octree) against its invariants.  Prints "ok"
 * and exits 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_pair(double xi, double yi, double zi, double hi, double xj, double yj, double zj);
int64_t oracle_row(const double *x, const double *y, const double *z, const double *h,
                   int64_t n, int64_t i, int32_t *out, int64_t cap);
void oracle_counts(const double *x, const double *y, const double *z, const double *h,
                   int64_t n, const int64_t *rows, int64_t m, int64_t *counts);
int64_t oracle_lists(const double *x, const double *y, const double *z, const double *h,
                     int64_t n, const int64_t *rows, int64_t m, int64_t *offsets,
                     int32_t *nbrs, int64_t cap);
int64_t oracle_cell_lists(const double *x, const double *y, const double *z, const double *h,
                          int64_t n, int64_t *counts, int64_t *offsets, int32_t *nbrs,
                          int64_t cap);
int64_t oracle_cell_check(const double *x, const double *y, const double *z, const double *h,
                          int64_t n, const int32_t *counts, const int64_t *offsets,
                          const int32_t *nbrs, int64_t *bad, int64_t max_bad);
double oracle_sph_shape(double d2, double h);
int64_t oracle_density(const double *x, const double *y, const double *z, const double *h,
                       const double *mass, int64_t n, int32_t exclude_self, double *rho,
                       int64_t *counts);
void oracle_build_tree(const double *x, const double *y, const double *z, int64_t n, int64_t s,
                       double alpha, double beta, int32_t max_depth, int32_t octree,
                       int64_t *leaf_cnt, int32_t *leaf_depth, int64_t leaf_cap,
                       int32_t *members, int64_t *b_hist, int64_t b_hist_len, int32_t *node_b,
                       int64_t *node_n, int32_t *node_depth, int64_t node_cap, int64_t *stats);

static uint64_t rng = 0x9e3779b97f4a7c15ull;
static double uni(void)
{
    rng ^= rng >> 12;
    rng ^= rng << 25;
    rng ^= rng >> 27;
    return (double)((rng * 0x2545f4914f6cdd1dull) >> 11) * 0x1p-53;
}

static int failures = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);               \
            fprintf(stderr, "\n");                      \
            ++failures;                                 \
        }                                               \
    } while (0)

static void one_set(int64_t n, int kind)
{
    double *x = malloc(sizeof(double) * (size_t)(n + 1));
    double *y = malloc(sizeof(double) * (size_t)(n + 1));
    double *z = malloc(sizeof(double) * (size_t)(n + 1));
    double *h = malloc(sizeof(double) * (size_t)(n + 1));
    double *m = malloc(sizeof(double) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) {
        if (kind == 0) {  /* uniform cube */
            x[i] = uni(); y[i] = uni(); z[i] = uni();
        } else if (kind == 1) {  /* clustered: sums of uniforms, some duplicates */
            x[i] = uni() + uni() + uni(); y[i] = uni() * uni(); z[i] = uni() - uni();
            if (i % 13 == 5) { x[i] = x[0]; y[i] = y[0]; z[i] = z[0]; }
        } else {  /* far from the origin, tiny spread */
            x[i] = 1e6 + 1e-3 * uni(); y[i] = -3e5 + 1e-3 * uni(); z[i] = 1e-3 * uni();
        }
        h[i] = (kind == 2 ? 1e-4 : 0.03) + (kind == 2 ? 2e-4 : 0.15) * uni();
        if (i % 7 == 3) h[i] = 0.0;
        m[i] = 0.5 + uni();
    }

    /* Brute force, all rows. */
    int64_t *off = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t cap = n * n + 1;
    int32_t *nb = malloc(sizeof(int32_t) * (size_t)cap);
    int64_t tot = oracle_lists(x, y, z, h, n, NULL, n, off, nb, cap);
    CHECK(tot == off[n], "lists total");
    CHECK(n == 0 || oracle_lists(x, y, z, h, n, NULL, n, off, nb, 0) == (tot > 0 ? -1 : 0),
          "lists with no room");
    tot = oracle_lists(x, y, z, h, n, NULL, n, off, nb, cap);

    /* One row by oracle_row and by pairs; counts of a subset of rows. */
    if (n > 0) {
        int64_t i = n / 2;
        int32_t *row = malloc(sizeof(int32_t) * (size_t)n);
        int64_t k = oracle_row(x, y, z, h, n, i, row, n);
        CHECK(k == off[i + 1] - off[i], "row length");
        CHECK(memcmp(row, nb + off[i], sizeof(int32_t) * (size_t)k) == 0, "row entries");
        int64_t k2 = 0;
        for (int64_t j = 0; j < n; ++j) k2 += oracle_pair(x[i], y[i], z[i], h[i], x[j], y[j], z[j]);
        CHECK(k2 == k, "pairs");
        int64_t rows[3] = {0, n - 1, i}, cnt[3];
        oracle_counts(x, y, z, h, n, rows, 3, cnt);
        for (int r = 0; r < 3; ++r)
            CHECK(cnt[r] == off[rows[r] + 1] - off[rows[r]], "subset count %d", r);
        free(row);
    }

    /* Cell list: identical lists. */
    int64_t *cc = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *co = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *cn = malloc(sizeof(int32_t) * (size_t)cap);
    int64_t ctot = oracle_cell_lists(x, y, z, h, n, cc, co, cn, cap);
    CHECK(ctot == tot, "cell total %lld vs %lld", (long long)ctot, (long long)tot);
    CHECK(memcmp(co, off, sizeof(int64_t) * (size_t)(n + 1)) == 0, "cell offsets");
    CHECK(memcmp(cn, nb, sizeof(int32_t) * (size_t)(tot > 0 ? tot : 0)) == 0, "cell lists");

    /* Row checker: clean, then with one planted error. */
    int32_t *c32 = malloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) c32[i] = (int32_t)(off[i + 1] - off[i]);
    int64_t bad[4];
    CHECK(oracle_cell_check(x, y, z, h, n, c32, off, nb, bad, 4) == 0, "check clean");
    if (tot > 0) {
        nb[tot / 2] ^= 1;
        CHECK(oracle_cell_check(x, y, z, h, n, c32, off, nb, bad, 4) >= 1, "check planted");
        nb[tot / 2] ^= 1;
    }

    /* Density against a direct sum over the brute-force rows. */
    for (int ex = 0; ex < 2; ++ex) {
        double *rho = malloc(sizeof(double) * (size_t)(n + 1));
        int64_t *dc = malloc(sizeof(int64_t) * (size_t)(n + 1));
        CHECK(oracle_density(x, y, z, h, m, n, ex, rho, dc) == 0, "density status");
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            int64_t k = 0;
            for (int64_t e = off[i]; e < off[i + 1]; ++e) {
                int64_t j = nb[e];
                if (ex && j == i) continue;
                double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
                s += m[j] * oracle_sph_shape((dx * dx + dy * dy) + dz * dz, h[i]);
                ++k;
            }
            double want = k ? s / (M_PI * h[i] * h[i] * h[i]) : 0.0;
            CHECK(dc[i] == k, "density count");
            CHECK(fabs(rho[i] - want) <= 1e-12 * fabs(want) + 1e-300, "density value");
        }
        free(rho);
        free(dc);
    }

    /* Algorithm 1 (and the octree): members a permutation, leaves cover n. */
    for (int oct = 0; oct < 2; ++oct) {
        int64_t lc = n + 64;
        int64_t *leaf_cnt = malloc(sizeof(int64_t) * (size_t)lc);
        int32_t *leaf_depth = malloc(sizeof(int32_t) * (size_t)lc);
        int32_t *members = malloc(sizeof(int32_t) * (size_t)(n + 1));
        int64_t b_hist[65];
        int32_t *node_b = malloc(sizeof(int32_t) * (size_t)lc);
        int64_t *node_n = malloc(sizeof(int64_t) * (size_t)lc);
        int32_t *node_depth = malloc(sizeof(int32_t) * (size_t)lc);
        int64_t st[8];
        oracle_build_tree(x, y, z, n, 8, 0.5, 0.5, 32, oct, leaf_cnt, leaf_depth, lc, members,
                          b_hist, 65, node_b, node_n, node_depth, lc, st);
        CHECK(st[6] == 0, "tree error %lld", (long long)st[6]);
        CHECK(st[5] == n, "members length");
        int64_t sum = 0;
        for (int64_t l = 0; l < st[1]; ++l) sum += leaf_cnt[l];
        CHECK(sum == n, "leaves cover n");
        char *seen = calloc((size_t)(n + 1), 1);
        for (int64_t i = 0; i < n; ++i) {
            int32_t v = members[i];
            CHECK(v >= 0 && v < n && !seen[v], "members permutation");
            if (v >= 0 && v < n) seen[v] = 1;
        }
        free(seen);
        free(leaf_cnt); free(leaf_depth); free(members); free(node_b); free(node_n);
        free(node_depth);
    }

    free(x); free(y); free(z); free(h); free(m); free(off); free(nb);
    free(cc); free(co); free(cn); free(c32);
}

int main(void)
{
    const int64_t sizes[] = {0, 1, 2, 17, 300, 1500};
    for (int k = 0; k < 3; ++k)
        for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; ++s) one_set(sizes[s], k);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}

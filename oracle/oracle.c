/*
 * CPU oracle for the b-tree neighbour search (Cavelan, Cabezon, Korndorfer,
 * Ciorba, "Finding Neighbors in a Forest: A b-tree for Smoothed Particle
 * Hydrodynamics Simulations", arXiv 1910.02639).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no source, header, table or helper with the GPU library.
 *
 * Two things are defined here:
 *
 *  1. The neighbour lists (Section 3.2, Algorithm 2, Eq. 5).  The tree only
 *     changes WHICH pairs get tested, never the test itself, so the result of
 *     FindNeighbors has a plain definition, written out as a brute force:
 *
 *        N(i) = { j in [0,n) : P64(i,j) }   listed in ascending j
 *        P64(i,j): dx = x_i - x_j ; dy = y_i - y_j ; dz = z_i - z_j
 *                  d2 = (dx*dx + dy*dy) + dz*dz     every op rounded, no FMA
 *                  r2 = (2*h_i) * (2*h_i)
 *                  P64 = d2 < r2                     (strict: "less than 2h")
 *
 *     The radius is the query particle's own 2h_p (Section 3.2).  The particle
 *     itself is in its own list when h_i > 0, as in Algorithm 2, which tests
 *     every particle of every cell in range.
 *
 *     The same lists are also computed by a multi-resolution cell list
 *     (exact, pinned to the brute force), fast enough to check every row of
 *     sets of millions of particles.
 *
 *  2. BuildTree (Section 3.1, Algorithm 1, Eqs. 1-4), as a plain recursion in
 *     the paper's order: branching factor (Eq. 1), distribute (Eqs. 2-3),
 *     ratio (Eq. 4), halve b while the ratio is too high, recurse on every
 *     sub-cell holding more than s particles.  It reports the tree shape and
 *     the particles of every leaf in a canonical depth-first order.  With
 *     the octree option every split uses b = 2 (the octree the paper
 *     compares against; Section 3.1 Step 3 reaches it when b halves to 2).
 *
 *  3. Two uses of the lists inside an SPH step, each a plain definition
 *     over the rows of part 1:
 *      - the density sum (SPH use of the search, Section 4.7; the paper fixes
 *        no kernel, this is the cubic spline of support 2h):
 *          rho_i = (sum_{j in N(i), ascending} m_j w(r_ij / h_i)) / (pi h_i^3),
 *          w(q) = (1 - 1.5 q^2) + 0.75 q^3 for q < 1, 0.25 (2 - q)^3 for
 *          1 <= q < 2, r_ij = sqrt(d2) with d2 as in P64, 0 for empty rows;
 *      - smoothing lengths adapted to a target neighbour count (the target
 *        of Table 3), in oracle/__init__.py on the counts of part 1.
 *
 * Readings where the paper is silent or inconsistent (each also listed in
 * the design notes):
 *   - distance test is strict (<), as the text says; Algorithm 2 prints <=;
 *   - Eq. 1 is evaluated exactly: b = smallest integer with b^3 * s >= n;
 *   - Eq. 4 counts sub-cells with n_j < alpha*s (text), compared in FP64;
 *   - halving happens when r > beta and b > 2, with b <- max(2, floor(b/2));
 *     Algorithm 1's "R < beta" test is read as the text's "r > beta";
 *   - Eq. 2 is evaluated as ((x - lo) / (hi - lo)) * b in FP64 and clamped to
 *     [0, b-1]; a zero extent maps every particle to sub-cell 0;
 *   - a sub-cell's box is lo + (w*c)/b .. lo + (w*(c+1))/b, w = hi - lo;
 *   - the root box is the tight per-axis bounding box of the particles;
 *   - a root holding n <= s particles is a single leaf;
 *   - a node at depth max_depth is a leaf whatever its size (depth guard);
 *   - sub-cells are visited in Morton order of their (x',y',z') coordinates
 *     (bit k of x' -> bit 3k, of y' -> 3k+1, of z' -> 3k+2).
 *
 * Build with: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* Part 1: the neighbour predicate and brute-force lists                     */
/* ------------------------------------------------------------------------ */

/* P64 (Section 3.2: "if the distance is less than 2h_p we add q"). */
static int p64(double xi, double yi, double zi, double hi,
               double xj, double yj, double zj)
{
    double dx = xi - xj;
    double dy = yi - yj;
    double dz = zi - zj;
    double dxx = dx * dx;
    double dyy = dy * dy;
    double dzz = dz * dz;
    double s1 = dxx + dyy;
    double d2 = s1 + dzz;
    double twoh = 2.0 * hi;
    double r2 = twoh * twoh;
    return d2 < r2;
}

int oracle_pair(double xi, double yi, double zi, double hi,
                double xj, double yj, double zj)
{
    return p64(xi, yi, zi, hi, xj, yj, zj);
}

/* Row i of the neighbour list, by testing every j in ascending order.
 * Writes at most cap entries to out (out may be NULL when cap == 0) and
 * returns the full row length. */
int64_t oracle_row(const double *x, const double *y, const double *z,
                   const double *h, int64_t n, int64_t i,
                   int32_t *out, int64_t cap)
{
    int64_t k = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (p64(x[i], y[i], z[i], h[i], x[j], y[j], z[j])) {
            if (k < cap) out[k] = (int32_t)j;
            ++k;
        }
    }
    return k;
}

/* Counts of the rows listed in rows[0..m) (all rows when rows == NULL,
 * then m must equal n).  Rows are independent, so they run in parallel. */
void oracle_counts(const double *x, const double *y, const double *z,
                   const double *h, int64_t n, const int64_t *rows, int64_t m,
                   int64_t *counts)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = rows ? rows[r] : r;
        counts[r] = oracle_row(x, y, z, h, n, i, NULL, 0);
    }
}

/* Lists of the rows in rows[0..m): offsets[m+1] is the exclusive prefix sum
 * of the counts; nbrs receives the rows back to back (capacity cap).
 * Returns the total, or -1 if cap is too small (nothing is written then). */
int64_t oracle_lists(const double *x, const double *y, const double *z,
                     const double *h, int64_t n, const int64_t *rows,
                     int64_t m, int64_t *offsets, int32_t *nbrs, int64_t cap)
{
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    oracle_counts(x, y, z, h, n, rows, m, cnt);
    offsets[0] = 0;
    for (int64_t r = 0; r < m; ++r) offsets[r + 1] = offsets[r] + cnt[r];
    int64_t total = offsets[m];
    free(cnt);
    if (total > cap) return -1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = rows ? rows[r] : r;
        oracle_row(x, y, z, h, n, i, nbrs + offsets[r],
                   offsets[r + 1] - offsets[r]);
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* Part 1b: the same lists by a multi-resolution cell list                   */
/* ------------------------------------------------------------------------ */
/*
 * An exact evaluation of the definition above that is fast enough for sets
 * of millions of particles (the brute force is O(n^2)).  The tree of the
 * paper only decides which pairs get tested; so does this cell list.  Every
 * pair it tests goes through the same P64, and every row is sorted.
 *
 * Cells.  Level l bins every particle into cubic cells of side c_l = c_0 2^l
 * with the index g_l(v) = floor((v - o) / c_l) per axis (FP64, o = the
 * smallest coordinate of the set on that axis, clamped to [0, G_l - 1]).
 * A level is the array of (cell key, index) pairs of all particles, sorted
 * by key; the key puts x above y above z, so one (x, y) column of cells is
 * one run of keys.  c_0 is the smallest positive h (raised if needed so
 * that no axis has more than 2^20 cells).
 *
 * Query i (R_i = 2 h_i > 0) uses the finest level with c_l >= h_i and scans
 * the cells g_l(fl(x_i - R_i)) .. g_l(fl(x_i + R_i)) on every axis, about
 * five per axis since 2 R_i / c_l <= 4.
 *
 * Why no neighbour is missed.  Take an axis and suppose x_j > fl(x_i + R).
 * Either fl(x_i + R) >= x_i + R, or x_i + R lies at or below the midpoint
 * between fl(x_i + R) and the next double, which x_j is at least; either
 * way x_j - x_i > R in real arithmetic.  Rounding is monotone and R = 2h is a
 * double, so |fl(x_i - x_j)| >= R, its rounded square is >= fl(R * R), and
 * adding the other two non-negative squares cannot make d2 smaller: d2 >=
 * r2 and P64 fails.  Likewise below.  So every neighbour satisfies
 * fl(x_i - R) <= x_j <= fl(x_i + R) on every axis, and since g_l is
 * non-decreasing (subtracting a constant, dividing by a positive constant
 * and floor all keep order; so does the clamp), its cell lies in the
 * scanned range.  A query with R_i = 0 has an empty row (d2 < 0 is false).
 */

static int cmp_i32(const void *a, const void *b);

typedef struct { uint64_t key; int32_t idx; int32_t pad; } cl_ent;

typedef struct {
    double c;          /* cell side                                         */
    int64_t g[3];      /* cells per axis                                    */
    cl_ent *ent;       /* n entries sorted by key, or NULL when unused      */
} cl_level;

typedef struct {
    const double *x, *y, *z, *h;
    int64_t n;
    double o[3];
    int nlev;
    cl_level lev[80];
    int8_t *qlev;      /* level of each query (-1: empty row)               */
} cl_grid;

static int cmp_cl(const void *a, const void *b)
{
    uint64_t u = ((const cl_ent *)a)->key, v = ((const cl_ent *)b)->key;
    if (u != v) return (u > v) - (u < v);
    int32_t p = ((const cl_ent *)a)->idx, q = ((const cl_ent *)b)->idx;
    return (p > q) - (p < q);
}

/* Cell index of coordinate v on one axis of a level. */
static int64_t cl_cell(double v, double o, double c, int64_t g)
{
    double t = floor((v - o) / c);
    if (!(t >= 0.0)) return 0;
    if (t > (double)(g - 1)) return g - 1;
    return (int64_t)t;
}

static uint64_t cl_key(int64_t a, int64_t b, int64_t c)
{
    return ((uint64_t)a << 42) | ((uint64_t)b << 21) | (uint64_t)c;
}

static void cl_free(cl_grid *G)
{
    for (int l = 0; l < G->nlev; ++l) free(G->lev[l].ent);
    free(G->qlev);
}

/* Builds the levels that some query uses.  Returns 0, or -1 when out of
 * memory. */
static int cl_build(cl_grid *G, const double *x, const double *y,
                    const double *z, const double *h, int64_t n)
{
    memset(G, 0, sizeof *G);
    G->x = x; G->y = y; G->z = z; G->h = h; G->n = n;
    G->qlev = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
    if (!G->qlev) return -1;
    if (n == 0) return 0;
    double lo[3] = { x[0], y[0], z[0] }, hi[3] = { x[0], y[0], z[0] };
    const double *xyz[3] = { x, y, z };
    for (int a = 0; a < 3; ++a)
        for (int64_t i = 1; i < n; ++i) {
            if (xyz[a][i] < lo[a]) lo[a] = xyz[a][i];
            if (xyz[a][i] > hi[a]) hi[a] = xyz[a][i];
        }
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) {
        G->o[a] = lo[a];
        if (hi[a] - lo[a] > ext) ext = hi[a] - lo[a];
    }
    double hmin = INFINITY, hmax = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (h[i] > 0.0) {
            if (h[i] < hmin) hmin = h[i];
            if (h[i] > hmax) hmax = h[i];
        }
    if (!(hmax > 0.0)) {                      /* every row is empty */
        for (int64_t i = 0; i < n; ++i) G->qlev[i] = -1;
        return 0;
    }
    double c0 = hmin;
    if (c0 < ext * 0x1p-20) c0 = ext * 0x1p-20;
    /* Levels up to the first whose side covers both the largest h and the
     * whole set (a single cell per axis). */
    int nlev = 1;
    for (double c = c0; (c < hmax || c < ext) && nlev < 80; c *= 2.0) ++nlev;
    G->nlev = nlev;
    for (int l = 0; l < nlev; ++l) {
        double c = ldexp(c0, l);
        G->lev[l].c = c;
        for (int a = 0; a < 3; ++a) {
            double gm = floor((hi[a] - lo[a]) / c) + 1.0;
            G->lev[l].g[a] = gm > 2097151.0 ? 2097151 : (int64_t)gm;
        }
    }
    int used[80] = { 0 };
    for (int64_t i = 0; i < n; ++i) {
        if (!(h[i] > 0.0)) { G->qlev[i] = -1; continue; }
        int l = 0;
        while (l < nlev - 1 && G->lev[l].c < h[i]) ++l;
        G->qlev[i] = (int8_t)l;
        used[l] = 1;
    }
    int err = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int l = 0; l < nlev; ++l) {
        if (!used[l]) continue;
        cl_level *L = &G->lev[l];
        cl_ent *e = (cl_ent *)malloc(sizeof(cl_ent) * (size_t)n);
        if (!e) {
            #pragma omp atomic write
            err = 1;
            continue;
        }
        for (int64_t i = 0; i < n; ++i) {
            e[i].key = cl_key(cl_cell(x[i], G->o[0], L->c, L->g[0]),
                              cl_cell(y[i], G->o[1], L->c, L->g[1]),
                              cl_cell(z[i], G->o[2], L->c, L->g[2]));
            e[i].idx = (int32_t)i;
            e[i].pad = 0;
        }
        qsort(e, (size_t)n, sizeof(cl_ent), cmp_cl);
        L->ent = e;
    }
    return err ? -1 : 0;
}

/* First entry of a level whose key is >= k. */
static int64_t cl_lower(const cl_ent *e, int64_t n, uint64_t k)
{
    int64_t a = 0, b = n;
    while (a < b) {
        int64_t m = a + (b - a) / 2;
        if (e[m].key < k) a = m + 1;
        else b = m;
    }
    return a;
}

/* Row i into *buf (grown as needed, capacity *cap); returns its length, or
 * -1 when out of memory.  The row is sorted ascending. */
static int64_t cl_row(const cl_grid *G, int64_t i, int32_t **buf, int64_t *cap)
{
    int l = G->qlev[i];
    if (l < 0) return 0;
    const cl_level *L = &G->lev[l];
    double xi = G->x[i], yi = G->y[i], zi = G->z[i], hi = G->h[i];
    double R = 2.0 * hi;
    double q[3] = { xi, yi, zi };
    int64_t a[3], b[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = cl_cell(q[k] - R, G->o[k], L->c, L->g[k]);
        b[k] = cl_cell(q[k] + R, G->o[k], L->c, L->g[k]);
    }
    int64_t m = 0;
    for (int64_t gx = a[0]; gx <= b[0]; ++gx)
        for (int64_t gy = a[1]; gy <= b[1]; ++gy) {
            uint64_t k0 = cl_key(gx, gy, a[2]), k1 = cl_key(gx, gy, b[2]);
            for (int64_t p = cl_lower(L->ent, G->n, k0);
                 p < G->n && L->ent[p].key <= k1; ++p) {
                int32_t j = L->ent[p].idx;
                if (!p64(xi, yi, zi, hi, G->x[j], G->y[j], G->z[j])) continue;
                if (m == *cap) {
                    int64_t nc = *cap ? 2 * *cap : 256;
                    int32_t *nb = (int32_t *)realloc(*buf, sizeof(int32_t) * (size_t)nc);
                    if (!nb) return -1;
                    *buf = nb;
                    *cap = nc;
                }
                (*buf)[m++] = j;
            }
        }
    qsort(*buf, (size_t)m, sizeof(int32_t), cmp_i32);
    return m;
}

/* The lists of all n rows by the cell list: counts[n], offsets[n+1] and,
 * when nbrs is not NULL, the rows back to back (capacity cap).  Returns the
 * total, -1 if cap is too small (nbrs untouched then), -2 if out of memory. */
int64_t oracle_cell_lists(const double *x, const double *y, const double *z,
                          const double *h, int64_t n, int64_t *counts,
                          int64_t *offsets, int32_t *nbrs, int64_t cap)
{
    cl_grid G;
    if (cl_build(&G, x, y, z, h, n)) { cl_free(&G); return -2; }
    int err = 0;
    for (int pass = 0; pass < 2 && !err; ++pass) {
        if (pass == 1) {
            offsets[0] = 0;
            for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + counts[i];
            if (!nbrs) break;
            if (offsets[n] > cap) { cl_free(&G); return -1; }
        }
        if (pass == 0)
            for (int64_t i = 0; i < n; ++i) counts[i] = 0;  /* empty rows */
        /* Queries level by level in cell order (neighbouring queries scan the
         * same cells). */
        for (int l = 0; l < G.nlev; ++l) {
            const cl_ent *e = G.lev[l].ent;
            if (!e) continue;
            #pragma omp parallel
            {
                int32_t *buf = NULL;
                int64_t bcap = 0;
                #pragma omp for schedule(dynamic, 1024)
                for (int64_t p = 0; p < n; ++p) {
                    int64_t i = e[p].idx;
                    if (G.qlev[i] != l) continue;
                    int64_t m = cl_row(&G, i, &buf, &bcap);
                    if (m < 0) {
                        #pragma omp atomic write
                        err = 1;
                        continue;
                    }
                    if (pass == 0) counts[i] = m;
                    else memcpy(nbrs + offsets[i], buf, sizeof(int32_t) * (size_t)m);
                }
                free(buf);
            }
        }
    }
    cl_free(&G);
    return err ? -2 : offsets[n];
}

/* Checks lists produced elsewhere (counts int32[n], offsets int64[n+1],
 * nbrs int32[offsets[n]]) row by row against the cell list.  Row i is wrong
 * when counts[i], offsets[i+1] - offsets[i] and the oracle's row length do
 * not all agree, or an entry differs.  Up to max_bad wrong rows are written
 * to bad (in no particular order).  Returns the number of wrong rows, or -2
 * when out of memory.  Queries are taken level by level in cell order, so
 * consecutive queries scan the same cells. */
int64_t oracle_cell_check(const double *x, const double *y, const double *z,
                          const double *h, int64_t n, const int32_t *counts,
                          const int64_t *offsets, const int32_t *nbrs,
                          int64_t *bad, int64_t max_bad)
{
    cl_grid G;
    if (cl_build(&G, x, y, z, h, n)) { cl_free(&G); return -2; }
    int64_t nbad = 0;
    int err = 0;
    if (n > 0 && offsets[0] != 0) {
        if (max_bad > 0) bad[0] = 0;
        nbad = 1;
    }
    /* Queries with an empty row: the lists must agree that they are. */
    for (int64_t i = 0; i < n; ++i)
        if (G.qlev[i] < 0 && (counts[i] != 0 || offsets[i + 1] != offsets[i])) {
            if (nbad < max_bad) bad[nbad] = i;
            ++nbad;
        }
    for (int l = 0; l < G.nlev; ++l) {
        const cl_ent *e = G.lev[l].ent;
        if (!e) continue;
        #pragma omp parallel
        {
            int32_t *buf = NULL;
            int64_t bcap = 0;
            #pragma omp for schedule(dynamic, 1024)
            for (int64_t p = 0; p < n; ++p) {
                int64_t i = e[p].idx;
                if (G.qlev[i] != l) continue;
                int64_t m = cl_row(&G, i, &buf, &bcap);
                if (m < 0) {
                    #pragma omp atomic write
                    err = 1;
                    continue;
                }
                int ok = counts[i] == m && offsets[i + 1] - offsets[i] == m &&
                         memcmp(nbrs + offsets[i], buf, sizeof(int32_t) * (size_t)m) == 0;
                if (!ok) {
                    int64_t k;
                    #pragma omp atomic capture
                    k = nbad++;
                    if (k < max_bad) bad[k] = i;
                }
            }
            free(buf);
        }
    }
    cl_free(&G);
    return err ? -2 : nbad;
}

/* ------------------------------------------------------------------------ */
/* Part 1c: the SPH density over the rows                                    */
/* ------------------------------------------------------------------------ */

/* Cubic spline shape w(q), q = r / h, from the squared distance d2:
 * r = sqrt(d2), q = r / h; w = (1 - 1.5 q^2) + 0.75 q^3 (q < 1),
 * 0.25 ((2 - q)^2 (2 - q)) (1 <= q < 2), 0 beyond.  W(r, h) = w / (pi h^3)
 * integrates to 1 over space. */
double oracle_sph_shape(double d2, double h)
{
    double r = sqrt(d2);
    double q = r / h;
    if (q < 1.0) {
        double q2 = q * q;
        double q3 = q2 * q;
        return (1.0 - 1.5 * q2) + 0.75 * q3;
    }
    if (q < 2.0) {
        double t = 2.0 - q;
        return 0.25 * ((t * t) * t);
    }
    return 0.0;
}

/* rho[i] = (sum over row i of N, ascending j, of m_j w(r_ij / h_i))
 * / (pi h_i^3), 0 for an empty row; mass NULL = unit masses; exclude_self
 * drops j = i from every row.  counts[i] (if not NULL) = the row length.
 * Rows from the cell list (part 1b).  Returns 0, or -2 when out of memory. */
int64_t oracle_density(const double *x, const double *y, const double *z,
                       const double *h, const double *mass, int64_t n,
                       int32_t exclude_self, double *rho, int64_t *counts)
{
    cl_grid G;
    if (cl_build(&G, x, y, z, h, n)) { cl_free(&G); return -2; }
    int err = 0;
    #pragma omp parallel
    {
        int32_t *buf = NULL;
        int64_t bcap = 0;
        #pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            int64_t m = cl_row(&G, i, &buf, &bcap);
            if (m < 0) {
                #pragma omp atomic write
                err = 1;
                continue;
            }
            double sum = 0.0;
            int64_t c = 0;
            for (int64_t k = 0; k < m; ++k) {
                int32_t j = buf[k];
                if (exclude_self && j == i) continue;
                double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
                double d2 = (dx * dx + dy * dy) + dz * dz;
                double w = oracle_sph_shape(d2, h[i]);
                sum += mass ? mass[j] * w : w;
                ++c;
            }
            rho[i] = c == 0 ? 0.0 : sum / (3.141592653589793 * ((h[i] * h[i]) * h[i]));
            if (counts) counts[i] = c;
        }
        free(buf);
    }
    cl_free(&G);
    return err ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Part 2: BuildTree (Algorithm 1) and the equations it uses                 */
/* ------------------------------------------------------------------------ */

/* Eq. 1: b = ceil((n/s)^(1/k)) for k = 3, evaluated exactly as the smallest
 * integer b >= 1 with b^3 * s >= n. */
int64_t oracle_eq1_branching(int64_t n, int64_t s)
{
    int64_t b = 1;
    while (b * b * b * s < n) ++b;
    return b;
}

/* Eq. 2: sub-cell coordinate of x in [lo, hi] split into b parts. */
int64_t oracle_eq2_subcell(double x, double lo, double hi, int64_t b)
{
    double w = hi - lo;
    if (!(w > 0.0)) return 0;
    double t = (x - lo) / w;
    double v = floor(t * (double)b);
    if (v < 0.0) return 0;
    if (v > (double)(b - 1)) return b - 1;
    return (int64_t)v;
}

/* Eq. 3: sub-cell id j = x'_1 + x'_2 W + x'_3 W^2 with W = b. */
int64_t oracle_eq3_cell_id(int64_t c1, int64_t c2, int64_t c3, int64_t b)
{
    return c1 + c2 * b + c3 * b * b;
}

/* Eq. 5: inclusive range of sub-cell coordinates a particle at x with
 * radius R = 2h must visit, on the same clamp as Eq. 2. */
void oracle_eq5_range(double x, double R, double lo, double hi, int64_t b,
                      int64_t *rmin, int64_t *rmax)
{
    *rmin = oracle_eq2_subcell(x - R, lo, hi, b);
    *rmax = oracle_eq2_subcell(x + R, lo, hi, b);
}

/* Morton code of sub-cell coordinates (visiting order of sub-cells). */
static uint64_t morton3(int64_t a, int64_t b, int64_t c)
{
    uint64_t m = 0;
    for (int k = 0; k < 21; ++k) {
        m |= (uint64_t)((a >> k) & 1) << (3 * k);
        m |= (uint64_t)((b >> k) & 1) << (3 * k + 1);
        m |= (uint64_t)((c >> k) & 1) << (3 * k + 2);
    }
    return m;
}

typedef struct {
    const double *x, *y, *z;
    int64_t s;
    double alpha, beta;
    int32_t max_depth;
    int32_t octree;           /* 1: b = 2 for every cell, no Eq. 1 / Eq. 4 */
    /* outputs */
    int64_t n_internal, n_leaves, depth, rounds, max_leaf;
    int64_t *b_hist;          /* b_hist[b] = internal nodes that chose b   */
    int64_t b_hist_len;
    int64_t *leaf_cnt;        /* leaves in canonical order                */
    int32_t *leaf_depth;
    int32_t *members;         /* original indices, leaf by leaf, ascending */
    int64_t members_len;
    int64_t leaf_cap;
    int32_t *node_b;          /* internal nodes in pre-order: b, n, depth */
    int64_t *node_n;
    int32_t *node_depth;
    int64_t node_cap;
    int error;
} tree_ctx;

static int cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

typedef struct { uint64_t key; int64_t cell; } order_ent;

static int cmp_order(const void *a, const void *b)
{
    uint64_t u = ((const order_ent *)a)->key, v = ((const order_ent *)b)->key;
    return (u > v) - (u < v);
}

static void emit_leaf(tree_ctx *t, const int32_t *idx, int64_t n, int32_t depth)
{
    if (t->n_leaves >= t->leaf_cap) { t->error = 1; return; }
    t->leaf_cnt[t->n_leaves] = n;
    t->leaf_depth[t->n_leaves] = depth;
    t->n_leaves++;
    memcpy(t->members + t->members_len, idx, sizeof(int32_t) * (size_t)n);
    qsort(t->members + t->members_len, (size_t)n, sizeof(int32_t), cmp_i32);
    t->members_len += n;
    if (depth > t->depth) t->depth = depth;
    if (n > t->max_leaf) t->max_leaf = n;
}

/* BuildTree(n, i) of Algorithm 1 on the cell with box [lo, hi] that holds
 * the particles idx[0..n). */
static void build_tree(tree_ctx *t, int32_t *idx, int64_t n,
                       const double lo[3], const double hi[3], int32_t depth)
{
    if (t->error) return;
    if (depth >= t->max_depth) { emit_leaf(t, idx, n, depth); return; }

    /* Step 1: branching factor (Eq. 1).  The octree halves every cell along
     * each axis (Section 2): b = 2 and no ratio test. */
    int64_t b = t->octree ? 2 : oracle_eq1_branching(n, t->s);
    int64_t *cnt = NULL;
    int64_t *cell_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (;;) {
        /* Step 2: distribute the particles over b^3 sub-cells (Eqs. 2-3). */
        int64_t nc = b * b * b;
        free(cnt);
        cnt = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
        for (int64_t p = 0; p < n; ++p) {
            int32_t q = idx[p];
            int64_t c1 = oracle_eq2_subcell(t->x[q], lo[0], hi[0], b);
            int64_t c2 = oracle_eq2_subcell(t->y[q], lo[1], hi[1], b);
            int64_t c3 = oracle_eq2_subcell(t->z[q], lo[2], hi[2], b);
            int64_t j = oracle_eq3_cell_id(c1, c2, c3, b);
            cell_of[p] = j;
            cnt[j]++;
        }
        /* Step 3: distribution ratio (Eq. 4) and halving. */
        int64_t under = 0;
        double thr = t->alpha * (double)t->s;
        for (int64_t j = 0; j < nc; ++j)
            if ((double)cnt[j] < thr) under++;
        double r = (double)under / (double)nc;
        if (!t->octree && r > t->beta && b > 2) {
            b = b / 2;
            if (b < 2) b = 2;
            t->rounds++;
            continue;
        }
        break;
    }

    /* Record this internal node (pre-order). */
    if (t->n_internal < t->node_cap) {
        t->node_b[t->n_internal] = (int32_t)b;
        t->node_n[t->n_internal] = n;
        t->node_depth[t->n_internal] = depth;
    } else {
        t->error = 1;
    }
    t->n_internal++;
    if (b < t->b_hist_len) t->b_hist[b]++;

    /* Sub-cells in Morton order of their coordinates. */
    int64_t nc = b * b * b;
    order_ent *ord = (order_ent *)malloc(sizeof(order_ent) * (size_t)nc);
    for (int64_t j = 0; j < nc; ++j) {
        int64_t c1 = j % b, c2 = (j / b) % b, c3 = j / (b * b);
        ord[j].key = morton3(c1, c2, c3);
        ord[j].cell = j;
    }
    qsort(ord, (size_t)nc, sizeof(order_ent), cmp_order);

    /* Group particle indices by sub-cell (counting sort). */
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
    start[0] = 0;
    for (int64_t j = 0; j < nc; ++j) start[j + 1] = start[j] + cnt[j];
    int32_t *grouped = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    memcpy(fill, start, sizeof(int64_t) * (size_t)nc);
    for (int64_t p = 0; p < n; ++p) grouped[fill[cell_of[p]]++] = idx[p];
    free(fill);
    free(cell_of);

    for (int64_t k = 0; k < nc && !t->error; ++k) {
        int64_t j = ord[k].cell;
        int64_t nj = cnt[j];
        if (nj == 0) continue;                      /* empty cells not stored */
        int32_t *sub = grouped + start[j];
        if (nj <= t->s) { emit_leaf(t, sub, nj, depth + 1); continue; }
        int64_t c[3] = { j % b, (j / b) % b, j / (b * b) };
        double clo[3], chi[3];
        for (int l = 0; l < 3; ++l) {
            double w = hi[l] - lo[l];
            clo[l] = lo[l] + (w * (double)c[l]) / (double)b;
            chi[l] = lo[l] + (w * (double)(c[l] + 1)) / (double)b;
        }
        build_tree(t, sub, nj, clo, chi, depth + 1);
    }
    free(grouped);
    free(start);
    free(ord);
    free(cnt);
}

/* Runs Algorithm 1 on all n particles (octree != 0: the classical octree,
 * every cell with more than s particles split into 2 x 2 x 2 sub-cells).
 * stats[0..7) = { n_internal, n_leaves, depth, rounds, max_leaf,
 *                 members_len, error, 0 }.
 * Caller provides leaf_cnt/leaf_depth with room for leaf_cap leaves,
 * members with room for n entries, b_hist with b_hist_len slots (zeroed
 * here), node_b/node_n/node_depth with room for node_cap internal nodes. */
void oracle_build_tree(const double *x, const double *y, const double *z,
                       int64_t n, int64_t s, double alpha, double beta,
                       int32_t max_depth, int32_t octree,
                       int64_t *leaf_cnt, int32_t *leaf_depth, int64_t leaf_cap,
                       int32_t *members, int64_t *b_hist, int64_t b_hist_len,
                       int32_t *node_b, int64_t *node_n, int32_t *node_depth,
                       int64_t node_cap, int64_t *stats)
{
    tree_ctx t;
    memset(&t, 0, sizeof t);
    t.x = x; t.y = y; t.z = z;
    t.s = s; t.alpha = alpha; t.beta = beta; t.max_depth = max_depth;
    t.octree = octree;
    t.b_hist = b_hist; t.b_hist_len = b_hist_len;
    t.leaf_cnt = leaf_cnt; t.leaf_depth = leaf_depth; t.leaf_cap = leaf_cap;
    t.members = members;
    t.node_b = node_b; t.node_n = node_n; t.node_depth = node_depth;
    t.node_cap = node_cap;
    for (int64_t k = 0; k < b_hist_len; ++k) b_hist[k] = 0;

    if (n > 0) {
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)i;
        if (n <= s) {
            emit_leaf(&t, idx, n, 0);
        } else {
            double lo[3] = { x[0], y[0], z[0] }, hi[3] = { x[0], y[0], z[0] };
            for (int64_t i = 1; i < n; ++i) {
                if (x[i] < lo[0]) lo[0] = x[i];
                if (x[i] > hi[0]) hi[0] = x[i];
                if (y[i] < lo[1]) lo[1] = y[i];
                if (y[i] > hi[1]) hi[1] = y[i];
                if (z[i] < lo[2]) lo[2] = z[i];
                if (z[i] > hi[2]) hi[2] = z[i];
            }
            build_tree(&t, idx, n, lo, hi, 0);
        }
        free(idx);
    }
    stats[0] = t.n_internal;
    stats[1] = t.n_leaves;
    stats[2] = t.depth;
    stats[3] = t.rounds;
    stats[4] = t.max_leaf;
    stats[5] = t.members_len;
    stats[6] = t.error;
    stats[7] = 0;
}

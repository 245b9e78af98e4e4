/*
 * btree.h -- C ABI of the MI355X (gfx950) b-tree neighbour search.
 *
 * Method: Cavelan, Cabezon, Korndorfer, Ciorba, "Finding Neighbors in a
 * Forest: A b-tree for Smoothed Particle Hydrodynamics Simulations"
 * (arXiv 1910.02639).  BuildTree is Algorithm 1 with Eqs. 1-4 (Section 3.1);
 * FindNeighbors is Algorithm 2 with Eq. 5 (Section 3.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Particle data (x, y, z, h), counts, offsets and nbrs are DEVICE
 *    pointers owned by the caller.  They must stay valid until the work
 *    queued on `hip_stream` has run.  The library never frees them and keeps
 *    no pointer to them after a call returns.
 *  - `hip_stream` is a hipStream_t passed as void* (NULL = null stream).
 *    All device work of a call is queued on that stream.
 *  - Coordinates and smoothing lengths are FP64, structure-of-arrays, one
 *    entry per particle, indexed 0..n-1 ("original index").
 *  - Every call returns a btree_status.  On failure the thread-local message
 *    of btree_last_error() says why.  No C++ exception crosses the ABI.
 *  - Host-side argument checks (NULL pointers, negative sizes, bad
 *    parameters) run before anything is queued.  Data checks (non-finite
 *    coordinates, h < 0 or non-finite) run on the device; when they fail the
 *    call returns BTREE_EINVAL and no caller-owned output has been written.
 *  - Distinct handles may be used from distinct host threads at once.  One
 *    handle must not be used by two threads at once.
 */
#ifndef BTREE_H
#define BTREE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BTREE_OK = 0,
    BTREE_EINVAL = -1,     /* bad argument or bad particle data            */
    BTREE_ENOMEM = -2,     /* a device allocation failed (for tests, the
                              environment variable BTREE_FAULT_ALLOC = k
                              fails the k-th allocation counted from the
                              last change of its value)                 */
    BTREE_EDEVICE = -3,    /* a HIP runtime call or kernel launch failed    */
    BTREE_EOVERFLOW = -4,  /* caller's output capacity below the total      */
    BTREE_ESTATE = -5      /* call made in a state that does not allow it   */
} btree_status;

typedef enum {
    BTREE_FP64 = 0,        /* every pair tested with the FP64 predicate     */
    BTREE_FP32_FILTER = 1  /* FP32 test with a rounding margin; pairs inside
                              the margin re-tested with the FP64 predicate  */
} btree_precision;

/* Tree and search parameters (Table 1 of the paper for s, alpha, beta). */
typedef struct {
    int32_t bucket_size;    /* s: a cell with more than s particles is split;
                               default 64, must be >= 1                       */
    double  alpha;          /* alpha: a sub-cell is "under-filled" when it
                               holds fewer than alpha*s particles (Eq. 4);
                               default 0.5, must be finite and >= 0           */
    double  beta;           /* beta: b is halved while the fraction of
                               under-filled sub-cells exceeds beta (Eq. 4);
                               default 0.5, must be finite                    */
    int32_t max_depth;      /* depth guard: a cell at this depth is a leaf
                               whatever its size; default 32, 0..64           */
    int32_t precision;      /* btree_precision; default BTREE_FP32_FILTER     */
    int32_t group_size;     /* queries per wavefront work item, 0 = library
                               choice (64); must be 0 or 64                   */
    int32_t timing;         /* 1: time each phase with HIP events recorded on
                               the caller's stream (btree_stats.phase_ms);
                               default 0                                      */
    int32_t exclude_self;   /* 1: row i does not list i itself (the method's
                               search, Algorithm 2, tests p against itself
                               and lists it when h_p > 0); default 0; in a
                               batch every set must agree                     */
    int32_t octree;         /* 1: every split uses b = 2 (the classical octree
                               of Section 2 that the paper compares against;
                               b = 2 is the floor of Section 3.1 step 3),
                               with no Eq. 1 / Eq. 4; default 0               */
    int32_t reserved[3];    /* must be zero                                   */
} btree_params;

/* Shape of a built tree and counters of the last search. */
typedef struct {
    int64_t n;              /* particles                                      */
    int64_t n_internal;     /* internal cells (split by Algorithm 1)          */
    int64_t n_leaves;       /* non-empty leaf cells                           */
    int64_t depth;          /* deepest leaf; the root is depth 0              */
    int64_t rounds;         /* halvings of b over all internal cells (Eq. 4)  */
    int64_t max_leaf;       /* largest leaf                                   */
    int64_t oversized;      /* leaves above s (made by the depth guard)       */
    int64_t n_chunks;       /* wavefront work items of the search             */
    int64_t b_hist[65];     /* b_hist[b] = internal cells with branching b,
                               b >= 64 counted in b_hist[64]                  */
    /* counters of the last btree_find_neighbors pass 1 on this handle:     */
    int64_t total;          /* neighbour entries                              */
    int64_t pair_tests;     /* candidate pairs tested (FP32 or FP64)          */
    int64_t fp64_confirms;  /* FP32-filter pairs re-tested in FP64            */
    int64_t brute_chunks;   /* queries that took the exhaustive path          */
    int64_t candidates;     /* culled candidates staged, summed over items    */
    /* with params.timing = 1, device time of each phase summed over the
       calls since btree_build (btree_rebuild keeps counting):
       [0] build, [1] search sweep kernel (walk, stage, test, rows or test
       words to the handle's scratch), [2] placement kernels (rows into the
       caller's CSR, expanded from the words or copied from the scratch; in
       the batched form the whole placement segment, exhaustive rows
       included), [3] whole pass 1, [4] whole pass 2;
       phase_calls counts the calls.                                      */
    double  phase_ms[5];
    int64_t phase_calls[5];
    int64_t split_items;    /* work items whose candidates overflowed shared
                               memory and were searched again in groups of 8
                               queries, then singly                            */
    int64_t brute_units;    /* units (1 to 64 queries of one set) that took
                               the exhaustive path; brute_chunks counts their
                               queries                                          */
    int64_t word_items;     /* work items of the main sweep whose rows pass 2
                               expanded from their test words (the items
                               whose words take less room than their rows)  */
    int64_t word_items_wide; /* of those, items with more than 8192 row
                               entries (expanded in windows)                  */
} btree_stats_t;

typedef struct btree_tree* btree_handle;

/* Fills *p with the defaults listed in btree_params.
 * Returns BTREE_EINVAL if p is NULL. */
btree_status btree_params_default(btree_params* p);

/* BuildTree (Algorithm 1, Eqs. 1-4).
 * x, y, z: device FP64 coordinates of n particles (n >= 0, n < 2^31).
 * p: parameters (NULL = defaults).  On success *out receives a handle that
 * owns a sorted copy of the particles and the tree; release it with
 * btree_destroy.  The root cell is the tight bounding box of the particles;
 * each cell is split into b^3 equal sub-cells, b from Eq. 1 halved while the
 * Eq. 4 ratio exceeds beta (b >= 2); sub-cells holding more than s
 * particles are split again; empty sub-cells are not stored.
 * Synchronises `hip_stream` (the level loop reads node counts on the host).
 * Errors: EINVAL (NULL x/y/z/out with n > 0, n < 0 or n >= 2^31, bad
 * parameters, non-finite coordinate), ENOMEM, EDEVICE. */
btree_status btree_build(const double* x, const double* y, const double* z,
                         int64_t n, const btree_params* p, void* hip_stream,
                         btree_handle* out);

/* BuildTree again on the handle `t` over new coordinates (n may differ),
 * with the handle's parameters, reusing its device memory where it is large
 * enough.  Same semantics and errors as btree_build; on failure the handle
 * holds no tree (a search returns BTREE_ESTATE) until a rebuild succeeds. */
btree_status btree_rebuild(btree_handle t, const double* x, const double* y,
                           const double* z, int64_t n, void* hip_stream);

/* FindNeighbors (Algorithm 2, Eq. 5) for every particle of the tree.
 * Row i lists, in ascending original index, every j with
 *     ((dx*dx + dy*dy) + dz*dz) < (2*h_i)*(2*h_i),
 *     dx = x_i - x_j (likewise dy, dz), FP64, each operation rounded,
 * i.e. the query particle's own radius 2h_i (gather form; i itself is listed
 * when h_i > 0).  Results are identical for every precision and parameter.
 *
 * h: device FP64 smoothing lengths (n entries, finite, >= 0).
 * counts: device int32[n], row lengths.
 * offsets: device int64[n+1], offsets[0] = 0, offsets[i+1] = offsets[i] +
 *          counts[i]; row i occupies nbrs[offsets[i] .. offsets[i+1]).
 * nbrs: device int32[capacity] or NULL.
 * total: host int64, receives offsets[n].
 *
 * Pass 1 (nbrs == NULL): writes counts, offsets and *total; synchronises
 *   the stream.  Remembers h, counts and offsets for pass 2.
 * Pass 2 (nbrs != NULL, right after pass 1 on this handle with the same h,
 *   counts and offsets, whose contents the caller has not changed): writes
 *   nbrs[0..total) and *total, without synchronising.
 * Otherwise (nbrs != NULL, no matching pass 1): runs both passes.
 * Errors: EINVAL (NULL h/counts/offsets/total with n > 0, bad h values),
 *   EOVERFLOW (capacity < total; nbrs untouched), ESTATE (NULL handle, or
 *   a handle whose last rebuild failed),
 *   ENOMEM, EDEVICE. */
btree_status btree_find_neighbors(btree_handle t, const double* h,
                                  int32_t* counts, int64_t* offsets,
                                  int32_t* nbrs, int64_t capacity,
                                  int64_t* total, void* hip_stream);

/* Fused SPH consumer: the density sum over each particle's neighbours,
 * computed inside the search with no list written (Section 4.7 uses the
 * search inside an SPH code; the paper fixes no kernel W, this one is the
 * cubic spline of support 2h):
 *     rho[i] = (sum over the j that row i would list of m_j w(r_ij / h_i))
 *              / (pi h_i^3),   rho[i] = 0 for an empty row,
 *     w(q) = (1 - 1.5 q^2) + 0.75 q^3 (q < 1), 0.25 (2 - q)^3 (1 <= q < 2),
 *     r_ij = sqrt((dx*dx + dy*dy) + dz*dz) from the FP64 coordinates,
 * the neighbour set exactly that of btree_find_neighbors (exclude_self
 * included).  Each term is rounded in a fixed order; terms are added in
 * ascending j per part of the row and the parts in a fixed order, so a
 * result is reproducible run to run and differs from a strictly sequential
 * sum by rounding only.
 * h: device FP64[n] (finite, >= 0); mass: device FP64[n] (original order) or
 * NULL for unit masses; rho: device FP64[n] (written); counts: device
 * int32[n] (written: row lengths) or NULL.  Synchronises the stream.
 * Errors: EINVAL (NULL h/rho with n > 0, bad h: nothing written), ESTATE,
 * ENOMEM, EDEVICE. */
btree_status btree_density(btree_handle t, const double* h, const double* mass,
                           double* rho, int32_t* counts, void* hip_stream);

/* Smoothing lengths adapted to a target neighbour count (the target
 * neighbours per particle of Table 3), on the handle's tree (h is an input
 * of the search, not of the tree).  Every particle repeats, independently:
 * c = its row length at its h (as btree_find_neighbors counts it); if
 * |c - target| <= tol it is done; else its h becomes the low end of its
 * bracket (c < target) or the high end (c > target), and h <- h f with
 * f = min(2, (5c + target) / (6c)) (f = 2 for c = 0), or the bracket's
 * midpoint (lo + hi) * 0.5 when h f would leave the bracket; each
 * operation rounded once.  Stops when every particle is done or after
 * max_iter rounds.
 * h: device FP64[n], read and overwritten; counts: device int32[n] or NULL,
 * receives the row lengths at the final h; iterations: host int32 or NULL,
 * receives the number of update rounds made.  A particle with h = 0
 * keeps it (its row stays empty).  Synchronises the stream once per
 * round.  Errors: EINVAL (target not finite and > 0, tol not finite and
 * >= 0, max_iter outside [0, 1000], NULL h, bad h values), ESTATE, ENOMEM,
 * EDEVICE. */
btree_status btree_adapt_h(btree_handle t, double* h, double target, double tol,
                           int32_t max_iter, int32_t* counts, int32_t* iterations,
                           void* hip_stream);

/* Tree shape and last-search counters.  Errors: EINVAL (NULL argument). */
btree_status btree_stats(btree_handle t, btree_stats_t* out);

/* Copies the leaf layout to HOST arrays (for inspection and tests):
 * leaf_beg[n_leaves], leaf_cnt[n_leaves], leaf_depth[n_leaves] in memory
 * order (depth-first, sub-cells in Morton order of their coordinates), and
 * order[n] = original index of the particle at each sorted position.  Any
 * pointer may be NULL to skip that array.  Synchronises `hip_stream`.
 * Errors: EINVAL (NULL handle), EDEVICE. */
btree_status btree_export(btree_handle t, int32_t* leaf_beg, int32_t* leaf_cnt,
                          int32_t* leaf_depth, int32_t* order,
                          void* hip_stream);

/* Releases the handle and all device memory it owns (NULL is a no-op).
 * Waits for work the handle queued to finish first. */
btree_status btree_destroy(btree_handle t);

/* ------------------------------------------------------------------------
 * Batched form: many independent particle sets, each with its own b-tree
 * (Algorithm 1) and its own neighbour lists (Algorithm 2), built and
 * searched together by a captured HIP graph per call.
 * ---------------------------------------------------------------------- */
typedef struct btree_batch* btree_batch_handle;

/* Plans a batch of nsets sets (1 <= nsets <= 2^20).  set_offsets: HOST
 * int64[nsets+1], set_offsets[0] = 0, non-decreasing, total below 2^31; set
 * k is particles [set_offsets[k], set_offsets[k+1]) of the concatenated
 * arrays (empty sets allowed).  per_set: HOST btree_params[nsets] (NULL =
 * defaults for every set); s, alpha, beta and max_depth may differ between
 * sets, precision and timing must not.  Allocates the device pools
 * of the batch; queues nothing.  Errors: EINVAL, ENOMEM, EDEVICE. */
btree_status btree_batch_create(int32_t nsets, const int64_t* set_offsets,
                                const btree_params* per_set,
                                btree_batch_handle* out);

/* BuildTree and FindNeighbors of every set of the batch.
 * x, y, z, h: device FP64[n_total], the sets concatenated.
 * counts: device int32[n_total]; offsets: device int64[n_total+1]; one CSR
 *   over all sets (offsets[0] = 0).  Rows of set k are rows set_offsets[k]
 *   .. set_offsets[k+1]-1; their entries are indices LOCAL to set k (0 is
 *   the set's first particle), ascending; each set's lists follow the
 *   previous set's.  Results per set are identical to btree_build +
 *   btree_find_neighbors on that set alone with the same parameters.
 * nbrs: device int32[capacity] (may be NULL when capacity = 0).
 * totals: HOST int64[nsets] or NULL, entries per set; total: HOST int64,
 *   their sum.
 * The work is a captured HIP graph, recorded on the first call with a given
 * set of pointers and capacity and replayed on later calls with the same
 * ones: five graph segments (build; search set-up; sweep; counts and
 * offsets; exhaustive rows, row placement and totals) launched back to
 * back on hip_stream with no host work between them (so that HIP events
 * between segments can time the steps).  The first call on a handle first runs an
 * eager build and count pass to size the pools.  The call waits for the
 * stream.  When a pool proves too small for new data, the handle grows it,
 * records the graph again and repeats the run.
 * Errors: EINVAL (NULL arrays with n_total > 0, capacity < 0, non-finite
 * coordinate, h < 0 or non-finite: then no caller output is written),
 * EOVERFLOW (capacity < total: counts, offsets, totals and *total are
 * written, nbrs is not), ESTATE (NULL handle), ENOMEM, EDEVICE. */
btree_status btree_batch_run(btree_batch_handle b, const double* x,
                             const double* y, const double* z,
                             const double* h, int32_t* counts,
                             int64_t* offsets, int32_t* nbrs,
                             int64_t capacity, int64_t* totals,
                             int64_t* total, void* hip_stream);

/* Shape of the batch's forest and counters of its last run, summed over
 * the sets (depth and max_leaf: maxima).  With timing = 1, phase_ms holds
 * device time of the graph runs (HIP events between segments; the first
 * call's sizing run is not counted), with the phases of btree_stats_t.
 * Errors: EINVAL (NULL argument). */
btree_status btree_batch_stats(btree_batch_handle b, btree_stats_t* out);

/* Graph launches made and graph recordings taken by the handle so far.
 * Errors: EINVAL (NULL argument). */
btree_status btree_batch_graph_counts(btree_batch_handle b, int64_t* launches,
                                      int64_t* recordings);

/* Releases the batch and its device memory (NULL is a no-op); waits for
 * the device first. */
btree_status btree_batch_destroy(btree_batch_handle b);

/* ------------------------------------------------------------------------
 * Autotuning of s, beta and alpha (the parameters of Table 1 and Eq. 4:
 * the bucket size and the empty-cell limit).  Results do not depend on the
 * parameters, so a tuner can only change speed.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n_bucket;       /* candidate bucket sizes s, 1..16              */
    int32_t bucket[16];
    int32_t n_beta;         /* candidate beta values, 1..8                  */
    double  beta[8];
    int32_t repeats;        /* timed runs per candidate (median), 1..100   */
    int32_t n_alpha;        /* candidate alpha values, 0..4 (0: the base
                               parameters' alpha only)                       */
    double  alpha[4];       /* finite and >= 0                               */
    int32_t reserved[2];    /* must be zero                                 */
} btree_tune_space;

/* Default space: s in {16, 24, 32, 48, 64, 96, 128, 192, 256}, beta in
 * {0.3, 0.5, 0.8}, alpha in {0.25, 0.5, 1}, 3 repeats.
 * Errors: EINVAL (NULL). */
btree_status btree_tune_space_default(btree_tune_space* space);

/* Times BuildTree + both FindNeighbors passes on the given particles for
 * every (s, beta, alpha) of `space` (NULL = default), other parameters from `base`
 * (NULL = defaults): the device time of the recorded graph of a one-set
 * batch (HIP events around its launch on hip_stream, so host round trips
 * of the eager path do not count), and returns in *best the parameters of
 * the fastest median and in *best_ms that median.
 * all_ms: HOST double[n_bucket * n_beta * max(n_alpha, 1)] (row-major:
 *   bucket, then beta, then alpha) or NULL.
 * Allocates its own device buffers; synchronises the stream.
 * Errors: EINVAL (bad arguments or data), ENOMEM, EDEVICE. */
btree_status btree_tune(const double* x, const double* y, const double* z,
                        const double* h, int64_t n, const btree_params* base,
                        const btree_tune_space* space, btree_params* best,
                        double* best_ms, double* all_ms, void* hip_stream);

/* ------------------------------------------------------------------------
 * Build and search with no device allocation.
 * ---------------------------------------------------------------------- */
#define BTREE_NOALLOC_MAX_N 65536       /* particles per call, at most       */
#define BTREE_NOALLOC_SCRATCH_MIB 128   /* fixed device scratch per GPU      */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as btree_build + btree_find_neighbors (both passes) + btree_destroy
 * on one set of n particles, with every tree, work-list and row buffer
 * carved from a fixed device array of BTREE_NOALLOC_SCRATCH_MIB MiB that the
 * library holds on each GPU it runs on from load until the process ends.
 * The call makes no hipMalloc or hipFree and allocates through no other
 * library; the caller passes inputs and outputs.
 *
 * x, y, z, h: device FP64[n], 0 <= n <= BTREE_NOALLOC_MAX_N.
 * p: parameters (NULL = defaults); timing must be 0.
 * counts: device int32[n]; offsets: device int64[n+1]; nbrs: device
 *   int32[capacity] (NULL allowed when capacity = 0); rows as in
 *   btree_find_neighbors.  total: host int64, receives offsets[n].
 * Synchronises hip_stream before returning.  Calls on one GPU share its
 * scratch: the library serialises calls from different host threads on
 * one device, and a call must not overlap other work that uses the
 * scratch (there is none besides this entry point).
 * Errors: EINVAL (n above BTREE_NOALLOC_MAX_N, NULL arrays, bad parameters
 *   or particle data: nothing written), EOVERFLOW (capacity < total: counts,
 *   offsets and *total written, nbrs not), ENOMEM (this input's tree, work
 *   lists and rows need more than the scratch holds; the message says how
 *   much; about 1 KB per particle plus 4 B per neighbour entry fit at the
 *   default bucket size, several times more at bucket sizes near 1), EDEVICE. */
btree_status btree_find_neighbors_noalloc(const double* x, const double* y,
                                          const double* z, const double* h,
                                          int64_t n, const btree_params* p,
                                          int32_t* counts, int64_t* offsets,
                                          int32_t* nbrs, int64_t capacity,
                                          int64_t* total, void* hip_stream);

/* Message of the last failed call on this host thread ("" if none). */
const char* btree_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BTREE_H */

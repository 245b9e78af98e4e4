/* Drives the host-side checks of the C ABI (include/btree.h) that run
 * before any device call, for a build of the library whose host code is
 * instrumented by AddressSanitizer and UndefinedBehaviorSanitizer: every
 * call must return the documented status, leave a message, and touch no
 * memory it does not own.  Needs no GPU.  Prints "ok" and exits 0 when
 * every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "btree.h"

static int failures = 0;
#define EXPECT(call, want)                                                          \
    do {                                                                            \
        btree_status got_ = (call);                                                 \
        if (got_ != (want)) {                                                       \
            fprintf(stderr, "FAIL line %d: %s = %d, want %d (%s)\n", __LINE__, #call, \
                    (int)got_, (int)(want), btree_last_error());                     \
            ++failures;                                                             \
        } else if ((want) != BTREE_OK && btree_last_error()[0] == '\0') {           \
            fprintf(stderr, "FAIL line %d: %s left no message\n", __LINE__, #call);  \
            ++failures;                                                             \
        }                                                                           \
    } while (0)

int main(void)
{
    const double* P = (const double*)(uintptr_t)64;  /* never dereferenced: checks come first */
    btree_params p, q;
    btree_handle t = NULL;
    EXPECT(btree_params_default(NULL), BTREE_EINVAL);
    EXPECT(btree_params_default(&p), BTREE_OK);

    /* btree_build: bad parameters and sizes. */
    q = p; q.bucket_size = 0;   EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    q = p; q.alpha = NAN;       EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    q = p; q.alpha = -1.0;      EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    q = p; q.beta = INFINITY;   EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    q = p; q.max_depth = 65;    EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    q = p; q.precision = 7;     EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    q = p; q.group_size = 32;   EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    q = p; q.exclude_self = 2;  EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    q = p; q.octree = -1;       EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    q = p; q.reserved[2] = 1;   EXPECT(btree_build(P, P, P, 100, &q, NULL, &t), BTREE_EINVAL);
    EXPECT(btree_build(P, P, P, -1, &p, NULL, &t), BTREE_EINVAL);
    EXPECT(btree_build(P, P, P, (int64_t)1 << 31, &p, NULL, &t), BTREE_EINVAL);
    EXPECT(btree_build(NULL, P, P, 100, &p, NULL, &t), BTREE_EINVAL);
    EXPECT(btree_build(P, P, P, 100, &p, NULL, NULL), BTREE_EINVAL);
    q = p; q.bucket_size = 1;
    EXPECT(btree_build(P, P, P, ((int64_t)1 << 31) - 2, &q, NULL, &t), BTREE_EINVAL);

    /* Calls on no handle. */
    int64_t total = 0;
    btree_stats_t st;
    EXPECT(btree_find_neighbors(NULL, NULL, NULL, NULL, NULL, 0, &total, NULL), BTREE_ESTATE);
    EXPECT(btree_density(NULL, NULL, NULL, NULL, NULL, NULL), BTREE_ESTATE);
    EXPECT(btree_adapt_h(NULL, NULL, 64.0, 0.0, 10, NULL, NULL, NULL), BTREE_ESTATE);
    EXPECT(btree_stats(NULL, &st), BTREE_EINVAL);
    EXPECT(btree_export(NULL, NULL, NULL, NULL, NULL, NULL), BTREE_EINVAL);
    EXPECT(btree_rebuild(NULL, P, P, P, 10, NULL), BTREE_ESTATE);
    EXPECT(btree_destroy(NULL), BTREE_OK);

    /* Batches. */
    btree_batch_handle b = NULL;
    int64_t offs[3] = {0, 5, 9};
    EXPECT(btree_batch_create(2, offs, NULL, NULL), BTREE_EINVAL);
    EXPECT(btree_batch_create(0, offs, NULL, &b), BTREE_EINVAL);
    EXPECT(btree_batch_create(2, NULL, NULL, &b), BTREE_EINVAL);
    int64_t bad1[3] = {1, 5, 9}, bad2[3] = {0, 5, 4}, bad3[2] = {0, (int64_t)1 << 31};
    EXPECT(btree_batch_create(2, bad1, NULL, &b), BTREE_EINVAL);
    EXPECT(btree_batch_create(2, bad2, NULL, &b), BTREE_EINVAL);
    EXPECT(btree_batch_create(1, bad3, NULL, &b), BTREE_EINVAL);
    btree_params two[2] = {p, p};
    two[1].precision = BTREE_FP64;
    EXPECT(btree_batch_create(2, offs, two, &b), BTREE_EINVAL);
    two[1] = p; two[1].bucket_size = 0;
    EXPECT(btree_batch_create(2, offs, two, &b), BTREE_EINVAL);
    two[1] = p; two[1].timing = 1;
    EXPECT(btree_batch_create(2, offs, two, &b), BTREE_EINVAL);
    two[1] = p; two[1].exclude_self = 1;
    EXPECT(btree_batch_create(2, offs, two, &b), BTREE_EINVAL);
    EXPECT(btree_batch_run(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, &total, NULL),
           BTREE_ESTATE);
    EXPECT(btree_batch_stats(NULL, &st), BTREE_EINVAL);
    EXPECT(btree_batch_graph_counts(NULL, NULL, NULL), BTREE_EINVAL);
    EXPECT(btree_batch_destroy(NULL), BTREE_OK);

    /* Tuner. */
    btree_tune_space sp;
    btree_params best;
    double ms = 0.0;
    EXPECT(btree_tune_space_default(NULL), BTREE_EINVAL);
    EXPECT(btree_tune_space_default(&sp), BTREE_OK);
    EXPECT(btree_tune(P, P, P, P, 10, NULL, NULL, NULL, &ms, NULL, NULL), BTREE_EINVAL);
    btree_tune_space bad = sp; bad.repeats = 0;
    EXPECT(btree_tune(P, P, P, P, 10, NULL, &bad, &best, &ms, NULL, NULL), BTREE_EINVAL);
    bad = sp; bad.bucket[1] = 0;
    EXPECT(btree_tune(P, P, P, P, 10, NULL, &bad, &best, &ms, NULL, NULL), BTREE_EINVAL);
    EXPECT(btree_tune(P, P, P, NULL, 10, NULL, NULL, &best, &ms, NULL, NULL), BTREE_EINVAL);

    /* The entry point that allocates nothing. */
    int32_t* C = (int32_t*)(uintptr_t)64;
    int64_t* O = (int64_t*)(uintptr_t)64;
    EXPECT(btree_find_neighbors_noalloc(P, P, P, P, 10, &p, C, O, NULL, 0, NULL, NULL),
           BTREE_EINVAL);
    EXPECT(btree_find_neighbors_noalloc(P, P, P, P, BTREE_NOALLOC_MAX_N + 1, &p, C, O, NULL, 0,
                                        &total, NULL), BTREE_EINVAL);
    EXPECT(btree_find_neighbors_noalloc(P, P, P, P, 10, &p, C, NULL, NULL, 0, &total, NULL),
           BTREE_EINVAL);
    EXPECT(btree_find_neighbors_noalloc(P, P, P, NULL, 10, &p, C, O, NULL, 0, &total, NULL),
           BTREE_EINVAL);
    EXPECT(btree_find_neighbors_noalloc(P, P, P, P, 10, &p, C, O, NULL, 5, &total, NULL),
           BTREE_EINVAL);
    q = p; q.timing = 1;
    EXPECT(btree_find_neighbors_noalloc(P, P, P, P, 10, &q, C, O, NULL, 0, &total, NULL),
           BTREE_EINVAL);

    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}

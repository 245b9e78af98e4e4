// Batched form: many independent particle sets built and searched by a
// captured HIP graph.  The sets share one control block, one set of pools
// and one launch sequence (set id in the top bits of the Morton key, per-set
// roots, work items tagged with their set), so the whole batch costs the
// launches of a single tree.  The sequence is recorded as a few graph
// segments (build, search steps) launched back to back with no host work
// between them, so HIP events on the caller's stream can time the steps.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"

namespace bt {

enum { kSegBuild = 0, kSegBegin, kSegSweep, kSegCounts, kSegPlace, kSegs };

struct Batch {
    Tree t;
    hipStream_t cs = nullptr;       // private stream the graph is captured on
    hipGraph_t graph[kSegs] = {};
    hipGraphExec_t exec[kSegs] = {};
    const void* key[7] = {};        // caller pointers baked into the graph
    int64_t key_cap = -1;
    bool primed = false;            // an eager run has sized the pools
    bool recorded = false;
    int64_t launches = 0;
    int64_t captures = 0;
    std::vector<int64_t> host_tot;  // per-set totals of the last run
    hipEvent_t e0 = nullptr, e1 = nullptr;  // around a launch, for tuning

    void drop_graph() {
        for (int k = 0; k < kSegs; ++k) {
            if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
            if (graph[k]) (void)hipGraphDestroy(graph[k]);
            exec[k] = nullptr;
            graph[k] = nullptr;
        }
        recorded = false;
    }
    ~Batch() {
        drop_graph();
        if (cs) (void)hipStreamDestroy(cs);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

namespace {

void check_set_params(const btree_params& p, const btree_params& p0) {
    if (p.bucket_size < 1) fail(BTREE_EINVAL, "bucket_size must be >= 1");
    if (!std::isfinite(p.alpha) || p.alpha < 0.0) fail(BTREE_EINVAL, "alpha must be finite and >= 0");
    if (!std::isfinite(p.beta)) fail(BTREE_EINVAL, "beta must be finite");
    if (p.max_depth < 0 || p.max_depth > 64) fail(BTREE_EINVAL, "max_depth must be in [0, 64]");
    if (p.precision != BTREE_FP64 && p.precision != BTREE_FP32_FILTER)
        fail(BTREE_EINVAL, "precision must be BTREE_FP64 or BTREE_FP32_FILTER");
    if (p.precision != p0.precision) fail(BTREE_EINVAL, "all sets of a batch need one precision");
    if (p.group_size != 0 && p.group_size != kGroup) fail(BTREE_EINVAL, "group_size must be 0 or 64");
    if (p.timing != 0 && p.timing != 1) fail(BTREE_EINVAL, "timing must be 0 or 1");
    if (p.timing != p0.timing) fail(BTREE_EINVAL, "all sets of a batch need one timing flag");
    if (p.exclude_self != 0 && p.exclude_self != 1) fail(BTREE_EINVAL, "exclude_self must be 0 or 1");
    if (p.exclude_self != p0.exclude_self)
        fail(BTREE_EINVAL, "all sets of a batch need one exclude_self flag");
    if (p.octree != 0 && p.octree != 1) fail(BTREE_EINVAL, "octree must be 0 or 1");
    for (int k = 0; k < 3; ++k)
        if (p.reserved[k] != 0) fail(BTREE_EINVAL, "reserved fields must be zero");
}

__global__ void k_zero_offsets(int64_t* __restrict__ offsets) {
    if (threadIdx.x == 0 && blockIdx.x == 0) offsets[0] = 0;
}

// Records one segment: whatever `queue` puts on the private stream.
template <class F>
void record(Batch& B, int seg, F&& queue) {
    BT_HIP(hipStreamBeginCapture(B.cs, hipStreamCaptureModeThreadLocal));
    try {
        queue(B.cs);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(B.cs, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    BT_HIP(hipStreamEndCapture(B.cs, &B.graph[seg]));
    BT_HIP(hipGraphInstantiate(&B.exec[seg], B.graph[seg], nullptr, nullptr, 0));
}

// Records build + search of every set.
void capture(Batch& B, const double* x, const double* y, const double* z, const double* h,
             int32_t* counts, int64_t* offsets, int32_t* nbrs, int64_t capacity) {
    Tree& t = B.t;
    B.drop_graph();
    record(B, kSegBuild, [&](hipStream_t s) { build_queue(t, x, y, z, (int)t.level_cap, false, s); });
    record(B, kSegBegin, [&](hipStream_t s) {
        find_begin(t, h, s);
        find_walk(t, h, t.chunk_cap, s);
    });
    record(B, kSegSweep, [&](hipStream_t s) { find_sweep(t, h, counts, t.chunk_cap, s); });
    record(B, kSegCounts, [&](hipStream_t s) { find_counts_end(t, h, counts, offsets, s); });
    record(B, kSegPlace, [&](hipStream_t s) {
        find_fill(t, counts, offsets, nbrs, capacity, t.tot.as<int64_t>(), false, s);
    });
    B.recorded = true;
    const void* k[7] = {x, y, z, h, counts, offsets, nbrs};
    std::memcpy(B.key, k, sizeof k);
    B.key_cap = capacity;
    ++B.captures;
}

// Launches the segments back to back on the caller's stream.
void launch(Batch& B, hipStream_t st) {
    Timer& T = B.t.timer;
    T.start(kPhBuild, st);
    BT_HIP(hipGraphLaunch(B.exec[kSegBuild], st));
    T.stop(kPhBuild, st);
    T.start(kPhPass1, st);
    BT_HIP(hipGraphLaunch(B.exec[kSegBegin], st));
    T.start(kPhSweep, st);
    BT_HIP(hipGraphLaunch(B.exec[kSegSweep], st));
    T.stop(kPhSweep, st);
    BT_HIP(hipGraphLaunch(B.exec[kSegCounts], st));
    T.stop(kPhPass1, st);
    T.start(kPhPass2, st);
    T.start(kPhPlace, st);
    BT_HIP(hipGraphLaunch(B.exec[kSegPlace], st));
    T.stop(kPhPlace, st);
    T.stop(kPhPass2, st);
    ++B.launches;
}

bool same_key(const Batch& B, const double* x, const double* y, const double* z, const double* h,
              const int32_t* counts, const int64_t* offsets, const int32_t* nbrs, int64_t cap) {
    const void* k[7] = {x, y, z, h, counts, offsets, nbrs};
    return B.recorded && std::memcmp(B.key, k, sizeof k) == 0 && B.key_cap == cap;
}

// First run: an eager build and count pass size the level count, the work
// item bound and the scratch for this batch.
int64_t prime(Batch& B, const double* x, const double* y, const double* z, const double* h,
              int32_t* counts, int64_t* offsets, hipStream_t st) {
    Tree& t = B.t;
    const bool timing = t.timer.on;
    t.timer.on = false;  // phase times count graph runs only
    build_tree(t, x, y, z, st);
    t.level_cap = std::max<int64_t>(1, std::min<int64_t>(t.levels_seen + 1, 66));
    t.chunk_cap = t.n_chunks + t.n_chunks / 4 + 64;
    const int64_t total = find_pass1(t, h, counts, offsets, st);
    t.timer.on = timing;
    B.primed = true;
    return total;
}

// Runs the recorded graph once (recording it first when the pointers or
// the capacity changed) and waits; on a pool overflow grows the pool,
// records again and repeats.  Fills host_ctl, host_stats and host_tot.
// With `ms`, the device time of the successful launch (HIP events around it).
void run_graph(Batch& B, const double* x, const double* y, const double* z, const double* h,
               int32_t* counts, int64_t* offsets, int32_t* nbrs, int64_t capacity, hipStream_t st,
               float* ms) {
    Tree& t = B.t;
    if (ms && !B.e0) {
        BT_HIP(hipEventCreate(&B.e0));
        BT_HIP(hipEventCreate(&B.e1));
    }
    for (int attempt = 0;; ++attempt) {
        if (!same_key(B, x, y, z, h, counts, offsets, nbrs, capacity))
            capture(B, x, y, z, h, counts, offsets, nbrs, capacity);
        if (ms) BT_HIP(hipEventRecord(B.e0, st));
        launch(B, st);
        if (ms) BT_HIP(hipEventRecord(B.e1, st));
        BT_HIP(hipMemcpyAsync(&t.host_ctl, t.ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(&t.host_stats, t.stats.p, sizeof(Stats), hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(B.host_tot.data(), t.tot.p, sizeof(int64_t) * t.nsets,
                              hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(t.host_stripes, t.stripes.p, sizeof t.host_stripes,
                              hipMemcpyDeviceToHost, st));
        BT_HIP(hipStreamSynchronize(st));
        const Ctl& c = t.host_ctl;
        if (c.data_bad & 1) fail(BTREE_EINVAL, "btree_batch_run: non-finite particle coordinate");
        if (c.data_bad & 2) fail(BTREE_EINVAL, "btree_batch_run: h must be finite and >= 0");
        const int ovf = c.overflow & ~kOvfCapacity;
        if (!ovf) break;
        if (attempt >= 8) fail(BTREE_ENOMEM, "btree_batch_run: pools kept overflowing");
        // Grow what was too small, then record again.
        if (ovf & (kOvfNodes | kOvfCtab | kOvfHist)) {
            if (ovf & kOvfNodes) t.node_cap *= 2;
            if (ovf & kOvfCtab) t.ctab_cap *= 2;
            if (ovf & kOvfHist) t.hist_cap *= 2;
            plan_sets(t, t.nsets, t.set_off.data(), t.set_prm.data());
        }
        if (ovf & kOvfLevels) t.level_cap = std::min<int64_t>(66, 2 * t.level_cap + 1);
        if (ovf & kOvfChunks) t.chunk_cap = (int64_t)c.n_chunks + c.n_chunks / 4 + 64;
        grow_pools(t, ovf);  // also sizes the walk results for the work-item bound
        B.drop_graph();
    }
    if (ms) BT_HIP(hipEventElapsedTime(ms, B.e0, B.e1));
    const Ctl& c = t.host_ctl;
    t.n_internal = c.n_nodes;
    t.n_leaves = c.n_leaves;
    t.n_chunks = c.n_chunks;
    t.ctab_len = c.ct_len;
    t.depth = c.depth;
    t.max_leaf = c.max_leaf;
    t.oversized = c.oversized;
    t.levels_seen = c.levels;
}

// Sets a handle up for `nsets` sets (offsets on the host, validated).
void setup(Batch& B, int32_t nsets, const int64_t* set_offsets, const btree_params* prm) {
    Tree& t = B.t;
    t.prm = prm[0];
    t.timer.on = prm[0].timing != 0;
    if (hipGetDevice(&t.device) != hipSuccess) t.device = 0;
    BT_HIP(hipStreamCreateWithFlags(&B.cs, hipStreamNonBlocking));
    plan_sets(t, nsets, set_offsets, prm);
    t.level_cap = 66;
    B.host_tot.assign((size_t)nsets, 0);
}

}  // namespace

}  // namespace bt

struct btree_batch {
    bt::Batch b;
};

using namespace bt;

template <class F>
static btree_status guarded_b(F&& f) {
    try {
        f();
        return BTREE_OK;
    } catch (const Fail& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return BTREE_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return BTREE_EDEVICE;
    }
}

extern "C" {

btree_status btree_batch_create(int32_t nsets, const int64_t* set_offsets,
                                const btree_params* per_set, btree_batch_handle* out) {
    return guarded_b([&] {
        if (!out) fail(BTREE_EINVAL, "btree_batch_create: out is NULL");
        *out = nullptr;
        if (nsets < 1 || nsets > (1 << 20)) fail(BTREE_EINVAL, "btree_batch_create: nsets must be in [1, 2^20]");
        if (!set_offsets) fail(BTREE_EINVAL, "btree_batch_create: set_offsets is NULL");
        if (set_offsets[0] != 0) fail(BTREE_EINVAL, "btree_batch_create: set_offsets[0] must be 0");
        for (int k = 0; k < nsets; ++k)
            if (set_offsets[k + 1] < set_offsets[k])
                fail(BTREE_EINVAL, "btree_batch_create: set_offsets must be non-decreasing");
        if (set_offsets[nsets] >= 0x7fffffffll)
            fail(BTREE_EINVAL, "btree_batch_create: total particles must be below 2^31");
        std::vector<btree_params> prm((size_t)nsets);
        for (int k = 0; k < nsets; ++k) {
            if (per_set) prm[k] = per_set[k];
            else btree_params_default(&prm[k]);
        }
        for (int k = 0; k < nsets; ++k) {
            check_set_params(prm[k], prm[0]);
            const int64_t nk = set_offsets[k + 1] - set_offsets[k];
            if ((nk + prm[k].bucket_size - 1) / prm[k].bucket_size > (1ll << 30))
                fail(BTREE_EINVAL, "btree_batch_create: n / bucket_size must not exceed 2^30");
        }
        btree_batch* H = new btree_batch();
        Batch& B = H->b;
        try {
            setup(B, nsets, set_offsets, prm.data());
        } catch (...) {
            delete H;
            throw;
        }
        *out = H;
        set_error("");
    });
}

btree_status btree_batch_run(btree_batch_handle H, const double* x, const double* y,
                             const double* z, const double* h, int32_t* counts, int64_t* offsets,
                             int32_t* nbrs, int64_t capacity, int64_t* totals, int64_t* total,
                             void* hip_stream) {
    return guarded_b([&] {
        Range range("btree_batch_run");
        if (!H) fail(BTREE_ESTATE, "btree_batch_run: NULL handle");
        Batch& B = H->b;
        Tree& t = B.t;
        const int64_t n = t.n;
        if (!total) fail(BTREE_EINVAL, "btree_batch_run: total is NULL");
        if (!offsets) fail(BTREE_EINVAL, "btree_batch_run: offsets is NULL");
        if (n > 0 && (!x || !y || !z || !h || !counts))
            fail(BTREE_EINVAL, "btree_batch_run: NULL particle or counts array");
        if (capacity < 0) fail(BTREE_EINVAL, "btree_batch_run: capacity < 0");
        if (capacity > 0 && !nbrs) fail(BTREE_EINVAL, "btree_batch_run: nbrs is NULL with capacity > 0");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        *total = 0;
        if (n == 0) {
            hipLaunchKernelGGL(k_zero_offsets, dim3(1), dim3(64), 0, st, offsets);
            BT_LAUNCH();
            BT_HIP(hipStreamSynchronize(st));
            if (totals)
                for (int k = 0; k < t.nsets; ++k) totals[k] = 0;
            set_error("");
            return;
        }
        if (!B.primed) (void)prime(B, x, y, z, h, counts, offsets, st);
        run_graph(B, x, y, z, h, counts, offsets, nbrs, capacity, st, nullptr);
        const Ctl& c = t.host_ctl;
        int64_t sum = 0;
        for (int k = 0; k < t.nsets; ++k) {
            sum += B.host_tot[k];
            if (totals) totals[k] = B.host_tot[k];
        }
        *total = sum;
        t.last_total = sum;
        if (c.overflow & kOvfCapacity)
            fail(BTREE_EOVERFLOW, "btree_batch_run: capacity " + std::to_string(capacity) +
                                      " < total " + std::to_string(sum));
        set_error("");
    });
}

btree_status btree_batch_stats(btree_batch_handle H, btree_stats_t* out) {
    if (!H || !out) {
        set_error("btree_batch_stats: NULL argument");
        return BTREE_EINVAL;
    }
    Batch& B = H->b;
    Tree& t = B.t;
    t.timer.fold_all();
    std::memset(out, 0, sizeof *out);
    out->n = t.n;
    out->n_internal = t.n_internal;
    out->n_leaves = t.n_leaves;
    out->depth = t.depth;
    out->rounds = (int64_t)t.host_stats.rounds;
    out->max_leaf = t.max_leaf;
    out->oversized = t.oversized;
    out->n_chunks = t.n_chunks;
    for (int k = 0; k < 65; ++k) out->b_hist[k] = (int64_t)t.host_stats.b_hist[k];
    out->total = t.last_total;
    out->pair_tests = (int64_t)ctr_total(t.host_stats, kCtrPairs);
    out->fp64_confirms = (int64_t)ctr_total(t.host_stats, kCtrConfirms);
    out->brute_chunks = (int64_t)ctr_total(t.host_stats, kCtrBrute);
    out->candidates = (int64_t)ctr_total(t.host_stats, kCtrCands);
    out->split_items = (int64_t)ctr_total(t.host_stats, kCtrSplit);
    out->word_items = (int64_t)ctr_total(t.host_stats, kCtrWords);
    out->word_items_wide = (int64_t)ctr_total(t.host_stats, kCtrWide);
    out->brute_units = (int64_t)t.host_ctl.nbunits;
    for (int k = 0; k < kPhases; ++k) {
        out->phase_ms[k] = t.timer.sum_ms[k];
        out->phase_calls[k] = t.timer.calls[k];
    }
    set_error("");
    return BTREE_OK;
}

btree_status btree_batch_graph_counts(btree_batch_handle H, int64_t* launches,
                                      int64_t* recordings) {
    if (!H || !launches || !recordings) {
        set_error("btree_batch_graph_counts: NULL argument");
        return BTREE_EINVAL;
    }
    *launches = H->b.launches;
    *recordings = H->b.captures;
    set_error("");
    return BTREE_OK;
}

btree_status btree_batch_destroy(btree_batch_handle H) {
    if (!H) return BTREE_OK;
    (void)hipDeviceSynchronize();
    delete H;
    return BTREE_OK;
}

btree_status btree_tune(const double* x, const double* y, const double* z, const double* h,
                        int64_t n, const btree_params* base, const btree_tune_space* space,
                        btree_params* best, double* best_ms, double* all_ms, void* hip_stream) {
    return guarded_b([&] {
        Range range("btree_tune");
        if (!best || !best_ms) fail(BTREE_EINVAL, "btree_tune: NULL best or best_ms");
        btree_params prm;
        if (base) prm = *base;
        else btree_params_default(&prm);
        prm.timing = 0;
        check_set_params(prm, prm);
        btree_tune_space sp;
        if (space) sp = *space;
        else btree_tune_space_default(&sp);
        if (sp.n_bucket < 1 || sp.n_bucket > 16 || sp.n_beta < 1 || sp.n_beta > 8 || sp.repeats < 1 ||
            sp.repeats > 100 || sp.n_alpha < 0 || sp.n_alpha > 4)
            fail(BTREE_EINVAL,
                 "btree_tune: space needs 1..16 buckets, 1..8 betas, 0..4 alphas, 1..100 repeats");
        if (n < 0 || n >= 0x7fffffffll) fail(BTREE_EINVAL, "btree_tune: n must be in [0, 2^31-1)");
        for (int k = 0; k < sp.n_bucket; ++k) {
            btree_params q = prm;
            q.bucket_size = sp.bucket[k];
            check_set_params(q, q);
            if ((n + q.bucket_size - 1) / q.bucket_size > (1ll << 30))
                fail(BTREE_EINVAL, "btree_tune: n / bucket_size must not exceed 2^30");
        }
        for (int k = 0; k < sp.n_beta; ++k)
            if (!std::isfinite(sp.beta[k])) fail(BTREE_EINVAL, "btree_tune: beta must be finite");
        for (int k = 0; k < sp.n_alpha; ++k)
            if (!std::isfinite(sp.alpha[k]) || sp.alpha[k] < 0.0)
                fail(BTREE_EINVAL, "btree_tune: alpha must be finite and >= 0");
        for (int k = 0; k < 2; ++k)
            if (sp.reserved[k] != 0) fail(BTREE_EINVAL, "btree_tune: reserved fields must be zero");
        // No alpha listed: the base parameters' alpha is the only candidate.
        const int na = sp.n_alpha > 0 ? sp.n_alpha : 1;
        if (n > 0 && (!x || !y || !z || !h)) fail(BTREE_EINVAL, "btree_tune: NULL particle array");
        *best = prm;
        *best_ms = 0.0;
        if (n == 0) {
            set_error("");
            return;
        }
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        // Outputs are the same for every candidate: one set of buffers.
        DBuf counts, offsets, nbrs;
        counts.reserve(sizeof(int32_t) * n);
        offsets.reserve(sizeof(int64_t) * (n + 1));
        const int64_t off[2] = {0, n};
        double best_t = INFINITY;
        for (int kb = 0; kb < sp.n_bucket; ++kb) {
            for (int kc = 0; kc < sp.n_beta * na; ++kc) {
                const int kt = kc / na, ka = kc % na;
                btree_params q = prm;
                q.bucket_size = sp.bucket[kb];
                q.beta = sp.beta[kt];
                if (sp.n_alpha > 0) q.alpha = sp.alpha[ka];
                // Device time of the recorded graph (build + both search
                // passes), as the batched form runs it: no host round trips.
                Batch B;
                setup(B, 1, off, &q);
                const int64_t tot = prime(B, x, y, z, h, counts.as<int32_t>(),
                                          offsets.as<int64_t>(), st);
                nbrs.reserve(sizeof(int32_t) * std::max<int64_t>(tot, 1));
                const int64_t cap = (int64_t)(nbrs.bytes / sizeof(int32_t));
                std::vector<double> ms;
                for (int r = 0; r <= sp.repeats; ++r) {  // run 0 records the graph
                    float v = 0.f;
                    run_graph(B, x, y, z, h, counts.as<int32_t>(), offsets.as<int64_t>(),
                              nbrs.as<int32_t>(), cap, st, &v);
                    if (r > 0) ms.push_back(v);
                }
                std::sort(ms.begin(), ms.end());
                const double med = ms[ms.size() / 2];
                if (all_ms) all_ms[(int64_t)kb * sp.n_beta * na + kc] = med;
                if (med < best_t) {
                    best_t = med;
                    *best = q;
                }
            }
        }
        best->timing = base ? base->timing : 0;
        *best_ms = best_t;
        set_error("");
    });
}

}  // extern "C"

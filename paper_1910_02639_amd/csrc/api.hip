// C ABI of libbtree: argument checks, handle lifetime, status codes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "common.h"

namespace bt {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

Arena*& current_arena() {
    static thread_local Arena* a = nullptr;
    return a;
}

// Makes an arena current on this host thread for the lifetime of the scope.
struct ArenaScope {
    Arena* prev;
    explicit ArenaScope(Arena* a) : prev(current_arena()) { current_arena() = a; }
    ~ArenaScope() { current_arena() = prev; }
};

// The scratch of the entry point that allocates no device memory: one
// fixed array per GPU, present from module load until the process ends.
// Host code must not use this name as a device address: each device's
// address comes from hipGetSymbolAddress (noalloc_scratch below).
constexpr size_t kNoAllocBytes = (size_t)BTREE_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static void* g_noalloc_ptr[kMaxDevices];
static std::mutex g_noalloc_mu[kMaxDevices];

// Device address of `scratch` on the current device `dev`, looked up once
// per device with that device current (the caller holds its mutex).
static char* noalloc_scratch(int dev) {
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            fail(BTREE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                    hipGetErrorString(e));
        g_noalloc_ptr[dev] = ptr;
    }
    return static_cast<char*>(g_noalloc_ptr[dev]);
}

static void check_params(const btree_params& p) {
    if (p.bucket_size < 1) fail(BTREE_EINVAL, "bucket_size must be >= 1");
    if (!std::isfinite(p.alpha) || p.alpha < 0.0) fail(BTREE_EINVAL, "alpha must be finite and >= 0");
    if (!std::isfinite(p.beta)) fail(BTREE_EINVAL, "beta must be finite");
    if (p.max_depth < 0 || p.max_depth > 64) fail(BTREE_EINVAL, "max_depth must be in [0, 64]");
    if (p.precision != BTREE_FP64 && p.precision != BTREE_FP32_FILTER)
        fail(BTREE_EINVAL, "precision must be BTREE_FP64 or BTREE_FP32_FILTER");
    if (p.group_size != 0 && p.group_size != kGroup) fail(BTREE_EINVAL, "group_size must be 0 or 64");
    if (p.timing != 0 && p.timing != 1) fail(BTREE_EINVAL, "timing must be 0 or 1");
    if (p.exclude_self != 0 && p.exclude_self != 1) fail(BTREE_EINVAL, "exclude_self must be 0 or 1");
    if (p.octree != 0 && p.octree != 1) fail(BTREE_EINVAL, "octree must be 0 or 1");
    for (int k = 0; k < 3; ++k)
        if (p.reserved[k] != 0) fail(BTREE_EINVAL, "reserved fields must be zero");
}

template <class F>
static btree_status guarded(F&& f) {
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

}  // namespace bt

// The opaque handle of the ABI wraps the tree.
struct btree_tree {
    bt::Tree t;
};

using namespace bt;

namespace bt {

static void check_n(int64_t n, const double* x, const double* y, const double* z, int32_t s) {
    if (n < 0 || n >= 0x7fffffffll) fail(BTREE_EINVAL, "n must be in [0, 2^31-1)");
    if (n > 0 && (!x || !y || !z)) fail(BTREE_EINVAL, "NULL coordinate array");
    if ((n + s - 1) / s > (1ll << 30)) fail(BTREE_EINVAL, "n / bucket_size must not exceed 2^30");
}

// (Re)builds the tree of t; the handle keeps its buffers.
static void do_build(Tree* t, const double* x, const double* y, const double* z, int64_t n,
                     hipStream_t st) {
    t->valid = false;
    t->n = n;
    t->p1_total = -1;
    t->p1_h = nullptr;
    t->p1_counts = nullptr;
    t->p1_offsets = nullptr;
    t->last_total = 0;
    t->n_internal = t->n_leaves = t->n_chunks = t->ctab_len = 0;
    t->depth = t->max_leaf = t->oversized = 0;
    t->root_code = kEmpty;
    t->host_stats = Stats{};
    t->timer.on = t->prm.timing != 0;
    t->stats.reserve(sizeof(Stats));
    t->timer.start(kPhBuild, st);
    if (n > 0) {
        const int64_t off[2] = {0, n};
        plan_sets(*t, 1, off, &t->prm);
        build_tree(*t, x, y, z, st);
    } else {
        BT_HIP(hipMemsetAsync(t->stats.p, 0, sizeof(Stats), st));
    }
    t->timer.stop(kPhBuild, st);
    BT_HIP(hipStreamSynchronize(st));
    t->valid = true;
}

}  // namespace bt

extern "C" {

btree_status btree_params_default(btree_params* p) {
    if (!p) {
        set_error("btree_params_default: NULL");
        return BTREE_EINVAL;
    }
    std::memset(p, 0, sizeof *p);
    p->bucket_size = 64;
    p->alpha = 0.5;
    p->beta = 0.5;
    p->max_depth = 32;
    p->precision = BTREE_FP32_FILTER;
    p->group_size = 0;
    set_error("");
    return BTREE_OK;
}

btree_status btree_build(const double* x, const double* y, const double* z, int64_t n,
                         const btree_params* p, void* hip_stream, btree_handle* out) {
    return guarded([&] {
        Range range("btree_build");
        if (!out) fail(BTREE_EINVAL, "btree_build: out is NULL");
        *out = nullptr;
        btree_params prm;
        if (p) prm = *p;
        else btree_params_default(&prm);
        check_params(prm);
        check_n(n, x, y, z, prm.bucket_size);
        btree_tree* H = new btree_tree();
        Tree* t = &H->t;
        t->prm = prm;
        if (hipGetDevice(&t->device) != hipSuccess) t->device = 0;
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        try {
            do_build(t, x, y, z, n, st);
        } catch (...) {
            (void)hipStreamSynchronize(st);
            delete H;
            throw;
        }
        *out = H;
        set_error("");
    });
}

btree_status btree_rebuild(btree_handle H, const double* x, const double* y, const double* z,
                           int64_t n, void* hip_stream) {
    return guarded([&] {
        Range range("btree_rebuild");
        if (!H) fail(BTREE_ESTATE, "btree_rebuild: NULL handle");
        Tree* t = &H->t;
        check_n(n, x, y, z, t->prm.bucket_size);
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        try {
            do_build(t, x, y, z, n, st);
        } catch (...) {
            (void)hipStreamSynchronize(st);
            t->valid = false;
            throw;
        }
        set_error("");
    });
}

btree_status btree_find_neighbors(btree_handle H, const double* h, int32_t* counts,
                                  int64_t* offsets, int32_t* nbrs, int64_t capacity,
                                  int64_t* total, void* hip_stream) {
    return guarded([&] {
        if (!H) fail(BTREE_ESTATE, "btree_find_neighbors: NULL handle");
        Tree* t = &H->t;
        if (!t->valid) fail(BTREE_ESTATE, "btree_find_neighbors: the handle holds no tree");
        if (!total) fail(BTREE_EINVAL, "btree_find_neighbors: total is NULL");
        if (!offsets) fail(BTREE_EINVAL, "btree_find_neighbors: offsets is NULL");
        if (t->n > 0 && (!h || !counts)) fail(BTREE_EINVAL, "btree_find_neighbors: NULL h or counts");
        if (capacity < 0) fail(BTREE_EINVAL, "btree_find_neighbors: capacity < 0");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        if (t->n == 0) {
            BT_HIP(hipMemsetAsync(offsets, 0, sizeof(int64_t), st));
            BT_HIP(hipStreamSynchronize(st));
            *total = 0;
            t->last_total = 0;
            set_error("");
            return;
        }
        const bool have_pass1 = t->p1_total >= 0 && t->p1_h == h && t->p1_counts == counts &&
                                t->p1_offsets == offsets;
        if (nbrs == nullptr || !have_pass1) {
            t->p1_total = -1;
            Range range("btree_find_neighbors pass 1");
            t->timer.start(kPhPass1, st);
            int64_t tot = find_pass1(*t, h, counts, offsets, st);
            t->timer.stop(kPhPass1, st);
            t->p1_h = h;
            t->p1_counts = counts;
            t->p1_offsets = offsets;
            t->p1_total = tot;
            t->last_total = tot;
        }
        *total = t->p1_total;
        if (nbrs != nullptr) {
            if (capacity < t->p1_total)
                fail(BTREE_EOVERFLOW, "btree_find_neighbors: capacity " + std::to_string(capacity) +
                                          " < total " + std::to_string(t->p1_total));
            Range range("btree_find_neighbors pass 2");
            t->timer.start(kPhPass2, st);
            find_pass2(*t, h, offsets, nbrs, st);
            t->timer.stop(kPhPass2, st);
        }
        set_error("");
    });
}

btree_status btree_density(btree_handle H, const double* h, const double* mass, double* rho,
                           int32_t* counts, void* hip_stream) {
    return guarded([&] {
        Range range("btree_density");
        if (!H) fail(BTREE_ESTATE, "btree_density: NULL handle");
        Tree* t = &H->t;
        if (!t->valid) fail(BTREE_ESTATE, "btree_density: the handle holds no tree");
        if (t->n > 0 && (!h || !rho)) fail(BTREE_EINVAL, "btree_density: NULL h or rho");
        if (t->n == 0) {
            set_error("");
            return;
        }
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        if (!counts) {
            t->aux_counts.reserve(sizeof(int32_t) * (size_t)t->n);
            counts = t->aux_counts.as<int32_t>();
        }
        t->p1_total = -1;  // a later pass 2 needs its own pass 1
        find_no_rows(*t, h, counts, mass, rho, st);
        set_error("");
    });
}

btree_status btree_adapt_h(btree_handle H, double* h, double target, double tol, int32_t max_iter,
                           int32_t* counts, int32_t* iterations, void* hip_stream) {
    return guarded([&] {
        Range range("btree_adapt_h");
        if (!H) fail(BTREE_ESTATE, "btree_adapt_h: NULL handle");
        Tree* t = &H->t;
        if (!t->valid) fail(BTREE_ESTATE, "btree_adapt_h: the handle holds no tree");
        if (t->n > 0 && !h) fail(BTREE_EINVAL, "btree_adapt_h: NULL h");
        if (!std::isfinite(target) || !(target > 0.0))
            fail(BTREE_EINVAL, "btree_adapt_h: target must be finite and > 0");
        if (!std::isfinite(tol) || tol < 0.0) fail(BTREE_EINVAL, "btree_adapt_h: tol must be finite and >= 0");
        if (max_iter < 0 || max_iter > 1000) fail(BTREE_EINVAL, "btree_adapt_h: max_iter must be in [0, 1000]");
        if (iterations) *iterations = 0;
        if (t->n == 0) {
            set_error("");
            return;
        }
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        if (!counts) {
            t->aux_counts.reserve(sizeof(int32_t) * (size_t)t->n);
            counts = t->aux_counts.as<int32_t>();
        }
        t->p1_total = -1;
        adapt_h_begin(*t, st);
        find_no_rows(*t, h, counts, nullptr, nullptr, st);
        int32_t it = 0;
        while (it < max_iter && adapt_h_step(*t, h, counts, target, tol, st) > 0) {
            ++it;
            find_no_rows(*t, h, counts, nullptr, nullptr, st);
        }
        if (iterations) *iterations = it;
        set_error("");
    });
}

btree_status btree_stats(btree_handle H, btree_stats_t* out) {
    if (!H || !out) {
        set_error("btree_stats: NULL argument");
        return BTREE_EINVAL;
    }
    Tree* t = &H->t;
    t->timer.fold_all();
    std::memset(out, 0, sizeof *out);
    out->n = t->n;
    out->n_internal = t->n_internal;
    out->n_leaves = t->n_leaves;
    out->depth = t->depth;
    out->rounds = (int64_t)t->host_stats.rounds;
    out->max_leaf = t->max_leaf;
    out->oversized = t->oversized;
    out->n_chunks = t->n_chunks;
    for (int k = 0; k < 65; ++k) out->b_hist[k] = (int64_t)t->host_stats.b_hist[k];
    out->total = t->last_total;
    out->pair_tests = (int64_t)ctr_total(t->host_stats, kCtrPairs);
    out->fp64_confirms = (int64_t)ctr_total(t->host_stats, kCtrConfirms);
    out->brute_chunks = (int64_t)ctr_total(t->host_stats, kCtrBrute);
    out->candidates = (int64_t)ctr_total(t->host_stats, kCtrCands);
    out->split_items = (int64_t)ctr_total(t->host_stats, kCtrSplit);
    out->word_items = (int64_t)ctr_total(t->host_stats, kCtrWords);
    out->word_items_wide = (int64_t)ctr_total(t->host_stats, kCtrWide);
    out->brute_units = (int64_t)t->host_ctl.nbunits;
    for (int k = 0; k < kPhases; ++k) {
        out->phase_ms[k] = t->timer.sum_ms[k];
        out->phase_calls[k] = t->timer.calls[k];
    }
    set_error("");
    return BTREE_OK;
}

btree_status btree_export(btree_handle H, int32_t* leaf_beg, int32_t* leaf_cnt,
                          int32_t* leaf_depth, int32_t* order, void* hip_stream) {
    return guarded([&] {
        if (!H) fail(BTREE_EINVAL, "btree_export: NULL handle");
        Tree* t = &H->t;
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const int64_t nl = t->n_leaves, n = t->n;
        if (n == 0) return;
        std::vector<Leaf> L((size_t)nl);
        if (leaf_beg || leaf_cnt)
            BT_HIP(hipMemcpyAsync(L.data(), t->leaves.p, sizeof(Leaf) * nl, hipMemcpyDeviceToHost, st));
        if (leaf_depth)
            BT_HIP(hipMemcpyAsync(leaf_depth, t->ldepth.p, sizeof(int32_t) * nl,
                                  hipMemcpyDeviceToHost, st));
        std::vector<double> P;
        if (order) {
            P.resize((size_t)n * 4);
            BT_HIP(hipMemcpyAsync(P.data(), t->pos.p, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, st));
        }
        BT_HIP(hipStreamSynchronize(st));
        for (int64_t l = 0; l < nl; ++l) {
            if (leaf_beg) leaf_beg[l] = L[l].beg;
            if (leaf_cnt) leaf_cnt[l] = L[l].cnt;
        }
        if (order)
            for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)P[(size_t)i * 4 + 3];
        set_error("");
    });
}

btree_status btree_destroy(btree_handle H) {
    if (!H) return BTREE_OK;
    (void)hipDeviceSynchronize();
    delete H;
    return BTREE_OK;
}

btree_status btree_find_neighbors_noalloc(const double* x, const double* y, const double* z,
                                          const double* h, int64_t n, const btree_params* p,
                                          int32_t* counts, int64_t* offsets, int32_t* nbrs,
                                          int64_t capacity, int64_t* total, void* hip_stream) {
    return guarded([&] {
        Range range("btree_find_neighbors_noalloc");
        if (!total) fail(BTREE_EINVAL, "btree_find_neighbors_noalloc: total is NULL");
        if (n < 0 || n > BTREE_NOALLOC_MAX_N)
            fail(BTREE_EINVAL, "btree_find_neighbors_noalloc: n = " + std::to_string(n) +
                                   " is outside [0, " + std::to_string(BTREE_NOALLOC_MAX_N) + "]");
        if (!offsets) fail(BTREE_EINVAL, "btree_find_neighbors_noalloc: offsets is NULL");
        if (n > 0 && (!h || !counts))
            fail(BTREE_EINVAL, "btree_find_neighbors_noalloc: NULL h or counts");
        if (capacity < 0 || (capacity > 0 && !nbrs))
            fail(BTREE_EINVAL, "btree_find_neighbors_noalloc: bad capacity or NULL nbrs");
        btree_params prm;
        if (p) prm = *p;
        else btree_params_default(&prm);
        check_params(prm);
        if (prm.timing) fail(BTREE_EINVAL, "btree_find_neighbors_noalloc: timing must be 0");
        check_n(n, x, y, z, prm.bucket_size);
        int dev = 0;
        BT_HIP(hipGetDevice(&dev));
        if (dev < 0 || dev >= kMaxDevices)
            fail(BTREE_EDEVICE, "btree_find_neighbors_noalloc: device id above 63");
        std::lock_guard<std::mutex> lock(g_noalloc_mu[dev]);
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        Arena arena;
        arena.base = noalloc_scratch(dev);
        arena.size = kNoAllocBytes;
        ArenaScope scope(&arena);
        // Every buffer of this tree is carved from the scratch; the tree's
        // host side lives on this call's stack.
        Tree t;
        t.prm = prm;
        t.device = dev;
        try {
            do_build(&t, x, y, z, n, st);
            if (n == 0) {
                BT_HIP(hipMemsetAsync(offsets, 0, sizeof(int64_t), st));
                *total = 0;
            } else {
                const int64_t tot = find_pass1(t, h, counts, offsets, st);
                *total = tot;
                if (capacity < tot)
                    fail(BTREE_EOVERFLOW, "btree_find_neighbors_noalloc: capacity " +
                                              std::to_string(capacity) + " < total " +
                                              std::to_string(tot));
                find_fill(t, counts, offsets, nbrs, capacity, nullptr, false, st);
            }
            // The next call on this device reuses the scratch.
            BT_HIP(hipStreamSynchronize(st));
        } catch (...) {
            (void)hipStreamSynchronize(st);
            throw;
        }
        set_error("");
    });
}

btree_status btree_tune_space_default(btree_tune_space* sp) {
    if (!sp) {
        set_error("btree_tune_space_default: NULL");
        return BTREE_EINVAL;
    }
    std::memset(sp, 0, sizeof *sp);
    const int32_t s[] = {16, 24, 32, 48, 64, 96, 128, 192, 256};
    sp->n_bucket = (int32_t)(sizeof s / sizeof s[0]);
    for (int k = 0; k < sp->n_bucket; ++k) sp->bucket[k] = s[k];
    const double b[] = {0.3, 0.5, 0.8};
    sp->n_beta = 3;
    for (int k = 0; k < 3; ++k) sp->beta[k] = b[k];
    const double a[] = {0.25, 0.5, 1.0};
    sp->n_alpha = 3;
    for (int k = 0; k < 3; ++k) sp->alpha[k] = a[k];
    sp->repeats = 3;
    set_error("");
    return BTREE_OK;
}

const char* btree_last_error(void) { return get_error(); }

}  // extern "C"

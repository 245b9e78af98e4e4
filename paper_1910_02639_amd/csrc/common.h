// Internal definitions shared by the HIP sources of libbtree (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>
#include <vector>

#include "btree.h"

namespace bt {

// ---------------------------------------------------------------------------
// Error plumbing: status codes out of the ABI, a thread-local message.
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* get_error();

struct Fail {
    btree_status code;
};

#define BT_HIP(call)                                                         \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) {                                              \
            ::bt::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            throw ::bt::Fail{e_ == hipErrorOutOfMemory ? BTREE_ENOMEM        \
                                                       : BTREE_EDEVICE};     \
        }                                                                    \
    } while (0)

#define BT_LAUNCH()                                                          \
    do {                                                                     \
        hipError_t e_ = hipGetLastError();                                   \
        if (e_ != hipSuccess) {                                              \
            ::bt::set_error(std::string("kernel launch: ") + hipGetErrorString(e_)); \
            throw ::bt::Fail{BTREE_EDEVICE};                                 \
        }                                                                    \
    } while (0)

[[noreturn]] inline void fail(btree_status code, const std::string& msg) {
    set_error(msg);
    throw Fail{code};
}

// Device buffer owned by a handle; grows on demand, never shrinks.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void reserve(size_t want) {
        if (want <= bytes) return;
        release();
        size_t b = want < 256 ? 256 : want;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            fail(e == hipErrorOutOfMemory ? BTREE_ENOMEM : BTREE_EDEVICE,
                 "hipMalloc of " + std::to_string(b) + " bytes: " + hipGetErrorString(e));
        }
        bytes = b;
    }
    // Grows to at least `want` bytes keeping the first `keep` bytes.
    void grow(size_t want, size_t keep, hipStream_t st) {
        if (want <= bytes) return;
        size_t b = want + want / 2;
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, b);
        if (e != hipSuccess)
            fail(e == hipErrorOutOfMemory ? BTREE_ENOMEM : BTREE_EDEVICE,
                 "hipMalloc of " + std::to_string(b) + " bytes: " + hipGetErrorString(e));
        if (p && keep) {
            e = hipMemcpyAsync(q, p, keep, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                (void)hipFree(q);
                fail(BTREE_EDEVICE, std::string("grow copy: ") + hipGetErrorString(e));
            }
        }
        release();
        p = q;
        bytes = b;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// Tree layout in HBM.
// ---------------------------------------------------------------------------
constexpr int32_t kEmpty = -1;         // child-table entry of an empty sub-cell
constexpr int32_t kLeafBit = 1 << 30;  // child-table entry flag: a leaf id

// An internal cell (split by Algorithm 1).  72 bytes.
struct Node {
    double lo[3];      // cell box
    double hi[3];
    int64_t ctab;      // offset of its dense b^3 child table (Eq. 3 order)
    int32_t b;         // branching factor per axis
    int32_t n;         // particles in the cell
    int32_t beg;       // first particle of the cell's segment
    int32_t depth;     // root = 0
};

struct Leaf {
    int32_t beg;       // first particle (sorted order)
    int32_t cnt;       // particles
};

// A search work item: up to kGroup consecutive particles of one leaf.
struct Chunk {
    int32_t beg;
    int32_t cnt;
};

constexpr int kGroup = 64;  // queries per work item (one per lane)

struct Stats {  // device-side counters
    unsigned long long rounds;
    unsigned long long pair_tests;
    unsigned long long confirms;
    unsigned long long brute;
    unsigned long long candidates;
    unsigned long long b_hist[65];
};

// Build workspace, kept by the handle so that rebuilds reuse its memory.
struct Work {
    DBuf P0, P1, pn0, pn1, part;
    DBuf hsize, hoff, hist, cstart, crank, cursor, bsel, selofs, nint, nleaf, ibase, lbase,
        ctsize, ctoff;
    DBuf mark, f, rank, l2, d2, newid, nc, coff;
    DBuf mk0, mk1, mv0, mv1, rcnt, roff;  // Morton sort
};

// Phases timed with HIP events when btree_params.timing is set.
enum Phase { kPhBuild = 0, kPhSweep = 1, kPhPlace = 2, kPhPass1 = 3, kPhPass2 = 4, kPhases = 5 };

struct Timer {
    hipEvent_t ev[kPhases][2] = {};
    bool pending[kPhases] = {};
    double sum_ms[kPhases] = {};
    int64_t calls[kPhases] = {};
    bool on = false;
    void fold(int ph) {
        if (!pending[ph]) return;
        float ms = 0.f;
        if (hipEventSynchronize(ev[ph][1]) == hipSuccess &&
            hipEventElapsedTime(&ms, ev[ph][0], ev[ph][1]) == hipSuccess) {
            sum_ms[ph] += ms;
            calls[ph] += 1;
        }
        pending[ph] = false;
    }
    void start(int ph, hipStream_t st) {
        if (!on) return;
        fold(ph);
        if (!ev[ph][0]) {
            (void)hipEventCreate(&ev[ph][0]);
            (void)hipEventCreate(&ev[ph][1]);
        }
        (void)hipEventRecord(ev[ph][0], st);
    }
    void stop(int ph, hipStream_t st) {
        if (!on) return;
        (void)hipEventRecord(ev[ph][1], st);
        pending[ph] = true;
    }
    void fold_all() {
        for (int k = 0; k < kPhases; ++k) fold(k);
    }
    ~Timer() {
        for (int k = 0; k < kPhases; ++k)
            for (int j = 0; j < 2; ++j)
                if (ev[k][j]) (void)hipEventDestroy(ev[k][j]);
    }
};

// The handle.
struct Tree {
    int64_t n = 0;
    bool valid = false;  // a tree is built
    btree_params prm{};
    int device = 0;

    DBuf pos;      // double4 per particle, tree order: x, y, z, (double)orig
    DBuf orig;     // double4 per particle, original order: x, y, z, 0
    DBuf nodes;    // Node[n_internal]
    DBuf ctab;     // int32 child tables
    DBuf leaves;   // Leaf[n_leaves], memory order
    DBuf ldepth;   // int32 per leaf
    DBuf lrange;   // int2 per leaf: smallest and largest original index
    DBuf chunks;   // Chunk[n_chunks]
    DBuf stats;    // Stats
    DBuf flag;     // int32 device flag (invalid data)
    DBuf cflag;    // int32 per chunk: exhaustive path needed
    DBuf scan_tmp; // scan block sums
    DBuf scal;     // small scalars (int64 total etc.)
    DBuf scratch;  // int32 rows of the search, in work-item order
    DBuf soff;     // int64 per particle: row start in scratch (-1: exhaustive path)
    Work ws;
    Timer timer;

    int64_t n_internal = 0, n_leaves = 0, n_chunks = 0, ctab_len = 0;
    int64_t scap = 0;  // scratch capacity, entries
    int64_t depth = 0, max_leaf = 0, oversized = 0;
    int32_t root_code = kEmpty;
    double rootbox[6] = {0, 0, 0, 0, 0, 0};
    Stats host_stats{};

    // pass-1 memory for pass 2
    const double* p1_h = nullptr;
    int32_t* p1_counts = nullptr;
    int64_t* p1_offsets = nullptr;
    int64_t p1_total = -1;
    int64_t last_total = 0;
};

// ---------------------------------------------------------------------------
// Helpers shared by build and search kernels.
// ---------------------------------------------------------------------------

// Eq. 2: sub-cell coordinate of x within [lo, hi] cut into b parts, clamped
// to [0, b-1]; a zero extent maps to 0.  The same function assigns particles
// at build time and computes the Eq. 5 range at search time, which makes the
// range complete: it is monotone in x, so fl(x_i - 2h) <= x_j <= fl(x_i + 2h)
// puts x_j's sub-cell inside the range.
__host__ __device__ inline int subcell(double x, double lo, double hi, int b) {
    double w = hi - lo;
    if (!(w > 0.0)) return 0;
    double t = (x - lo) / w;
    double v = floor(t * (double)b);
    if (v < 0.0) return 0;
    if (v > (double)(b - 1)) return b - 1;
    return (int)v;
}

// Box of sub-cell c along one axis: lo + (w*c)/b .. lo + (w*(c+1))/b.
__host__ __device__ inline double cell_edge(double lo, double hi, int c, int b) {
    double w = hi - lo;
    return lo + (w * (double)c) / (double)b;
}

// Eq. 1 evaluated exactly: smallest b >= 1 with b^3 * s >= n.
__host__ __device__ inline int branching(int64_t n, int64_t s) {
    double g = cbrt((double)n / (double)s);
    int64_t b = (int64_t)g;
    if (b < 1) b = 1;
    while (b > 1 && (b - 1) * (b - 1) * (b - 1) * s >= n) --b;
    while (b * b * b * s < n) ++b;
    return (int)b;
}

// Next branching factor of the halving loop (Eq. 4 step): max(2, b/2).
__host__ __device__ inline int halve(int b) { return b / 2 < 2 ? 2 : b / 2; }

// Spread the low 10 bits of v to every third bit (Morton interleave).
__host__ __device__ inline uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__host__ __device__ inline uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0x030000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}

// Spread the low 21 bits of v to every third bit of a 64-bit word.
__host__ __device__ inline uint64_t spread3_64(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__host__ __device__ inline uint64_t compact3_64(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return v;
}

// Host-side helpers implemented in the .hip sources.
// Exclusive prefix sums, out[n] = total.  When guard is non-null and *guard
// is set on the device, nothing is written to out.
void scan_exclusive_i32(const int32_t* in, int64_t* out, int64_t n, Tree& t,
                        hipStream_t st, const int* guard = nullptr);
void scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, Tree& t,
                        hipStream_t st, const int* guard = nullptr);

void radix_sort_pairs(uint32_t* k0, int32_t* v0, uint32_t* k1, int32_t* v1, int64_t n, int bits,
                      Tree& t, DBuf& cnt, DBuf& off, hipStream_t st);
void build_tree(Tree& t, const double* x, const double* y, const double* z,
                hipStream_t st);
int64_t find_pass1(Tree& t, const double* h, int32_t* counts, int64_t* offsets,
                   hipStream_t st);
void find_pass2(Tree& t, const double* h, const int64_t* offsets, int32_t* nbrs,
                hipStream_t st);

inline unsigned grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 0x7fffffff) g = 0x7fffffff;
    return (unsigned)g;
}

}  // namespace bt

// Internal definitions shared by the HIP sources of libbtree (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

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

// A named roctx range over a scope (a phase of an entry point), seen by
// rocprofv3 --marker-trace; inert when no tool is attached.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

[[noreturn]] inline void fail(btree_status code, const std::string& msg) {
    set_error(msg);
    throw Fail{code};
}

// A device region that buffers are carved from instead of hipMalloc: a bump
// allocator over [base, base + size), for the entry point that allocates no
// device memory.  Nothing carved is ever freed; the region is reused from
// its start by the next call.
struct Arena {
    char* base = nullptr;  // device address of the region
    size_t size = 0;       // bytes
    size_t used = 0;       // bytes handed out so far
};

// The arena this host thread's buffers come from, or null (hipMalloc).
Arena*& current_arena();

inline void* arena_take(Arena* a, size_t b) {
    const size_t at = (a->used + 255) & ~(size_t)255;
    if (at > a->size || b > a->size - at)
        fail(BTREE_ENOMEM, "the no-allocation scratch (" + std::to_string(a->size) +
                               " bytes) is exhausted: " + std::to_string(b) +
                               " more bytes needed after " + std::to_string(a->used));
    a->used = at + b;
    return a->base + at;
}

// hipMalloc behind a fault hook for tests of the allocation-failure paths:
// while the environment variable BTREE_FAULT_ALLOC holds k >= 1, the k-th
// device allocation counted from the last change of its value fails with
// BTREE_ENOMEM (later ones succeed).  Unset or not a positive integer: no
// effect.
inline void device_malloc(void** p, size_t b) {
    static std::mutex mu;
    static std::string seen;
    static long long count = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        const char* v = std::getenv("BTREE_FAULT_ALLOC");
        const std::string now = v ? v : "";
        if (now != seen) {
            seen = now;
            count = 0;
        }
        const long long k = v ? std::atoll(v) : 0;
        if (k > 0 && ++count == k) {
            *p = nullptr;
            fail(BTREE_ENOMEM, "device allocation " + std::to_string(k) + " of " +
                                   std::to_string(b) + " bytes failed by BTREE_FAULT_ALLOC");
        }
    }
    hipError_t e = hipMalloc(p, b);
    if (e != hipSuccess) {
        *p = nullptr;
        fail(e == hipErrorOutOfMemory ? BTREE_ENOMEM : BTREE_EDEVICE,
             "hipMalloc of " + std::to_string(b) + " bytes: " + hipGetErrorString(e));
    }
}

// Device buffer owned by a handle; grows on demand, never shrinks.  While
// an arena is current on the host thread, memory is carved from it (and
// `borrowed`: never freed).
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p && !borrowed) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        borrowed = false;
    }
    void reserve(size_t want) {
        if (want <= bytes) return;
        release();
        size_t b = want < 256 ? 256 : want;
        if (Arena* a = current_arena()) {
            p = arena_take(a, b);
            bytes = b;
            borrowed = true;
            return;
        }
        device_malloc(&p, b);
        bytes = b;
    }
    // Grows to at least `want` bytes keeping the first `keep` bytes.
    void grow(size_t want, size_t keep, hipStream_t st) {
        if (want <= bytes) return;
        size_t b = want + want / 2;
        void* q = nullptr;
        Arena* a = current_arena();
        if (a) {
            q = arena_take(a, b);
        } else {
            device_malloc(&q, b);
        }
        if (p && keep) {
            hipError_t e = hipMemcpyAsync(q, p, keep, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                if (!a) (void)hipFree(q);
                fail(BTREE_EDEVICE, std::string("grow copy: ") + hipGetErrorString(e));
            }
        }
        release();
        p = q;
        bytes = b;
        borrowed = a != nullptr;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// Tree layout in HBM.
// ---------------------------------------------------------------------------
constexpr int32_t kEmpty = -1;         // child-table entry of an empty sub-cell
constexpr int32_t kLeafBit = 1 << 30;  // child-table entry flag: a leaf id

// An internal cell (split by Algorithm 1).  80 bytes.
struct Node {
    double lo[3];      // cell box
    double hi[3];
    int64_t ctab;      // offset of its dense b^3 child table (Eq. 3 order)
    int32_t b;         // branching factor per axis
    int32_t n;         // particles in the cell
    int32_t beg;       // first particle of the cell's segment
    int32_t depth;     // root = 0
    int32_t set;       // particle set the cell belongs to
    int32_t pad;
};

struct Leaf {
    int32_t beg;       // first particle (sorted order)
    int32_t cnt;       // particles
};

// A search work item: up to kGroup consecutive particles of one leaf.
struct Chunk {
    int32_t beg;
    int32_t cnt;
    int32_t set;
    int32_t pad;
};

constexpr int kGroup = 64;  // queries per work item (one per lane)


// One independent particle set (a batch holds several, a tree one).
struct SetDev {
    int64_t beg;       // first particle, original and sorted numbering
    int64_t n;         // particles
    double alpha, beta;
    int32_t s;         // bucket size
    int32_t max_depth;
    int32_t root;      // child code of the root cell (node id, leaf id | kLeafBit, or kEmpty)
    int32_t octree;    // 1: b = 2 at every split (no Eq. 1 / Eq. 4)
    double box[6];     // root box: lo x, y, z, hi x, y, z
};

// First branching factor tried for a cell of n particles of set S: Eq. 1,
// or 2 for the octree.
__host__ __device__ inline int branching(int64_t n, int64_t s);
__host__ __device__ inline int first_branching(int64_t n, const SetDev& S) {
    return S.octree ? 2 : branching(n, S.s);
}

// Tiles of at most kTileN particles, never straddling two sets.
struct Tile {
    int32_t set;
    int32_t pad;
    int64_t beg, end;
};
constexpr int64_t kTileN = 8192;

// Overflow bits of Ctl::overflow (a pool was too small for this input).
enum { kOvfNodes = 1, kOvfLeaves = 2, kOvfCtab = 4, kOvfHist = 8, kOvfLevels = 16,
       kOvfScratch = 32, kOvfCapacity = 64, kOvfChunks = 128, kOvfWalk = 256 };
// A build that overflowed a pool left an incomplete tree: the search must
// not walk it.  Work items beyond the launched grid leave counts unset: the
// lists must not be placed.
constexpr int kOvfTree = kOvfNodes | kOvfLeaves | kOvfCtab | kOvfHist | kOvfLevels;

// Device control block of a build and its search: every level reads its
// cell range from here, so no host round trip is needed between launches.
struct Ctl {
    int32_t cur_nb, cur_ne;     // cells of the level being split
    int32_t lvm;                // cur_ne - cur_nb (a device length for scans)
    uint32_t nsplit;            // work items split for overflowing (atomic)
    int32_t next_nb, next_ne;   // cells of the next level
    int32_t n_nodes, n_leaves;  // allocated so far
    int64_t ct_len;             // child-table entries allocated
    int64_t hist_len;           // histogram entries of the current level
    int32_t lv_int0, lv_leaf0;  // first node / leaf id given to this level's children
    int64_t lv_ct0;             // first child-table entry of this level
    int32_t level_ok;           // the current level fits its pools
    int32_t overflow;           // kOvf* bits
    int32_t data_bad;           // non-finite coordinate or h
    int32_t n_chunks;           // search work items
    int32_t depth;              // deepest leaf
    int32_t max_leaf;           // largest leaf
    int32_t oversized;          // leaves above their set's s
    int32_t levels;             // levels that had cells to split
    uint32_t queue;             // next search work item (atomic)
    uint32_t nbrute;            // work items on the exhaustive path (atomic)
    uint32_t nsplit2, nsplit3;  // units left for the second and third split levels (atomic)
    uint32_t split_take[3];     // next unit of each split level to start (atomic)
    uint32_t nbunits;           // exhaustive-path units after regrouping by set
    uint32_t nbtasks;           // exhaustive count-pass tasks (unit x span of its set)
    int64_t bspan;              // candidates per exhaustive count-pass task
    int32_t bfill_tasks;        // 1: the exhaustive fill pass also runs by tasks
    uint32_t nadapt;            // h adaptation: particles whose h changed (atomic)
};

// Allocation from the search's pools (row scratch, walk lists) goes through
// kStripes independent cursors, one per 128-byte line, each over its own
// 1/kStripes of the pool: one counter shared by every workgroup of the chip
// would serialise its atomics.
constexpr int kStripes = 64;
constexpr int64_t kDenseTaskCap = 16384;  // exhaustive tasks whose counts the fill pass reuses
constexpr int kStripeStride = 16;  // uint64 per cursor slot

// Device-side counters.  The search's counters are added to once per work
// item, so they are striped like the cursors (work item -> stripe_of its
// first particle): one line shared by every workgroup serialises their
// atomics, which then bound the whole sweep.  The host sums the stripes.
enum { kCtrPairs = 0, kCtrCands, kCtrConfirms, kCtrBrute, kCtrSplit, kCtrWords, kCtrWide,
       kCtrCount };
struct Stats {
    unsigned long long rounds;
    unsigned long long b_hist[65];
    alignas(128) unsigned long long ctr[kStripes][kStripeStride];
};
static_assert(kCtrCount <= kStripeStride, "counters must fit a stripe's line");

inline unsigned long long ctr_total(const Stats& s, int k) {
    unsigned long long v = 0;
    for (int i = 0; i < kStripes; ++i) v += s.ctr[i][k];
    return v;
}

constexpr int kPersistBlocks = 2048;  // grid of the persistent per-cell / per-item kernels

// Build workspace, kept by the handle so that rebuilds reuse its memory.
struct Work {
    DBuf P0, P1, part;
    DBuf tcnt, toff;  // per cell of a level: particle chunks, and their offsets
    DBuf hsize, hoff, hist, cstart, crank, cursor, bsel, selofs, nint, nleaf, ibase, lbase,
        ctsize, ctoff;
    DBuf mark, f, rank, newid, nc, coff;
    DBuf mk0, mk1, mv0, mv1, rcnt, roff;  // Morton sort
    DBuf tiles, settile;                   // ingest tiles and their first tile per set
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
    DBuf leaves2, ldepth2;  // the other copy (leaf renumbering ping-pongs)
    DBuf sets;     // SetDev[nsets]
    DBuf ctl;      // Ctl
    DBuf tot;      // int64 per set boundary: offsets at set starts (batch totals)
    DBuf lrange;   // int2 per leaf: smallest and largest original index
    DBuf chunks;   // Chunk[n_chunks]
    DBuf stats;    // Stats
    DBuf split;    // three lists of Chunk (leaf_cap each): units of the split levels
    DBuf split_ci; // int32 per entry of the first list: the work item it came from
    DBuf blist;    // Chunk per unit (1 to 64 queries of one set) listed for the exhaustive path
    DBuf bq;       // tree positions of the exhaustive path's queries, grouped by set
    DBuf bset;     // per set: listed queries, fill cursor, query, unit and count-task offsets
    DBuf btab;     // per exhaustive count task and lane: the lane's hits in the task's span
    DBuf scan_tmp; // scan block sums
    DBuf scratch;  // int32 rows of the search, in work-item order
    DBuf soff;     // int64 per particle: row start in scratch (-1: exhaustive path)
    DBuf stripes;  // uint64 cursors: kStripes for the scratch, then kStripes for the walk lists
    DBuf hs;       // double per particle: h in tree order (filled by each search)
    DBuf whdr;     // int4 per work item: walk result header
    DBuf ibox;     // per work item: box E and the FP32 filter's item-wide bounds (64 bytes)
    DBuf irec;     // per work item: where pass 1 left its test words and candidates
    DBuf wl;       // int2 pool: candidate leaves (first particle, count) of every item
    DBuf aux_counts;  // int32 per particle, when a caller passes no counts buffer
    DBuf adapt_br;    // double2 per particle: bracket (lo, hi) of the h adaptation
    Work ws;
    Timer timer;

    int64_t n_internal = 0, n_leaves = 0, n_chunks = 0, ctab_len = 0;
    int64_t scap = 0;  // scratch capacity, entries
    int64_t chunk_cap = 0;  // work items a captured search launches for
    int64_t sweep_cap = 0;  // item bound of the last rows pass 1 (its pass 2 uses the same)
    int64_t wl_cap = 0;     // entries of the walk-list pool
    int64_t wl_need = 0;    // pool size the last walk needed, when the pool was too small
    unsigned long long host_stripes[2 * kStripes * kStripeStride] = {};
    // sets and pool capacities
    int32_t nsets = 1;
    std::vector<int64_t> set_off;        // nsets + 1, host
    std::vector<btree_params> set_prm;   // per set
    int64_t ntiles = 0;
    int64_t node_cap = 0, ctab_cap = 0, hist_cap = 0, leaf_cap = 0, level_cap = 0;
    int32_t levels_seen = 0;
    Ctl host_ctl{};
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
    if (!(v >= 0.0)) return 0;  // below the box (or not a number)
    if (v > (double)(b - 1)) return b - 1;
    return (int)v;
}

// subcell() in two steps, for several b on one cell: the fraction
// t = (x - lo) / w does not depend on b (0 for a zero extent, which then
// maps to sub-cell 0 as above), and subcell_of(t, b) equals
// subcell(x, lo, hi, b) bit for bit.
__host__ __device__ inline double subcell_frac(double x, double lo, double hi) {
    double w = hi - lo;
    if (!(w > 0.0)) return 0.0;
    return (x - lo) / w;
}

__host__ __device__ inline int subcell_of(double t, int b) {
    double v = floor(t * (double)b);
    if (!(v >= 0.0)) return 0;
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
void scan_reserve(Tree& t, int64_t ncap);
// Two or three device-length int64 scans of one length in one launch
// sequence; need scan_reserve(t, 3 * ncap + 4 * 2048).
void scan2_dev_i64(const int64_t* in0, int64_t* out0, const int64_t* in1, int64_t* out1,
                   const int32_t* nptr, int64_t ncap, Tree& t, hipStream_t st);
void scan3_dev_i64(const int64_t* in0, int64_t* out0, const int64_t* in1, int64_t* out1,
                   const int64_t* in2, int64_t* out2, const int32_t* nptr, int64_t ncap,
                   Tree& t, hipStream_t st);
void scan_dev_i32(const int32_t* in, int64_t* out, const int32_t* nptr, int64_t ncap, Tree& t,
                  hipStream_t st);
void scan_dev_i64(const int64_t* in, int64_t* out, const int32_t* nptr, int64_t ncap, Tree& t,
                  hipStream_t st);

// Sets the handle up for nsets sets (offsets on the host) and sizes all pools.
void plan_sets(Tree& t, int32_t nsets, const int64_t* set_off, const btree_params* prm);
// Queues BuildTree of every set; `levels` level groups (no host reads when
// eager is false).  With eager, the host stops as soon as a level is empty.
void build_queue(Tree& t, const double* x, const double* y, const double* z, int levels,
                 bool eager, hipStream_t st);
// Eager build: queue, wait, grow pools and redo on overflow.
void build_tree(Tree& t, const double* x, const double* y, const double* z,
                hipStream_t st);
// Steps of the search, each queued without host reads (a captured graph
// may hold them): reset and h check; the sweep over `grid` work items;
// exhaustive counts and the offsets scan; placement of the rows into nbrs
// of `capacity` entries (nothing written if they do not fit); exhaustive
// rows and per-set totals (when `totals` is non-null).
void find_begin(Tree& t, const double* h, hipStream_t st);
void find_walk(Tree& t, const double* h, int64_t grid, hipStream_t st);
void find_sweep(Tree& t, const double* h, int32_t* counts, int64_t grid, hipStream_t st);
void find_counts_end(Tree& t, const double* h, int32_t* counts, int64_t* offsets, hipStream_t st);
void find_place(Tree& t, const int32_t* counts, const int64_t* offsets, int32_t* nbrs,
                int64_t capacity, hipStream_t st);
void find_fill(Tree& t, const int32_t* counts, const int64_t* offsets, int32_t* nbrs,
               int64_t capacity, int64_t* totals, bool time_place, hipStream_t st);
// Sizes the search scratch for at least `entries` list entries.
void find_reserve(Tree& t, int64_t entries);
// Grows the scratch and walk-list pools from the stripe cursors in
// t.host_stripes after a search reported these overflow bits.
void grow_pools(Tree& t, int overflow);
int64_t find_pass1(Tree& t, const double* h, int32_t* counts, int64_t* offsets,
                   hipStream_t st);
// A search pass that writes counts (rho null) or counts and the fused SPH
// densities (mass null: unit masses), no rows; synchronises the stream.
void find_no_rows(Tree& t, const double* h, int32_t* counts, const double* mass, double* rho,
                  hipStream_t st);
// The h adaptation: brackets cleared, then one round per call on counts
// taken at h (original order); a round returns how many h changed
// (synchronises the stream).
void adapt_h_begin(Tree& t, hipStream_t st);
int64_t adapt_h_step(Tree& t, double* h, const int32_t* counts, double target, double tol,
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

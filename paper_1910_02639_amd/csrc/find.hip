// FindNeighbors on the device (Section 3.2, Algorithm 2, Eq. 5).
//
// Work item: up to 64 consecutive particles of one leaf (the paper's
// blocked, cache-reusing search, recast for a GPU: a leaf's particles share
// one tree walk and one staged candidate set).  Pass 1 writes every query's
// count and keeps each item's result in a scratch buffer (its test words and
// ordered candidates, or its rows, whichever is smaller); pass 2 puts the
// rows into the caller's CSR arrays once the offsets are known.
//
//  1. k_walk, one wavefront per item: box E = [min_i fl(x_i - 2h_i),
//     max_i fl(x_i + 2h_i)]; walk (Algorithm 2 with Eq. 5 applied to E),
//     breadth first: each internal cell's sub-cell range on every axis is
//     [f(E_lo), f(E_hi)] with the build's own Eq. 2 function f.  The
//     candidate leaves go to a pool in global memory, E and the FP32
//     filter's item-wide bounds to a record per item; the walk also checks
//     that h is finite and >= 0.
//  2. k_sweep, one workgroup of 4 wavefronts per item (lane q of every
//     wavefront holds query q): the particles of the candidate leaves that
//     lie inside E are staged into LDS (every true neighbour of every query
//     lies inside E) and put in original index order; wavefront w sweeps
//     its quarter of them for its 64 queries (LDS reads broadcast to all
//     lanes), one bit per (query, candidate); the item then stores its
//     words and candidates, or each lane writes its row in ascending index,
//     to the scratch.
//  3. Items whose candidates do not fit the LDS budget are searched again
//     by k_sweep_split (the whole item with a larger budget, then parts of
//     8 queries, then single queries), and what still does not fit by an
//     exhaustive FP64 sweep of the query's set in index order (k_dense).
//  4. Pass 2: k_expand expands the items' words into the CSR rows (through
//     a shared-memory image of each item's rows, copied out row by row);
//     k_place copies the rows kept in the scratch.
//
// Two arithmetic forms of the pair test, with identical results:
//  * FP64: the exact predicate ((dx*dx + dy*dy) + dz*dz) < (2h)*(2h).
//  * FP32 filter: coordinates relative to the centre c of E, a = fl32(x_i
//    - c), b = fl32(x_j - c), t = fl32(a - b), D = fl32(|t|^2).  With
//    per-axis bounds S_l >= |x_i - c| + |x_j - c|, the staging error per
//    axis is at most u'*S_l (u' = 2^-24 + 2^-52), so |t| is within
//    eta = u'*|S| of |x_i - x_j| up to a relative u, and D within gamma_3
//    of |t|^2.  The FP64 predicate can only differ from the real one inside
//    |x_i - x_j|^2 in R^2 (1 -/+ 8 v), v = 2^-53.  Hence
//        D < T_lo = (1 - g3)(1 - u)^2 (R(1 - 2^-48) - eta)_+^2  => neighbour
//        D > T_hi = (1 + g3)(1 + u)^2 (R(1 + 2^-48) + eta)^2    => not one
//    (thresholds rounded outwards to FP32, with an absolute slack of
//    8*2^-126 for flushed subnormals); pairs in between are decided by the
//    FP64 predicate on the original coordinates.  Items whose spread or
//    radius reaches 2^60 (where FP32 squares could overflow) take FP64
//    arithmetic.
//    The words of the main test fold the threshold into the sum: with
//    T = fl32(R^2), E = fl(tz^2 + fl(ty^2 + fl(tx^2 - T))) (three FMAs) is
//    within kap (|t|^2 + T) + ea of |t|^2 - T (kap = 3u (1 + 2^-20)), so a
//    margin M (set-up in sweep_item) makes E < -M certify a neighbour and
//    E >= M a non-neighbour; the bit is E's sign bit and a word whose
//    smallest |E| is at most M is classified again candidate by candidate.
#include "prim.h"

#include <algorithm>
#include <cfloat>

namespace bt {

namespace {

constexpr int kWG = 256;
constexpr int kWaves = kWG / 64;
constexpr int kLMax = 512;   // candidate leaves per item
constexpr int kSMax = 256;   // walk stack entries
constexpr int kCMax = 1536;  // staged candidates per item (both forms)
// An item of the main sweep leaves its test words for k_expand when
// their size times kBitsNum / kBitsDen is below the size of its rows.
constexpr int kBitsNum = 1, kBitsDen = 1;
constexpr int kRowBuf = 8192;  // entries of k_expand's shared-memory row image
constexpr int kBuckets = 256;       // original-index buckets of the staged list
constexpr int kBucketSortMax = 48;  // a fuller bucket sorts the whole item instead

enum { kCount = 0, kFill = 1, kDens = 2 };  // exhaustive path: count, rows, density

// The FP64 predicate of the method, every operation rounded.
__device__ __forceinline__ bool p64(double xi, double yi, double zi, double R, double xj,
                                    double yj, double zj) {
    double dx = __dsub_rn(xi, xj);
    double dy = __dsub_rn(yi, yj);
    double dz = __dsub_rn(zi, zj);
    double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    return d2 < __dmul_rn(R, R);
}

// Bit accumulation of the pair tests: word = 2*word + (d < lo) and
// lword = 2*lword + (d < hi) for four consecutive candidates, with one
// compare and one add-with-carry per bit (the compare's lane mask is the
// carry-in).  All eight compares are issued before the first add so every
// mask is read at least six instructions after it is written.
__device__ __forceinline__ void push4_f32(uint32_t& word, uint32_t& lword, float d0, float d1,
                                          float d2, float d3, float lo, float hi) {
    uint64_t m0, m1, m2, m3, n0, n1, n2, n3, c;
    asm volatile(
        "v_cmp_lt_f32_e64 %[m0], %[d0], %[lo]\n\t"
        "v_cmp_lt_f32_e64 %[n0], %[d0], %[hi]\n\t"
        "v_cmp_lt_f32_e64 %[m1], %[d1], %[lo]\n\t"
        "v_cmp_lt_f32_e64 %[n1], %[d1], %[hi]\n\t"
        "v_cmp_lt_f32_e64 %[m2], %[d2], %[lo]\n\t"
        "v_cmp_lt_f32_e64 %[n2], %[d2], %[hi]\n\t"
        "v_cmp_lt_f32_e64 %[m3], %[d3], %[lo]\n\t"
        "v_cmp_lt_f32_e64 %[n3], %[d3], %[hi]\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m0]\n\t"
        "v_addc_co_u32_e64 %[l], %[c], %[l], %[l], %[n0]\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m1]\n\t"
        "v_addc_co_u32_e64 %[l], %[c], %[l], %[l], %[n1]\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m2]\n\t"
        "v_addc_co_u32_e64 %[l], %[c], %[l], %[l], %[n2]\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m3]\n\t"
        "v_addc_co_u32_e64 %[l], %[c], %[l], %[l], %[n3]"
        : [w] "+v"(word), [l] "+v"(lword), [m0] "=&s"(m0), [m1] "=&s"(m1), [m2] "=&s"(m2),
          [m3] "=&s"(m3), [n0] "=&s"(n0), [n1] "=&s"(n1), [n2] "=&s"(n2), [n3] "=&s"(n3),
          [c] "=&s"(c)
        : [d0] "v"(d0), [d1] "v"(d1), [d2] "v"(d2), [d3] "v"(d3), [lo] "v"(lo), [hi] "v"(hi));
}

// One candidate (tails of a block): same bits, two wait states spelled out.
__device__ __forceinline__ void push1_f32(uint32_t& word, uint32_t& lword, float d, float lo,
                                          float hi) {
    uint64_t m, n, c;
    asm volatile(
        "v_cmp_lt_f32_e64 %[m], %[d], %[lo]\n\t"
        "v_cmp_lt_f32_e64 %[n], %[d], %[hi]\n\t"
        "s_nop 1\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m]\n\t"
        "v_addc_co_u32_e64 %[l], %[c], %[l], %[l], %[n]"
        : [w] "+v"(word), [l] "+v"(lword), [m] "=&s"(m), [n] "=&s"(n), [c] "=&s"(c)
        : [d] "v"(d), [lo] "v"(lo), [hi] "v"(hi));
}

// word = 2*word + (d < r2) for four / one candidates of the FP64 form.
__device__ __forceinline__ void push4_f64(uint32_t& word, double d0, double d1, double d2,
                                          double d3, double r2) {
    uint64_t m0, m1, m2, m3, c;
    asm volatile(
        "v_cmp_lt_f64_e64 %[m0], %[d0], %[r]\n\t"
        "v_cmp_lt_f64_e64 %[m1], %[d1], %[r]\n\t"
        "v_cmp_lt_f64_e64 %[m2], %[d2], %[r]\n\t"
        "v_cmp_lt_f64_e64 %[m3], %[d3], %[r]\n\t"
        "s_nop 1\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m0]\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m1]\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m2]\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m3]"
        : [w] "+v"(word), [m0] "=&s"(m0), [m1] "=&s"(m1), [m2] "=&s"(m2), [m3] "=&s"(m3),
          [c] "=&s"(c)
        : [d0] "v"(d0), [d1] "v"(d1), [d2] "v"(d2), [d3] "v"(d3), [r] "v"(r2));
}

__device__ __forceinline__ void push1_f64(uint32_t& word, double d, double r2) {
    uint64_t m, c;
    asm volatile(
        "v_cmp_lt_f64_e64 %[m], %[d], %[r]\n\t"
        "s_nop 1\n\t"
        "v_addc_co_u32_e64 %[w], %[c], %[w], %[w], %[m]"
        : [w] "+v"(word), [m] "=&s"(m), [c] "=&s"(c)
        : [d] "v"(d), [r] "v"(r2));
}

__device__ __forceinline__ float f32_down(double d) {
    float f = (float)d;
    if ((double)f > d) f = nextafterf(f, -INFINITY);
    return f;
}

__device__ __forceinline__ float f32_up(double d) {
    float f = (float)d;
    if ((double)f < d) f = nextafterf(f, INFINITY);
    return f;
}

template <bool F32> struct Ent;
template <> struct Ent<true> {
    using T = float4;
    __device__ static int key(float4 e) { return __float_as_int(e.w); }
    __device__ static void pad(float4& e) { e.w = __int_as_float(0x7fffffff); }
};
template <> struct Ent<false> {
    using T = double4;
    __device__ static int key(double4 e) { return e.w > 2147483647.0 ? 0x7fffffff : (int)e.w; }
    __device__ static void pad(double4& e) { e.w = 4294967296.0; }
};

// Walk (Algorithm 2 with Eq. 5 applied to the box E) by one wavefront:
// from the root code, every internal cell's sub-cell range on each axis is
// [f(E_lo), f(E_hi)] with the build's own Eq. 2 function f (lanes 0..5
// compute the six bounds); lanes then take one sub-cell of the range each.
// Leaves in range go to list[0..n), internal sub-cells to the stack.
// Returns n, or -1 when the list or the stack overflowed; kmin and kmax
// receive the smallest and largest original index over the listed leaves.
template <int LMAX>
__device__ __forceinline__ int walk_wave(int32_t root_code, const double elo[3],
                                         const double ehi[3], const Node* __restrict__ nodes,
                                         const int32_t* __restrict__ ctab,
                                         const int2* __restrict__ lrange,
                                         int32_t* __restrict__ s_stack,
                                         int32_t* __restrict__ s_leaf, int& kmin, int& kmax) {
    const int lane = lane_id();
    int top = 0, nleaf = 0, ovf = 0;
    if (root_code & kLeafBit) {
        if (lane == 0) s_leaf[0] = root_code & ~kLeafBit;
        nleaf = 1;
    } else {
        if (lane == 0) s_stack[0] = root_code;
        top = 1;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    while (top > 0 && !ovf) {
        --top;
        const int node = __builtin_amdgcn_readfirstlane(s_stack[top]);
        const Node N = nodes[node];
        const int b = N.b;
        const int ax3 = lane < 3 ? lane : lane - 3;
        const double ev = lane == 0 ? elo[0] : lane == 1 ? elo[1] : lane == 2 ? elo[2]
                        : lane == 3 ? ehi[0] : lane == 4 ? ehi[1] : ehi[2];
        const double nlo = ax3 == 0 ? N.lo[0] : ax3 == 1 ? N.lo[1] : N.lo[2];
        const double nhi = ax3 == 0 ? N.hi[0] : ax3 == 1 ? N.hi[1] : N.hi[2];
        const int r = lane < 6 ? subcell(ev, nlo, nhi, b) : 0;
        const int rlo0 = __shfl(r, 0, 64), rlo1 = __shfl(r, 1, 64), rlo2 = __shfl(r, 2, 64);
        const int nx = __builtin_amdgcn_readfirstlane(__shfl(r, 3, 64) - rlo0 + 1);
        const int ny = __builtin_amdgcn_readfirstlane(__shfl(r, 4, 64) - rlo1 + 1);
        const int nz = __builtin_amdgcn_readfirstlane(__shfl(r, 5, 64) - rlo2 + 1);
        const int nxy = nx * ny;
        const int T = nxy * nz;
        for (int k0 = 0; k0 < T; k0 += 64) {
            const int k = k0 + lane;
            int32_t code = kEmpty;
            if (k < T) {
                const int iz = k / nxy;
                const int rem = k - iz * nxy;
                const int iy = rem / nx;
                const int ix = rem - iy * nx;
                code = ctab[N.ctab + (rlo0 + ix) +
                            (int64_t)b * ((rlo1 + iy) + (int64_t)b * (rlo2 + iz))];
            }
            const bool isl = code != kEmpty && (code & kLeafBit);
            const bool isi = code != kEmpty && !(code & kLeafBit);
            const uint64_t ml = __ballot(isl);
            const uint64_t mi = __ballot(isi);
            if (isl) {
                const int p = nleaf + lanes_below(ml);
                if (p < LMAX) s_leaf[p] = code & ~kLeafBit;
            }
            if (isi) {
                const int p = top + lanes_below(mi);
                if (p < kSMax) s_stack[p] = code;
            }
            nleaf += __popcll(ml);
            top += __popcll(mi);
            if (nleaf > LMAX || top > kSMax) {
                ovf = 1;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // Index range of the candidate leaves.
    int mn = 0x7fffffff, mx = -1;
    if (!ovf) {
        for (int li = lane; li < nleaf; li += 64) {
            const int2 rr = lrange[s_leaf[li]];
            mn = min(mn, rr.x);
            mx = max(mx, rr.y);
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        mn = min(mn, __shfl_xor(mn, d, 64));
        mx = max(mx, __shfl_xor(mx, d, 64));
    }
    kmin = mn;
    kmax = mx;
    return ovf ? -1 : nleaf;
}

// Box E of a work item (lane q holds query q, valid when qv):
// [min fl(x_i - R_i), max fl(x_i + R_i)] per axis.
__device__ __forceinline__ void item_box(bool qv, const double4& qp, double R, double elo[3],
                                         double ehi[3]) {
    const double q3[3] = {qp.x, qp.y, qp.z};
    for (int l = 0; l < 3; ++l) {
        elo[l] = wave_min(qv ? q3[l] - R : INFINITY);
        ehi[l] = wave_max(qv ? q3[l] + R : -INFINITY);
    }
}

// The item-wide part of the FP32 filter's set-up: the norm bound |S| of the
// per-axis staging bounds and the largest radius (derivation at the top of
// the file).  The walk computes it with the box and keeps both per item, so
// the main sweep's four wavefronts need not reduce them again.
struct ItemBox {
    double lo[3], hi[3];
    double sn, rmax;
};

// Where pass 1 left a main-sweep work item's result for pass 2 (off < 0:
// nowhere, the item's rows went through the split path or did not fit):
// at scratch[off], the test words, word g of query q at g * qs + q (qs: the
// item's queries), then its C candidates' set-local indices in ascending
// order.  Bit 31 - j of word g is the pair (query, candidate 32 g + j).
struct ItemRows {
    int64_t off;
    int32_t C;
    int32_t qs;
};

__device__ __forceinline__ void item_bounds(bool qv, const double4& qp, double R,
                                            const double elo[3], const double ehi[3],
                                            double& sn, double& rmax) {
    const double up = 1.0 + 0x1p-50;
    const double c3[3] = {elo[0] + (ehi[0] - elo[0]) * 0.5, elo[1] + (ehi[1] - elo[1]) * 0.5,
                          elo[2] + (ehi[2] - elo[2]) * 0.5};
    const double q3[3] = {qp.x, qp.y, qp.z};
    double S[3];
    for (int l = 0; l < 3; ++l) {
        const double mb = fmax(c3[l] - elo[l], ehi[l] - c3[l]) * up;
        const double ma = wave_max(qv ? fabs(q3[l] - c3[l]) : 0.0) * up;
        S[l] = (ma + mb) * up;
    }
    sn = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]) * up;
    rmax = wave_max(R);
}

// Stripe of a pool (scratch, walk lists) that a unit starting at sorted position `beg`
// allocates from: a function of the unit alone, so that a search repeated
// over the same data asks each stripe for the same amount.
__device__ __forceinline__ int stripe_of(int beg) {
    return (int)(((uint32_t)beg * 2654435761u) >> 26) & (kStripes - 1);
}

// Work item of workgroup b.  Workgroups are dealt to the chip's 8 XCDs in
// turn (XCD b mod 8), each with its own L2, and work items next to each
// other in tree order share most candidate leaves.  So the items are cut
// into blocks of kXcdBlock, dealt to the XCDs in turn: the r-th workgroup
// of XCD x takes item (r / K) 8K + x K + r mod K (K = kXcdBlock), so a
// block's items meet in one L2 while every XCD still gets a share of every
// part of the item list (their costs vary widely along it).  The grid must
// cover the items rounded up to a multiple of 8K (xcd_grid); returns n (no
// item) past the end.  n must not exceed the items the per-item buffers
// hold (callers pass min(items, capacity)): the id is not bounded by the
// grid size.
constexpr int kXcdBlock = 16;

__device__ __forceinline__ int xcd_item(unsigned b, int n) {
    const unsigned r = b >> 3, x = b & 7u;
    const int64_t ci = (int64_t)(r / kXcdBlock) * (8 * kXcdBlock) + (int64_t)x * kXcdBlock +
                       (r % kXcdBlock);
    return ci < n ? (int)ci : n;
}

// Grid for xcd_item over `items` work items: a multiple of 8 kXcdBlock.
inline unsigned xcd_grid(int64_t items) {
    constexpr int64_t q = 8 * kXcdBlock;
    int64_t g = std::max<int64_t>(1, items);
    g = (g + q - 1) / q * q;
    return (unsigned)std::min<int64_t>(g, 0x7fffff00);
}

// The walk as a kernel of its own, one wavefront per work item, breadth
// first: all cells of the current tree level are expanded together (lane j
// computes the Eq. 5 ranges of frontier cell j; then the sub-cells of all
// ranges, numbered by a prefix sum, are read from the child tables one per
// lane), so the chain of dependent loads is two per level rather than two
// per cell.  Result per item: a header {first entry, leaf count (negative:
// overflow), smallest index, largest index} and the candidate leaves as
// (first particle, count) pairs.
constexpr int kLMaxWalk = 512;  // candidate leaves per item
constexpr int kFMax = 128;      // cells of one frontier

__global__ __launch_bounds__(64) void k_walk(const Chunk* __restrict__ chunks,
                                             const double4* __restrict__ pos,
                                             const Node* __restrict__ nodes,
                                             const int32_t* __restrict__ ctab,
                                             const Leaf* __restrict__ leaves,
                                             const int2* __restrict__ lrange,
                                             const SetDev* __restrict__ sets,
                                             const double* __restrict__ h,
                                             double* __restrict__ hs,
                                             int4* __restrict__ whdr, int2* __restrict__ wl,
                                             int64_t wl_cap, unsigned long long* __restrict__ wcur,
                                             ItemBox* __restrict__ ibox, Ctl* __restrict__ ctl,
                                             const int item_cap) {
    __shared__ int32_t s_front[2][kFMax];
    __shared__ int32_t s_pref[kFMax + 1];
    __shared__ int64_t s_tab[kFMax];      // child-table offset of frontier cell j
    __shared__ uint32_t s_geo[kFMax][3];  // 16-bit pairs: (b, start x), (start y, z), (size x, y)
    __shared__ int32_t s_leaf[kLMaxWalk];
    if (ctl->data_bad || (ctl->overflow & kOvfTree)) return;
    // Items past the per-item buffers (a replay with more items than it was
    // recorded for) are left alone; the sweep reports the overflow.
    const int nit = min(ctl->n_chunks, item_cap);
    const int ci = xcd_item(blockIdx.x, nit);
    if (ci >= nit) return;
    const Chunk ch = chunks[ci];
    const int lane = threadIdx.x;
    const bool qv = lane < ch.cnt;
    const double4 qp = qv ? pos[ch.beg + lane] : make_double4(0.0, 0.0, 0.0, 0.0);
    // h of the item's particles, also kept in tree order for the later
    // search kernels (the work items cover every particle once).
    double hv = 0.0;
    if (qv) {
        hv = h[(int)qp.w];
        hs[ch.beg + lane] = hv;
    }
    // h must be finite and >= 0 (the work items cover every particle once);
    // the later kernels write nothing once the flag is up.
    if (__ballot(qv && !(hv >= 0.0 && isfinite(hv))) && lane == 0) atomicOr(&ctl->data_bad, 2);
    const double R = 2.0 * hv;
    double elo[3], ehi[3];
    item_box(qv, qp, R, elo, ehi);
    {
        double sn, rmax;
        item_bounds(qv, qp, R, elo, ehi, sn, rmax);
        // Eight doubles, one per lane (the values are uniform).
        const double f[8] = {elo[0], elo[1], elo[2], ehi[0], ehi[1], ehi[2], sn, rmax};
        double v = f[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) v = lane == k ? f[k] : v;
        if (lane < 8) reinterpret_cast<double*>(ibox + ci)[lane] = v;
    }
    const int32_t root_code = __builtin_amdgcn_readfirstlane(sets[ch.set].root);

    int nleaf = 0, nf = 0, cur = 0;
    bool ovf = false;
    if (root_code & kLeafBit) {
        if (lane == 0) s_leaf[0] = root_code & ~kLeafBit;
        nleaf = 1;
    } else {
        if (lane == 0) s_front[0][0] = root_code;
        nf = 1;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    while (nf > 0 && !ovf) {
        // Ranges of the frontier cells (Eq. 5 with the build's Eq. 2).
        int carry = 0;
        for (int j0 = 0; j0 < nf; j0 += 64) {
            const int j = j0 + lane;
            int T = 0;
            if (j < nf) {
                const Node N = nodes[s_front[cur][j]];
                int r[6];
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    r[l] = subcell(elo[l], N.lo[l], N.hi[l], N.b);
                    r[3 + l] = subcell(ehi[l], N.lo[l], N.hi[l], N.b);
                }
                const int nx = r[3] - r[0] + 1, ny = r[4] - r[1] + 1, nz = r[5] - r[2] + 1;
                T = nx * ny * nz;
                s_tab[j] = N.ctab;
                s_geo[j][0] = (uint32_t)N.b | ((uint32_t)r[0] << 16);
                s_geo[j][1] = (uint32_t)r[1] | ((uint32_t)r[2] << 16);
                s_geo[j][2] = (uint32_t)nx | ((uint32_t)ny << 16);
            }
            const int inc = wave_incl_scan(T);
            if (j < nf) s_pref[j] = carry + inc - T;
            carry += __shfl(inc, 63, 64);
            if (carry > (1 << 28)) ovf = true;  // absurdly wide level: the item is split
        }
        if (ovf) break;
        if (lane == 0) s_pref[nf] = carry;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // Sub-cells of all ranges, one per lane.
        const int total = __builtin_amdgcn_readfirstlane(carry);
        int nnext = 0;
        for (int k0 = 0; k0 < total; k0 += 64) {
            const int k = k0 + lane;
            int32_t code = kEmpty;
            if (k < total) {
                int lo = 0, hi = nf - 1;  // frontier cell j: s_pref[j] <= k < s_pref[j + 1]
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_pref[mid] <= k) lo = mid;
                    else hi = mid - 1;
                }
                const uint32_t g0 = s_geo[lo][0], g1 = s_geo[lo][1], g2 = s_geo[lo][2];
                const int b = g0 & 0xffff, nx = g2 & 0xffff, nxy = nx * (int)(g2 >> 16);
                const int e = k - s_pref[lo];
                const int iz = e / nxy;
                const int rem = e - iz * nxy;
                const int iy = rem / nx;
                const int ix = rem - iy * nx;
                code = ctab[s_tab[lo] + ((int)(g0 >> 16) + ix) +
                            (int64_t)b * (((int)(g1 & 0xffff) + iy) + (int64_t)b * ((int)(g1 >> 16) + iz))];
            }
            const bool isl = code != kEmpty && (code & kLeafBit);
            const bool isi = code != kEmpty && !(code & kLeafBit);
            const uint64_t ml = __ballot(isl);
            const uint64_t mi = __ballot(isi);
            if (isl) {
                const int q = nleaf + lanes_below(ml);
                if (q < kLMaxWalk) s_leaf[q] = code & ~kLeafBit;
            }
            if (isi) {
                const int q = nnext + lanes_below(mi);
                if (q < kFMax) s_front[cur ^ 1][q] = code;
            }
            nleaf += __popcll(ml);
            nnext += __popcll(mi);
            if (nleaf > kLMaxWalk || nnext > kFMax) {
                ovf = true;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        cur ^= 1;
        nf = nnext;
    }
    int nl = ovf ? -1 : nleaf;
    unsigned long long off = 0;
    if (nl > 0) {
        const int stripe = stripe_of(ch.beg);
        const int64_t region = wl_cap / kStripes;
        if (lane == 0) off = atomicAdd(&wcur[stripe * kStripeStride], (unsigned long long)nl);
        off = __shfl(off, 0, 64);
        if ((int64_t)(off + nl) > region) {  // stripe full: the item is split, the host grows it
            if (lane == 0) atomicOr(&ctl->overflow, kOvfWalk);
            nl = -2;
        }
        off += (unsigned long long)(stripe * region);
    }
    int mn = 0x7fffffff, mx = -1;
    if (nl > 0)
        for (int li = lane; li < nl; li += 64) {
            const int id = s_leaf[li];
            const Leaf L = leaves[id];
            const int2 rr = lrange[id];
            wl[off + li] = make_int2(L.beg, L.cnt);
            mn = min(mn, rr.x);
            mx = max(mx, rr.y);
        }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        mn = min(mn, __shfl_xor(mn, d, 64));
        mx = max(mx, __shfl_xor(mx, d, 64));
    }
    if (lane == 0) whdr[ci] = make_int4((int)off, nl, mn, mx);
}

// One work item of the sweep: walk, stage, order by original index, test,
// rows out.  Called by every thread of the workgroup with the same item.
// Returns 0 when done.  When the item's candidates do not fit the
// shared-memory budget it writes nothing and returns their number (kHuge
// when the walk itself overflowed), and the caller splits the item.
constexpr int kHuge = 1 << 30;

constexpr int kNoCount = kHuge + 1;  // overflow of the leaf list, candidates not counted

// WALK: 0 = walk here; 1 = take the walk kernel's list of item ci; 2 = take
// it when ci >= 0 and the list is whole and fits, else walk here.
constexpr int kSubGroup = 8;  // queries per sub-item of a split work item

// What a search pass writes per query: the row (to the scratch, placed
// later), the count only (h adaptation), or the count and the fused SPH
// density sum over the row (no row materialised).
enum { kOutRows = 0, kOutCount = 1, kOutDensity = 2 };

// Caller buffers of the density form: masses (original order; null = unit
// masses) and the densities written.
struct DensOut {
    const double* mass;
    double* rho;
};

// Shape of the cubic-spline SPH kernel (the M4 B-spline: support 2h,
// W(r, h) = w(r / h) / (pi h^3)), evaluated from the squared distance of a
// pair with every operation rounded in this order:
//   r = sqrt(d2), q = r / h,
//   q < 1: (1 - 1.5 q^2) + 0.75 q^3,  1 <= q < 2: 0.25 ((2 - q)^2 (2 - q)).
__device__ __forceinline__ double sph_shape(double d2, double h) {
    const double q = __ddiv_rn(__dsqrt_rn(d2), h);
    if (q < 1.0) {
        const double q2 = __dmul_rn(q, q);
        return __dadd_rn(__dsub_rn(1.0, __dmul_rn(1.5, q2)), __dmul_rn(0.75, __dmul_rn(q2, q)));
    }
    if (q < 2.0) {
        const double t = __dsub_rn(2.0, q);
        return __dmul_rn(0.25, __dmul_rn(__dmul_rn(t, t), t));
    }
    return 0.0;
}

// m_j w(r_ij / h_i) of one neighbour j (key = its original index) of the
// query at (x, y, z) with smoothing length h, from FP64 coordinates.
__device__ __forceinline__ double sph_term(double x, double y, double z, double h, int key,
                                           const double4* __restrict__ src,
                                           const double* __restrict__ mass) {
    const double4 o = src[key];  // either particle copy: .w is the original index
    const double dx = __dsub_rn(x, o.x), dy = __dsub_rn(y, o.y), dz = __dsub_rn(z, o.z);
    const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    const double w = sph_shape(d2, h);
    return mass ? __dmul_rn(mass[(int)o.w], w) : w;
}

// Density from the sum of the terms of a row: sum / (pi h^3); 0 for an
// empty row.
__device__ __forceinline__ double sph_density(double sum, int count, double h) {
    if (count == 0) return 0.0;
    return __ddiv_rn(sum, __dmul_rn(3.141592653589793, __dmul_rn(__dmul_rn(h, h), h)));
}

// SMALL: units of at most kSubGroup queries test with lane = candidate.
template <bool F32, int WALK, int CMAX = kCMax, int LMAX = kLMax, bool SMALL = false,
          int OUT = kOutRows>
__device__ __forceinline__ int sweep_item(const int ci, const Chunk ch,
                                          const int4* __restrict__ whdr,
                                          const int2* __restrict__ wl,
                                          const ItemBox* __restrict__ ibox,
                                          const double4* __restrict__ pos,
                                           const double4* __restrict__ orig,
                                           const Node* __restrict__ nodes,
                                           const int32_t* __restrict__ ctab,
                                           const Leaf* __restrict__ leaves,
                                           const int2* __restrict__ lrange,
                                           const SetDev* __restrict__ sets,
                                           const double* __restrict__ h,
                                           int32_t* __restrict__ counts,
                                           int64_t* __restrict__ soff,
                                           int32_t* __restrict__ scratch, int64_t scap,
                                           unsigned long long* __restrict__ scur, int stripe,
                                           Ctl* __restrict__ ctl, Stats* __restrict__ stats,
                                           const int excl, const DensOut dout,
                                           ItemRows* __restrict__ irec) {
    using E = typename Ent<F32>::T;
    // The main sweep's rows form leaves the test words and the ordered
    // candidates for pass 2 (k_expand), which writes the rows straight into
    // the caller's CSR once the offsets are known; the split levels write
    // rows to the scratch (k_place copies them).
    constexpr bool kBits = OUT == kOutRows && WALK == 1 && !SMALL;
    // The density form never lists indices: its entries carry the tree
    // position instead of the original index, so the coordinates of a term
    // (and of an FP64 confirmation) come from the tree-ordered copy, whose
    // entries for one item lie in a few nearby leaves, not from scattered
    // places in the caller's order.  Candidates are then ordered by tree
    // position (the sum's order, fixed for a given tree).
    constexpr bool kTreeKeys = OUT == kOutDensity;
    const double4* __restrict__ const src = kTreeKeys ? pos : orig;
    constexpr int kMaxW = ((CMAX / kWaves) + 31) / 32;  // bit words per lane and wavefront
    __shared__ E s_cand[CMAX];
    __shared__ int32_t s_cnt[kWaves][64];
    // Walk stack and candidate-leaf list; once the candidates are staged the
    // same memory holds the permutation that orders them by original index.
    __shared__ __align__(16) int32_t s_walk[kSMax + LMAX];
    int32_t* const s_stack = s_walk;
    int32_t* const s_leaf = s_walk + kSMax;
    int2* const s_linfo = reinterpret_cast<int2*>(s_walk);  // prewalked: (first, count)
    constexpr int kLPre = (kSMax + LMAX) / 2;
    uint16_t* const s_perm = reinterpret_cast<uint16_t*>(s_walk);
    static_assert(2 * (kSMax + LMAX) >= CMAX, "permutation must fit the walk area");
    // Bucket sizes, then bucket starts; placement cursors, then bucket ends.
    // Once the test is over (after a barrier) the density form keeps its
    // per-wavefront sums in the same memory.
    __shared__ __align__(16) int32_t s_bk[2 * kBuckets];
    int32_t* const s_bcnt = s_bk;
    int32_t* const s_bcur = s_bk + kBuckets;
    static_assert(2 * kBuckets * sizeof(int32_t) >= kWaves * 64 * sizeof(double),
                  "the density sums must fit the bucket arrays");
    __shared__ int32_t s_qoff[64];
    __shared__ int64_t s_scan[kWaves + 1];
    __shared__ int s_nleaf, s_ovf, s_kmin, s_kmax, s_C, s_big, s_total, s_bits, s_rows_total;
    __shared__ unsigned long long s_base;

    // The item's set: its root, and the base that makes indices set-local.
    const int32_t root_code = __builtin_amdgcn_readfirstlane(sets[ch.set].root);
    const int sbeg = __builtin_amdgcn_readfirstlane((int)sets[ch.set].beg);
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);

    // The walk kernel's list of candidate leaves, when this item has one: it
    // does not depend on the queries, so its loads go first.
    int4 hd = make_int4(0, -1, 0, 0);
    if (WALK != 0 && ci >= 0) hd = whdr[ci];
    const bool pre = WALK == 1 || (WALK == 2 && hd.y >= 0 && hd.y <= kLPre);
    if (pre && hd.y >= 0 && hd.y <= kLPre)
        for (int li = t; li < hd.y; li += kWG) s_linfo[li] = wl[hd.x + li];

    // Queries: lane q of every wavefront holds query q of the item.
    const bool qv = lane < ch.cnt;
    const double4 qp = qv ? pos[ch.beg + lane] : make_double4(0.0, 0.0, 0.0, 0.0);
    const int qidx = (int)qp.w;
    const int qkey = kTreeKeys ? ch.beg + lane : qidx;  // the query's own entry
    const double R = qv ? 2.0 * h[ch.beg + lane] : 0.0;

    // Box E of the item and the filter's item-wide bounds: from the walk
    // kernel's record when the item has one, else reduced here.
    double elo[3], ehi[3], sn = 0.0, rmax = 0.0;
    if (WALK == 1 || (WALK == 2 && ci >= 0 && ibox != nullptr)) {
        const ItemBox ib = ibox[ci];
        for (int l = 0; l < 3; ++l) {
            elo[l] = ib.lo[l];
            ehi[l] = ib.hi[l];
        }
        sn = ib.sn;
        rmax = ib.rmax;
    } else {
        item_box(qv, qp, R, elo, ehi);
        if (F32) item_bounds(qv, qp, R, elo, ehi, sn, rmax);
    }

    // FP32 filter set-up (derivation at the top of the file).  tlo, thi:
    // the thresholds on D (the lane-per-candidate test of small units);
    // nT, tM: the threshold and margin of the three-FMA test of the words.
    float ax = 0.f, ay = 0.f, az = 0.f, tlo = -1.f, thi = -1.f, nT = 1.f, tM = -1.f;
    double cx = 0.0, cy = 0.0, cz = 0.0;
    bool unsafe = false;
    if (F32) {
        cx = elo[0] + (ehi[0] - elo[0]) * 0.5;
        cy = elo[1] + (ehi[1] - elo[1]) * 0.5;
        cz = elo[2] + (ehi[2] - elo[2]) * 0.5;
        // Every square, product and threshold below stays under 2^128.
        unsafe = !(sn < 0x1p60 && rmax < 0x1p60);
        const double u = 0x1p-24;
        const double eta = (0x1p-24 + 0x1p-52) * sn * (1.0 + 0x1p-40) + 8.0 * 0x1p-126;
        const double g3 = 3.0 * u / (1.0 - 3.0 * u);
        if (qv) {
            double A = R * (1.0 - 0x1p-48) - eta;
            if (A < 0.0) A = 0.0;
            const double tl =
                (1.0 - g3) * (1.0 - u) * (1.0 - u) * A * A * (1.0 - 0x1p-40) - 8.0 * 0x1p-126;
            const double B = R * (1.0 + 0x1p-48) + eta;
            const double th =
                (1.0 + g3) * (1.0 + u) * (1.0 + u) * B * B * (1.0 + 0x1p-40) + 8.0 * 0x1p-126;
            tlo = tl > 0.0 ? f32_down(tl) : 0.0f;
            thi = f32_up(th);
            // Three-FMA test: E = fl(tz^2 + fl(ty^2 + fl(tx^2 - T))), T = fl32(R^2).
            // Each FMA rounds once, so |E - (|t|^2 - T)| <= kap (|t|^2 + T) + ea
            // with kap = 3u (1 + 2^-20) and ea an absolute slack for results
            // flushed to zero.  The filter's bounds on |t|^2 are Qlo (below it
            // the pair is a neighbour) and Qhi (at or above it, not one): D's
            // thresholds above are Qlo and Qhi widened by gamma_3.  Hence
            //   E < -M => |t|^2 < (T (1 + kap) - M + ea) / (1 - kap) <= Qlo,
            //   E >= M => |t|^2 >= (T (1 - kap) + M - ea) / (1 + kap) >= Qhi,
            // for M = max(T (1 + kap) + ea - Qlo (1 - kap),
            //             Qhi (1 + kap) - T (1 - kap) + ea),
            // computed in FP64 with a slack of 2^-48 (T + Qhi) for its own
            // roundings (the difference cancels) and rounded up to FP32.
            // A pair with |E| <= M is decided by the FP64 predicate.
            const double Td = (double)(float)(R * R);
            const double kap = 3.0 * u * (1.0 + 0x1p-20);
            const double ea = 16.0 * 0x1p-126;
            const double Qlo = (1.0 - u) * (1.0 - u) * A * A * (1.0 - 0x1p-40);
            const double Qhi = (1.0 + u) * (1.0 + u) * B * B * (1.0 + 0x1p-40);
            const double m1 = Td * (1.0 + kap) + ea - Qlo * (1.0 - kap);
            const double m2 = Qhi * (1.0 + kap) - Td * (1.0 - kap) + ea;
            nT = -(float)Td;
            tM = f32_up((m1 > m2 ? m1 : m2) + (Td + Qhi) * 0x1p-48);
            ax = (float)(qp.x - cx);
            ay = (float)(qp.y - cy);
            az = (float)(qp.z - cz);
        }
    }
    const double r2q = qv ? __dmul_rn(R, R) : -1.0;

    for (int b = t; b < kBuckets; b += kWG) s_bcnt[b] = 0;
    if (t == 0) {
        s_C = 0;
        s_big = 0;
    }

    // Candidate leaves: from the walk kernel's list (fetched at the top), or
    // walked here by wavefront 0.
    if (pre) {
        const int nl = hd.y;
        if (t == 0) {
            s_nleaf = nl;
            s_ovf = unsafe ? 1 : (nl < 0 || nl > kLPre) ? 2 : 0;
            s_kmin = hd.z;
            s_kmax = hd.w;
        }
    } else if (w == 0) {
        int mn, mx;
        const int nl = walk_wave<LMAX>(root_code, elo, ehi, nodes, ctab, lrange, s_stack, s_leaf,
                                       mn, mx);
        if (lane == 0) {
            s_nleaf = nl;
            s_ovf = (nl < 0 || unsafe) ? 1 : 0;
            s_kmin = mn;
            s_kmax = mx;
        }
    }
    __syncthreads();
    if (s_ovf) return s_ovf == 2 ? kNoCount : kHuge;
    const int nleaf = __builtin_amdgcn_readfirstlane(s_nleaf);
    const int kmin = __builtin_amdgcn_readfirstlane(s_kmin);
    const int kmax = __builtin_amdgcn_readfirstlane(s_kmax);
    // Buckets of the original index: a monotone map of [kmin, kmax] onto
    // 0..255, so sorting each bucket sorts the whole candidate list.  The
    // density form's keys (tree positions) cluster in the few leaves of the
    // item, so there a multiplicative hash spreads them over the buckets:
    // the order is then fixed for a given tree, not ascending, which is all
    // the sum needs.
    const float binv = (float)kBuckets / (float)((int64_t)kmax - kmin + 1);

    // (first particle, count) of candidate leaf li.
    auto leaf_at = [&](int li) -> int2 {
        if (pre) return s_linfo[li];
        const Leaf L = leaves[s_leaf[li]];
        return make_int2(L.beg, L.cnt);
    };

    // Wavefront w visits the 64-particle chunks of candidate leaves w,
    // w + kWaves, ... in order; the next chunk's load is issued before the
    // current chunk is used, so two loads are in flight per wavefront.
    auto visit = [&](auto&& body) {
        int li = w, p0 = 0;
        int2 L = li < nleaf ? leaf_at(li) : make_int2(0, 0);
        bool vn = li < nleaf && lane < L.y;
        double4 Pn = vn ? pos[L.x + lane] : make_double4(0.0, 0.0, 0.0, 0.0);
        if (kTreeKeys) Pn.w = (double)(L.x + lane);
        while (li < nleaf) {
            const double4 P = Pn;
            const bool v = vn;
            p0 += 64;
            if (p0 >= L.y) {
                li += kWaves;
                p0 = 0;
                if (li < nleaf) L = leaf_at(li);
            }
            vn = li < nleaf && p0 + lane < L.y;
            Pn = vn ? pos[L.x + p0 + lane] : make_double4(0.0, 0.0, 0.0, 0.0);
            if (kTreeKeys) Pn.w = (double)(L.x + p0 + lane);
            const bool in = v && P.x >= elo[0] && P.x <= ehi[0] && P.y >= elo[1] &&
                            P.y <= ehi[1] && P.z >= elo[2] && P.z <= ehi[2];
            body(P, in);
        }
    };

    auto entry = [&](const double4& P) -> E {
        if constexpr (F32)
            return make_float4((float)(P.x - cx), (float)(P.y - cy), (float)(P.z - cz),
                               __int_as_float((int)P.w));
        else
            return P;
    };
    auto bucket = [&](int key) -> int {
        if constexpr (kTreeKeys) return (int)(((uint32_t)key * 2654435761u) >> 24);
        else return min(kBuckets - 1, (int)((float)(key - kmin) * binv));
    };
    static_assert(kBuckets == 256, "the hash takes the top 8 bits");
    constexpr int kPer = (CMAX + kWG - 1) / kWG;
    constexpr bool kPhys = kPer <= 6;  // six entries per thread fit in registers

    // Stage, pass 1: count candidates inside E per index bucket.  With up to
    // six entries per thread the candidates also go to shared memory here,
    // in arrival order (past the budget they are only counted).
    if constexpr (kPhys) {
        visit([&](const double4& P, bool in) {
            const uint64_t m = __ballot(in);
            int b = 0;
            if (lane == 0 && m) b = atomicAdd(&s_C, (int)__popcll(m));
            b = __builtin_amdgcn_readfirstlane(b);  // every lane is active: lane 0's value
            if (in) {
                atomicAdd(&s_bcnt[bucket((int)P.w)], 1);
                const int slot = b + lanes_below(m);
                if (slot < CMAX) s_cand[slot] = entry(P);
            }
        });
    } else {
        int myC = 0;
        visit([&](const double4& P, bool in) {
            if (in) atomicAdd(&s_bcnt[bucket((int)P.w)], 1);
            myC += __popcll(__ballot(in));
        });
        if (lane == 0) atomicAdd(&s_C, myC);
    }
    __syncthreads();
    const int C = __builtin_amdgcn_readfirstlane(s_C);
    if (C > CMAX) return C;
    int bstart, bcount;
    {
        int64_t tot;
        bcount = s_bcnt[t];
        bstart = (int)block_excl_scan<kWG>(bcount, s_scan, &tot);
        s_bcur[t] = bstart;
        if (bcount > kBucketSortMax) s_big = 1;
        __syncthreads();
        s_bcnt[t] = bstart;
    }
    __syncthreads();
    // A crowded bucket sorts the whole list with a bitonic network padded to
    // a power of two; if that does not fit the buffer, take the exhaustive path.
    if (s_big) {
        int P2 = 1;
        while (P2 < C) P2 <<= 1;
        if (P2 > CMAX) return C;
    }

    // Stage, pass 2: each candidate into its bucket; from shared memory
    // through registers (all slots are taken before any entry is written),
    // or, with the split kernels' larger budget, from global memory again.
    if constexpr (kPhys) {
        // Six named entries (an array here would leave registers).
        auto take = [&](int p) -> E { return s_cand[p < C ? p : 0]; };
        auto slot = [&](int p, const E e) -> int {
            return p < C ? atomicAdd(&s_bcur[bucket(Ent<F32>::key(e))], 1) : -1;
        };
        const E v0 = take(t), v1 = take(t + kWG), v2 = take(t + 2 * kWG);
        const E v3 = take(t + 3 * kWG), v4 = take(t + 4 * kWG), v5 = take(t + 5 * kWG);
        const int s0 = slot(t, v0), s1 = slot(t + kWG, v1), s2 = slot(t + 2 * kWG, v2);
        const int s3 = slot(t + 3 * kWG, v3), s4 = slot(t + 4 * kWG, v4);
        const int s5 = slot(t + 5 * kWG, v5);
        __syncthreads();
        if (s0 >= 0) s_cand[s0] = v0;
        if (s1 >= 0) s_cand[s1] = v1;
        if (s2 >= 0) s_cand[s2] = v2;
        if (s3 >= 0) s_cand[s3] = v3;
        if (s4 >= 0) s_cand[s4] = v4;
        if (s5 >= 0) s_cand[s5] = v5;
    } else {
        visit([&](const double4& P, bool in) {
            if (in) s_cand[atomicAdd(&s_bcur[bucket((int)P.w)], 1)] = entry(P);
        });
    }
    __syncthreads();

    // Order by original index.  Keys are distinct, so a candidate's rank is
    // its bucket's start plus the number of smaller keys in its bucket.  With
    // the main kernel's budget each entry then moves to its rank; with the
    // split kernel's larger one, s_perm[rank] = its slot instead.  An item
    // with a crowded bucket is sorted whole in place.
    if (!s_big && kPhys) {
        // Entries move to their ranks through registers: all ranks are
        // taken before any entry is overwritten.
        // Rank of entry e from slot p (or -1 past the list).
        auto rank_of = [&](int p, const E e) -> int {
            const int key = Ent<F32>::key(e);
            const int bk = bucket(key);
            const int b1 = p < C ? s_bcur[bk] : 0;
            int r = s_bcnt[bk];
            for (int q = r; q < b1; ++q) r += Ent<F32>::key(s_cand[q]) < key;
            return p < C ? r : -1;
        };
        auto at = [&](int p) -> E { return s_cand[p < C ? p : 0]; };
        const E e0 = at(t);
        const E e1 = at(t + kWG);
        const E e2 = at(t + 2 * kWG);
        const E e3 = at(t + 3 * kWG);
        const E e4 = at(t + 4 * kWG);
        const E e5 = at(t + 5 * kWG);
        const int d0 = rank_of(t, e0);
        const int d1 = rank_of(t + kWG, e1);
        const int d2 = rank_of(t + 2 * kWG, e2);
        const int d3 = rank_of(t + 3 * kWG, e3);
        const int d4 = rank_of(t + 4 * kWG, e4);
        const int d5 = rank_of(t + 5 * kWG, e5);
        __syncthreads();
        if (d0 >= 0) s_cand[d0] = e0;
        if (d1 >= 0) s_cand[d1] = e1;
        if (d2 >= 0) s_cand[d2] = e2;
        if (d3 >= 0) s_cand[d3] = e3;
        if (d4 >= 0) s_cand[d4] = e4;
        if (d5 >= 0) s_cand[d5] = e5;
    } else if (!s_big) {
        for (int p = t; p < C; p += kWG) {
            const int key = Ent<F32>::key(s_cand[p]);
            const int bk = bucket(key);
            const int b1 = s_bcur[bk];
            int r = s_bcnt[bk];
            for (int q = r; q < b1; ++q) r += Ent<F32>::key(s_cand[q]) < key;
            s_perm[r] = (uint16_t)p;
        }
    } else {
        int P2 = 1;
        while (P2 < C) P2 <<= 1;
        for (int k = C + t; k < P2; k += kWG) Ent<F32>::pad(s_cand[k]);
        __syncthreads();
        for (int kk = 2; kk <= P2; kk <<= 1) {
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int a = t; a < P2; a += kWG) {
                    const int c = a ^ j;
                    if (c > a) {
                        const E ea = s_cand[a], ec = s_cand[c];
                        const bool upw = (a & kk) == 0;
                        if ((Ent<F32>::key(ea) > Ent<F32>::key(ec)) == upw) {
                            s_cand[a] = ec;
                            s_cand[c] = ea;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (!kPhys)
            for (int p = t; p < C; p += kWG) s_perm[p] = (uint16_t)p;
    }
    __syncthreads();
    // Candidate k in index order.
    auto cand = [&](int k) -> E { return kPhys ? s_cand[k] : s_cand[s_perm[k]]; };

    // A unit of at most kSubGroup queries (split levels 2 and 3) would use
    // that many lanes of each wavefront in the layout below.  It tests with
    // lane = candidate instead: for each query in turn, wavefront w takes its
    // quarter of the 64-candidate chunks, a ballot gives the chunk's hits in
    // index order, and a lane prefix places them in the row.  Counts first;
    // the rows pass tests again (cheap at this size).
    const bool small = SMALL && ch.cnt <= kSubGroup;
    const int nch = (C + 63) >> 6;
    const int ch0 = (nch * w) / kWaves, ch1 = (nch * (w + 1)) / kWaves;  // this wavefront's chunks
    // Query q's data, broadcast from lane q by the whole wavefront (a
    // cross-lane read from a lane that is inactive returns 0, so this is
    // never done under a branch).
    struct Q {
        double x, y, z, R, r2;
        float ax, ay, az, lo, hi;
        int idx;
    };
    auto query = [&](int q) -> Q {
        return Q{__shfl(qp.x, q, 64), __shfl(qp.y, q, 64), __shfl(qp.z, q, 64), __shfl(R, q, 64),
                 __shfl(r2q, q, 64),  __shfl(ax, q, 64),   __shfl(ay, q, 64),   __shfl(az, q, 64),
                 __shfl(tlo, q, 64),  __shfl(thi, q, 64),  __shfl(qkey, q, 64)};
    };
    // Hits of query Qd among chunk c.
    auto chunk_hits = [&](const Q& Qd, int c, unsigned long long& nconf) -> uint64_t {
        const int k = c * 64 + lane;
        const bool v = k < C;
        const E e = cand(v ? k : 0);
        if constexpr (F32) {
            const float tx = Qd.ax - e.x, ty = Qd.ay - e.y, tz = Qd.az - e.z;
            const float D = fmaf(tz, tz, fmaf(ty, ty, tx * tx));
            uint64_t lo = __ballot(v && D < Qd.lo);
            const uint64_t band = __ballot(v && D < Qd.hi) & ~lo;
            if (band) {
                nconf += __popcll(band);
                bool ok = false;
                if ((band >> lane) & 1) {
                    const double4 o = src[Ent<F32>::key(e)];
                    ok = p64(Qd.x, Qd.y, Qd.z, Qd.R, o.x, o.y, o.z);
                }
                lo |= __ballot(ok);
            }
            if (excl) lo &= ~__ballot(v && Ent<F32>::key(e) == Qd.idx);
            return lo;
        } else {
            const double dx = __dsub_rn(Qd.x, e.x), dy = __dsub_rn(Qd.y, e.y);
            const double dz = __dsub_rn(Qd.z, e.z);
            const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                        __dmul_rn(dz, dz));
            uint64_t m = __ballot(v && d2 < Qd.r2);
            if (excl) m &= ~__ballot(v && Ent<F32>::key(e) == Qd.idx);
            return m;
        }
    };

    // Test: wavefront w sweeps candidates [k0, k1) (32-aligned) for its 64
    // queries; one bit per (query, candidate), first candidate in the top
    // bit of each 32-candidate word.  FP32 form: `word` collects D < T_lo
    // (certain neighbours), `lword` collects D < T_hi (possible ones); the
    // bits of lword & ~word are decided by the FP64 predicate.  D >= T_hi
    // rules a pair out: below T_hi's real-valued bound whenever the pair
    // could be a neighbour.
    const int B = ((C + kWaves * 32 - 1) / (kWaves * 32)) * 32;
    const int k0 = w * B;
    const int k1 = min(k0 + B, C);
    const int nw = (k1 > k0) ? (k1 - k0 + 31) >> 5 : 0;  // words of this wavefront, <= kMaxW
    // The words of a lane live in registers as a shift queue: each new word
    // enters at the top, so after nw words they sit in wq[kMaxW - nw ..].
    uint32_t wq[kMaxW];
#pragma unroll
    for (int i = 0; i < kMaxW; ++i) wq[i] = 0u;
    int hits = 0;
    unsigned long long conf = 0;   // FP64 confirmations, the same in every lane
    unsigned long long lconf = 0;  // ... counted per lane (words of the three-FMA test)
    // (Density form: lane q's sum of query q's terms over the wavefront's
    // part.)
    double dacc = 0.0;
    if (small) {
        if (lane >= ch.cnt) s_cnt[w][lane] = 0;
        for (int q = 0; q < ch.cnt; ++q) {
            const Q Qd = query(q);
            int hq = 0;
            double dq = 0.0;
            for (int c = ch0; c < ch1; ++c) {
                const uint64_t m = chunk_hits(Qd, c, conf);
                hq += __popcll(m);
                if constexpr (OUT == kOutDensity) {
                    double term = 0.0;
                    if ((m >> lane) & 1)
                        term = sph_term(Qd.x, Qd.y, Qd.z, 0.5 * Qd.R,
                                        Ent<F32>::key(cand(c * 64 + lane)), src, dout.mass);
                    dq += wave_sum(term);
                }
            }
            if (lane == 0) s_cnt[w][q] = hq;
            if (OUT == kOutDensity && lane == q) dacc = dq;
        }
    }
    for (int kw = k0; !small && kw < k1; kw += 32) {
        const int m = min(32, k1 - kw);
        uint32_t word = 0;
        if constexpr (F32) {
            // Bit = sign of E (the three-FMA test, set-up above), entering at
            // the bottom of the word; mn = the word's smallest |E|.
            float mn = INFINITY;
            auto test = [&](const float4& e) {
                const float tx = ax - e.x, ty = ay - e.y, tz = az - e.z;
                const float E = fmaf(tz, tz, fmaf(ty, ty, fmaf(tx, tx, nT)));
                word = __builtin_amdgcn_alignbit(word, __float_as_uint(E), 31);
                mn = fminf(mn, fabsf(E));
            };
            if (m == 32) {
                for (int g = 0; g < 32; g += 8) {
                    float4 e[8];
                    if constexpr (kPhys) {
#pragma unroll
                        for (int j = 0; j < 8; ++j) e[j] = s_cand[kw + g + j];
                    } else {
                        const uint4 pk = *reinterpret_cast<const uint4*>(s_perm + kw + g);
                        const uint32_t pw[4] = {pk.x, pk.y, pk.z, pk.w};
#pragma unroll
                        for (int j = 0; j < 8; ++j)
                            e[j] = s_cand[(pw[j >> 1] >> (16 * (j & 1))) & 0xffffu];
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j) test(e[j]);
                }
            } else {
                for (int j = 0; j < m; ++j) test(cand(kw + j));
                word <<= (32 - m);
            }
            // A word holding a pair with |E| <= M: every candidate of it is
            // classified again (E < -M: neighbour, E >= M: not; otherwise
            // the FP64 predicate decides).
            if (__ballot(mn <= tM)) {
                if (mn <= tM) {
                    uint32_t nwd = 0;
                    for (int j = 0; j < m; ++j) {
                        const float4 e = cand(kw + j);
                        const float tx = ax - e.x, ty = ay - e.y, tz = az - e.z;
                        const float E = fmaf(tz, tz, fmaf(ty, ty, fmaf(tx, tx, nT)));
                        uint32_t bit;
                        if (E < -tM) {
                            bit = 1u;
                        } else if (E >= tM) {
                            bit = 0u;
                        } else {
                            ++lconf;
                            const double4 o = src[__float_as_int(e.w)];
                            bit = p64(qp.x, qp.y, qp.z, R, o.x, o.y, o.z) ? 1u : 0u;
                        }
                        nwd = (nwd << 1) | bit;
                    }
                    word = m == 32 ? nwd : nwd << (32 - m);
                }
            }
        } else {
            if (m == 32) {
                for (int g = 0; g < 32; g += 4) {
                    double4 e[4];
                    if constexpr (kPhys) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) e[j] = s_cand[kw + g + j];
                    } else {
                        const uint2 pk = *reinterpret_cast<const uint2*>(s_perm + kw + g);
                        const uint32_t pw[2] = {pk.x, pk.y};
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            e[j] = s_cand[(pw[j >> 1] >> (16 * (j & 1))) & 0xffffu];
                    }
                    double d2[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const double dx = __dsub_rn(qp.x, e[j].x);
                        const double dy = __dsub_rn(qp.y, e[j].y);
                        const double dz = __dsub_rn(qp.z, e[j].z);
                        d2[j] = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                          __dmul_rn(dz, dz));
                    }
                    push4_f64(word, d2[0], d2[1], d2[2], d2[3], r2q);
                }
            } else {
                for (int j = 0; j < m; ++j) {
                    const double4 e = cand(kw + j);
                    const double dx = __dsub_rn(qp.x, e.x);
                    const double dy = __dsub_rn(qp.y, e.y);
                    const double dz = __dsub_rn(qp.z, e.z);
                    push1_f64(word, __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                              __dmul_rn(dz, dz)), r2q);
                }
                word <<= (32 - m);
            }
        }
        hits += __popc(word);
#pragma unroll
        for (int i = 0; i + 1 < kMaxW; ++i) wq[i] = wq[i + 1];
        wq[kMaxW - 1] = word;
    }
    // exclude_self: the query's own bit is cleared before anything is
    // counted, so counts, row offsets and rows all leave it out.  The query
    // lies inside its item's box, so it is one of the candidates; its place
    // in the ordered list is found by bisection on the keys, or (hashed
    // buckets of the density form) by a scan of its own bucket, whose range
    // the ordering kept.
    if (excl && !small && qv && r2q > 0.0 && C > 0) {
        int lo = 0;
        if (kTreeKeys && !s_big) {
            const int b = bucket(qkey);
            lo = s_bcur[b];
            for (int q = s_bcnt[b]; q < s_bcur[b]; ++q)
                if (Ent<F32>::key(cand(q)) == qkey) {
                    lo = q;
                    break;
                }
        } else {
            int hi = C - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (Ent<F32>::key(cand(mid)) < qkey) lo = mid + 1;
                else hi = mid;
            }
        }
        if (lo >= k0 && lo < k1 && Ent<F32>::key(cand(lo)) == qkey) {
            const int slot = kMaxW - nw + ((lo - k0) >> 5);
            const uint32_t bit = 0x80000000u >> ((lo - k0) & 31);
#pragma unroll
            for (int i = 0; i < kMaxW; ++i)
                if (i == slot && (wq[i] & bit)) {
                    wq[i] &= ~bit;
                    --hits;
                }
        }
    }
    if (__ballot(lconf != 0ull)) conf += wave_sum(lconf);
    if (lane == 0 && conf) atomicAdd(&stats->ctr[stripe][kCtrConfirms], conf);
    if (!small) s_cnt[w][lane] = hits;
    if constexpr (OUT == kOutDensity) {
        // The lane's hits in its part, in ascending index.
        if (!small) {
            // The words are taken four at a time (128 candidates): the loop
            // over one block runs as long as its busiest lane, so larger
            // blocks leave fewer lanes idle.  Each neighbour's coordinates
            // (and mass) are loaded one hit ahead of their use, so a load is
            // in flight while the previous term is evaluated; the coordinates
            // come from the tree-ordered copy (the entries' keys are tree
            // positions).  The terms are added in ascending candidate order.
            static_assert(kMaxW % 4 == 0, "words are taken four at a time");
            double acc = 0.0;
            const int wbase = kMaxW - nw;  // slots below it hold zeros
            const double hq = 0.5 * R;
#pragma unroll
            for (int i = 0; i < kMaxW; i += 4) {
                uint64_t wa = qv ? ((uint64_t)wq[i] << 32) | wq[i + 1] : 0ull;
                uint64_t wb = qv ? ((uint64_t)wq[i + 2] << 32) | wq[i + 3] : 0ull;
                const int kb = k0 + 32 * (i - wbase);  // the candidate of wa's top bit
                // The block's next hit (its candidate number), or -1.
                auto pop = [&]() -> int {
                    const bool ua = wa != 0ull;
                    const uint64_t x = ua ? wa : wb;
                    if (x == 0ull) return -1;
                    const int j = __clzll(x);
                    const uint64_t bit = 0x8000000000000000ull >> j;
                    if (ua) wa ^= bit;
                    else wb ^= bit;
                    return kb + j + (ua ? 0 : 64);
                };
                int k = pop();
                double4 o = make_double4(0.0, 0.0, 0.0, 0.0);
                double mj = 1.0;
                if (k >= 0) {
                    o = src[Ent<F32>::key(cand(k))];
                    if (dout.mass) mj = dout.mass[(int)o.w];
                }
                while (k >= 0) {
                    const int kn = pop();
                    double4 on = o;
                    double mn = mj;
                    if (kn >= 0) {
                        on = src[Ent<F32>::key(cand(kn))];
                        if (dout.mass) mn = dout.mass[(int)on.w];
                    }
                    const double dx = __dsub_rn(qp.x, o.x), dy = __dsub_rn(qp.y, o.y);
                    const double dz = __dsub_rn(qp.z, o.z);
                    const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                                __dmul_rn(dz, dz));
                    const double wv = sph_shape(d2, hq);
                    acc += dout.mass ? __dmul_rn(mj, wv) : wv;
                    o = on;
                    mj = mn;
                    k = kn;
                }
            }
            dacc = acc;
        }
    }
    __syncthreads();
    if constexpr (OUT == kOutDensity) {
        // Every wavefront is past its last use of the buckets: the other
        // wavefronts' sums go there for wavefront 0.
        double* const s_dens = reinterpret_cast<double*>(s_bk);
        if (w != 0) s_dens[w * 64 + lane] = dacc;
        __syncthreads();
    }
    if constexpr (OUT != kOutRows) {
        // Counts (and densities: the wavefronts' parts added in order); no
        // rows.
        if (w == 0) {
            int c = 0;
#pragma unroll
            for (int k = 0; k < kWaves; ++k) c += s_cnt[k][lane];
            if (qv) counts[qidx] = c;
            if constexpr (OUT == kOutDensity) {
                const double* const s_dens = reinterpret_cast<const double*>(s_bk);
                const double sum = ((dacc + s_dens[64 + lane]) + s_dens[128 + lane]) +
                                   s_dens[192 + lane];
                if (qv) dout.rho[qidx] = sph_density(sum, c, 0.5 * R);
            }
            if (lane == 0) {
                unsigned long long tests = (unsigned long long)C * (unsigned long long)ch.cnt;
                atomicAdd(&stats->ctr[stripe][kCtrPairs], tests);
                atomicAdd(&stats->ctr[stripe][kCtrCands], (unsigned long long)C);
            }
        }
        return 0;
    }

    // Row lengths, then one scratch allocation for the item: its rows, or
    // (main sweep) its test words and candidates when they take less room
    // than the rows (k_expand's cost goes with the items, k_place's with
    // the rows, so items of few queries or few hits keep their rows).
    if (w == 0) {
        int c = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) c += s_cnt[k][lane];
        if (!qv) c = 0;
        const int inc = wave_incl_scan(c);
        s_qoff[lane] = inc - c;
        const int rows_total = __builtin_amdgcn_readlane(inc, 63);
        int total = rows_total;
        bool use_bits = false;
        if constexpr (kBits) {
            const int btotal = ((C + 31) >> 5) * ch.cnt + C;
            use_bits = kBitsNum * btotal < kBitsDen * total;
            if (use_bits) total = btotal;
        }
        if (lane == 0) {
            s_bits = use_bits ? 1 : 0;
            s_rows_total = rows_total;
            s_total = total;
            s_base = atomicAdd(&scur[stripe * kStripeStride], (unsigned long long)total);
            atomicAdd(&stats->ctr[stripe][kCtrPairs], (unsigned long long)C * (unsigned long long)ch.cnt);
            atomicAdd(&stats->ctr[stripe][kCtrCands], (unsigned long long)C);
        }
        if (qv) counts[qidx] = c;
    }
    __syncthreads();
    const int64_t region = scap / kStripes;  // this stripe's share of the scratch
    const int64_t rbase = (int64_t)s_base;
    const int64_t base = rbase + (int64_t)stripe * region;
    if (rbase + s_total > region) {
        // Scratch too small this time: counts are right; the rows are redone
        // once the scratch has grown to the need the cursors now hold.
        if (t == 0) atomicOr(&ctl->overflow, kOvfScratch);
        if (kBits && t == 0) irec[ci] = ItemRows{-1, 0, 0};
        if (w == 0 && qv) soff[qidx] = -2;
        return 0;
    }
    if (kBits && s_bits) {
        // Words: wavefront w's g-th word of query q at (w B / 32 + g) qs + q,
        // stored by the item's lanes together; then the candidates.
        const int qs = ch.cnt;
        const int g0 = k0 >> 5;
#pragma unroll
        for (int i = 0; i < kMaxW; ++i) {
            const int wi = i - (kMaxW - nw);
            if (wi >= 0 && qv) scratch[base + (int64_t)(g0 + wi) * qs + lane] = (int32_t)wq[i];
        }
        const int64_t kbase = base + (int64_t)((C + 31) >> 5) * qs;
        for (int k = t; k < C; k += kWG) scratch[kbase + k] = Ent<F32>::key(cand(k)) - sbeg;
        if (w == 0 && qv) soff[qidx] = -3;  // k_place leaves the row to k_expand
        if (t == 0) {
            irec[ci] = ItemRows{base, C, qs};
            atomicAdd(&stats->ctr[stripe][kCtrWords], 1ull);
            if (s_rows_total > kRowBuf) atomicAdd(&stats->ctr[stripe][kCtrWide], 1ull);
        }
        return 0;
    }
    if (kBits && t == 0) irec[ci] = ItemRows{-1, 0, 0};  // rows through k_place
    if (w == 0 && qv) soff[qidx] = base + s_qoff[lane];
    if (small) {
        unsigned long long unused = 0;
        const uint64_t below = (1ull << lane) - 1ull;
        for (int q = 0; q < ch.cnt; ++q) {
            const Q Qd = query(q);
            int64_t at = base + s_qoff[q];
            for (int k = 0; k < w; ++k) at += s_cnt[k][q];
            for (int c = ch0; c < ch1; ++c) {
                const uint64_t m = chunk_hits(Qd, c, unused);
                if ((m >> lane) & 1)
                    scratch[at + __popcll(m & below)] = Ent<F32>::key(cand(c * 64 + lane)) - sbeg;
                at += __popcll(m);
            }
        }
        return 0;
    }
    // Rows: lane q of wavefront w writes the hits of its block right after
    // those of the blocks of lower wavefronts (ascending original index).
    // Every lane writes a row of its own, so the stores are scattered: once
    // the lane's position is 16-byte aligned it collects four entries and
    // writes them with one store.  (Assembling the item's rows in shared
    // memory for coalesced stores was slower: the extra barriers put every
    // wavefront's extraction on the item's critical path.)
    if (qv) {
        int64_t at0 = base + s_qoff[lane];
        for (int k = 0; k < w; ++k) at0 += s_cnt[k][lane];
        // Positions from here on are relative to the lane's first entry;
        // `head` entries go one by one up to the first 16-byte boundary.
        int32_t* const row = scratch + at0;
        int head = (int)((4 - (at0 & 3)) & 3);
        int at = 0;
        int32_t b0 = 0, b1 = 0, b2 = 0, b3 = 0;
        int nb = 0;
#pragma unroll
        for (int i = 0; i < kMaxW; ++i) {
            const int wi = i - (kMaxW - nw);  // word index within the block
            if (wi >= 0) {
                uint32_t word = wq[i];
                const int kb = k0 + 32 * wi;
                while (word) {
                    const int j = __clz(word);
                    word &= ~(0x80000000u >> j);
                    const int32_t v = Ent<F32>::key(cand(kb + j)) - sbeg;
                    if (head > 0) {
                        row[at++] = v;
                        --head;
                        continue;
                    }
                    b0 = b1;
                    b1 = b2;
                    b2 = b3;
                    b3 = v;
                    if (++nb == 4) {
                        *reinterpret_cast<int4*>(row + at) = make_int4(b0, b1, b2, b3);
                        at += 4;
                        nb = 0;
                    }
                }
            }
        }
        // The last one to three entries sit at the top of the buffer.
        if (nb == 3) {
            row[at] = b1;
            row[at + 1] = b2;
            row[at + 2] = b3;
        } else if (nb == 2) {
            row[at] = b2;
            row[at + 1] = b3;
        } else if (nb == 1) {
            row[at] = b3;
        }
    }
    return 0;
}

// The sweep: workgroup g takes work item g.  The grid is the host's bound on
// the item count (exact after an eager build; a captured graph uses a bound
// with a margin and reports an item count above it as an overflow).  Items
// whose candidates overflow the shared-memory budget are listed for
// k_sweep_split.
template <bool F32, int OUT>
__global__ __launch_bounds__(kWG) void k_sweep(const Chunk* __restrict__ chunks,
                                               const double4* __restrict__ pos,
                                               const double4* __restrict__ orig,
                                               const Node* __restrict__ nodes,
                                               const int32_t* __restrict__ ctab,
                                               const Leaf* __restrict__ leaves,
                                               const int2* __restrict__ lrange,
                                               const SetDev* __restrict__ sets,
                                               const double* __restrict__ h,
                                               int32_t* __restrict__ counts,
                                               int64_t* __restrict__ soff,
                                               int32_t* __restrict__ scratch, int64_t scap,
                                               unsigned long long* __restrict__ scur,
                                               Ctl* __restrict__ ctl, Chunk* __restrict__ split,
                                               int32_t* __restrict__ split_ci,
                                               const int4* __restrict__ whdr,
                                               const int2* __restrict__ wl,
                                               const ItemBox* __restrict__ ibox,
                                               Stats* __restrict__ stats, const int excl,
                                               const DensOut dout, ItemRows* __restrict__ irec,
                                               const int item_cap) {
    if (ctl->data_bad || (ctl->overflow & kOvfTree)) return;
    // More items than the per-item buffers hold (a replay recorded for fewer):
    // the host grows them and records again.
    const int nch = ctl->n_chunks;
    if (blockIdx.x == 0 && threadIdx.x == 0 && nch > item_cap) atomicOr(&ctl->overflow, kOvfChunks);
    const int nit = min(nch, item_cap);
    const int ci = xcd_item(blockIdx.x, nit);
    if (ci >= nit) return;
    const Chunk ch = chunks[ci];
    const int C = sweep_item<F32, 1, kCMax, kLMax, false, OUT>(
        ci, ch, whdr, wl, ibox, pos, orig, nodes, ctab, leaves, lrange, sets, h, counts, soff,
        scratch, scap, scur, stripe_of(ch.beg), ctl, stats, excl, dout, irec);
    if (C && threadIdx.x == 0) {
        if (OUT == kOutRows) irec[ci] = ItemRows{-1, 0, 0};
        const uint32_t k = atomicAdd(&ctl->nsplit, 1u);
        split[k] = Chunk{ch.beg, ch.cnt, ch.set, C};
        split_ci[k] = ci;
        atomicAdd(&stats->ctr[stripe_of(ch.beg)][kCtrSplit], 1ull);
    }
}

// Shared-memory budget of the split kernel: it runs rarely, so it trades
// occupancy for capacity (FP32 form 64 KB of candidates, FP64 form 96 KB).
template <bool F32> constexpr int kCMaxSplit = F32 ? 4096 : 3072;
constexpr int kLMaxSplit = 2048;

// Lists a unit (up to 64 queries of one set) for the exhaustive path.
__device__ __forceinline__ void to_brute(const Chunk q, const double4* __restrict__ pos,
                                         int64_t* __restrict__ soff, Ctl* __restrict__ ctl,
                                         Chunk* __restrict__ brute, int32_t* __restrict__ bcnt,
                                         Stats* __restrict__ stats) {
    if (threadIdx.x < q.cnt) soff[(int)pos[q.beg + threadIdx.x].w] = -1;
    if (threadIdx.x == 0) {
        brute[atomicAdd(&ctl->nbrute, 1u)] = Chunk{q.beg, q.cnt, q.set, 0};
        atomicAdd(&bcnt[q.set], q.cnt);
        atomicAdd(&stats->ctr[stripe_of(q.beg)][kCtrBrute], (unsigned long long)q.cnt);
    }
}

// Work items that overflowed are searched again in three levels, each a
// launch persistent over its list, so that the units of one item run in
// parallel on different workgroups:
//   level 1: the whole item, with the larger shared-memory budget;
//   level 2: its sub-items of kSubGroup queries (each with its own box E);
//   level 3: single queries.
// A unit that still overflows goes to the next level, and from level 3 to
// the exhaustive path.  In a set of at most kDenseSet particles, a unit
// whose overflowing candidate count exceeds a quarter of the set goes to the
// exhaustive path at once: its box covers so much of the set that a sweep
// over the whole (small) set costs little more, and smaller boxes would
// overflow too.  In larger sets a sweep of the whole set by one workgroup
// would be long, so units there go down to single queries first.
constexpr int64_t kDenseSet = 32768;
// Split levels from this one take their units from a counter; level 1
// keeps a fixed stride over its list (measured faster there).
constexpr int kDynFrom = 2;

template <bool F32, int LEVEL, int OUT>
__global__ __launch_bounds__(kWG) void k_sweep_split(const Chunk* __restrict__ in,
                                                     Chunk* __restrict__ next,
                                                     const int32_t* __restrict__ split_ci,
                                                     const int4* __restrict__ whdr,
                                                     const int2* __restrict__ wl,
                                                     const ItemBox* __restrict__ ibox,
                                                     const double4* __restrict__ pos,
                                                     const double4* __restrict__ orig,
                                                     const Node* __restrict__ nodes,
                                                     const int32_t* __restrict__ ctab,
                                                     const Leaf* __restrict__ leaves,
                                                     const int2* __restrict__ lrange,
                                                     const SetDev* __restrict__ sets,
                                                     const double* __restrict__ h,
                                                     int32_t* __restrict__ counts,
                                                     int64_t* __restrict__ soff,
                                                     int32_t* __restrict__ scratch, int64_t scap,
                                                     unsigned long long* __restrict__ scur,
                                                     Ctl* __restrict__ ctl,
                                                     Chunk* __restrict__ brute,
                                                     int32_t* __restrict__ bcnt,
                                                     Stats* __restrict__ stats, const int excl,
                                                     const DensOut dout) {
    if (ctl->data_bad || (ctl->overflow & kOvfTree)) return;
    // Units of this level: level 1 takes each listed item whole; levels 2
    // and 3 cut each listed unit into parts of kSubGroup queries or of one.
    constexpr int kPart = LEVEL == 1 ? kGroup : LEVEL == 2 ? kSubGroup : 1;
    constexpr int kParts = LEVEL == 1 ? 1 : LEVEL == 2 ? kGroup / kSubGroup : kSubGroup;
    const uint32_t nin = LEVEL == 1 ? ctl->nsplit : LEVEL == 2 ? ctl->nsplit2 : ctl->nsplit3;
    const uint64_t units = (uint64_t)nin * kParts;
    // The parts of levels 2 and 3 differ widely in cost, so there a
    // workgroup that is done with a unit takes the next one from a counter
    // (a fixed stride over the list left a few workgroups with long chains
    // of heavy units).  Every workgroup's first unit is its own index, so a
    // short list costs no atomics.
    constexpr bool kDynamic = LEVEL >= kDynFrom;
    __shared__ uint32_t s_take;
    bool first = true;
    for (uint64_t us = blockIdx.x;; us += gridDim.x) {
        __syncthreads();  // the previous unit is done with the shared memory
        uint64_t u = us;
        if (kDynamic && !first) {
            if (threadIdx.x == 0) s_take = atomicAdd(&ctl->split_take[LEVEL - 1], 1u);
            __syncthreads();
            u = (uint64_t)gridDim.x + s_take;
        }
        first = false;
        if (u >= units) break;
        const Chunk src = in[u / kParts];
        const int q0 = (int)(u % kParts) * kPart;
        if (q0 >= src.cnt) continue;  // uniform: the unit is empty
        const Chunk unit{src.beg + q0, min(kPart, src.cnt - q0), src.set, 0};
        const int64_t nset = sets[unit.set].n;
        if (LEVEL == 1 && nset <= kDenseSet && src.pad != kNoCount && 4 * (int64_t)src.pad > nset) {
            to_brute(unit, pos, soff, ctl, brute, bcnt, stats);
            continue;
        }
        if (LEVEL == 1 && src.pad < kHuge && src.pad > kCMaxSplit<F32>) {
            // The main sweep counted the candidates inside this item's box
            // (the same box here): more than this budget too, so the item
            // goes on to the parts without being staged again.
            if (threadIdx.x == 0)
                next[atomicAdd(&ctl->nsplit2, 1u)] = Chunk{unit.beg, unit.cnt, unit.set, src.pad};
            continue;
        }
        // Level 1 takes the item whole: its walk list, if whole, still holds.
        const int ci = LEVEL == 1 ? split_ci[u] : -1;
        const int C = sweep_item<F32, 2, kCMaxSplit<F32>, kLMaxSplit, (LEVEL >= 2), OUT>(
            ci, unit, whdr, wl, LEVEL == 1 ? ibox : nullptr, pos, orig, nodes, ctab, leaves, lrange,
            sets, h, counts, soff, scratch, scap, scur, stripe_of(unit.beg), ctl, stats, excl,
            dout, nullptr);
        if (!C) continue;
        __syncthreads();
        if (LEVEL == 3 || (nset <= kDenseSet && C != kNoCount && 4 * (int64_t)C > nset)) {
            to_brute(unit, pos, soff, ctl, brute, bcnt, stats);
        } else if (threadIdx.x == 0) {
            uint32_t* cnt = LEVEL == 1 ? &ctl->nsplit2 : &ctl->nsplit3;
            next[atomicAdd(cnt, 1u)] = Chunk{unit.beg, unit.cnt, unit.set, C};
        }
    }
}

// Rows from the scratch into the CSR array (original order).  A wavefront
// takes 64 consecutive rows (lane r loads row r's length, source and
// destination) and copies them four at a time with all its lanes, so every
// load and store is coalesced and no lane searches for its row; the first
// 128 entries of the four rows are loaded before any is stored, so that
// eight loads per lane are in flight.  Rows taken by the exhaustive path,
// rows that k_expand writes from an item's words and rows without room in
// the scratch (soff < 0) count as empty here.  Nothing is written when the
// rows do not fit the caller's capacity.
__device__ __forceinline__ int64_t readlane64(int64_t v, int j) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), j);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__global__ __launch_bounds__(kWG) void k_place(const int32_t* __restrict__ counts,
                                               const int64_t* __restrict__ soff,
                                               const int64_t* __restrict__ offsets,
                                               const int32_t* __restrict__ scratch,
                                               int32_t* __restrict__ nbrs, int64_t n,
                                               int64_t capacity, Ctl* __restrict__ ctl) {
    if (ctl->data_bad || (ctl->overflow & (kOvfTree | kOvfChunks))) return;
    if (offsets[n] > capacity) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctl->overflow, kOvfCapacity);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int64_t wid = ((int64_t)blockIdx.x * kWG + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * kWG) >> 6;
    for (int64_t r0 = wid * 64; r0 < n; r0 += nw * 64) {
        const int64_t i = r0 + lane;
        int64_t so = 0, o = 0;
        int c = 0;
        if (i < n) {
            so = soff[i];
            o = offsets[i];
            c = so >= 0 ? counts[i] : 0;
            if (so < 0) so = 0;
        }
        for (int j0 = 0; j0 < 64; j0 += 4) {
            const int c0 = __builtin_amdgcn_readlane(c, j0);
            const int c1 = __builtin_amdgcn_readlane(c, j0 + 1);
            const int c2 = __builtin_amdgcn_readlane(c, j0 + 2);
            const int c3 = __builtin_amdgcn_readlane(c, j0 + 3);
            if ((c0 | c1 | c2 | c3) == 0) continue;
            const int64_t s0 = readlane64(so, j0), s1 = readlane64(so, j0 + 1);
            const int64_t s2 = readlane64(so, j0 + 2), s3 = readlane64(so, j0 + 3);
            const int64_t d0 = readlane64(o, j0), d1 = readlane64(o, j0 + 1);
            const int64_t d2 = readlane64(o, j0 + 2), d3 = readlane64(o, j0 + 3);
            const int ka = lane, kb = lane + 64;
            const int32_t a0 = ka < c0 ? scratch[s0 + ka] : 0, b0 = kb < c0 ? scratch[s0 + kb] : 0;
            const int32_t a1 = ka < c1 ? scratch[s1 + ka] : 0, b1 = kb < c1 ? scratch[s1 + kb] : 0;
            const int32_t a2 = ka < c2 ? scratch[s2 + ka] : 0, b2 = kb < c2 ? scratch[s2 + kb] : 0;
            const int32_t a3 = ka < c3 ? scratch[s3 + ka] : 0, b3 = kb < c3 ? scratch[s3 + kb] : 0;
            if (ka < c0) nbrs[d0 + ka] = a0;
            if (kb < c0) nbrs[d0 + kb] = b0;
            if (ka < c1) nbrs[d1 + ka] = a1;
            if (kb < c1) nbrs[d1 + kb] = b1;
            if (ka < c2) nbrs[d2 + ka] = a2;
            if (kb < c2) nbrs[d2 + kb] = b2;
            if (ka < c3) nbrs[d3 + ka] = a3;
            if (kb < c3) nbrs[d3 + kb] = b3;
            // Entries past the first 128 of a row.
            for (int k = lane + 128; k < c0; k += 64) nbrs[d0 + k] = scratch[s0 + k];
            for (int k = lane + 128; k < c1; k += 64) nbrs[d1 + k] = scratch[s1 + k];
            for (int k = lane + 128; k < c2; k += 64) nbrs[d2 + k] = scratch[s2 + k];
            for (int k = lane + 128; k < c3; k += 64) nbrs[d3 + k] = scratch[s3 + k];
        }
    }
}

// Pass 2 of the main sweep's work items: the test words and ordered
// candidates that pass 1 left in the scratch (ItemRows) are expanded into
// the caller's CSR rows, which saves the scratch round trip of the rows
// (they are several times larger than the words).  The expansion is the
// sweep's: lane q of wavefront w takes query q's words over w's quarter of
// the candidates and puts its hits after those of the lower wavefronts
// (ascending original index) into a shared-memory image of the item's rows,
// as 16-bit candidate numbers; then each wavefront copies whole rows out
// with consecutive lanes on consecutive entries, so that the lines inside a
// row are written together and leave the L2 whole (only a row's two end
// lines are partial; rows stored lane by lane, 16 bytes of 64 different rows
// per store, took 1.5-2 times as long).  Rows longer than the image go
// through it in windows of kRowBuf entries.  A row is written only when its words hold
// exactly the count pass 1 recorded, so every store stays inside the row's
// own range of the CSR.
__global__ __launch_bounds__(kWG) void k_expand(const Chunk* __restrict__ chunks,
                                                const ItemRows* __restrict__ irec,
                                                const double4* __restrict__ pos,
                                                const int32_t* __restrict__ counts,
                                                const int64_t* __restrict__ offsets,
                                                const int32_t* __restrict__ scratch, int64_t scap,
                                                int32_t* __restrict__ nbrs, int64_t n,
                                                int64_t capacity, const Ctl* __restrict__ ctl,
                                                const int item_cap, const unsigned blocks) {
    constexpr int kMaxW = ((kCMax / kWaves) + 31) / 32;
    static_assert(kCMax <= 65536, "candidate numbers are 16-bit");
    __shared__ int32_t s_key[kCMax];
    __shared__ uint16_t s_rows[kRowBuf];
    __shared__ int32_t s_cnt[kWaves][64];
    __shared__ int32_t s_cq[64];
    __shared__ int64_t s_dst[64];
    // Nothing is written after a failed pass 1 or when the rows do not fit
    // (k_place raises that flag).
    if (ctl->data_bad || (ctl->overflow & (kOvfTree | kOvfChunks | kOvfScratch))) return;
    if (offsets[n] > capacity) return;
    const int nit = min(ctl->n_chunks, item_cap);
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    // The stride keeps each workgroup on its XCD in the sweep's item order.
    for (unsigned b = blockIdx.x; b < blocks; b += gridDim.x) {
        const int ci = xcd_item(b, nit);
        if (ci >= nit) continue;
        const ItemRows r = irec[ci];
        const Chunk ch = chunks[ci];
        const int C = r.C, qs = r.qs;
        const int64_t nwt = (C + 31) >> 5;
        if (r.off < 0 || C <= 0 || C > kCMax || qs != ch.cnt || r.off + nwt * qs + C > scap)
            continue;
        const int32_t* const words = scratch + r.off;
        const int32_t* const keys = words + nwt * qs;
        const bool qv = lane < qs;
        // Wavefront 0 fetches the queries' counts and destinations while
        // every wavefront fetches its words.
        int cq = -1;
        int64_t dq = 0;
        if (w == 0 && qv) {
            const int qidx = (int)pos[ch.beg + lane].w;
            cq = counts[qidx];
            dq = offsets[qidx];
        }
        __syncthreads();  // the previous item is done with the shared memory
        for (int k = t; k < C; k += kWG) s_key[k] = keys[k];
        // This wavefront's block of candidates, as in the sweep.
        const int B = ((C + kWaves * 32 - 1) / (kWaves * 32)) * 32;
        const int k0 = w * B;
        const int k1 = min(k0 + B, C);
        const int nw = (k1 > k0) ? (k1 - k0 + 31) >> 5 : 0;
        uint32_t wq[kMaxW];
        int hits = 0;
#pragma unroll
        for (int i = 0; i < kMaxW; ++i) {
            wq[i] = (i < nw && qv) ? (uint32_t)words[((k0 >> 5) + i) * (int64_t)qs + lane] : 0u;
            hits += __popc(wq[i]);
        }
        s_cnt[w][lane] = hits;
        if (w == 0) {
            s_cq[lane] = cq;
            s_dst[lane] = dq;
        }
        __syncthreads();
        // Every wavefront: row lengths (0 for a row that does not match its
        // count) and their offsets in the item's row image.
        int tot = 0, before = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            const int c = s_cnt[k][lane];
            tot += c;
            if (k < w) before += c;
        }
        const int len = (qv && tot == s_cq[lane]) ? tot : 0;
        const int inc = wave_incl_scan(len);
        const int qoff = inc - len;
        const int total = __builtin_amdgcn_readlane(inc, 63);
        const int lo = qoff + before;  // this lane's first entry in the image
        for (int r0 = 0; r0 < total; r0 += kRowBuf) {
            const int r1 = r0 + kRowBuf;
            if (len > 0 && lo < r1 && lo + hits > r0) {
                // The common case, the whole image at once, needs no bounds
                // per entry.
                const bool whole = total <= kRowBuf;
                int at = lo - r0;
#pragma unroll
                for (int i = 0; i < kMaxW; ++i) {
                    if (i < nw) {
                        uint32_t word = wq[i];
                        const int kb = k0 + 32 * i;
                        if (whole) {
                            while (word) {
                                const int j = __clz(word);
                                word &= ~(0x80000000u >> j);
                                s_rows[at++] = (uint16_t)(kb + j);
                            }
                        } else {
                            while (word) {
                                const int j = __clz(word);
                                word &= ~(0x80000000u >> j);
                                if (at >= 0 && at < kRowBuf) s_rows[at] = (uint16_t)(kb + j);
                                ++at;
                            }
                        }
                    }
                }
            }
            __syncthreads();
            // Whole rows (their parts in this window) out, one wavefront per row.
            for (int q = w; q < qs; q += kWaves) {
                const int lq = __builtin_amdgcn_readlane(len, q);
                if (lq <= 0) continue;
                const int sq = __builtin_amdgcn_readlane(qoff, q);
                const int a = max(sq, r0), e = min(sq + lq, r1);
                int32_t* const dst = nbrs + s_dst[q];
                for (int j = a + lane; j < e; j += 64) dst[j - sq] = s_key[s_rows[j - r0]];
            }
            if (r1 < total) __syncthreads();  // the image is refilled
        }
    }
}

// The exhaustive path takes its queries in units of up to 64 queries of one
// set.  The split levels list units of 1, 8 or 64 queries; before the
// sweep they are regrouped by set into full units, so that every lane of
// the sweep has a query.  The count pass cuts each unit's sweep over its set
// into spans of kDenseSpan candidates, one workgroup each, so that a large
// set does not make one workgroup the critical path; the fill pass uses the
// same spans when their counts fit the task table (else whole units).
// `bset` holds, for
// nsets sets: listed queries [0, nsets), fill cursors [nsets, 2 nsets),
// query offsets [2 nsets, 3 nsets + 1), unit offsets [3 nsets + 1,
// 4 nsets + 2) and count-task offsets [4 nsets + 2, 5 nsets + 3).
constexpr int kDenseTile = 768;
constexpr int64_t kDenseSpan = 12 * kDenseTile;

__device__ __forceinline__ int64_t dense_spans(int64_t nset, int64_t span) {
    return nset > 0 ? (nset + span - 1) / span : 1;
}

// Query, unit and count-task offsets per set (one workgroup).
__global__ __launch_bounds__(kWG) void k_brute_plan(int32_t* __restrict__ bset, int nsets,
                                                    const SetDev* __restrict__ sets,
                                                    Ctl* __restrict__ ctl) {
    __shared__ int64_t sh[kWaves + 1];
    const int32_t* cnt = bset;
    int32_t* fill = bset + nsets;
    int32_t* off = bset + 2 * nsets;
    int32_t* uoff = off + nsets + 1;
    int32_t* toff = uoff + nsets + 1;
    // Span of a count task: kDenseSpan, or the whole set should the tasks
    // not be countable in 32 bits.
    int64_t all = 0;
    for (int s = threadIdx.x; s < nsets; s += kWG)
        all += (cnt[s] + kGroup - 1) / kGroup * dense_spans(sets[s].n, kDenseSpan);
    all = block_sum<kWG>(all, sh);
    const int64_t span = all <= INT32_MAX ? kDenseSpan : (int64_t)INT32_MAX;
    int64_t qrun = 0, urun = 0, trun = 0;
    for (int s0 = 0; s0 < nsets; s0 += kWG) {
        const int s = s0 + (int)threadIdx.x;
        const int64_t c = s < nsets ? cnt[s] : 0;
        const int64_t units = (c + kGroup - 1) / kGroup;
        const int64_t tasks = s < nsets ? units * dense_spans(sets[s].n, span) : 0;
        int64_t tq, tu, tt;
        const int64_t eq = block_excl_scan<kWG>(c, sh, &tq);
        const int64_t eu = block_excl_scan<kWG>(units, sh, &tu);
        const int64_t et = block_excl_scan<kWG>(tasks, sh, &tt);
        if (s < nsets) {
            off[s] = (int32_t)(qrun + eq);
            uoff[s] = (int32_t)(urun + eu);
            toff[s] = (int32_t)(trun + et);
            fill[s] = 0;
        }
        qrun += tq;
        urun += tu;
        trun += tt;
    }
    if (threadIdx.x == 0) {
        off[nsets] = (int32_t)qrun;
        uoff[nsets] = (int32_t)urun;
        toff[nsets] = (int32_t)trun;
        ctl->nbunits = (uint32_t)urun;
        ctl->nbtasks = (uint32_t)trun;
        ctl->bspan = span;
        ctl->bfill_tasks = trun <= kDenseTaskCap ? 1 : 0;
    }
}

// The listed units' queries into their set's segment of `bq` (one
// wavefront per listed unit; the order inside a set is free).
__global__ __launch_bounds__(kWG) void k_brute_group(const Chunk* __restrict__ blist,
                                                     const Ctl* __restrict__ ctl,
                                                     int32_t* __restrict__ bset, int nsets,
                                                     int32_t* __restrict__ bq,
                                                     const double4* __restrict__ pos,
                                                     int32_t* __restrict__ counts) {
    int32_t* fill = bset + nsets;
    const int32_t* off = bset + 2 * nsets;
    const uint32_t nb = ctl->nbrute;
    const int lane = lane_id();
    const int64_t nw = ((int64_t)gridDim.x * kWG) >> 6;
    for (int64_t k = ((int64_t)blockIdx.x * kWG + threadIdx.x) >> 6; k < nb; k += nw) {
        const Chunk ch = blist[k];
        int base = 0;
        if (lane == 0) base = atomicAdd(&fill[ch.set], ch.cnt);
        base = __shfl(base, 0, 64);
        if (lane < ch.cnt) {
            bq[off[ch.set] + base + lane] = ch.beg + lane;
            counts[(int)pos[ch.beg + lane].w] = 0;  // the count pass adds its spans
        }
    }
}

// Exhaustive sweep of the regrouped units (lane q of every wavefront holds
// query q of the unit): the set's particles, already in original index
// order in `orig`, pass through shared memory in tiles of kDenseTile;
// wavefront w tests its quarter of each tile with the FP64 predicate, one
// bit per (query, candidate).  Count mode adds the bits of one span of the
// set to the query's count and, when the tasks fit kDenseTaskCap, records
// it per task and lane; fill mode then runs by the same tasks and writes
// each row in ascending index at offsets[i] plus the hits of the unit's
// earlier spans, earlier tiles and lower wavefronts (else it sweeps the
// whole set per unit).  Persistent over the tasks or units.
constexpr int kDenseWords = kDenseTile / kWaves / 32;  // words per wavefront and tile

template <int MODE>
__global__ __launch_bounds__(kWG) void k_dense(const int32_t* __restrict__ bq,
                                               const int32_t* __restrict__ bset, int nsets,
                                               int32_t* __restrict__ btab,
                                               const SetDev* __restrict__ sets,
                                               const double4* __restrict__ pos,
                                               const double4* __restrict__ orig,
                                               const double* __restrict__ h,
                                               int32_t* __restrict__ counts,
                                               const int64_t* __restrict__ offsets, int64_t n,
                                               int64_t capacity, int32_t* __restrict__ nbrs,
                                               Ctl* __restrict__ ctl, const int excl,
                                               const DensOut dout) {
    __shared__ double4 s_c[kDenseTile];
    __shared__ int32_t s_cnt[kWaves][64];
    if (ctl->data_bad || (ctl->overflow & kOvfTree)) return;
    if (MODE == kFill && ((ctl->overflow & kOvfChunks) || offsets[n] > capacity)) return;
    const int32_t* bcnt = bset;
    const int32_t* off = bset + 2 * nsets;
    const int32_t* uoff = off + nsets + 1;
    const int32_t* toff = uoff + nsets + 1;
    // The density form takes each unit whole (one workgroup adds all of a
    // query's terms, in a fixed order).
    const bool by_task = MODE == kCount || (MODE == kFill && ctl->bfill_tasks);
    const int32_t* woff = by_task ? toff : uoff;  // first task / unit of each set
    const uint32_t nwork = by_task ? ctl->nbtasks : ctl->nbunits;
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    for (uint32_t u = blockIdx.x; u < nwork; u += gridDim.x) {
        // Set of task u: the last set whose first task is at most u.
        int slo = 0, shi = nsets - 1;
        while (slo < shi) {
            const int mid = (slo + shi + 1) >> 1;
            if ((uint32_t)woff[mid] <= u) slo = mid;
            else shi = mid - 1;
        }
        const int set = slo;
        const int64_t jb = sets[set].beg, jn = sets[set].n;
        const int64_t span = by_task ? ctl->bspan : jn;
        const int64_t spans = by_task ? dense_spans(jn, span) : 1;
        const int64_t local = (int64_t)u - woff[set];
        const int j = (int)(local / spans);             // unit within the set
        const int64_t ks = local % spans;               // span within the unit
        const int64_t c0 = ks * span;                   // this task's candidates [c0, c1)
        const int64_t c1 = min(jn, c0 + span);
        const int qcnt = min(kGroup, bcnt[set] - kGroup * j);
        const bool qv = lane < qcnt;
        const int qpos = qv ? bq[off[set] + kGroup * j + lane] : 0;
        const double4 qp = qv ? pos[qpos] : make_double4(0.0, 0.0, 0.0, 0.0);
        const int qidx = (int)qp.w;
        const double R = qv ? 2.0 * h[qpos] : 0.0;
        const double r2 = qv ? __dmul_rn(R, R) : -1.0;  // nothing is below -1
        int64_t run = (MODE == kFill && qv) ? offsets[qidx] : 0;
        if (MODE == kFill && by_task && qv)
            for (int64_t k = 0; k < ks; ++k) run += btab[((int64_t)u - ks + k) * 64 + lane];
        int64_t hits = 0;
        double dsum = 0.0;  // density form: this lane's terms, tile by tile
        for (int64_t t0 = c0; t0 < c1; t0 += kDenseTile) {
            __syncthreads();  // the previous tile is no longer read
            for (int i = t; i < kDenseTile; i += kWG) {
                const int64_t j = t0 + i;
                s_c[i] = j < c1 ? orig[jb + j] : make_double4(NAN, NAN, NAN, 0.0);
            }
            __syncthreads();
            uint32_t wd[kDenseWords];
            int mine = 0;
#pragma unroll
            for (int b = 0; b < kDenseWords; ++b) {
                uint32_t word = 0;
                const int k0 = w * (kDenseTile / kWaves) + 32 * b;
                for (int g = 0; g < 32; g += 4) {
                    double4 e[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) e[j] = s_c[k0 + g + j];
                    double d2[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const double dx = __dsub_rn(qp.x, e[j].x);
                        const double dy = __dsub_rn(qp.y, e[j].y);
                        const double dz = __dsub_rn(qp.z, e[j].z);
                        d2[j] = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                          __dmul_rn(dz, dz));
                    }
                    push4_f64(word, d2[0], d2[1], d2[2], d2[3], r2);
                }
                if (excl) {  // the query's own bit (its index local to the set)
                    const int64_t d = (int64_t)qidx - jb - (t0 + k0);
                    if (d >= 0 && d < 32) word &= ~(0x80000000u >> d);
                }
                wd[b] = word;
                mine += __popc(word);
            }
            if (MODE == kCount || MODE == kDens) {
                hits += mine;
                if (MODE == kDens && qv) {
#pragma unroll
                    for (int b = 0; b < kDenseWords; ++b) {
                        uint32_t word = wd[b];
                        const int k0 = w * (kDenseTile / kWaves) + 32 * b;
                        while (word) {
                            const int j = __clz(word);
                            word &= ~(0x80000000u >> j);
                            dsum += sph_term(qp.x, qp.y, qp.z, 0.5 * R,
                                             (int)(jb + t0 + k0 + j), orig, dout.mass);
                        }
                    }
                }
            } else {
                s_cnt[w][lane] = mine;
                __syncthreads();
                int64_t at = run;
                int tot = 0;
#pragma unroll
                for (int v = 0; v < kWaves; ++v) {
                    const int c = s_cnt[v][lane];
                    if (v < w) at += c;
                    tot += c;
                }
                if (qv) {
#pragma unroll
                    for (int b = 0; b < kDenseWords; ++b) {
                        uint32_t word = wd[b];
                        const int64_t k0 = t0 + w * (kDenseTile / kWaves) + 32 * b;
                        while (word) {
                            const int j = __clz(word);
                            word &= ~(0x80000000u >> j);
                            nbrs[at++] = (int32_t)(k0 + j);
                        }
                    }
                }
                run += tot;
            }
        }
        if (MODE == kCount) {
            __syncthreads();
            s_cnt[w][lane] = (int)hits;
            __syncthreads();
            if (w == 0) {
                const int tot = s_cnt[0][lane] + s_cnt[1][lane] + s_cnt[2][lane] + s_cnt[3][lane];
                if (qv) atomicAdd(&counts[qidx], tot);
                if (ctl->bfill_tasks) btab[(int64_t)u * 64 + lane] = qv ? tot : 0;
            }
        }
        if constexpr (MODE == kDens) {
            __shared__ double s_ds[kWaves][64];
            __syncthreads();
            s_cnt[w][lane] = (int)hits;
            s_ds[w][lane] = dsum;
            __syncthreads();
            if (w == 0 && qv) {
                const int tot = s_cnt[0][lane] + s_cnt[1][lane] + s_cnt[2][lane] + s_cnt[3][lane];
                counts[qidx] = tot;
                const double sum = ((s_ds[0][lane] + s_ds[1][lane]) + s_ds[2][lane]) + s_ds[3][lane];
                dout.rho[qidx] = sph_density(sum, tot, 0.5 * R);
            }
        }
        __syncthreads();
    }
}

// Clears the search's part of the control block and the search counters.
__global__ void k_find_reset(Ctl* __restrict__ ctl, Stats* __restrict__ stats,
                             unsigned long long* __restrict__ stripes, int32_t* __restrict__ bcnt,
                             int nsets) {
    if (threadIdx.x < 2 * kStripes) stripes[threadIdx.x * kStripeStride] = 0;
    for (int s = threadIdx.x; s < nsets; s += blockDim.x) bcnt[s] = 0;
    if (threadIdx.x == 0) {
        ctl->queue = 0;
        ctl->nsplit = 0;
        ctl->nsplit2 = 0;
        ctl->nsplit3 = 0;
        for (int k = 0; k < 3; ++k) ctl->split_take[k] = 0;
        ctl->nbrute = 0;
        ctl->nbunits = 0;
        ctl->nbtasks = 0;
        ctl->nadapt = 0;
        ctl->data_bad &= 1;  // keep a bad coordinate seen by the build
        ctl->overflow &= ~(kOvfScratch | kOvfCapacity | kOvfChunks | kOvfWalk);
    }
    if (threadIdx.x < kStripes)
        for (int k = 0; k < kCtrCount; ++k) stats->ctr[threadIdx.x][k] = 0;
}

// Brackets of the h adaptation: lo = 0 and hi = +inf (none known yet).
__global__ void k_adapt_init(double2* __restrict__ br, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        br[i] = make_double2(0.0, INFINITY);
}

// One round of the h adaptation (original order).  A particle with h > 0
// whose count c is off the target T by more than tol records its h as the
// lower (c < T) or upper (c > T) end of its bracket, and proposes h f with
// f = min(2, (5c + T) / (6c)) (2 when c = 0): half the first-order step
// towards (T / c)^(1/3) around c = T.  A proposal that leaves the bracket
// is replaced by the bracket's midpoint, so a particle whose band
// [T - tol, T + tol] is reachable cannot cycle.  Basic operations only,
// each rounded once, so every platform takes the same steps.
__global__ void k_adapt_h(const int32_t* __restrict__ counts, double* __restrict__ h,
                          double2* __restrict__ br, int64_t n, double target, double tol,
                          Ctl* __restrict__ ctl) {
    unsigned mine = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double c = (double)counts[i];
        const double hv = h[i];
        if (fabs(__dsub_rn(c, target)) <= tol || hv == 0.0) continue;  // done, or cannot move
        double2 b = br[i];
        if (c < target) b.x = hv;
        else b.y = hv;
        double f = 2.0;
        if (c > 0.0)
            f = fmin(2.0, __ddiv_rn(__dadd_rn(__dmul_rn(5.0, c), target), __dmul_rn(6.0, c)));
        double p = __dmul_rn(hv, f);
        if (p >= b.y || p <= b.x) p = __dmul_rn(__dadd_rn(b.x, b.y), 0.5);
        h[i] = p;
        br[i] = b;
        ++mine;
    }
    // One atomic per workgroup (the grid strides over the particles).
    __shared__ unsigned s_mine[kWG / 64];
    mine = wave_sum(mine);
    if (lane_id() == 0) s_mine[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int k = 0; k < kWG / 64; ++k) tot += s_mine[k];
        if (tot) atomicAdd(&ctl->nadapt, tot);
    }
}

// Lists per set: totals[k] = offsets[end of set k] - offsets[start of set k].
__global__ void k_set_totals(const int64_t* __restrict__ offsets, const SetDev* __restrict__ sets,
                             int nsets, int64_t* __restrict__ totals) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nsets; k += gridDim.x * blockDim.x)
        totals[k] = offsets[sets[k].beg + sets[k].n] - offsets[sets[k].beg];
}

constexpr unsigned kBruteGrid = 512;
constexpr unsigned kExpandGrid = 1u << 30;  // k_expand: one workgroup per item
constexpr int64_t kWalkPerItem = 64;  // mean leaf entries per item the walk pool holds
constexpr unsigned kSplitGrid = 1024;

// item_cap: work items the per-item buffers hold (the grid covers them).
template <bool F32, int OUT>
void launch_sweep(Tree& t, const double* h, int32_t* counts, int item_cap, DensOut dout,
                  hipStream_t st) {
    const unsigned grid = xcd_grid(item_cap);
    hipLaunchKernelGGL((k_sweep<F32, OUT>), dim3(grid), dim3(kWG), 0, st, t.chunks.as<Chunk>(),
                       t.pos.as<double4>(), t.orig.as<double4>(), t.nodes.as<Node>(),
                       t.ctab.as<int32_t>(), t.leaves.as<Leaf>(), t.lrange.as<int2>(),
                       t.sets.as<SetDev>(), t.hs.as<double>(), counts, t.soff.as<int64_t>(),
                       t.scratch.as<int32_t>(), t.scap, t.stripes.as<unsigned long long>(),
                       t.ctl.as<Ctl>(), t.split.as<Chunk>(), t.split_ci.as<int32_t>(),
                       t.whdr.as<int4>(), t.wl.as<int2>(), t.ibox.as<ItemBox>(),
                       t.stats.as<Stats>(), t.prm.exclude_self, dout, t.irec.as<ItemRows>(),
                       item_cap);
    BT_LAUNCH();
}

template <bool F32, int LEVEL, int OUT>
void launch_split_level(Tree& t, const double* h, int32_t* counts, const Chunk* in, Chunk* next,
                        DensOut dout, hipStream_t st) {
    hipLaunchKernelGGL((k_sweep_split<F32, LEVEL, OUT>), dim3(kSplitGrid), dim3(kWG), 0, st, in,
                       next, t.split_ci.as<int32_t>(), t.whdr.as<int4>(), t.wl.as<int2>(),
                       t.ibox.as<ItemBox>(), t.pos.as<double4>(), t.orig.as<double4>(),
                       t.nodes.as<Node>(), t.ctab.as<int32_t>(), t.leaves.as<Leaf>(), t.lrange.as<int2>(),
                       t.sets.as<SetDev>(), t.hs.as<double>(), counts, t.soff.as<int64_t>(),
                       t.scratch.as<int32_t>(), t.scap, t.stripes.as<unsigned long long>(),
                       t.ctl.as<Ctl>(), t.blist.as<Chunk>(), t.bset.as<int32_t>(),
                       t.stats.as<Stats>(), t.prm.exclude_self, dout);
    BT_LAUNCH();
}

template <bool F32, int OUT>
void launch_split(Tree& t, const double* h, int32_t* counts, DensOut dout, hipStream_t st) {
    Chunk* l1 = t.split.as<Chunk>();
    Chunk* l2 = l1 + t.leaf_cap;
    Chunk* l3 = l2 + t.leaf_cap;
    launch_split_level<F32, 1, OUT>(t, h, counts, l1, l2, dout, st);
    launch_split_level<F32, 2, OUT>(t, h, counts, l2, l3, dout, st);
    launch_split_level<F32, 3, OUT>(t, h, counts, l3, nullptr, dout, st);
}

template <int MODE>
void launch_dense(Tree& t, int32_t* counts, const int64_t* offsets, int64_t capacity,
                  int32_t* nbrs, DensOut dout, hipStream_t st) {
    hipLaunchKernelGGL((k_dense<MODE>), dim3(kBruteGrid), dim3(kWG), 0, st, t.bq.as<int32_t>(),
                       t.bset.as<int32_t>(), (int)t.nsets, t.btab.as<int32_t>(),
                       t.sets.as<SetDev>(), t.pos.as<double4>(), t.orig.as<double4>(),
                       t.hs.as<double>(), counts, offsets, t.n, capacity, nbrs, t.ctl.as<Ctl>(),
                       t.prm.exclude_self, dout);
    BT_LAUNCH();
}

// Split levels and the exhaustive path's plan, regrouping and sweep of one
// search pass (OUT: what it writes).
template <int OUT>
void counts_tail(Tree& t, const double* h, int32_t* counts, DensOut dout, hipStream_t st) {
    if (t.prm.precision == BTREE_FP32_FILTER) launch_split<true, OUT>(t, h, counts, dout, st);
    else launch_split<false, OUT>(t, h, counts, dout, st);
    hipLaunchKernelGGL(k_brute_plan, dim3(1), dim3(kWG), 0, st, t.bset.as<int32_t>(),
                       (int)t.nsets, t.sets.as<SetDev>(), t.ctl.as<Ctl>());
    BT_LAUNCH();
    hipLaunchKernelGGL(k_brute_group, dim3(kBruteGrid), dim3(kWG), 0, st, t.blist.as<Chunk>(),
                       t.ctl.as<Ctl>(), t.bset.as<int32_t>(), (int)t.nsets, t.bq.as<int32_t>(),
                       t.pos.as<double4>(), counts);
    BT_LAUNCH();
    if (OUT == kOutDensity)
        launch_dense<kDens>(t, counts, nullptr, 0, nullptr, dout, st);
    else
        launch_dense<kCount>(t, counts, nullptr, 0, nullptr, dout, st);
}

}  // namespace

void find_reserve(Tree& t, int64_t entries) {
    t.soff.reserve(sizeof(int64_t) * std::max<int64_t>(t.n, 1));
    t.stripes.reserve(sizeof(unsigned long long) * 2 * kStripes * kStripeStride);
    t.hs.reserve(sizeof(double) * std::max<int64_t>(t.n, 1));
    // Walk results: a header per work item and a pool of leaf entries (an
    // item that does not fit the pool is searched by the split path).
    const int64_t items = std::max<int64_t>(std::max(t.n_chunks, t.chunk_cap), 1);
    t.whdr.reserve(sizeof(int4) * items);
    t.ibox.reserve(sizeof(ItemBox) * items);
    t.irec.reserve(sizeof(ItemRows) * items);
    const int64_t wl_want = std::max(kWalkPerItem * items, t.wl_need);
    if (t.wl_cap < wl_want) {
        t.wl.release();
        t.wl_cap = 0;
        t.wl.reserve(sizeof(int2) * wl_want);
        t.wl_cap = wl_want;
    }
    if (entries > t.scap) {
        t.scratch.release();
        t.scap = 0;
        t.scratch.reserve(sizeof(int32_t) * entries);
        t.scap = entries;
    }
}

void find_begin(Tree& t, const double* h, hipStream_t st) {
    hipLaunchKernelGGL(k_find_reset, dim3(1), dim3(2 * kStripes), 0, st, t.ctl.as<Ctl>(),
                       t.stats.as<Stats>(), t.stripes.as<unsigned long long>(),
                       t.bset.as<int32_t>(), (int)t.nsets);
    BT_LAUNCH();
}

void find_walk(Tree& t, const double* h, int64_t grid, hipStream_t st) {
    const int cap = (int)std::min<int64_t>(std::max<int64_t>(grid, 1), INT32_MAX);
    const unsigned g = xcd_grid(cap);
    hipLaunchKernelGGL(k_walk, dim3(g), dim3(64), 0, st, t.chunks.as<Chunk>(), t.pos.as<double4>(),
                       t.nodes.as<Node>(), t.ctab.as<int32_t>(), t.leaves.as<Leaf>(),
                       t.lrange.as<int2>(), t.sets.as<SetDev>(), h, t.hs.as<double>(),
                       t.whdr.as<int4>(),
                       t.wl.as<int2>(), t.wl_cap,
                       t.stripes.as<unsigned long long>() + kStripes * kStripeStride,
                       t.ibox.as<ItemBox>(), t.ctl.as<Ctl>(), cap);
    BT_LAUNCH();
}

void find_sweep(Tree& t, const double* h, int32_t* counts, int64_t grid, hipStream_t st) {
    const int cap = (int)std::min<int64_t>(std::max<int64_t>(grid, 1), INT32_MAX);
    t.sweep_cap = cap;
    const DensOut none{nullptr, nullptr};
    if (t.prm.precision == BTREE_FP32_FILTER) launch_sweep<true, kOutRows>(t, h, counts, cap, none, st);
    else launch_sweep<false, kOutRows>(t, h, counts, cap, none, st);
}

void find_counts_end(Tree& t, const double* h, int32_t* counts, int64_t* offsets, hipStream_t st) {
    counts_tail<kOutRows>(t, h, counts, DensOut{nullptr, nullptr}, st);
    scan_exclusive_i32(counts, offsets, t.n, t, st, &t.ctl.as<Ctl>()->data_bad);
}

// A search pass that writes counts, or counts and densities, and no rows:
// queued, then one host read of the control block for errors.  A walk-list
// pool found too small is grown for the next pass (the items that did not
// fit were searched by the split levels, so this pass is complete).
void find_no_rows(Tree& t, const double* h, int32_t* counts, const double* mass, double* rho,
                  hipStream_t st) {
    find_reserve(t, std::max<int64_t>(t.scap, 1));
    const DensOut d{mass, rho};
    const int g = (int)std::max<int64_t>(t.n_chunks, 1);  // items the buffers hold
    find_begin(t, h, st);
    find_walk(t, h, t.n_chunks, st);
    t.timer.start(kPhSweep, st);
    if (rho) {
        if (t.prm.precision == BTREE_FP32_FILTER) launch_sweep<true, kOutDensity>(t, h, counts, g, d, st);
        else launch_sweep<false, kOutDensity>(t, h, counts, g, d, st);
    } else {
        if (t.prm.precision == BTREE_FP32_FILTER) launch_sweep<true, kOutCount>(t, h, counts, g, d, st);
        else launch_sweep<false, kOutCount>(t, h, counts, g, d, st);
    }
    t.timer.stop(kPhSweep, st);
    if (rho) counts_tail<kOutDensity>(t, h, counts, d, st);
    else counts_tail<kOutCount>(t, h, counts, d, st);
    BT_HIP(hipMemcpyAsync(&t.host_ctl, t.ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    BT_HIP(hipMemcpyAsync(&t.host_stats, t.stats.p, sizeof(Stats), hipMemcpyDeviceToHost, st));
    BT_HIP(hipMemcpyAsync(t.host_stripes, t.stripes.p, sizeof t.host_stripes,
                          hipMemcpyDeviceToHost, st));
    BT_HIP(hipStreamSynchronize(st));
    if (t.host_ctl.data_bad & 2) fail(BTREE_EINVAL, "h must be finite and >= 0");
    if (t.host_ctl.overflow & kOvfChunks) fail(BTREE_EDEVICE, "work items out of date");
    if (t.host_ctl.overflow & kOvfWalk) grow_pools(t, kOvfWalk);
}

void find_place(Tree& t, const int32_t* counts, const int64_t* offsets, int32_t* nbrs,
                int64_t capacity, hipStream_t st) {
    const int64_t waves = (t.n + 63) / 64;
    unsigned grid = grid_for(waves < 1 ? 1 : waves, kWG / 64);
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_place, dim3(grid), dim3(kWG), 0, st, counts, t.soff.as<int64_t>(), offsets,
                       t.scratch.as<int32_t>(), nbrs, t.n, capacity, t.ctl.as<Ctl>());
    BT_LAUNCH();
}

// Pass 2: the rows of the exhaustive path, then the rows from the scratch
// into the caller's CSR (k_place, bound by HBM); the two write disjoint
// rows.  Then the per-set totals, when asked for.  `time_place` times
// k_place alone (not inside a graph capture).
void find_fill(Tree& t, const int32_t* counts, const int64_t* offsets, int32_t* nbrs,
               int64_t capacity, int64_t* totals, bool time_place, hipStream_t st) {
    // The kernels below read counts and offsets of every particle (nbrs may
    // be null with a capacity of 0: nothing is written then).
    if (t.n > 0 && (!counts || !offsets))
        fail(BTREE_EDEVICE, "find_fill: counts or offsets missing");
    launch_dense<kFill>(t, nullptr, offsets, capacity, nbrs, DensOut{nullptr, nullptr}, st);
    if (time_place) t.timer.start(kPhPlace, st);
    if (t.n > 0 && t.sweep_cap > 0) {
        const int cap = (int)t.sweep_cap;
        const unsigned blocks = xcd_grid(cap);
        hipLaunchKernelGGL(k_expand, dim3(std::min(blocks, kExpandGrid)), dim3(kWG), 0, st,
                           t.chunks.as<Chunk>(), t.irec.as<ItemRows>(), t.pos.as<double4>(),
                           counts, offsets, t.scratch.as<int32_t>(), t.scap, nbrs, t.n,
                           capacity, t.ctl.as<Ctl>(), cap, blocks);
        BT_LAUNCH();
    }
    find_place(t, counts, offsets, nbrs, capacity, st);
    if (time_place) t.timer.stop(kPhPlace, st);
    if (totals) {
        hipLaunchKernelGGL(k_set_totals, dim3(grid_for(t.nsets, 256)), dim3(256), 0, st, offsets,
                           t.sets.as<SetDev>(), t.nsets, totals);
        BT_LAUNCH();
    }
}

void grow_pools(Tree& t, int overflow) {
    int64_t sneed = 0, wneed = 0;
    for (int k = 0; k < kStripes; ++k) {
        sneed = std::max<int64_t>(sneed, (int64_t)t.host_stripes[k * kStripeStride]);
        wneed = std::max<int64_t>(wneed, (int64_t)t.host_stripes[(kStripes + k) * kStripeStride]);
    }
    // Every stripe gets the largest stripe's need, with room.
    if (overflow & kOvfWalk) t.wl_need = std::max(2 * t.wl_cap, kStripes * (wneed + wneed / 4 + 64));
    find_reserve(t, (overflow & kOvfScratch)
                        ? std::max(t.scap + t.scap / 2, kStripes * (sneed + sneed / 8 + 1024))
                        : t.scap);
}

int64_t find_pass1(Tree& t, const double* h, int32_t* counts, int64_t* offsets, hipStream_t st) {
    if (t.scap == 0) find_reserve(t, std::max<int64_t>(t.n * 128, 1 << 20));
    else find_reserve(t, t.scap);
    int64_t total = 0;
    for (int attempt = 0; attempt < 4; ++attempt) {
        find_begin(t, h, st);
        find_walk(t, h, t.n_chunks, st);
        t.timer.start(kPhSweep, st);
        find_sweep(t, h, counts, t.n_chunks, st);
        t.timer.stop(kPhSweep, st);
        find_counts_end(t, h, counts, offsets, st);
        BT_HIP(hipMemcpyAsync(&total, offsets + t.n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(&t.host_ctl, t.ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(&t.host_stats, t.stats.p, sizeof(Stats), hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(t.host_stripes, t.stripes.p, sizeof t.host_stripes,
                              hipMemcpyDeviceToHost, st));
        BT_HIP(hipStreamSynchronize(st));
        if (t.host_ctl.data_bad & 2) fail(BTREE_EINVAL, "btree_find_neighbors: h must be finite and >= 0");
        if (t.host_ctl.overflow & kOvfChunks) fail(BTREE_EDEVICE, "btree_find_neighbors: work items out of date");
        if (!(t.host_ctl.overflow & (kOvfScratch | kOvfWalk))) break;
        if (attempt == 3)
            fail(BTREE_EDEVICE, "btree_find_neighbors: scratch sizing failed (overflow bits " +
                                    std::to_string(t.host_ctl.overflow) + ", scratch " +
                                    std::to_string(t.scap) + ", walk pool " +
                                    std::to_string(t.wl_cap) + ")");
        // Rows or walk lists did not fit: grow to the exact need, search again.
        grow_pools(t, t.host_ctl.overflow);
    }
    return total;
}

void adapt_h_begin(Tree& t, hipStream_t st) {
    t.adapt_br.reserve(sizeof(double2) * (size_t)std::max<int64_t>(t.n, 1));
    hipLaunchKernelGGL(k_adapt_init, dim3(std::min<unsigned>(grid_for(t.n, 256), 4096u)),
                       dim3(256), 0, st, t.adapt_br.as<double2>(), t.n);
    BT_LAUNCH();
}

int64_t adapt_h_step(Tree& t, double* h, const int32_t* counts, double target, double tol,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_adapt_h, dim3(std::min<unsigned>(grid_for(t.n, kWG), 4096u)), dim3(kWG),
                       0, st, counts, h, t.adapt_br.as<double2>(), t.n, target, tol,
                       t.ctl.as<Ctl>());
    BT_LAUNCH();
    BT_HIP(hipMemcpyAsync(&t.host_ctl, t.ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    BT_HIP(hipStreamSynchronize(st));
    return (int64_t)t.host_ctl.nadapt;
}

void find_pass2(Tree& t, const double* h, const int64_t* offsets, int32_t* nbrs, hipStream_t st) {
    (void)h;  // pass 1 kept h in tree order
    find_fill(t, t.p1_counts, offsets, nbrs, INT64_MAX, nullptr, true, st);
}

}  // namespace bt

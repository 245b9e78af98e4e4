// BuildTree on the device (Section 3.1, Algorithm 1, Eqs. 1-4), for one or
// many independent particle sets at once.
//
// The recursion of Algorithm 1 runs level by level: every cell that still
// holds more than s particles at depth L (in any set) is split in the same
// group of launches.  Per level:
//   1. each cell lists its branching candidates b0 (Eq. 1), b0/2, ..., 2;
//   2. one pass over the cell's particles histograms all candidates at once
//      (Eqs. 2-3); the halving loop of Step 3 depends only on these
//      histograms, so computing them together gives the same b as halving
//      one round at a time;
//   3. the first candidate whose Eq. 4 ratio does not exceed beta (or b = 2)
//      is kept;
//   4. the kept histogram is scanned in Morton order of the sub-cell
//      coordinates, giving every non-empty sub-cell a segment of the cell's
//      particle range; sub-cells above s become cells of the next level,
//      the others leaves;
//   5. particles are scattered into their sub-cell segments.
// Cell ranges, pool use and counters live in a device control block (Ctl):
// the per-cell kernels loop over the range they read there, so a whole build
// can be queued without host reads (and captured in a graph).  Pools are
// sized from bounds; a level that would not fit raises an overflow bit and
// stops the build, and the host grows the pools and builds again.
//
// Before the levels, particles are put in Morton order of their set's root
// box (the paper reorders particles along the walk curve for locality; here
// it also lets neighbouring lanes share sub-cells and combine atomics).
// Particles ping-pong between two buffers; a leaf made at depth d keeps its
// particles in buffer d % 2 until the final pass sorts each leaf along a
// 63-bit Morton curve and writes the tree-ordered copy.
#include "prim.h"

#include <algorithm>
#include <cmath>

namespace bt {

namespace {

constexpr int kT = 256;

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// Zeroes a[0 .. *len) and b[0 .. *len), the length read on the device.

__global__ void k_ctl_reset(Ctl* __restrict__ ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Ctl c{};
        *ctl = c;
    }
}

// A1: validate coordinates, original-order copy (.w = the particle's index),
// bounding-box partials per tile.
__global__ __launch_bounds__(kT) void k_ingest(const double* __restrict__ x,
                                               const double* __restrict__ y,
                                               const double* __restrict__ z,
                                               const Tile* __restrict__ tiles,
                                               double4* __restrict__ orig,
                                               double* __restrict__ part, Ctl* __restrict__ ctl) {
    const Tile T = tiles[blockIdx.x];
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int64_t i = T.beg + threadIdx.x; i < T.end; i += kT) {
        const double a = x[i], b = y[i], c = z[i];
        bad |= !(isfinite(a) && isfinite(b) && isfinite(c));
        orig[i] = make_double4(a, b, c, (double)i);  // .w: the index, as in the tree copy
        mn[0] = fmin(mn[0], a); mx[0] = fmax(mx[0], a);
        mn[1] = fmin(mn[1], b); mx[1] = fmax(mx[1], b);
        mn[2] = fmin(mn[2], c); mx[2] = fmax(mx[2], c);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctl->data_bad, 1);
    __shared__ double sh[6][kT / 64];
    const int w = threadIdx.x >> 6;
    for (int k = 0; k < 3; ++k) {
        const double a = wave_min(mn[k]);
        const double b = wave_max(mx[k]);
        if (lane_id() == 0) { sh[k][w] = a; sh[3 + k][w] = b; }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = sh[threadIdx.x][0];
        for (int k = 1; k < kT / 64; ++k)
            v = threadIdx.x < 3 ? fmin(v, sh[threadIdx.x][k]) : fmax(v, sh[threadIdx.x][k]);
        part[blockIdx.x * 6 + threadIdx.x] = v;
    }
}

// A2: root box of each set (tight per-axis bounding box).
__global__ __launch_bounds__(64) void k_setbox(const double* __restrict__ part,
                                               const int64_t* __restrict__ settile,
                                               SetDev* __restrict__ sets) {
    const int k = blockIdx.x;
    const int64_t t0 = settile[k], t1 = settile[k + 1];
    for (int c = 0; c < 6; ++c) {
        double v = c < 3 ? INFINITY : -INFINITY;
        for (int64_t i = t0 + threadIdx.x; i < t1; i += 64)
            v = c < 3 ? fmin(v, part[i * 6 + c]) : fmax(v, part[i * 6 + c]);
        v = c < 3 ? wave_min(v) : wave_max(v);
        if (threadIdx.x == 0) sets[k].box[c] = (t1 > t0) ? v : 0.0;
    }
}

// A3: sort key = set id above a Morton code of the particle in its set's
// root box (Eq. 2 with b = 2^abits per axis).
__global__ __launch_bounds__(kT) void k_morton(const double4* __restrict__ orig,
                                               const Tile* __restrict__ tiles,
                                               const SetDev* __restrict__ sets, int abits,
                                               uint32_t* __restrict__ keys,
                                               int32_t* __restrict__ vals) {
    const Tile T = tiles[blockIdx.x];
    const SetDev& S = sets[T.set];
    const int B = 1 << abits;
    const uint32_t top = (uint32_t)T.set << (3 * abits);
    for (int64_t i = T.beg + threadIdx.x; i < T.end; i += kT) {
        const double4 q = orig[i];
        const uint32_t kx = (uint32_t)subcell(q.x, S.box[0], S.box[3], B);
        const uint32_t ky = (uint32_t)subcell(q.y, S.box[1], S.box[4], B);
        const uint32_t kz = (uint32_t)subcell(q.z, S.box[2], S.box[5], B);
        keys[i] = top | spread3(kx) | (spread3(ky) << 1) | (spread3(kz) << 2);
        vals[i] = (int32_t)i;
    }
}

// Root cell of every set: an internal cell if it holds more than s particles
// (and the depth guard allows a split), else a single leaf.
__global__ void k_roots(SetDev* __restrict__ sets, int nsets, Node* __restrict__ nodes,
                        Leaf* __restrict__ leaves, int32_t* __restrict__ ldepth,
                        Ctl* __restrict__ ctl) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int ni = 0, li = 0;
    for (int k = 0; k < nsets; ++k) {
        SetDev& S = sets[k];
        if (S.n == 0) {
            S.root = kEmpty;
        } else if (S.n > S.s && S.max_depth > 0) {
            Node R;
            for (int c = 0; c < 3; ++c) { R.lo[c] = S.box[c]; R.hi[c] = S.box[3 + c]; }
            R.ctab = -1; R.b = 0; R.n = (int32_t)S.n; R.beg = (int32_t)S.beg; R.depth = 0;
            R.set = k; R.pad = 0;
            nodes[ni] = R;
            S.root = ni++;
        } else {
            leaves[li] = Leaf{(int32_t)S.beg, (int32_t)S.n};
            ldepth[li] = 0;
            S.root = (li++) | kLeafBit;
        }
    }
    ctl->n_nodes = ni;
    ctl->n_leaves = li;
    ctl->cur_nb = 0;
    ctl->cur_ne = ni;
    ctl->lvm = ni;
    ctl->ct_len = 0;
}

// Particles in Morton order; those of sets with an internal root start in it.
__global__ __launch_bounds__(kT) void k_gather(const double4* __restrict__ orig,
                                               const int32_t* __restrict__ perm,
                                               const Tile* __restrict__ tiles,
                                               double4* __restrict__ P0) {
    const Tile T = tiles[blockIdx.x];
    // Eight particles per thread and step, so that eight independent
    // index -> particle load chains are in flight.
    constexpr int kU = 8;
    for (int64_t k0 = T.beg + threadIdx.x; k0 < T.end; k0 += kT * kU) {
        int32_t i[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t k = k0 + u * kT;
            i[u] = k < T.end ? perm[k] : -1;
        }
        double4 q[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (i[u] >= 0) q[u] = orig[i[u]];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (i[u] < 0) continue;
            const int64_t k = k0 + u * kT;
            P0[k] = make_double4(q[u].x, q[u].y, q[u].z, (double)i[u]);
        }
    }
}

// ---------------------------------------------------------------------------
// Level kernels.  The cells of the level are nodes [cur_nb, cur_ne).
// ---------------------------------------------------------------------------

// The histogram and scatter kernels take tasks of up to kRunR consecutive
// particles of one cell (the particles follow the Morton curve inside each
// cell).  The cell's bins, up to kLdsBins / kLdsHistBins of them, are
// counted in shared memory and added to global memory once per task; the
// other bins use global atomics, one per distinct bin and wavefront.
// Without this, the coarse bins of a large cell (b = 2: eight bins for
// millions of particles) serialise millions of same-address atomics.
constexpr int kRunPer = 8;
constexpr int kRunR = kT * kRunPer;
constexpr int kLdsBins = 8192;      // scatter: int32 counters
constexpr int kLdsHistBins = 16384;  // histogram: two 16-bit counters per word (<= kRunR each)

// Step 1: histogram size of all branching candidates of each cell, and its
// number of particle tasks.  The cell's b field holds the first candidate
// (Eq. 1) until k_select replaces it with the chosen one.
__global__ void k_candidates(Node* __restrict__ nodes, const SetDev* __restrict__ sets,
                             const Ctl* __restrict__ ctl, int64_t* __restrict__ hsize,
                             int64_t* __restrict__ tcnt) {
    const int64_t nb = ctl->cur_nb, m = ctl->lvm;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Node& N = nodes[nb + i];
        const int b = first_branching(N.n, sets[N.set]);
        nodes[nb + i].b = b;
        int64_t sum = 0;
        for (int bb = b;; bb = halve(bb)) {
            sum += (int64_t)bb * bb * bb;
            if (bb == 2) break;
        }
        hsize[i] = sum;
        tcnt[i] = ((int64_t)N.n + kRunR - 1) / kRunR;
    }
}

// Histogram length of the level (stop the build if it exceeds the pool),
// and the histogram and slot cursors cleared up to it.  Every workgroup
// derives the length itself; the first records it.
__global__ void k_hist_zero(Ctl* __restrict__ ctl, const int64_t* __restrict__ hoff, int64_t cap,
                            int32_t* __restrict__ hist, int32_t* __restrict__ cursor) {
    const int64_t m = ctl->lvm;
    const int64_t len = m > 0 ? hoff[m] : 0;
    const bool ok = m > 0 && len <= cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (m > 0 && !ok) ctl->overflow |= kOvfHist;
        ctl->level_ok = ok ? 1 : 0;
        ctl->hist_len = ok ? len : 0;
    }
    if (!ok) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        hist[i] = 0;
        cursor[i] = 0;
    }
}

// Cell of task u of the level: the last cell whose first task is at most u.
__device__ __forceinline__ int64_t task_cell(const int64_t* __restrict__ toff, int64_t m, int64_t u) {
    int64_t lo = 0, hi = m - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (toff[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Adds 1 per active lane to a 16-bit counter packed two to a word in shared
// memory.  A wavefront whose active lanes all hit one bin adds with one
// atomic (the common case for coarse bins, where per-lane atomics would all
// conflict on one address).
__device__ __forceinline__ void lds_inc16(uint32_t* w, int32_t bin, bool active) {
    const uint64_t act = __ballot(active);
    if (!act) return;
    const int first = __ffsll((unsigned long long)act) - 1;
    const int32_t b0 = __shfl(bin, first, 64);
    if (__ballot(active && bin == b0) == act) {
        if (lane_id() == first) atomicAdd(&w[b0 >> 1], (uint32_t)__popcll(act) << ((b0 & 1) * 16));
    } else if (active) {
        atomicAdd(&w[bin >> 1], 1u << ((bin & 1) * 16));
    }
}

// Rank of each active lane among the task's particles of its bin, from
// int32 counters in shared memory (one atomic when the wavefront's active
// lanes share one bin).
__device__ __forceinline__ int32_t lds_rank(int32_t* cnt, int32_t bin, bool active) {
    const uint64_t act = __ballot(active);
    if (!act) return 0;
    const int first = __ffsll((unsigned long long)act) - 1;
    const int32_t b0 = __shfl(bin, first, 64);
    if (__ballot(active && bin == b0) == act) {
        int32_t base = 0;
        if (lane_id() == first) base = atomicAdd(&cnt[b0], (int32_t)__popcll(act));
        base = __shfl(base, first, 64);
        return base + lanes_below(act);
    }
    return active ? atomicAdd(&cnt[bin], 1) : 0;
}

static_assert(kRunR < 65536, "a task's count per bin must fit 16 bits");

// Step 2: one histogram per candidate b (Eqs. 2 and 3), persistent over the
// level's tasks.  Shared window: the last kLdsHistBins bins of the cell's
// candidates (the small b, whose bins are the crowded ones).
__global__ __launch_bounds__(kT) void k_histogram(const double4* __restrict__ P,
                                                  const Node* __restrict__ nodes,
                                                  const Ctl* __restrict__ ctl,
                                                  const int64_t* __restrict__ hoff,
                                                  const int64_t* __restrict__ toff,
                                                  int32_t* __restrict__ hist) {
    if (!ctl->level_ok) return;
    __shared__ uint32_t s_bin[kLdsHistBins / 2];
    const int32_t nb = ctl->cur_nb;
    const int64_t m = ctl->lvm;
    const int64_t ntask = toff[m];
    for (int64_t u = blockIdx.x; u < ntask; u += gridDim.x) {
        const int64_t ci = task_cell(toff, m, u);
        const Node& N = nodes[nb + ci];
        const int64_t p0 = (int64_t)N.beg + (u - toff[ci]) * kRunR;
        const int64_t p1 = min((int64_t)N.beg + N.n, p0 + kRunR);
        const int64_t h0 = hoff[ci], h1 = hoff[ci + 1];
        const int64_t wlo = max(h0, h1 - kLdsHistBins);
        const int32_t wwords = (int32_t)((h1 - wlo + 1) >> 1);
        const int b0 = N.b;  // Eq. 1, set by k_candidates
        int ncand = 0;
        for (int b = b0;; b = halve(b)) {
            ++ncand;
            if (b == 2) break;
        }
        __syncthreads();  // the previous task's flush is done with s_bin
        for (int i = threadIdx.x; i < wwords; i += kT) s_bin[i] = 0;
        __syncthreads();
#pragma unroll 1
        for (int j = 0; j < kRunPer; ++j) {
            const int64_t p = p0 + j * kT + threadIdx.x;
            const bool act = p < p1;
            double tx = 0.0, ty = 0.0, tz = 0.0;
            if (act) {
                const double4 q = P[p];
                // Eq. 2 fractions per axis: the same for every candidate b.
                tx = subcell_frac(q.x, N.lo[0], N.hi[0]);
                ty = subcell_frac(q.y, N.lo[1], N.hi[1]);
                tz = subcell_frac(q.z, N.lo[2], N.hi[2]);
            }
            int64_t off = h0;
            int bb = b0;
            for (int k = 0; k < ncand; ++k) {
                const int64_t key = off + subcell_of(tx, bb) +
                                    (int64_t)bb * (subcell_of(ty, bb) + (int64_t)bb * subcell_of(tz, bb));
                off += (int64_t)bb * bb * bb;
                bb = halve(bb);
                const bool local = act && key >= wlo;
                lds_inc16(s_bin, (int32_t)(key - wlo), local);
                wave_agg_inc(hist, key, act && !local);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < wwords; i += kT) {
            const uint32_t v = s_bin[i];
            if (v & 0xffffu) atomicAdd(&hist[wlo + 2 * i], (int32_t)(v & 0xffffu));
            if (v >> 16) atomicAdd(&hist[wlo + 2 * i + 1], (int32_t)(v >> 16));
        }
    }
}

// Step 3: Eq. 4 ratio r = #{n_j < alpha*s} / b^3; halve while r > beta.
__global__ __launch_bounds__(kT) void k_select(Node* __restrict__ nodes,
                                               const SetDev* __restrict__ sets,
                                               const Ctl* __restrict__ ctl,
                                               const int64_t* __restrict__ hoff,
                                               const int32_t* __restrict__ hist,
                                               int32_t* __restrict__ bsel,
                                               int64_t* __restrict__ selofs,
                                               Stats* __restrict__ stats) {
    __shared__ int64_t sh[kT / 64 + 1];
    // Statistics summed per workgroup and sent once at the end: atomics on
    // one address are serialised, and a level can hold thousands of cells.
    __shared__ unsigned s_bh[65];
    __shared__ unsigned s_rounds;
    if (!ctl->level_ok) return;
    const int64_t nb = ctl->cur_nb, m = ctl->lvm;
    if ((int64_t)blockIdx.x >= m) return;  // uniform: no cell for this workgroup
    for (int k = threadIdx.x; k < 65; k += kT) s_bh[k] = 0;
    if (threadIdx.x == 0) s_rounds = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        const int64_t node = nb + i;
        const SetDev& S = sets[nodes[node].set];
        const double thr = S.alpha * (double)S.s;
        int64_t off = hoff[i];
        int rounds = 0;
        int bb = first_branching(nodes[node].n, S);
        for (;; bb = halve(bb), ++rounds) {
            const int64_t nc = (int64_t)bb * bb * bb;
            int64_t under = 0;
            for (int64_t c = threadIdx.x; c < nc; c += kT)
                under += ((double)hist[off + c] < thr) ? 1 : 0;
            under = block_sum<kT>(under, sh);
            const double r = (double)under / (double)nc;
            if (!(r > S.beta && bb > 2)) break;
            off += nc;
        }
        if (threadIdx.x == 0) {
            bsel[i] = bb;
            selofs[i] = off;
            nodes[node].b = bb;
            s_rounds += (unsigned)rounds;
            s_bh[bb < 64 ? bb : 64] += 1u;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 65; k += kT)
        if (s_bh[k]) atomicAdd(&stats->b_hist[k], (unsigned long long)s_bh[k]);
    if (threadIdx.x == 0 && s_rounds) atomicAdd(&stats->rounds, (unsigned long long)s_rounds);
}

constexpr int kChildItems = 4;

// Step 4a: sub-cell segments in Morton order of (x', y', z'); ranks of the
// sub-cells that become cells (n_j > s, below the depth guard) and leaves.
__global__ __launch_bounds__(kT) void k_children(const Node* __restrict__ nodes,
                                                 const SetDev* __restrict__ sets,
                                                 const Ctl* __restrict__ ctl,
                                                 const int32_t* __restrict__ bsel,
                                                 const int64_t* __restrict__ selofs,
                                                 const int32_t* __restrict__ hist,
                                                 int32_t* __restrict__ cstart,
                                                 int32_t* __restrict__ crank,
                                                 int64_t* __restrict__ nint,
                                                 int64_t* __restrict__ nleaf,
                                                 int64_t* __restrict__ ctsize) {
    __shared__ int64_t sh[kT / 64 + 1];
    if (!ctl->level_ok) return;
    const int64_t nb = ctl->cur_nb, m = ctl->lvm;
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        const Node& N = nodes[nb + i];
        const SetDev& S = sets[N.set];
        const int s = S.s;
        const int b = bsel[i];
        const int64_t off = selofs[i];
        const bool can_split = N.depth + 1 < S.max_depth;
        int p2 = 1;
        while (p2 < b) p2 <<= 1;
        const uint64_t ncodes = (uint64_t)p2 * p2 * p2;
        int64_t carry_n = 0, carry_i = 0, carry_l = 0;
        for (uint64_t m0 = 0; m0 < ncodes; m0 += (uint64_t)kT * kChildItems) {
            int64_t cell[kChildItems];
            int64_t cnt[kChildItems];
            int flags[kChildItems];  // 1 = internal, 2 = leaf
            int64_t packed = 0;
#pragma unroll
            for (int k = 0; k < kChildItems; ++k) {
                const uint64_t mc = m0 + (uint64_t)threadIdx.x * kChildItems + k;
                cell[k] = -1;
                cnt[k] = 0;
                flags[k] = 0;
                if (mc < ncodes) {
                    const uint64_t cx = compact3_64(mc), cy = compact3_64(mc >> 1),
                                   cz = compact3_64(mc >> 2);
                    if (cx < (uint64_t)b && cy < (uint64_t)b && cz < (uint64_t)b) {
                        cell[k] = (int64_t)cx + (int64_t)b * ((int64_t)cy + (int64_t)b * (int64_t)cz);
                        cnt[k] = hist[off + cell[k]];
                        if (cnt[k] > s && can_split) flags[k] = 1;
                        else if (cnt[k] > 0) flags[k] = 2;
                    }
                }
                packed += cnt[k] | ((int64_t)(flags[k] == 1) << 34) | ((int64_t)(flags[k] == 2) << 48);
            }
            int64_t tot;
            const int64_t ex = block_excl_scan<kT>(packed, sh, &tot);
            int64_t en = ex & ((1ll << 34) - 1);
            int64_t ei = (ex >> 34) & 0x3fff;
            int64_t el = (ex >> 48) & 0x3fff;
#pragma unroll
            for (int k = 0; k < kChildItems; ++k) {
                if (cell[k] >= 0) {
                    cstart[off + cell[k]] = (int32_t)(carry_n + en);
                    if (flags[k] == 1) crank[off + cell[k]] = (int32_t)(carry_i + ei);
                    if (flags[k] == 2) crank[off + cell[k]] = (int32_t)(carry_l + el);
                }
                en += cnt[k];
                ei += flags[k] == 1;
                el += flags[k] == 2;
            }
            carry_n += tot & ((1ll << 34) - 1);
            carry_i += (tot >> 34) & 0x3fff;
            carry_l += (tot >> 48) & 0x3fff;
        }
        if (threadIdx.x == 0) {
            nint[i] = carry_i;
            nleaf[i] = carry_l;
            ctsize[i] = (int64_t)b * b * b;
        }
    }
}

// Ids for the level's children; stop the build if a pool would overflow.
__global__ void k_level_alloc(Ctl* __restrict__ ctl, const int64_t* __restrict__ ibase,
                              const int64_t* __restrict__ lbase,
                              const int64_t* __restrict__ ctoff, int64_t node_cap,
                              int64_t leaf_cap, int64_t ctab_cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t m = ctl->lvm;
    if (!ctl->level_ok || m == 0) {
        ctl->level_ok = 0;
        ctl->next_nb = ctl->next_ne = ctl->cur_ne;
        return;
    }
    const int64_t new_int = ibase[m], new_leaf = lbase[m], new_ct = ctoff[m];
    int ovf = 0;
    if (ctl->n_nodes + new_int > node_cap) ovf |= kOvfNodes;
    if (ctl->n_leaves + new_leaf > leaf_cap) ovf |= kOvfLeaves;
    if (ctl->ct_len + new_ct > ctab_cap) ovf |= kOvfCtab;
    if (ovf) {
        ctl->overflow |= ovf;
        ctl->level_ok = 0;
        ctl->next_nb = ctl->next_ne = ctl->cur_ne;
        return;
    }
    ctl->lv_int0 = ctl->n_nodes;
    ctl->lv_leaf0 = ctl->n_leaves;
    ctl->lv_ct0 = ctl->ct_len;
    ctl->n_nodes += (int32_t)new_int;
    ctl->n_leaves += (int32_t)new_leaf;
    ctl->ct_len += new_ct;
    ctl->next_nb = ctl->cur_ne;
    ctl->next_ne = ctl->cur_ne + (int32_t)new_int;
}

// Step 4b: child tables, next-level cells and new leaves.
__global__ __launch_bounds__(kT) void k_emit(Node* __restrict__ nodes,
                                             const SetDev* __restrict__ sets,
                                             const Ctl* __restrict__ ctl,
                                             const int32_t* __restrict__ bsel,
                                             const int64_t* __restrict__ selofs,
                                             const int32_t* __restrict__ hist,
                                             const int32_t* __restrict__ cstart,
                                             const int32_t* __restrict__ crank,
                                             const int64_t* __restrict__ int_base,
                                             const int64_t* __restrict__ leaf_base,
                                             const int64_t* __restrict__ ctoff,
                                             int32_t* __restrict__ ctab, Leaf* __restrict__ leaves,
                                             int32_t* __restrict__ ldepth) {
    if (!ctl->level_ok) return;
    const int64_t nb = ctl->cur_nb, m = ctl->lvm;
    const int64_t int0 = ctl->lv_int0, leaf0 = ctl->lv_leaf0, ct0 = ctl->lv_ct0;
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        const int64_t node = nb + i;
        const Node N = nodes[node];
        const SetDev& S = sets[N.set];
        const int b = bsel[i];
        const int64_t off = selofs[i];
        const int64_t ct = ct0 + ctoff[i];
        const bool can_split = N.depth + 1 < S.max_depth;
        if (threadIdx.x == 0) nodes[node].ctab = ct;
        const int64_t nc = (int64_t)b * b * b;
        for (int64_t c = threadIdx.x; c < nc; c += kT) {
            const int64_t cnt = hist[off + c];
            int32_t code = kEmpty;
            if (cnt > S.s && can_split) {
                const int64_t id = int0 + int_base[i] + crank[off + c];
                const int cx = (int)(c % b), cy = (int)((c / b) % b), cz = (int)(c / ((int64_t)b * b));
                Node C;
                C.lo[0] = cell_edge(N.lo[0], N.hi[0], cx, b);
                C.hi[0] = cell_edge(N.lo[0], N.hi[0], cx + 1, b);
                C.lo[1] = cell_edge(N.lo[1], N.hi[1], cy, b);
                C.hi[1] = cell_edge(N.lo[1], N.hi[1], cy + 1, b);
                C.lo[2] = cell_edge(N.lo[2], N.hi[2], cz, b);
                C.hi[2] = cell_edge(N.lo[2], N.hi[2], cz + 1, b);
                C.ctab = -1;
                C.b = 0;
                C.n = (int32_t)cnt;
                C.beg = N.beg + cstart[off + c];
                C.depth = N.depth + 1;
                C.set = N.set;
                C.pad = 0;
                nodes[id] = C;
                code = (int32_t)id;
            } else if (cnt > 0) {
                const int64_t lid = leaf0 + leaf_base[i] + crank[off + c];
                leaves[lid] = Leaf{N.beg + cstart[off + c], (int32_t)cnt};
                ldepth[lid] = N.depth + 1;
                code = (int32_t)lid | kLeafBit;
            }
            ctab[ct + c] = code;
        }
    }
}

// Step 5: scatter each particle of a cell into its sub-cell segment,
// persistent over the level's tasks.  When the cell's b^3 fits kLdsBins,
// particles take a rank in their sub-cell from shared counters and each
// sub-cell reserves the task's slots with one global atomic; otherwise slots
// are taken per wavefront and sub-cell.  Particles that end in leaves stay
// in the destination array, those of next-level cells are read from it by
// the next level.
__global__ __launch_bounds__(kT) void k_scatter(const double4* __restrict__ Psrc,
                                                double4* __restrict__ Pdst,
                                                const Node* __restrict__ nodes,
                                                const Ctl* __restrict__ ctl,
                                                const int32_t* __restrict__ bsel,
                                                const int64_t* __restrict__ selofs,
                                                const int32_t* __restrict__ cstart,
                                                int32_t* __restrict__ cursor,
                                                const int64_t* __restrict__ toff, int64_t n) {
    if (!ctl->level_ok) return;
    __shared__ int32_t s_cnt[kLdsBins];  // counts, then the task's first slot
    const int32_t nb = ctl->cur_nb;
    const int64_t m = ctl->lvm;
    const int64_t ntask = toff[m];
    for (int64_t u = blockIdx.x; u < ntask; u += gridDim.x) {
        const int64_t ci = task_cell(toff, m, u);
        const Node& N = nodes[nb + ci];
        const int64_t p0 = (int64_t)N.beg + (u - toff[ci]) * kRunR;
        const int64_t p1 = min((int64_t)N.beg + N.n, p0 + kRunR);
        const int b = bsel[ci];
        const int64_t sel = selofs[ci];
        const int32_t wlen = (int64_t)b * b * b <= kLdsBins ? b * b * b : 0;
        __syncthreads();  // the previous task is done with s_cnt
        for (int i = threadIdx.x; i < wlen; i += kT) s_cnt[i] = 0;
        __syncthreads();
        // Particles with a shared-memory rank wait in registers for their
        // sub-cell's first slot.
        double4 q[kRunPer];
        int64_t dst[kRunPer];  // start of the sub-cell's segment; -1: nothing pending
        int32_t bin[kRunPer], rank[kRunPer];
#pragma unroll
        for (int j = 0; j < kRunPer; ++j) {
            const int64_t p = p0 + j * kT + threadIdx.x;
            const bool act = p < p1;
            int64_t key = 0, start = 0;
            int32_t c = 0;
            double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
            if (act) {
                v = Psrc[p];
                const int cx = subcell(v.x, N.lo[0], N.hi[0], b);
                const int cy = subcell(v.y, N.lo[1], N.hi[1], b);
                const int cz = subcell(v.z, N.lo[2], N.hi[2], b);
                c = cx + b * (cy + b * cz);
                key = sel + c;
                start = (int64_t)N.beg + cstart[key];
            }
            const bool local = act && wlen > 0;
            dst[j] = local ? start : -1;
            q[j] = v;
            bin[j] = c;
            rank[j] = lds_rank(s_cnt, c, local);
            const int32_t slot = wave_agg_slot(cursor, key, act && !local);
            if (act && !local) Pdst[start + slot] = v;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < wlen; i += kT) {
            const int32_t v = s_cnt[i];
            if (v) s_cnt[i] = atomicAdd(&cursor[sel + i], v);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRunPer; ++j) {
            if (dst[j] < 0) continue;
            const int64_t d = dst[j] + s_cnt[bin[j]] + rank[j];
            if ((uint64_t)d >= (uint64_t)n) continue;  // cannot happen; keeps a slot error off memory
            Pdst[d] = q[j];
        }
    }
}

// The next level becomes the current one.
__global__ void k_level_advance(Ctl* __restrict__ ctl, int level, int level_cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (ctl->lvm > 0 && ctl->level_ok) ctl->levels = level + 1;
    ctl->cur_nb = ctl->next_nb;
    ctl->cur_ne = ctl->next_ne;
    ctl->lvm = ctl->cur_ne - ctl->cur_nb;
    if (level + 1 >= level_cap && ctl->lvm > 0) ctl->overflow |= kOvfLevels;
}

// ---------------------------------------------------------------------------
// After the levels: leaves in memory order, sorted, and cut into work items.
// ---------------------------------------------------------------------------

// Leaves in particle order.  Every leaf is non-empty and leaves do not
// overlap, so their first particles are distinct: one bit per particle marks
// them, and a leaf's new id is the number of marks before its own (a scan
// over the words' bit counts, then a count inside the word).
__global__ void k_mark_bits(const Leaf* __restrict__ leaves, const Ctl* __restrict__ ctl,
                            uint32_t* __restrict__ bits) {
    const int64_t nl = ctl->n_leaves;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nl;
         l += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = leaves[l].beg;
        atomicOr(&bits[p >> 5], 1u << (p & 31));
    }
}

__global__ void k_popc(const uint32_t* __restrict__ bits, int64_t nw, int32_t* __restrict__ pc) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nw;
         k += (int64_t)gridDim.x * blockDim.x)
        pc[k] = __popc(bits[k]);
}

__global__ void k_relabel_leaves(const uint32_t* __restrict__ bits, const int64_t* __restrict__ pre,
                                 const Ctl* __restrict__ ctl, const Leaf* __restrict__ lin,
                                 const int32_t* __restrict__ din, Leaf* __restrict__ lout,
                                 int32_t* __restrict__ dout, int32_t* __restrict__ newid) {
    const int64_t nl = ctl->n_leaves;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nl;
         l += (int64_t)gridDim.x * blockDim.x) {
        const Leaf L = lin[l];
        const int32_t w = L.beg >> 5;
        const int64_t r = pre[w] + __popc(bits[w] & ((1u << (L.beg & 31)) - 1u));
        lout[r] = L;
        dout[r] = din[l];
        newid[l] = (int32_t)r;
    }
}

__global__ void k_relabel_ctab(int32_t* __restrict__ ctab, const Ctl* __restrict__ ctl,
                               const int32_t* __restrict__ newid, SetDev* __restrict__ sets,
                               int nsets) {
    const int64_t len = ctl->ct_len;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = ctab[k];
        if (c != kEmpty && (c & kLeafBit)) ctab[k] = newid[c & ~kLeafBit] | kLeafBit;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int s = 0; s < nsets; ++s) {
            const int32_t c = sets[s].root;
            if (c != kEmpty && (c & kLeafBit)) sets[s].root = newid[c & ~kLeafBit] | kLeafBit;
        }
    }
}

// Set that owns sorted position p (sets are contiguous and ascending).
__device__ __forceinline__ int set_of(const SetDev* __restrict__ sets, int nsets, int64_t p) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sets[mid].beg <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

constexpr int kSortMax = 1024;  // leaves up to this size are Morton-sorted

__device__ __forceinline__ uint64_t grid21(double x, double lo, double scale) {
    const double v = (x - lo) * scale;
    if (!(v >= 0.0)) return 0;
    return v >= 2097151.0 ? 2097151ull : (uint64_t)v;
}

// 63-bit Morton key of a particle on its set's root box (21-bit grid per
// axis; any monotone map will do: the key only orders particles inside a
// leaf, so that consecutive particles, hence work items, are compact).
__device__ __forceinline__ uint64_t leaf_key(const double4& q, const SetDev& S, double sx,
                                             double sy, double sz) {
    return spread3_64(grid21(q.x, S.box[0], sx)) | (spread3_64(grid21(q.y, S.box[1], sy)) << 1) |
           (spread3_64(grid21(q.z, S.box[2], sz)) << 2);
}

constexpr int kWaveSort = 512;  // leaves up to this size are sorted by one wavefront

// Leaves of at most kWaveSort particles, one wavefront per leaf, into the
// tree-ordered array with their smallest and largest original index.  A
// leaf of at most one work item (kGroup particles) keeps the order it has:
// the order inside a work item is free.  A larger one is put in Morton order
// on a 128^3 grid over the leaf's own bounding box, so that its work items
// (consecutive runs of kGroup) are compact.  The sort key is one 32-bit word,
// the 21-bit grid code above the particle's 9-bit position in the leaf
// (unique keys, and the position comes back out of the key), sorted by a
// bitonic network in the wavefront's slice of shared memory, which needs no
// workgroup barrier.
__global__ __launch_bounds__(kT) void k_leaf_wave(const Leaf* __restrict__ leaves,
                                                  const int32_t* __restrict__ ldepth,
                                                  const Ctl* __restrict__ ctl,
                                                  const double4* __restrict__ P0,
                                                  const double4* __restrict__ P1,
                                                  double4* __restrict__ pos,
                                                  int2* __restrict__ lrange) {
    static_assert(kWaveSort <= 512, "the position in the leaf takes 9 bits of the key");
    __shared__ uint32_t s_key[kT / 64][kWaveSort];
    uint32_t* const key = s_key[threadIdx.x >> 6];
    const int64_t nl = ctl->n_leaves;
    const int lane = lane_id();
    const int64_t nw = ((int64_t)gridDim.x * kT) >> 6;
    for (int64_t li = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6; li < nl; li += nw) {
        const Leaf L = leaves[li];
        if (L.cnt > kWaveSort) continue;  // uniform over the wavefront; k_leaf_final
        const double4* src = (ldepth[li] & 1) ? P1 : P0;
        int mn = 0x7fffffff, mx = -1;
        if (L.cnt <= kGroup) {
            if (lane < L.cnt) {
                const double4 q = src[L.beg + lane];
                pos[L.beg + lane] = q;
                mn = mx = (int)q.w;
            }
        } else {
            double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int k = lane; k < L.cnt; k += 64) {
                const double4 q = src[L.beg + k];
                lo[0] = fmin(lo[0], q.x);
                hi[0] = fmax(hi[0], q.x);
                lo[1] = fmin(lo[1], q.y);
                hi[1] = fmax(hi[1], q.y);
                lo[2] = fmin(lo[2], q.z);
                hi[2] = fmax(hi[2], q.z);
                mn = min(mn, (int)q.w);
                mx = max(mx, (int)q.w);
            }
            double sc[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                lo[d] = wave_min(lo[d]);
                hi[d] = wave_max(hi[d]);
                sc[d] = 128.0 / fmax(hi[d] - lo[d], 1e-300);
            }
            int P = 2 * kGroup;
            while (P < L.cnt) P <<= 1;
            for (int k = lane; k < P; k += 64) {
                uint32_t kv = 0xffffffffu;
                if (k < L.cnt) {
                    const double4 q = src[L.beg + k];
                    const double g[3] = {q.x, q.y, q.z};
                    uint32_t c[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const double v = (g[d] - lo[d]) * sc[d];
                        c[d] = v >= 127.0 ? 127u : (v >= 0.0 ? (uint32_t)v : 0u);
                    }
                    kv = ((spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2)) << 9) |
                         (uint32_t)k;
                }
                key[k] = kv;
            }
            wave_lds_sync();
            for (int kk = 2; kk <= P; kk <<= 1) {
                for (int j = kk >> 1; j > 0; j >>= 1) {
                    // Pair t: a has bit j clear, c = a + j.
                    for (int t = lane; t < P / 2; t += 64) {
                        const int a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                        const int c = a | j;
                        const uint32_t ka = key[a], kc = key[c];
                        const uint32_t small = min(ka, kc), large = max(ka, kc);
                        const bool up = (a & kk) == 0;
                        key[a] = up ? small : large;
                        key[c] = up ? large : small;
                    }
                    wave_lds_sync();
                }
            }
            for (int k = lane; k < L.cnt; k += 64) pos[L.beg + k] = src[L.beg + (key[k] & 511u)];
            wave_lds_sync();  // the next leaf reuses the slice
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            mn = min(mn, __shfl_xor(mn, d, 64));
            mx = max(mx, __shfl_xor(mx, d, 64));
        }
        if (lane == 0) lrange[li] = make_int2(mn, mx);
    }
}

// Leaves above kWaveSort particles (a cell at the depth guard, or a large
// s), one workgroup per leaf: Morton-sorted on the set's root box (ties by
// original index) into the tree-ordered particle array, with the leaf's
// smallest and largest original index.
__global__ __launch_bounds__(kT) void k_leaf_final(const Leaf* __restrict__ leaves,
                                                   const int32_t* __restrict__ ldepth,
                                                   const Ctl* __restrict__ ctl,
                                                   const SetDev* __restrict__ sets, int nsets,
                                                   const double4* __restrict__ P0,
                                                   const double4* __restrict__ P1,
                                                   double4* __restrict__ pos,
                                                   int2* __restrict__ lrange) {
    __shared__ uint64_t key[kSortMax];
    __shared__ int32_t val[kSortMax];
    __shared__ int32_t ord[kSortMax];
    __shared__ int32_t red[2][kT / 64];
    __shared__ int32_t s_big[kT];
    __shared__ int s_nbig;
    const int64_t nl = ctl->n_leaves;
    // Each workgroup lists the large leaves of a range of kT leaves (one
    // load per thread), then orders them one after the other.
    for (int64_t base = (int64_t)blockIdx.x * kT; base < nl; base += (int64_t)gridDim.x * kT) {
        if (threadIdx.x == 0) s_nbig = 0;
        __syncthreads();
        {
            const int64_t l = base + threadIdx.x;
            if (l < nl && leaves[l].cnt > kWaveSort) s_big[atomicAdd(&s_nbig, 1)] = (int32_t)l;
        }
        __syncthreads();
        const int nbig = s_nbig;
        for (int bi = 0; bi < nbig; ++bi) {
            const int64_t li = s_big[bi];
            const Leaf L = leaves[li];
            const double4* src = (ldepth[li] & 1) ? P1 : P0;
            const SetDev& S = sets[set_of(sets, nsets, L.beg)];
            {
                int mn = 0x7fffffff, mx = -1;
                for (int k = threadIdx.x; k < L.cnt; k += kT) {
                    const int v = (int)src[L.beg + k].w;
                    mn = min(mn, v);
                    mx = max(mx, v);
                }
#pragma unroll
                for (int d = 32; d > 0; d >>= 1) {
                    mn = min(mn, __shfl_xor(mn, d, 64));
                    mx = max(mx, __shfl_xor(mx, d, 64));
                }
                if (lane_id() == 0) { red[0][threadIdx.x >> 6] = mn; red[1][threadIdx.x >> 6] = mx; }
                __syncthreads();
                if (threadIdx.x == 0) {
                    for (int k = 1; k < kT / 64; ++k) { mn = min(mn, red[0][k]); mx = max(mx, red[1][k]); }
                    lrange[li] = make_int2(mn, mx);
                }
            }
            // A leaf too large to sort here keeps the order of the Morton pre-sort.
            if (L.cnt > kSortMax) {
                for (int k = threadIdx.x; k < L.cnt; k += kT) pos[L.beg + k] = src[L.beg + k];
                __syncthreads();
                continue;
            }
            const double sx = (double)(1 << 21) / fmax(S.box[3] - S.box[0], 1e-300);
            const double sy = (double)(1 << 21) / fmax(S.box[4] - S.box[1], 1e-300);
            const double sz = (double)(1 << 21) / fmax(S.box[5] - S.box[2], 1e-300);
            int P = 1;
            while (P < L.cnt) P <<= 1;
            for (int k = threadIdx.x; k < P; k += kT) {
                if (k < L.cnt) {
                    const double4 q = src[L.beg + k];
                    key[k] = leaf_key(q, S, sx, sy, sz);
                    val[k] = (int32_t)q.w;
                } else {
                    key[k] = ~0ull;
                    val[k] = 0x7fffffff;
                }
                ord[k] = k;
            }
            __syncthreads();
            for (int kk = 2; kk <= P; kk <<= 1) {
                for (int j = kk >> 1; j > 0; j >>= 1) {
                    for (int a = threadIdx.x; a < P; a += kT) {
                        const int c = a ^ j;
                        if (c > a) {
                            const bool up = (a & kk) == 0;
                            const bool gt = key[a] > key[c] || (key[a] == key[c] && val[a] > val[c]);
                            if (gt == up) {
                                const uint64_t tk = key[a]; key[a] = key[c]; key[c] = tk;
                                const int32_t tv = val[a]; val[a] = val[c]; val[c] = tv;
                                const int32_t to = ord[a]; ord[a] = ord[c]; ord[c] = to;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int k = threadIdx.x; k < L.cnt; k += kT) pos[L.beg + k] = src[L.beg + ord[k]];
            __syncthreads();
        }
        __syncthreads();  // s_nbig is reset for the next range
    }
}

__global__ void k_leaf_stats(const Leaf* __restrict__ leaves, const int32_t* __restrict__ ldepth,
                             const SetDev* __restrict__ sets, int nsets, Ctl* __restrict__ ctl) {
    __shared__ int red[3][4];
    const int64_t nl = ctl->n_leaves;
    // Reduced over the workgroup first (the loop bound is uniform over it,
    // so every lane takes part): atomics on one address are serialised.
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < nl;
         b0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = b0 + threadIdx.x;
        int d = 0, c = 0, o = 0;
        if (l < nl) {
            const Leaf L = leaves[l];
            d = ldepth[l];
            c = L.cnt;
            o = L.cnt > sets[set_of(sets, nsets, L.beg)].s ? 1 : 0;
        }
#pragma unroll
        for (int k = 32; k > 0; k >>= 1) {
            d = max(d, __shfl_xor(d, k, 64));
            c = max(c, __shfl_xor(c, k, 64));
            o += __shfl_xor(o, k, 64);
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[0][w] = d;
            red[1][w] = c;
            red[2][w] = o;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
                d = max(d, red[0][k]);
                c = max(c, red[1][k]);
                o += red[2][k];
            }
            if (d > ctl->depth) atomicMax(&ctl->depth, d);
            if (c > ctl->max_leaf) atomicMax(&ctl->max_leaf, c);
            if (o > 0) atomicAdd(&ctl->oversized, o);
        }
        __syncthreads();
    }
}

__global__ void k_chunk_count(const Leaf* __restrict__ leaves, const Ctl* __restrict__ ctl,
                              int32_t* __restrict__ nc) {
    const int64_t nl = ctl->n_leaves;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nl;
         l += (int64_t)gridDim.x * blockDim.x)
        nc[l] = (leaves[l].cnt + kGroup - 1) / kGroup;
}

__global__ void k_chunk_emit(const Leaf* __restrict__ leaves, Ctl* __restrict__ ctl,
                             const SetDev* __restrict__ sets, int nsets,
                             const int64_t* __restrict__ coff, Chunk* __restrict__ chunks) {
    const int64_t nl = ctl->n_leaves;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->n_chunks = (int32_t)coff[nl];
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nl;
         l += (int64_t)gridDim.x * blockDim.x) {
        const Leaf L = leaves[l];
        const int set = set_of(sets, nsets, L.beg);
        int64_t c = coff[l];
        for (int k = 0; k < L.cnt; k += kGroup) {
            const int cnt = L.cnt - k < kGroup ? L.cnt - k : kGroup;
            chunks[c++] = Chunk{L.beg + k, cnt, set, 0};
        }
    }
}

int ceil_log2(int64_t v) {
    int k = 0;
    while ((int64_t(1) << k) < v) ++k;
    return k;
}

}  // namespace

void plan_sets(Tree& t, int32_t nsets, const int64_t* set_off_in, const btree_params* prm_in) {
    // Copies first: the inputs may be the handle's own vectors.
    std::vector<int64_t> off_copy(set_off_in, set_off_in + nsets + 1);
    std::vector<btree_params> prm_copy(prm_in, prm_in + nsets);
    t.nsets = nsets;
    t.set_off = off_copy;
    t.set_prm = prm_copy;
    const int64_t* set_off = t.set_off.data();
    const btree_params* prm = t.set_prm.data();
    t.n = set_off[nsets];
    const int64_t n = t.n;
    // Tiles that never straddle two sets.
    std::vector<Tile> tiles;
    std::vector<int64_t> settile(nsets + 1, 0);
    for (int k = 0; k < nsets; ++k) {
        settile[k] = (int64_t)tiles.size();
        for (int64_t b = set_off[k]; b < set_off[k + 1]; b += kTileN)
            tiles.push_back(Tile{k, 0, b, std::min(set_off[k + 1], b + kTileN)});
    }
    settile[nsets] = (int64_t)tiles.size();
    t.ntiles = settile[nsets];
    if (tiles.empty()) tiles.push_back(Tile{0, 0, 0, 0});
    t.ws.tiles.reserve(sizeof(Tile) * tiles.size());
    t.ws.settile.reserve(sizeof(int64_t) * settile.size());
    BT_HIP(hipMemcpy(t.ws.tiles.p, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice));
    BT_HIP(hipMemcpy(t.ws.settile.p, settile.data(), sizeof(int64_t) * settile.size(),
                     hipMemcpyHostToDevice));
    std::vector<SetDev> sd(nsets);
    int64_t node_b = 0, ctab_b = 0, hist_b = 0;
    for (int k = 0; k < nsets; ++k) {
        SetDev S{};
        S.beg = set_off[k];
        S.n = set_off[k + 1] - set_off[k];
        S.alpha = prm[k].alpha;
        S.beta = prm[k].beta;
        S.s = prm[k].bucket_size;
        S.max_depth = prm[k].max_depth;
        S.root = kEmpty;
        S.octree = prm[k].octree;
        sd[k] = S;
        // Cells of one level are disjoint and hold more than s particles each.
        const int64_t q = S.n / (S.s + 1) + 1;
        node_b += 2 * q + 8;
        // b0^3 < 8 n/s for a cell of n > s particles, so a level's child tables
        // and candidate histograms are O(n/s) (histograms: 8/7 of b0^3 plus
        // the odd halving steps).
        ctab_b += 32 * (S.n / S.s + 1) + 64;
        hist_b += 12 * (S.n / S.s + 1) + 96 * q;
    }
    t.sets.reserve(sizeof(SetDev) * nsets);
    BT_HIP(hipMemcpy(t.sets.p, sd.data(), sizeof(SetDev) * nsets, hipMemcpyHostToDevice));
    if (t.node_cap < node_b + 1024) t.node_cap = node_b + 1024;
    if (t.ctab_cap < ctab_b + 4096) t.ctab_cap = ctab_b + 4096;
    if (t.hist_cap < hist_b + 4096) t.hist_cap = hist_b + 4096;
    t.leaf_cap = n + nsets + 1;
    // Pools and workspaces, sized once so that queued builds allocate nothing.
    Work& W = t.ws;
    const int64_t nn = std::max<int64_t>(n, 1);
    W.P0.reserve(sizeof(double4) * nn);
    W.P1.reserve(sizeof(double4) * nn);
    W.part.reserve(sizeof(double) * 6 * std::max<int64_t>(t.ntiles, 1));
    W.mk0.reserve(sizeof(uint32_t) * nn);
    W.mk1.reserve(sizeof(uint32_t) * nn);
    W.mv0.reserve(sizeof(int32_t) * nn);
    W.mv1.reserve(sizeof(int32_t) * nn);
    const int64_t rtiles = (nn + 4095) / 4096;
    W.rcnt.reserve(sizeof(int32_t) * 256 * rtiles);
    W.roff.reserve(sizeof(int64_t) * (256 * rtiles + 1));
    const int64_t nc = t.node_cap;
    W.hsize.reserve(sizeof(int64_t) * nc);
    W.tcnt.reserve(sizeof(int64_t) * nc);
    W.toff.reserve(sizeof(int64_t) * (nc + 1));
    W.hoff.reserve(sizeof(int64_t) * (nc + 1));
    W.bsel.reserve(sizeof(int32_t) * nc);
    W.selofs.reserve(sizeof(int64_t) * nc);
    W.nint.reserve(sizeof(int64_t) * nc);
    W.nleaf.reserve(sizeof(int64_t) * nc);
    W.ctsize.reserve(sizeof(int64_t) * nc);
    W.ibase.reserve(sizeof(int64_t) * (nc + 1));
    W.lbase.reserve(sizeof(int64_t) * (nc + 1));
    W.ctoff.reserve(sizeof(int64_t) * (nc + 1));
    W.hist.reserve(sizeof(int32_t) * t.hist_cap);
    W.cstart.reserve(sizeof(int32_t) * t.hist_cap);
    W.crank.reserve(sizeof(int32_t) * t.hist_cap);
    W.cursor.reserve(sizeof(int32_t) * t.hist_cap);
    W.mark.reserve(sizeof(int32_t) * nn);
    W.f.reserve(sizeof(int32_t) * nn);
    W.rank.reserve(sizeof(int64_t) * (nn + 1));
    W.newid.reserve(sizeof(int32_t) * t.leaf_cap);
    W.nc.reserve(sizeof(int32_t) * t.leaf_cap);
    W.coff.reserve(sizeof(int64_t) * (t.leaf_cap + 1));
    t.orig.reserve(sizeof(double4) * nn);
    t.pos.reserve(sizeof(double4) * nn);
    t.nodes.reserve(sizeof(Node) * nc);
    t.ctab.reserve(sizeof(int32_t) * t.ctab_cap);
    t.leaves.reserve(sizeof(Leaf) * t.leaf_cap);
    t.ldepth.reserve(sizeof(int32_t) * t.leaf_cap);
    t.leaves2.reserve(sizeof(Leaf) * t.leaf_cap);
    t.ldepth2.reserve(sizeof(int32_t) * t.leaf_cap);
    t.lrange.reserve(sizeof(int2) * t.leaf_cap);
    t.chunks.reserve(sizeof(Chunk) * t.leaf_cap);
    t.split.reserve(3 * sizeof(Chunk) * t.leaf_cap);
    t.split_ci.reserve(sizeof(int32_t) * t.leaf_cap);
    t.blist.reserve(sizeof(Chunk) * t.leaf_cap);
    t.bq.reserve(sizeof(int32_t) * nn);
    t.bset.reserve(sizeof(int32_t) * (5 * (int64_t)nsets + 3));
    t.btab.reserve(sizeof(int32_t) * 64 * kDenseTaskCap);
    t.ctl.reserve(sizeof(Ctl));
    t.stats.reserve(sizeof(Stats));
    t.tot.reserve(sizeof(int64_t) * (nsets + 1));
    t.soff.reserve(sizeof(int64_t) * nn);
    scan_reserve(t, std::max<int64_t>(std::max<int64_t>(3 * nc + 4 * 2048, t.leaf_cap),
                                      256 * rtiles + 1));
    scan_reserve(t, nn + 1);
}

void build_queue(Tree& t, const double* x, const double* y, const double* z, int levels,
                 bool eager, hipStream_t st) {
    const int64_t n = t.n;
    Work& W = t.ws;
    Ctl* ctl = t.ctl.as<Ctl>();
    Stats* dstats = t.stats.as<Stats>();
    const unsigned nt = (unsigned)std::max<int64_t>(t.ntiles, 1);
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st, ctl);
    BT_LAUNCH();
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, reinterpret_cast<int32_t*>(dstats),
                       (int64_t)(sizeof(Stats) / sizeof(int32_t)), 0);
    BT_LAUNCH();
    if (t.ntiles > 0) {
        hipLaunchKernelGGL(k_ingest, dim3(nt), dim3(kT), 0, st, x, y, z, W.tiles.as<Tile>(),
                           t.orig.as<double4>(), W.part.as<double>(), ctl);
        BT_LAUNCH();
    }
    hipLaunchKernelGGL(k_setbox, dim3(t.nsets), dim3(64), 0, st, W.part.as<double>(),
                       W.settile.as<int64_t>(), t.sets.as<SetDev>());
    BT_LAUNCH();
    hipLaunchKernelGGL(k_roots, dim3(1), dim3(64), 0, st, t.sets.as<SetDev>(), t.nsets,
                       t.nodes.as<Node>(), t.leaves.as<Leaf>(), t.ldepth.as<int32_t>(), ctl);
    BT_LAUNCH();
    if (t.ntiles > 0) {
        // The pre-sort only gives the level kernels locality, so 24 key bits
        // (three radix passes) do: the set id above a Morton code on a grid of
        // 2^abits cells per axis of the set's root box.
        const int setbits = ceil_log2(t.nsets);
        const int abits = std::max(0, std::min(10, (24 - setbits) / 3));
        const int kbits = ((setbits + 3 * abits + 7) / 8) * 8;
        hipLaunchKernelGGL(k_morton, dim3(nt), dim3(kT), 0, st, t.orig.as<double4>(),
                           W.tiles.as<Tile>(), t.sets.as<SetDev>(), abits, W.mk0.as<uint32_t>(),
                           W.mv0.as<int32_t>());
        BT_LAUNCH();
        radix_sort_pairs(W.mk0.as<uint32_t>(), W.mv0.as<int32_t>(), W.mk1.as<uint32_t>(),
                         W.mv1.as<int32_t>(), n, kbits, t, W.rcnt, W.roff, st);
        hipLaunchKernelGGL(k_gather, dim3(nt), dim3(kT), 0, st, t.orig.as<double4>(),
                           W.mv0.as<int32_t>(), W.tiles.as<Tile>(), W.P0.as<double4>());
        BT_LAUNCH();
    }

    DBuf* Ps[2] = {&W.P0, &W.P1};
    // Histogram and scatter: persistent over the level's tasks.
    const unsigned gR =
        (unsigned)std::min<int64_t>(kPersistBlocks, std::max<int64_t>(1, (n + kRunR - 1) / kRunR));
    const int64_t nc = t.node_cap;
    int level = 0;
    for (; level < levels; ++level) {
        const int par = level & 1;
        hipLaunchKernelGGL(k_candidates, dim3(kPersistBlocks), dim3(256), 0, st, t.nodes.as<Node>(),
                           t.sets.as<SetDev>(), ctl, W.hsize.as<int64_t>(), W.tcnt.as<int64_t>());
        BT_LAUNCH();
        scan2_dev_i64(W.hsize.as<int64_t>(), W.hoff.as<int64_t>(), W.tcnt.as<int64_t>(),
                      W.toff.as<int64_t>(), &ctl->lvm, nc, t, st);
        hipLaunchKernelGGL(k_hist_zero, dim3(kPersistBlocks), dim3(256), 0, st, ctl,
                           W.hoff.as<int64_t>(), t.hist_cap, W.hist.as<int32_t>(),
                           W.cursor.as<int32_t>());
        BT_LAUNCH();
        hipLaunchKernelGGL(k_histogram, dim3(gR), dim3(kT), 0, st, Ps[par]->as<double4>(),
                           t.nodes.as<Node>(), ctl, W.hoff.as<int64_t>(), W.toff.as<int64_t>(),
                           W.hist.as<int32_t>());
        BT_LAUNCH();
        hipLaunchKernelGGL(k_select, dim3(kPersistBlocks), dim3(kT), 0, st, t.nodes.as<Node>(),
                           t.sets.as<SetDev>(), ctl, W.hoff.as<int64_t>(), W.hist.as<int32_t>(),
                           W.bsel.as<int32_t>(), W.selofs.as<int64_t>(), dstats);
        BT_LAUNCH();
        hipLaunchKernelGGL(k_children, dim3(kPersistBlocks), dim3(kT), 0, st, t.nodes.as<Node>(),
                           t.sets.as<SetDev>(), ctl, W.bsel.as<int32_t>(), W.selofs.as<int64_t>(),
                           W.hist.as<int32_t>(), W.cstart.as<int32_t>(), W.crank.as<int32_t>(),
                           W.nint.as<int64_t>(), W.nleaf.as<int64_t>(), W.ctsize.as<int64_t>());
        BT_LAUNCH();
        scan3_dev_i64(W.nint.as<int64_t>(), W.ibase.as<int64_t>(), W.nleaf.as<int64_t>(),
                      W.lbase.as<int64_t>(), W.ctsize.as<int64_t>(), W.ctoff.as<int64_t>(),
                      &ctl->lvm, nc, t, st);
        hipLaunchKernelGGL(k_level_alloc, dim3(1), dim3(64), 0, st, ctl, W.ibase.as<int64_t>(),
                           W.lbase.as<int64_t>(), W.ctoff.as<int64_t>(), t.node_cap, t.leaf_cap,
                           t.ctab_cap);
        BT_LAUNCH();
        hipLaunchKernelGGL(k_emit, dim3(kPersistBlocks), dim3(kT), 0, st, t.nodes.as<Node>(),
                           t.sets.as<SetDev>(), ctl, W.bsel.as<int32_t>(), W.selofs.as<int64_t>(),
                           W.hist.as<int32_t>(), W.cstart.as<int32_t>(), W.crank.as<int32_t>(),
                           W.ibase.as<int64_t>(), W.lbase.as<int64_t>(), W.ctoff.as<int64_t>(),
                           t.ctab.as<int32_t>(), t.leaves.as<Leaf>(), t.ldepth.as<int32_t>());
        BT_LAUNCH();
        hipLaunchKernelGGL(k_scatter, dim3(gR), dim3(kT), 0, st, Ps[par]->as<double4>(),
                           Ps[par ^ 1]->as<double4>(), t.nodes.as<Node>(), ctl,
                           W.bsel.as<int32_t>(), W.selofs.as<int64_t>(), W.cstart.as<int32_t>(),
                           W.cursor.as<int32_t>(), W.toff.as<int64_t>(), n);
        BT_LAUNCH();
        hipLaunchKernelGGL(k_level_advance, dim3(1), dim3(64), 0, st, ctl, level, levels);
        BT_LAUNCH();
        if (eager) {
            int32_t m = 0;
            BT_HIP(hipMemcpyAsync(&m, &ctl->lvm, sizeof m, hipMemcpyDeviceToHost, st));
            BT_HIP(hipStreamSynchronize(st));
            if (m == 0) break;
        }
    }

    // Leaves renumbered in memory order (depth-first, sub-cells in Morton order).
    const int64_t nwords = (std::max<int64_t>(n, 1) + 31) / 32;
    hipLaunchKernelGGL(k_fill_i32, dim3(kPersistBlocks), dim3(256), 0, st, W.mark.as<int32_t>(),
                       nwords, 0);
    BT_LAUNCH();
    hipLaunchKernelGGL(k_mark_bits, dim3(kPersistBlocks), dim3(256), 0, st, t.leaves.as<Leaf>(),
                       ctl, W.mark.as<uint32_t>());
    BT_LAUNCH();
    hipLaunchKernelGGL(k_popc, dim3(kPersistBlocks), dim3(256), 0, st, W.mark.as<uint32_t>(),
                       nwords, W.f.as<int32_t>());
    BT_LAUNCH();
    scan_exclusive_i32(W.f.as<int32_t>(), W.rank.as<int64_t>(), nwords, t, st);
    hipLaunchKernelGGL(k_relabel_leaves, dim3(kPersistBlocks), dim3(256), 0, st,
                       W.mark.as<uint32_t>(), W.rank.as<int64_t>(), ctl, t.leaves.as<Leaf>(),
                       t.ldepth.as<int32_t>(), t.leaves2.as<Leaf>(), t.ldepth2.as<int32_t>(),
                       W.newid.as<int32_t>());
    BT_LAUNCH();
    hipLaunchKernelGGL(k_relabel_ctab, dim3(kPersistBlocks), dim3(256), 0, st, t.ctab.as<int32_t>(),
                       ctl, W.newid.as<int32_t>(), t.sets.as<SetDev>(), t.nsets);
    BT_LAUNCH();
    std::swap(t.leaves.p, t.leaves2.p);
    std::swap(t.leaves.bytes, t.leaves2.bytes);
    std::swap(t.ldepth.p, t.ldepth2.p);
    std::swap(t.ldepth.bytes, t.ldepth2.bytes);

    // Leaf ordering: a wavefront per leaf, with enough wavefronts that each
    // takes only a few leaves (its steps are chains of dependent loads).
    hipLaunchKernelGGL(k_leaf_wave, dim3(4 * kPersistBlocks), dim3(kT), 0, st, t.leaves.as<Leaf>(),
                       t.ldepth.as<int32_t>(), ctl, W.P0.as<double4>(), W.P1.as<double4>(),
                       t.pos.as<double4>(), t.lrange.as<int2>());
    BT_LAUNCH();
    hipLaunchKernelGGL(k_leaf_final, dim3(kPersistBlocks), dim3(kT), 0, st, t.leaves.as<Leaf>(),
                       t.ldepth.as<int32_t>(), ctl, t.sets.as<SetDev>(), t.nsets,
                       W.P0.as<double4>(), W.P1.as<double4>(), t.pos.as<double4>(),
                       t.lrange.as<int2>());
    BT_LAUNCH();
    hipLaunchKernelGGL(k_leaf_stats, dim3(kPersistBlocks), dim3(256), 0, st, t.leaves.as<Leaf>(),
                       t.ldepth.as<int32_t>(), t.sets.as<SetDev>(), t.nsets, ctl);
    BT_LAUNCH();
    hipLaunchKernelGGL(k_chunk_count, dim3(kPersistBlocks), dim3(256), 0, st, t.leaves.as<Leaf>(),
                       ctl, W.nc.as<int32_t>());
    BT_LAUNCH();
    scan_dev_i32(W.nc.as<int32_t>(), W.coff.as<int64_t>(), &ctl->n_leaves, t.leaf_cap, t, st);
    hipLaunchKernelGGL(k_chunk_emit, dim3(kPersistBlocks), dim3(256), 0, st, t.leaves.as<Leaf>(),
                       ctl, t.sets.as<SetDev>(), t.nsets, W.coff.as<int64_t>(),
                       t.chunks.as<Chunk>());
    BT_LAUNCH();
}

void build_tree(Tree& t, const double* x, const double* y, const double* z, hipStream_t st) {
    // A first build reads the next level's size after every level and stops
    // at the last one.  A rebuild queues the previous tree's level count
    // plus one with no host read in between (an empty level costs only its
    // launches); a tree that needs more sets kOvfLevels, and the build is
    // done again level by level.
    bool eager = t.levels_seen <= 0;
    SetDev s0;
    for (int attempt = 0;; ++attempt) {
        const int levels = eager ? 66 : (int)std::min<int64_t>(66, t.levels_seen + 1);
        build_queue(t, x, y, z, levels, eager, st);
        BT_HIP(hipMemcpyAsync(&t.host_ctl, t.ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(&t.host_stats, t.stats.p, sizeof(Stats), hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(&s0, t.sets.p, sizeof(SetDev), hipMemcpyDeviceToHost, st));
        BT_HIP(hipStreamSynchronize(st));
        const Ctl& c = t.host_ctl;
        if (c.data_bad) fail(BTREE_EINVAL, "btree_build: non-finite particle coordinate");
        if (!c.overflow) break;
        if (attempt >= 6) fail(BTREE_ENOMEM, "btree_build: tree pools kept overflowing");
        // Grow what overflowed and build again.
        if (c.overflow & kOvfLevels) eager = true;
        if (c.overflow & kOvfNodes) t.node_cap *= 2;
        if (c.overflow & kOvfCtab) t.ctab_cap *= 2;
        if (c.overflow & kOvfHist) t.hist_cap *= 2;
        plan_sets(t, t.nsets, t.set_off.data(), t.set_prm.data());
    }
    const Ctl& c = t.host_ctl;
    t.n_internal = c.n_nodes;
    t.n_leaves = c.n_leaves;
    t.n_chunks = c.n_chunks;
    t.ctab_len = c.ct_len;
    t.depth = c.depth;
    t.max_leaf = c.max_leaf;
    t.oversized = c.oversized;
    t.levels_seen = c.levels;
    t.root_code = s0.root;
    for (int k = 0; k < 6; ++k) t.rootbox[k] = s0.box[k];
}

}  // namespace bt

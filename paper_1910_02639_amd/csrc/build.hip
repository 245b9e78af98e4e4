// BuildTree on the device (Section 3.1, Algorithm 1, Eqs. 1-4).
//
// The recursion of Algorithm 1 is run level by level: every cell that still
// holds more than s particles at depth L is split in the same set of
// launches.  Per level:
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
// Particles ping-pong between two buffers; a leaf made at depth d keeps its
// particles in buffer d % 2 until the final pass sorts each leaf along a
// 63-bit Morton curve of the root box and writes the tree-ordered copy.
#include "prim.h"

#include <algorithm>
#include <cmath>

namespace bt {

namespace {

constexpr int kT = 256;
constexpr int kIngestBlocks = 1024;

// A1: validate coordinates, keep an original-order copy, bounding-box
// partials per block.
__global__ __launch_bounds__(kT) void k_ingest(const double* __restrict__ x,
                                               const double* __restrict__ y,
                                               const double* __restrict__ z, int64_t n,
                                               double4* __restrict__ orig,
                                               double* __restrict__ part, int* __restrict__ flag) {
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        double a = x[i], b = y[i], c = z[i];
        bad |= !(isfinite(a) && isfinite(b) && isfinite(c));
        orig[i] = make_double4(a, b, c, 0.0);
        mn[0] = fmin(mn[0], a); mx[0] = fmax(mx[0], a);
        mn[1] = fmin(mn[1], b); mx[1] = fmax(mx[1], b);
        mn[2] = fmin(mn[2], c); mx[2] = fmax(mx[2], c);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(flag, 1);
    __shared__ double sh[6][kT / 64];
    const int w = threadIdx.x >> 6;
    for (int k = 0; k < 3; ++k) {
        double a = wave_min(mn[k]);
        double b = wave_max(mx[k]);
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

// A3: 30-bit Morton key of each particle on the root box (10 bits per axis,
// the Eq. 2 function with b = 1024).
__global__ __launch_bounds__(kT) void k_morton(const double4* __restrict__ orig, int64_t n,
                                               const double* __restrict__ box,
                                               uint32_t* __restrict__ keys,
                                               int32_t* __restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const double4 q = orig[i];
    uint32_t kx = (uint32_t)subcell(q.x, box[0], box[3], 1024);
    uint32_t ky = (uint32_t)subcell(q.y, box[1], box[4], 1024);
    uint32_t kz = (uint32_t)subcell(q.z, box[2], box[5], 1024);
    keys[i] = spread3(kx) | (spread3(ky) << 1) | (spread3(kz) << 2);
    vals[i] = (int32_t)i;
}

// Particles in Morton order, all in the root cell (node 0).
__global__ __launch_bounds__(kT) void k_gather(const double4* __restrict__ orig,
                                               const int32_t* __restrict__ perm, int64_t n,
                                               double4* __restrict__ P0,
                                               int32_t* __restrict__ pnode) {
    int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (k >= n) return;
    const int32_t i = perm[k];
    const double4 q = orig[i];
    P0[k] = make_double4(q.x, q.y, q.z, (double)i);
    pnode[k] = 0;
}

__global__ __launch_bounds__(64) void k_rootbox(const double* __restrict__ part, int nparts,
                                                double* __restrict__ box) {
    for (int k = 0; k < 6; ++k) {
        double v = k < 3 ? INFINITY : -INFINITY;
        for (int i = threadIdx.x; i < nparts; i += 64)
            v = k < 3 ? fmin(v, part[i * 6 + k]) : fmax(v, part[i * 6 + k]);
        v = k < 3 ? wave_min(v) : wave_max(v);
        if (threadIdx.x == 0) box[k] = v;
    }
}

// Step 1: histogram size of all branching candidates of each active cell.
__global__ void k_candidates(const Node* __restrict__ nodes, int64_t nb, int64_t m, int32_t s,
                             int64_t* __restrict__ hsize) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int b = branching(nodes[nb + i].n, s);
    int64_t sum = 0;
    for (int bb = b;; bb = halve(bb)) {
        sum += (int64_t)bb * bb * bb;
        if (bb == 2) break;
    }
    hsize[i] = sum;
}

// Step 2: one histogram per candidate b (Eqs. 2 and 3).  Lanes of a
// wavefront that fall in the same sub-cell share one atomic.
__global__ __launch_bounds__(kT) void k_histogram(const double4* __restrict__ P,
                                                  const int32_t* __restrict__ pnode, int64_t n,
                                                  const Node* __restrict__ nodes, int64_t nb,
                                                  int64_t ne, int32_t s,
                                                  const int64_t* __restrict__ hoff,
                                                  int32_t* __restrict__ hist) {
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int32_t node = p < n ? pnode[p] : -1;
    const bool act = node >= nb && node < ne;
    Node N;
    double4 q = make_double4(0.0, 0.0, 0.0, 0.0);
    int bb = 2, ncand = 0;
    int64_t off = 0;
    if (act) {
        N = nodes[node];
        q = P[p];
        off = hoff[node - nb];
        bb = branching(N.n, s);
        for (int b = bb;; b = halve(b)) {
            ++ncand;
            if (b == 2) break;
        }
    }
    int maxc = ncand;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) maxc = max(maxc, __shfl_xor(maxc, d, 64));
    for (int k = 0; k < maxc; ++k) {
        const bool a = act && k < ncand;
        int64_t bin = 0;
        if (a) {
            int cx = subcell(q.x, N.lo[0], N.hi[0], bb);
            int cy = subcell(q.y, N.lo[1], N.hi[1], bb);
            int cz = subcell(q.z, N.lo[2], N.hi[2], bb);
            bin = off + cx + (int64_t)bb * (cy + (int64_t)bb * cz);
            off += (int64_t)bb * bb * bb;
            bb = halve(bb);
        }
        wave_agg_inc(hist, bin, a);
    }
}

// Step 3: Eq. 4 ratio r = #{n_j < alpha*s} / b^3; halve while r > beta.
__global__ __launch_bounds__(kT) void k_select(Node* __restrict__ nodes, int64_t nb, int32_t s,
                                               double alpha, double beta,
                                               const int64_t* __restrict__ hoff,
                                               const int32_t* __restrict__ hist,
                                               int32_t* __restrict__ bsel,
                                               int64_t* __restrict__ selofs,
                                               Stats* __restrict__ stats) {
    __shared__ int64_t sh[kT / 64 + 1];
    const int64_t i = blockIdx.x;
    const int64_t node = nb + i;
    const double thr = alpha * (double)s;
    int64_t off = hoff[i];
    int rounds = 0;
    int bb = branching(nodes[node].n, s);
    for (;; bb = halve(bb), ++rounds) {
        int64_t nc = (int64_t)bb * bb * bb;
        int64_t under = 0;
        for (int64_t c = threadIdx.x; c < nc; c += kT) under += ((double)hist[off + c] < thr) ? 1 : 0;
        under = block_sum<kT>(under, sh);
        double r = (double)under / (double)nc;
        if (!(r > beta && bb > 2)) break;
        off += nc;
    }
    if (threadIdx.x == 0) {
        bsel[i] = bb;
        selofs[i] = off;
        nodes[node].b = bb;
        atomicAdd(&stats->rounds, (unsigned long long)rounds);
        atomicAdd(&stats->b_hist[bb < 64 ? bb : 64], 1ull);
    }
}

constexpr int kChildItems = 4;

// Step 4a: sub-cell segments in Morton order of (x', y', z'); ranks of the
// sub-cells that become cells (n_j > s, below the depth guard) and leaves.
__global__ __launch_bounds__(kT) void k_children(const Node* __restrict__ nodes, int64_t nb,
                                                 int32_t s, int32_t max_depth,
                                                 const int32_t* __restrict__ bsel,
                                                 const int64_t* __restrict__ selofs,
                                                 const int32_t* __restrict__ hist,
                                                 int32_t* __restrict__ cstart,
                                                 int32_t* __restrict__ crank,
                                                 int64_t* __restrict__ nint,
                                                 int64_t* __restrict__ nleaf) {
    __shared__ int64_t sh[kT / 64 + 1];
    const int64_t i = blockIdx.x;
    const int b = bsel[i];
    const int64_t off = selofs[i];
    const bool can_split = nodes[nb + i].depth + 1 < max_depth;
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
            uint64_t mc = m0 + (uint64_t)threadIdx.x * kChildItems + k;
            cell[k] = -1;
            cnt[k] = 0;
            flags[k] = 0;
            if (mc < ncodes) {
                uint64_t cx = compact3_64(mc), cy = compact3_64(mc >> 1), cz = compact3_64(mc >> 2);
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
        int64_t ex = block_excl_scan<kT>(packed, sh, &tot);
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
    }
}

__global__ void k_ctsize(const int32_t* __restrict__ bsel, int64_t m, int64_t* __restrict__ ctsize) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t b = bsel[i];
    ctsize[i] = b * b * b;
}

// Step 4b: child tables, next-level cells and new leaves.
__global__ __launch_bounds__(kT) void k_emit(Node* __restrict__ nodes, int64_t nb, int64_t ne,
                                             int32_t s, int32_t max_depth,
                                             const int32_t* __restrict__ bsel,
                                             const int64_t* __restrict__ selofs,
                                             const int32_t* __restrict__ hist,
                                             const int32_t* __restrict__ cstart,
                                             const int32_t* __restrict__ crank,
                                             const int64_t* __restrict__ int_base,
                                             const int64_t* __restrict__ leaf_base,
                                             const int64_t* __restrict__ ctoff, int64_t ct0,
                                             int64_t leaf0, int32_t* __restrict__ ctab,
                                             Leaf* __restrict__ leaves,
                                             int32_t* __restrict__ ldepth) {
    const int64_t i = blockIdx.x;
    const int64_t node = nb + i;
    const Node N = nodes[node];
    const int b = bsel[i];
    const int64_t off = selofs[i];
    const int64_t ct = ct0 + ctoff[i];
    const bool can_split = N.depth + 1 < max_depth;
    if (threadIdx.x == 0) nodes[node].ctab = ct;
    const int64_t nc = (int64_t)b * b * b;
    for (int64_t c = threadIdx.x; c < nc; c += kT) {
        int64_t cnt = hist[off + c];
        int32_t code = kEmpty;
        if (cnt > s && can_split) {
            int64_t id = ne + int_base[i] + crank[off + c];
            int cx = (int)(c % b), cy = (int)((c / b) % b), cz = (int)(c / ((int64_t)b * b));
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
            nodes[id] = C;
            code = (int32_t)id;
        } else if (cnt > 0) {
            int64_t lid = leaf0 + leaf_base[i] + crank[off + c];
            leaves[lid] = Leaf{N.beg + cstart[off + c], (int32_t)cnt};
            ldepth[lid] = N.depth + 1;
            code = (int32_t)lid | kLeafBit;
        }
        ctab[ct + c] = code;
    }
}

// Step 5: scatter each particle of an active cell into its sub-cell segment
// (slots handed out per wavefront and sub-cell).
__global__ __launch_bounds__(kT) void k_scatter(const double4* __restrict__ Psrc,
                                                double4* __restrict__ Pdst,
                                                const int32_t* __restrict__ pn_src,
                                                int32_t* __restrict__ pn_dst, int64_t n,
                                                const Node* __restrict__ nodes, int64_t nb,
                                                int64_t ne, const int32_t* __restrict__ bsel,
                                                const int64_t* __restrict__ selofs,
                                                const int32_t* __restrict__ cstart,
                                                int32_t* __restrict__ cursor,
                                                const int32_t* __restrict__ ctab) {
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int32_t node = p < n ? pn_src[p] : -1;
    const bool act = node >= nb && node < ne;
    int64_t hbin = 0, c = 0, nbeg = 0, nct = 0;
    double4 q = make_double4(0.0, 0.0, 0.0, 0.0);
    if (act) {
        const Node N = nodes[node];
        const int64_t i = node - nb;
        const int b = bsel[i];
        q = Psrc[p];
        int cx = subcell(q.x, N.lo[0], N.hi[0], b);
        int cy = subcell(q.y, N.lo[1], N.hi[1], b);
        int cz = subcell(q.z, N.lo[2], N.hi[2], b);
        c = cx + (int64_t)b * (cy + (int64_t)b * cz);
        hbin = selofs[i] + c;
        nbeg = N.beg;
        nct = N.ctab;
    }
    const int32_t slot = wave_agg_slot(cursor, hbin, act);
    if (!act) return;
    const int64_t dest = nbeg + cstart[hbin] + slot;
    Pdst[dest] = q;
    const int32_t code = ctab[nct + c];
    pn_dst[dest] = (code & kLeafBit) ? -1 : code;
}

// Leaves in memory order: mark each leaf's first particle.
__global__ void k_mark_leaves(const Leaf* __restrict__ leaves, int64_t nl,
                              int32_t* __restrict__ mark) {
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nl) mark[leaves[l].beg] = (int32_t)l;
}

__global__ void k_mark_flags(const int32_t* __restrict__ mark, int64_t n, int32_t* __restrict__ f) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) f[p] = mark[p] >= 0 ? 1 : 0;
}

// New id of every leaf = rank of its first particle; permute the table.
__global__ void k_relabel_leaves(const int32_t* __restrict__ mark, const int64_t* __restrict__ rank,
                                 int64_t n, const Leaf* __restrict__ lin,
                                 const int32_t* __restrict__ din, Leaf* __restrict__ lout,
                                 int32_t* __restrict__ dout, int32_t* __restrict__ newid) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t old = mark[p];
    if (old < 0) return;
    int64_t r = rank[p];
    lout[r] = lin[old];
    dout[r] = din[old];
    newid[old] = (int32_t)r;
}

__global__ void k_relabel_ctab(int32_t* __restrict__ ctab, int64_t len,
                               const int32_t* __restrict__ newid) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    int32_t c = ctab[k];
    if (c != kEmpty && (c & kLeafBit)) ctab[k] = newid[c & ~kLeafBit] | kLeafBit;
}

constexpr int kSortMax = 1024;  // leaves up to this size are Morton-sorted

// Final pass: each leaf, Morton-sorted on the root box (ties by original
// index), into the tree-ordered particle array.
__global__ __launch_bounds__(kT) void k_leaf_final(const Leaf* __restrict__ leaves,
                                                   const int32_t* __restrict__ ldepth,
                                                   const double4* __restrict__ P0,
                                                   const double4* __restrict__ P1,
                                                   double4* __restrict__ pos, double blo0,
                                                   double blo1, double blo2, double bhi0,
                                                   double bhi1, double bhi2,
                                                   int2* __restrict__ lrange) {
    __shared__ uint64_t key[kSortMax];
    __shared__ int32_t val[kSortMax];
    __shared__ int32_t ord[kSortMax];
    __shared__ int32_t red[2][kT / 64];
    const Leaf L = leaves[blockIdx.x];
    const double4* src = (ldepth[blockIdx.x] & 1) ? P1 : P0;
    // Smallest and largest original index of the leaf (bounds the index
    // range of the candidates a search stages from it).
    {
        int mn = 0x7fffffff, mx = -1;
        for (int k = threadIdx.x; k < L.cnt; k += kT) {
            int v = (int)src[L.beg + k].w;
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
            lrange[blockIdx.x] = make_int2(mn, mx);
        }
    }
    if (L.cnt > kSortMax) {
        for (int k = threadIdx.x; k < L.cnt; k += kT) pos[L.beg + k] = src[L.beg + k];
        return;
    }
    int P = 1;
    while (P < L.cnt) P <<= 1;
    for (int k = threadIdx.x; k < P; k += kT) {
        if (k < L.cnt) {
            double4 q = src[L.beg + k];
            const int B = 1 << 21;
            uint64_t kx = (uint64_t)subcell(q.x, blo0, bhi0, B);
            uint64_t ky = (uint64_t)subcell(q.y, blo1, bhi1, B);
            uint64_t kz = (uint64_t)subcell(q.z, blo2, bhi2, B);
            key[k] = spread3_64(kx) | (spread3_64(ky) << 1) | (spread3_64(kz) << 2);
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
                int c = a ^ j;
                if (c > a) {
                    bool up = (a & kk) == 0;
                    bool gt = key[a] > key[c] || (key[a] == key[c] && val[a] > val[c]);
                    if (gt == up) {
                        uint64_t tk = key[a]; key[a] = key[c]; key[c] = tk;
                        int32_t tv = val[a]; val[a] = val[c]; val[c] = tv;
                        int32_t to = ord[a]; ord[a] = ord[c]; ord[c] = to;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int k = threadIdx.x; k < L.cnt; k += kT) pos[L.beg + k] = src[L.beg + ord[k]];
}

__global__ void k_leaf_stats(const Leaf* __restrict__ leaves, const int32_t* __restrict__ ldepth,
                             int64_t nl, int32_t s, int32_t* __restrict__ out3) {
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl) return;
    atomicMax(&out3[0], ldepth[l]);
    atomicMax(&out3[1], leaves[l].cnt);
    if (leaves[l].cnt > s) atomicAdd(&out3[2], 1);
}

__global__ void k_chunk_count(const Leaf* __restrict__ leaves, int64_t nl, int32_t* __restrict__ nc) {
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nl) nc[l] = (leaves[l].cnt + kGroup - 1) / kGroup;
}

__global__ void k_chunk_emit(const Leaf* __restrict__ leaves, int64_t nl,
                             const int64_t* __restrict__ coff, Chunk* __restrict__ chunks) {
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl) return;
    Leaf L = leaves[l];
    int64_t c = coff[l];
    for (int k = 0; k < L.cnt; k += kGroup) {
        int cnt = L.cnt - k < kGroup ? L.cnt - k : kGroup;
        chunks[c++] = Chunk{L.beg + k, cnt};
    }
}

template <class T>
T read1(const void* dptr, hipStream_t st) {
    T v;
    BT_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, st));
    BT_HIP(hipStreamSynchronize(st));
    return v;
}

}  // namespace

void build_tree(Tree& t, const double* x, const double* y, const double* z, hipStream_t st) {
    const int64_t n = t.n;
    const int32_t s = t.prm.bucket_size;
    const int32_t maxd = t.prm.max_depth;

    t.stats.reserve(sizeof(Stats));
    BT_HIP(hipMemsetAsync(t.stats.p, 0, sizeof(Stats), st));
    t.flag.reserve(sizeof(int32_t) * 4);
    BT_HIP(hipMemsetAsync(t.flag.p, 0, sizeof(int32_t) * 4, st));

    Work& W = t.ws;
    DBuf &P0 = W.P0, &P1 = W.P1, &pn0 = W.pn0, &pn1 = W.pn1, &part = W.part;
    P0.reserve(sizeof(double4) * n);
    P1.reserve(sizeof(double4) * n);
    pn0.reserve(sizeof(int32_t) * n);
    pn1.reserve(sizeof(int32_t) * n);
    t.orig.reserve(sizeof(double4) * n);
    t.pos.reserve(sizeof(double4) * n);
    int nblk = (int)std::min<int64_t>(kIngestBlocks, (n + kT - 1) / kT);
    part.reserve(sizeof(double) * 6 * nblk + 6 * sizeof(double));
    double* rootbox_d = part.as<double>() + 6 * nblk;
    hipLaunchKernelGGL(k_ingest, dim3(nblk), dim3(kT), 0, st, x, y, z, n, t.orig.as<double4>(),
                       part.as<double>(), t.flag.as<int>());
    BT_LAUNCH();
    hipLaunchKernelGGL(k_rootbox, dim3(1), dim3(64), 0, st, part.as<double>(), nblk, rootbox_d);
    BT_LAUNCH();
    BT_HIP(hipMemcpyAsync(t.rootbox, rootbox_d, sizeof(double) * 6, hipMemcpyDeviceToHost, st));
    int flag = read1<int>(t.flag.p, st);
    if (flag) fail(BTREE_EINVAL, "btree_build: non-finite particle coordinate");

    // Morton order of the particles (keys and permutation use the node-id
    // and histogram buffers of the level loop as scratch).
    {
        W.mk0.reserve(sizeof(uint32_t) * n);
        W.mk1.reserve(sizeof(uint32_t) * n);
        W.mv0.reserve(sizeof(int32_t) * n);
        W.mv1.reserve(sizeof(int32_t) * n);
        hipLaunchKernelGGL(k_morton, dim3(grid_for(n, kT)), dim3(kT), 0, st, t.orig.as<double4>(), n,
                           rootbox_d, W.mk0.as<uint32_t>(), W.mv0.as<int32_t>());
        BT_LAUNCH();
        radix_sort_pairs(W.mk0.as<uint32_t>(), W.mv0.as<int32_t>(), W.mk1.as<uint32_t>(),
                         W.mv1.as<int32_t>(), n, 32, t, W.rcnt, W.roff, st);
        hipLaunchKernelGGL(k_gather, dim3(grid_for(n, kT)), dim3(kT), 0, st, t.orig.as<double4>(),
                           W.mv0.as<int32_t>(), n, P0.as<double4>(), pn0.as<int32_t>());
        BT_LAUNCH();
    }

    // Level loop state.
    int64_t nodes_cap = 1024, leaves_cap = 1024, ctab_cap = 4096;
    t.nodes.reserve(sizeof(Node) * nodes_cap);
    t.leaves.reserve(sizeof(Leaf) * leaves_cap);
    t.ldepth.reserve(sizeof(int32_t) * leaves_cap);
    t.ctab.reserve(sizeof(int32_t) * ctab_cap);
    int64_t n_nodes = 0, n_leaves = 0, ct_len = 0;

    if (n <= s || maxd == 0) {
        Leaf L{0, (int32_t)n};
        int32_t d0 = 0;
        BT_HIP(hipMemcpyAsync(t.leaves.p, &L, sizeof(Leaf), hipMemcpyHostToDevice, st));
        BT_HIP(hipMemcpyAsync(t.ldepth.p, &d0, sizeof(int32_t), hipMemcpyHostToDevice, st));
        n_leaves = 1;
        t.root_code = 0 | kLeafBit;
    } else {
        Node R;
        for (int k = 0; k < 3; ++k) { R.lo[k] = t.rootbox[k]; R.hi[k] = t.rootbox[3 + k]; }
        R.ctab = -1; R.b = 0; R.n = (int32_t)n; R.beg = 0; R.depth = 0;
        BT_HIP(hipMemcpyAsync(t.nodes.p, &R, sizeof(Node), hipMemcpyHostToDevice, st));
        n_nodes = 1;
        t.root_code = 0;
    }

    DBuf &hsize = W.hsize, &hoff = W.hoff, &hist = W.hist, &cstart = W.cstart, &crank = W.crank,
         &cursor = W.cursor, &bsel = W.bsel, &selofs = W.selofs, &nint = W.nint,
         &nleaf = W.nleaf, &ibase = W.ibase, &lbase = W.lbase, &ctsize = W.ctsize,
         &ctoff = W.ctoff;
    int64_t nb = 0, ne = n_nodes;
    DBuf* Ps[2] = {&P0, &P1};
    DBuf* Ns[2] = {&pn0, &pn1};
    int par = 0;
    Stats* dstats = t.stats.as<Stats>();
    for (int level = 0; ne > nb && level < maxd; ++level) {
        const int64_t m = ne - nb;
        hsize.reserve(sizeof(int64_t) * m);
        hoff.reserve(sizeof(int64_t) * (m + 1));
        hipLaunchKernelGGL(k_candidates, dim3(grid_for(m, 256)), dim3(256), 0, st,
                           t.nodes.as<Node>(), nb, m, s, hsize.as<int64_t>());
        BT_LAUNCH();
        scan_exclusive_i64(hsize.as<int64_t>(), hoff.as<int64_t>(), m, t, st);
        const int64_t htot = read1<int64_t>(hoff.as<int64_t>() + m, st);
        hist.reserve(sizeof(int32_t) * htot);
        cstart.reserve(sizeof(int32_t) * htot);
        crank.reserve(sizeof(int32_t) * htot);
        cursor.reserve(sizeof(int32_t) * htot);
        BT_HIP(hipMemsetAsync(hist.p, 0, sizeof(int32_t) * htot, st));
        BT_HIP(hipMemsetAsync(cursor.p, 0, sizeof(int32_t) * htot, st));
        hipLaunchKernelGGL(k_histogram, dim3(grid_for(n, kT)), dim3(kT), 0, st,
                           Ps[par]->as<double4>(), Ns[par]->as<int32_t>(), n, t.nodes.as<Node>(),
                           nb, ne, s, hoff.as<int64_t>(), hist.as<int32_t>());
        BT_LAUNCH();
        bsel.reserve(sizeof(int32_t) * m);
        selofs.reserve(sizeof(int64_t) * m);
        hipLaunchKernelGGL(k_select, dim3((unsigned)m), dim3(kT), 0, st, t.nodes.as<Node>(), nb, s,
                           t.prm.alpha, t.prm.beta, hoff.as<int64_t>(), hist.as<int32_t>(),
                           bsel.as<int32_t>(), selofs.as<int64_t>(), dstats);
        BT_LAUNCH();
        nint.reserve(sizeof(int64_t) * m);
        nleaf.reserve(sizeof(int64_t) * m);
        hipLaunchKernelGGL(k_children, dim3((unsigned)m), dim3(kT), 0, st, t.nodes.as<Node>(), nb,
                           s, maxd, bsel.as<int32_t>(), selofs.as<int64_t>(), hist.as<int32_t>(),
                           cstart.as<int32_t>(), crank.as<int32_t>(), nint.as<int64_t>(),
                           nleaf.as<int64_t>());
        BT_LAUNCH();
        ibase.reserve(sizeof(int64_t) * (m + 1));
        lbase.reserve(sizeof(int64_t) * (m + 1));
        ctsize.reserve(sizeof(int64_t) * m);
        ctoff.reserve(sizeof(int64_t) * (m + 1));
        scan_exclusive_i64(nint.as<int64_t>(), ibase.as<int64_t>(), m, t, st);
        scan_exclusive_i64(nleaf.as<int64_t>(), lbase.as<int64_t>(), m, t, st);
        hipLaunchKernelGGL(k_ctsize, dim3(grid_for(m, 256)), dim3(256), 0, st, bsel.as<int32_t>(),
                           m, ctsize.as<int64_t>());
        BT_LAUNCH();
        scan_exclusive_i64(ctsize.as<int64_t>(), ctoff.as<int64_t>(), m, t, st);
        int64_t tots[3];
        BT_HIP(hipMemcpyAsync(&tots[0], ibase.as<int64_t>() + m, 8, hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(&tots[1], lbase.as<int64_t>() + m, 8, hipMemcpyDeviceToHost, st));
        BT_HIP(hipMemcpyAsync(&tots[2], ctoff.as<int64_t>() + m, 8, hipMemcpyDeviceToHost, st));
        BT_HIP(hipStreamSynchronize(st));
        const int64_t new_int = tots[0], new_leaf = tots[1], new_ct = tots[2];
        if (ct_len + new_ct >= (int64_t)kLeafBit || n_nodes + new_int >= (int64_t)kLeafBit)
            fail(BTREE_ENOMEM, "btree_build: tree exceeds 2^30 cells or child-table entries");
        t.nodes.grow(sizeof(Node) * (n_nodes + new_int), sizeof(Node) * n_nodes, st);
        t.leaves.grow(sizeof(Leaf) * (n_leaves + new_leaf), sizeof(Leaf) * n_leaves, st);
        t.ldepth.grow(sizeof(int32_t) * (n_leaves + new_leaf), sizeof(int32_t) * n_leaves, st);
        t.ctab.grow(sizeof(int32_t) * (ct_len + new_ct), sizeof(int32_t) * ct_len, st);
        hipLaunchKernelGGL(k_emit, dim3((unsigned)m), dim3(kT), 0, st, t.nodes.as<Node>(), nb, ne, s,
                           maxd, bsel.as<int32_t>(), selofs.as<int64_t>(), hist.as<int32_t>(),
                           cstart.as<int32_t>(), crank.as<int32_t>(), ibase.as<int64_t>(),
                           lbase.as<int64_t>(), ctoff.as<int64_t>(), ct_len, n_leaves,
                           t.ctab.as<int32_t>(), t.leaves.as<Leaf>(), t.ldepth.as<int32_t>());
        BT_LAUNCH();
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, kT)), dim3(kT), 0, st,
                           Ps[par]->as<double4>(), Ps[par ^ 1]->as<double4>(),
                           Ns[par]->as<int32_t>(), Ns[par ^ 1]->as<int32_t>(), n,
                           t.nodes.as<Node>(), nb, ne, bsel.as<int32_t>(), selofs.as<int64_t>(),
                           cstart.as<int32_t>(), cursor.as<int32_t>(), t.ctab.as<int32_t>());
        BT_LAUNCH();
        par ^= 1;
        n_nodes += new_int;
        n_leaves += new_leaf;
        ct_len += new_ct;
        nb = ne;
        ne = n_nodes;
    }
    t.n_internal = n_nodes;
    t.n_leaves = n_leaves;
    t.ctab_len = ct_len;

    // Leaf ids in memory order (depth-first, sub-cells in Morton order).
    {
        DBuf &mark = W.mark, &f = W.f, &rank = W.rank, &l2 = W.l2, &d2 = W.d2, &newid = W.newid;
        mark.reserve(sizeof(int32_t) * n);
        f.reserve(sizeof(int32_t) * n);
        rank.reserve(sizeof(int64_t) * (n + 1));
        l2.reserve(sizeof(Leaf) * n_leaves);
        d2.reserve(sizeof(int32_t) * n_leaves);
        newid.reserve(sizeof(int32_t) * n_leaves);
        BT_HIP(hipMemsetAsync(mark.p, 0xff, sizeof(int32_t) * n, st));
        hipLaunchKernelGGL(k_mark_leaves, dim3(grid_for(n_leaves, 256)), dim3(256), 0, st,
                           t.leaves.as<Leaf>(), n_leaves, mark.as<int32_t>());
        BT_LAUNCH();
        hipLaunchKernelGGL(k_mark_flags, dim3(grid_for(n, 256)), dim3(256), 0, st,
                           mark.as<int32_t>(), n, f.as<int32_t>());
        BT_LAUNCH();
        scan_exclusive_i32(f.as<int32_t>(), rank.as<int64_t>(), n, t, st);
        hipLaunchKernelGGL(k_relabel_leaves, dim3(grid_for(n, 256)), dim3(256), 0, st,
                           mark.as<int32_t>(), rank.as<int64_t>(), n, t.leaves.as<Leaf>(),
                           t.ldepth.as<int32_t>(), l2.as<Leaf>(), d2.as<int32_t>(),
                           newid.as<int32_t>());
        BT_LAUNCH();
        if (ct_len > 0) {
            hipLaunchKernelGGL(k_relabel_ctab, dim3(grid_for(ct_len, 256)), dim3(256), 0, st,
                               t.ctab.as<int32_t>(), ct_len, newid.as<int32_t>());
            BT_LAUNCH();
        }
        BT_HIP(hipMemcpyAsync(t.leaves.p, l2.p, sizeof(Leaf) * n_leaves, hipMemcpyDeviceToDevice, st));
        BT_HIP(hipMemcpyAsync(t.ldepth.p, d2.p, sizeof(int32_t) * n_leaves, hipMemcpyDeviceToDevice, st));
        if (t.root_code != kEmpty && (t.root_code & kLeafBit)) t.root_code = 0 | kLeafBit;
        BT_HIP(hipStreamSynchronize(st));
    }

    t.lrange.reserve(sizeof(int2) * n_leaves);
    hipLaunchKernelGGL(k_leaf_final, dim3((unsigned)n_leaves), dim3(kT), 0, st,
                       t.leaves.as<Leaf>(), t.ldepth.as<int32_t>(), P0.as<double4>(),
                       P1.as<double4>(), t.pos.as<double4>(), t.rootbox[0], t.rootbox[1],
                       t.rootbox[2], t.rootbox[3], t.rootbox[4], t.rootbox[5],
                       t.lrange.as<int2>());
    BT_LAUNCH();

    // Shape statistics.
    BT_HIP(hipMemsetAsync(t.flag.as<int32_t>() + 1, 0, sizeof(int32_t) * 3, st));
    hipLaunchKernelGGL(k_leaf_stats, dim3(grid_for(n_leaves, 256)), dim3(256), 0, st,
                       t.leaves.as<Leaf>(), t.ldepth.as<int32_t>(), n_leaves, s,
                       t.flag.as<int32_t>() + 1);
    BT_LAUNCH();
    int32_t ls[3];
    BT_HIP(hipMemcpyAsync(ls, t.flag.as<int32_t>() + 1, sizeof ls, hipMemcpyDeviceToHost, st));

    // Work items: every leaf cut into pieces of at most kGroup particles.
    {
        DBuf &nc = W.nc, &coff = W.coff;
        nc.reserve(sizeof(int32_t) * n_leaves);
        coff.reserve(sizeof(int64_t) * (n_leaves + 1));
        hipLaunchKernelGGL(k_chunk_count, dim3(grid_for(n_leaves, 256)), dim3(256), 0, st,
                           t.leaves.as<Leaf>(), n_leaves, nc.as<int32_t>());
        BT_LAUNCH();
        scan_exclusive_i32(nc.as<int32_t>(), coff.as<int64_t>(), n_leaves, t, st);
        t.n_chunks = read1<int64_t>(coff.as<int64_t>() + n_leaves, st);
        t.chunks.reserve(sizeof(Chunk) * t.n_chunks);
        hipLaunchKernelGGL(k_chunk_emit, dim3(grid_for(n_leaves, 256)), dim3(256), 0, st,
                           t.leaves.as<Leaf>(), n_leaves, coff.as<int64_t>(), t.chunks.as<Chunk>());
        BT_LAUNCH();
        t.cflag.reserve(sizeof(int32_t) * t.n_chunks);
    }
    BT_HIP(hipMemcpyAsync(&t.host_stats, dstats, sizeof(Stats), hipMemcpyDeviceToHost, st));
    BT_HIP(hipStreamSynchronize(st));
    t.depth = ls[0];
    t.max_leaf = ls[1];
    t.oversized = ls[2];
}

}  // namespace bt

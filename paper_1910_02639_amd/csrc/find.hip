// FindNeighbors on the device (Section 3.2, Algorithm 2, Eq. 5).
//
// Work item: up to 64 consecutive particles of one leaf (the paper's
// blocked, cache-reusing search, recast for a GPU: a leaf's particles share
// one tree walk and one staged candidate set).  A workgroup of 4 wavefronts
// takes one work item; lane q of every wavefront holds query q.
//
//  1. Box E = [min_i fl(x_i - 2h_i), max_i fl(x_i + 2h_i)] of the item.
//  2. Walk (Algorithm 2 with Eq. 5 applied to E): from the root, each
//     internal cell's sub-cell range on every axis is [f(E_lo), f(E_hi)]
//     with the build's own Eq. 2 function f; leaves in range go to a
//     candidate list, internal sub-cells to a stack, all in LDS.
//  3. Stage: the particles of the candidate leaves that lie inside E are
//     compacted into LDS (wavefront ballot + lane prefix).  Every true
//     neighbour of every query of the item lies inside E.
//  4. Test: wavefront w sweeps its quarter of the staged candidates for its
//     64 queries, LDS reads broadcast to all lanes.
//  5. Count pass: per-query counts.  Fill pass: the staged candidates are
//     first sorted by original index; hits are recorded as one bit per
//     (query, candidate) in LDS, then each lane walks its bits in order and
//     writes its row, which therefore comes out in ascending index.
// Items whose candidate set does not fit the LDS budget (or whose walk
// overflows its stack) are flagged in the count pass and handled by an
// exhaustive FP64 sweep in original index order.
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
//    FP64 predicate on the original coordinates.
#include "prim.h"

#include <cfloat>

namespace bt {

namespace {

constexpr int kWG = 256;
constexpr int kWaves = kWG / 64;
constexpr int kLMax = 1024;  // candidate leaves per item
constexpr int kSMax = 512;   // walk stack entries
constexpr int kCMax = 2048;  // staged candidates per item (both forms)

enum { kCount = 0, kFill = 1 };

// The FP64 predicate of the method, every operation rounded.
__device__ __forceinline__ bool p64(double xi, double yi, double zi, double R, double xj,
                                    double yj, double zj) {
    double dx = __dsub_rn(xi, xj);
    double dy = __dsub_rn(yi, yj);
    double dz = __dsub_rn(zi, zj);
    double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    return d2 < __dmul_rn(R, R);
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
    __device__ static int key(const float4& e) { return __float_as_int(e.w); }
    __device__ static void pad(float4& e) { e.w = __int_as_float(0x7fffffff); }
};
template <> struct Ent<false> {
    using T = double4;
    __device__ static int key(const double4& e) { return e.w > 2147483647.0 ? 0x7fffffff : (int)e.w; }
    __device__ static void pad(double4& e) { e.w = 4294967296.0; }
};

template <bool F32, int MODE>
__global__ __launch_bounds__(kWG) void k_find(const Chunk* __restrict__ chunks,
                                              const double4* __restrict__ pos,
                                              const double4* __restrict__ orig,
                                              const Node* __restrict__ nodes,
                                              const int32_t* __restrict__ ctab,
                                              const Leaf* __restrict__ leaves, int32_t root_code,
                                              const double* __restrict__ h,
                                              int32_t* __restrict__ counts,
                                              const int64_t* __restrict__ offsets,
                                              int32_t* __restrict__ nbrs,
                                              int32_t* __restrict__ cflag,
                                              const int* __restrict__ dflag,
                                              Stats* __restrict__ stats) {
    using E = typename Ent<F32>::T;
    __shared__ E s_cand[kCMax];
    __shared__ uint32_t s_bits[MODE == kFill ? (kCMax / 32) * 64 : 1];
    __shared__ int32_t s_stack[kSMax];
    __shared__ int32_t s_leaf[kLMax];
    __shared__ int32_t s_cnt[kWaves][64];
    __shared__ int s_top, s_nleaf, s_ovf, s_cur, s_C;

    if (*dflag) return;
    const int64_t ci = blockIdx.x;
    if (MODE == kFill && cflag[ci]) return;
    const Chunk ch = chunks[ci];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;

    // Query of this lane.
    const bool qv = lane < ch.cnt;
    const double4 qp = qv ? pos[ch.beg + lane] : make_double4(0.0, 0.0, 0.0, 0.0);
    const int qidx = (int)qp.w;
    const double R = qv ? 2.0 * h[qidx] : 0.0;

    // Box E of the item.
    double elo[3], ehi[3];
    {
        double q3[3] = {qp.x, qp.y, qp.z};
        for (int l = 0; l < 3; ++l) {
            elo[l] = wave_min(qv ? q3[l] - R : INFINITY);
            ehi[l] = wave_max(qv ? q3[l] + R : -INFINITY);
        }
    }

    // FP32 filter set-up (see the derivation at the top of the file).
    float ax = 0.f, ay = 0.f, az = 0.f, tlo = -1.f, thi = -1.f;
    double cx = 0.0, cy = 0.0, cz = 0.0;
    bool unsafe = false;
    if (F32) {
        cx = elo[0] + (ehi[0] - elo[0]) * 0.5;
        cy = elo[1] + (ehi[1] - elo[1]) * 0.5;
        cz = elo[2] + (ehi[2] - elo[2]) * 0.5;
        const double up = 1.0 + 0x1p-50;
        double S[3];
        double c3[3] = {cx, cy, cz};
        double q3[3] = {qp.x, qp.y, qp.z};
        for (int l = 0; l < 3; ++l) {
            double mb = fmax(c3[l] - elo[l], ehi[l] - c3[l]) * up;
            double ma = wave_max(qv ? fabs(q3[l] - c3[l]) : 0.0) * up;
            S[l] = (ma + mb) * up;
        }
        double sn = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]) * up;
        double rmax = wave_max(R);
        unsafe = !(sn < 0x1p100 && rmax < 0x1p100);
        const double u = 0x1p-24;
        const double eta = (0x1p-24 + 0x1p-52) * sn * (1.0 + 0x1p-40) + 8.0 * 0x1p-126;
        const double g3 = 3.0 * u / (1.0 - 3.0 * u);
        if (qv) {
            double A = R * (1.0 - 0x1p-48) - eta;
            if (A < 0.0) A = 0.0;
            double tl = (1.0 - g3) * (1.0 - u) * (1.0 - u) * A * A * (1.0 - 0x1p-40) - 8.0 * 0x1p-126;
            double B = R * (1.0 + 0x1p-48) + eta;
            double th = (1.0 + g3) * (1.0 + u) * (1.0 + u) * B * B * (1.0 + 0x1p-40) + 8.0 * 0x1p-126;
            tlo = tl > 0.0 ? f32_down(tl) : 0.0f;
            thi = f32_up(th);
            ax = (float)(qp.x - cx);
            ay = (float)(qp.y - cy);
            az = (float)(qp.z - cz);
        }
    }
    const double r2q = qv ? __dmul_rn(R, R) : -1.0;

    // Walk.
    if (t == 0) {
        s_top = 0;
        s_nleaf = 0;
        s_ovf = unsafe ? 1 : 0;
        s_C = 0;
        if (root_code & kLeafBit) {
            s_leaf[0] = root_code & ~kLeafBit;
            s_nleaf = 1;
        } else {
            s_stack[0] = root_code;
            s_top = 1;
        }
    }
    __syncthreads();
    for (;;) {
        if (t == 0) s_cur = (s_top > 0 && !s_ovf) ? s_stack[--s_top] : -1;
        __syncthreads();
        const int node = s_cur;
        if (node < 0) break;
        const Node N = nodes[node];
        const int b = N.b;
        int rlo[3], rhi[3];
        for (int l = 0; l < 3; ++l) {
            rlo[l] = subcell(elo[l], N.lo[l], N.hi[l], b);
            rhi[l] = subcell(ehi[l], N.lo[l], N.hi[l], b);
        }
        const int nx = rhi[0] - rlo[0] + 1, ny = rhi[1] - rlo[1] + 1, nz = rhi[2] - rlo[2] + 1;
        const int64_t T = (int64_t)nx * ny * nz;
        for (int64_t k = t; k < T; k += kWG) {
            int ix = rlo[0] + (int)(k % nx);
            int iy = rlo[1] + (int)((k / nx) % ny);
            int iz = rlo[2] + (int)(k / ((int64_t)nx * ny));
            int32_t code = ctab[N.ctab + ix + (int64_t)b * (iy + (int64_t)b * iz)];
            if (code == kEmpty) continue;
            if (code & kLeafBit) {
                int p = atomicAdd(&s_nleaf, 1);
                if (p < kLMax) s_leaf[p] = code & ~kLeafBit;
                else s_ovf = 1;
            } else {
                int p = atomicAdd(&s_top, 1);
                if (p < kSMax) s_stack[p] = code;
                else s_ovf = 1;
            }
        }
        __syncthreads();
    }

    // Stage the candidates inside E.
    const int nleaf = s_nleaf < kLMax ? s_nleaf : kLMax;
    if (!s_ovf) {
        for (int li = w; li < nleaf; li += kWaves) {
            const Leaf L = leaves[s_leaf[li]];
            for (int p0 = 0; p0 < L.cnt; p0 += 64) {
                const bool v = p0 + lane < L.cnt;
                double4 P = v ? pos[L.beg + p0 + lane] : make_double4(0.0, 0.0, 0.0, 0.0);
                const bool in = v && P.x >= elo[0] && P.x <= ehi[0] && P.y >= elo[1] &&
                                P.y <= ehi[1] && P.z >= elo[2] && P.z <= ehi[2];
                const uint64_t m = __ballot(in);
                if (m == 0) continue;
                int base = 0;
                if (lane == 0) base = atomicAdd(&s_C, __popcll(m));
                base = __shfl(base, 0, 64);
                if (in) {
                    int slot = base + lanes_below(m);
                    if (slot < kCMax) {
                        if constexpr (F32) {
                            s_cand[slot] = make_float4((float)(P.x - cx), (float)(P.y - cy),
                                                       (float)(P.z - cz),
                                                       __int_as_float((int)P.w));
                        } else {
                            s_cand[slot] = P;
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    const int C = s_C;
    if (s_ovf || C > kCMax) {
        if (MODE == kCount && t == 0) {
            cflag[ci] = 1;
            atomicAdd(&stats->brute, 1ull);
        }
        return;
    }

    if (MODE == kFill) {
        // Sort the staged candidates by original index (bitonic, in LDS).
        int P2 = 1;
        while (P2 < C) P2 <<= 1;
        for (int k = C + t; k < P2; k += kWG) Ent<F32>::pad(s_cand[k]);
        __syncthreads();
        for (int kk = 2; kk <= P2; kk <<= 1) {
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int a = t; a < P2; a += kWG) {
                    int c = a ^ j;
                    if (c > a) {
                        E ea = s_cand[a], ec = s_cand[c];
                        bool upw = (a & kk) == 0;
                        if ((Ent<F32>::key(ea) > Ent<F32>::key(ec)) == upw) {
                            s_cand[a] = ec;
                            s_cand[c] = ea;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

    // Test: wavefront w sweeps candidates [k0, k1), 32-aligned blocks.
    const int B = ((C + kWaves * 32 - 1) / (kWaves * 32)) * 32;
    const int k0 = w * B;
    const int k1 = (k0 + B < C) ? k0 + B : C;
    int cnt = 0;
    unsigned long long conf = 0;
    for (int kw = k0; kw < k1; kw += 32) {
        uint32_t word = 0;
        const int kend = (kw + 32 < k1) ? kw + 32 : k1;
        for (int k = kw; k < kend; ++k) {
            const E e = s_cand[k];
            bool acc;
            if constexpr (F32) {
                float tx = ax - e.x, ty = ay - e.y, tz = az - e.z;
                float D = fmaf(tz, tz, fmaf(ty, ty, tx * tx));
                acc = D < tlo;
                const bool band = !acc && D <= thi;
                const uint64_t bm = __ballot(band);
                if (bm) {
                    if (band) {
                        const double4 o = orig[__float_as_int(e.w)];
                        acc = p64(qp.x, qp.y, qp.z, R, o.x, o.y, o.z);
                    }
                    conf += __popcll(bm);
                }
            } else {
                double dx = __dsub_rn(qp.x, e.x);
                double dy = __dsub_rn(qp.y, e.y);
                double dz = __dsub_rn(qp.z, e.z);
                double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                      __dmul_rn(dz, dz));
                acc = d2 < r2q;
            }
            word |= (uint32_t)acc << (k - kw);
        }
        cnt += __popc(word);
        if (MODE == kFill) s_bits[(kw >> 5) * 64 + lane] = word;
    }
    s_cnt[w][lane] = cnt;
    __syncthreads();

    if (MODE == kCount) {
        if (w == 0 && qv) {
            int tot = 0;
            for (int k = 0; k < kWaves; ++k) tot += s_cnt[k][lane];
            counts[qidx] = tot;
        }
        if (lane == 0 && conf) atomicAdd(&stats->confirms, conf);
        if (t == 0) {
            atomicAdd(&stats->pair_tests, (unsigned long long)C * (unsigned long long)ch.cnt);
            atomicAdd(&stats->candidates, (unsigned long long)C);
        }
    } else {
        // Rows out, one query per wavefront iteration: lane k owns bit word k
        // (candidates 32k .. 32k+31, ascending original index), so a row is
        // written as consecutive runs by consecutive lanes.
        const int nwords = (C + 31) >> 5;
        const int64_t myoff = qv ? offsets[qidx] : 0;
        const int64_t myend = qv ? offsets[qidx + 1] : 0;
        for (int q = w; q < ch.cnt; q += kWaves) {
            uint32_t word = lane < nwords ? s_bits[lane * 64 + q] : 0u;
            const int pc = __popc(word);
            const int inc = wave_incl_scan(pc);
            int64_t at = __shfl(myoff, q, 64) + (inc - pc);
            const int64_t end = __shfl(myend, q, 64);
            while (word) {
                const int bpos = __ffs(word) - 1;
                word &= word - 1;
                if (at < end) nbrs[at] = Ent<F32>::key(s_cand[lane * 32 + bpos]);
                ++at;
            }
        }
    }
}

// Exhaustive path for flagged items: every j in original index order.
template <int MODE>
__global__ __launch_bounds__(kWG) void k_brute(const Chunk* __restrict__ chunks,
                                               const int32_t* __restrict__ cflag,
                                               const double4* __restrict__ pos,
                                               const double4* __restrict__ orig, int64_t n,
                                               const double* __restrict__ h,
                                               int32_t* __restrict__ counts,
                                               const int64_t* __restrict__ offsets,
                                               int32_t* __restrict__ nbrs,
                                               const int* __restrict__ dflag) {
    __shared__ int64_t sh[kWaves + 1];
    const int64_t ci = blockIdx.x;
    if (*dflag || !cflag[ci]) return;
    const Chunk ch = chunks[ci];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int q = 0; q < ch.cnt; ++q) {
        const double4 qp = pos[ch.beg + q];
        const int qidx = (int)qp.w;
        const double R = 2.0 * h[qidx];
        int64_t run = MODE == kFill ? offsets[qidx] : 0;
        const int64_t end = MODE == kFill ? offsets[qidx + 1] : 0;
        int64_t mine = 0;
        for (int64_t j0 = 0; j0 < n; j0 += kWG) {
            const int64_t j = j0 + t;
            bool acc = false;
            if (j < n) {
                const double4 o = orig[j];
                acc = p64(qp.x, qp.y, qp.z, R, o.x, o.y, o.z);
            }
            if (MODE == kCount) {
                mine += acc;
            } else {
                const uint64_t m = __ballot(acc);
                if (lane == 0) sh[w] = __popcll(m);
                __syncthreads();
                int64_t before = 0, tot = 0;
                for (int k = 0; k < kWaves; ++k) {
                    if (k < w) before += sh[k];
                    tot += sh[k];
                }
                const int64_t at = run + before + lanes_below(m);
                if (acc && at < end) nbrs[at] = (int32_t)j;
                run += tot;
                __syncthreads();
            }
        }
        if (MODE == kCount) {
            int64_t tot = block_sum<kWG>(mine, sh);
            if (t == 0) counts[qidx] = (int32_t)tot;
        }
    }
}

__global__ void k_check_h(const double* __restrict__ h, int64_t n, int* __restrict__ dflag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v = h[i];
        bad |= !(v >= 0.0 && isfinite(v));
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(dflag, 1);
}

template <bool F32, int MODE>
void launch_find(Tree& t, const double* h, int32_t* counts, const int64_t* offsets,
                 int32_t* nbrs, hipStream_t st) {
    const int ph = MODE == kCount ? kPhCount : kPhFill;
    t.timer.start(ph, st);
    hipLaunchKernelGGL((k_find<F32, MODE>), dim3((unsigned)t.n_chunks), dim3(kWG), 0, st,
                       t.chunks.as<Chunk>(), t.pos.as<double4>(), t.orig.as<double4>(),
                       t.nodes.as<Node>(), t.ctab.as<int32_t>(), t.leaves.as<Leaf>(),
                       t.root_code, h, counts, offsets, nbrs, t.cflag.as<int32_t>(),
                       t.flag.as<int>(), t.stats.as<Stats>());
    BT_LAUNCH();
    t.timer.stop(ph, st);
    hipLaunchKernelGGL((k_brute<MODE>), dim3((unsigned)t.n_chunks), dim3(kWG), 0, st,
                       t.chunks.as<Chunk>(), t.cflag.as<int32_t>(), t.pos.as<double4>(),
                       t.orig.as<double4>(), t.n, h, counts, offsets, nbrs, t.flag.as<int>());
    BT_LAUNCH();
}

}  // namespace

int64_t find_pass1(Tree& t, const double* h, int32_t* counts, int64_t* offsets, hipStream_t st) {
    const bool f32 = t.prm.precision == BTREE_FP32_FILTER;
    BT_HIP(hipMemsetAsync(t.flag.p, 0, sizeof(int32_t), st));
    BT_HIP(hipMemsetAsync(t.cflag.p, 0, sizeof(int32_t) * t.n_chunks, st));
    BT_HIP(hipMemsetAsync(&t.stats.as<Stats>()->pair_tests, 0, 4 * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_check_h, dim3(grid_for(t.n, 256) < 2048 ? grid_for(t.n, 256) : 2048),
                       dim3(256), 0, st, h, t.n, t.flag.as<int>());
    BT_LAUNCH();
    if (f32) launch_find<true, kCount>(t, h, counts, nullptr, nullptr, st);
    else launch_find<false, kCount>(t, h, counts, nullptr, nullptr, st);
    scan_exclusive_i32(counts, offsets, t.n, t, st, t.flag.as<int>());
    int64_t total = 0;
    int flag = 0;
    BT_HIP(hipMemcpyAsync(&total, offsets + t.n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    BT_HIP(hipMemcpyAsync(&flag, t.flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
    BT_HIP(hipMemcpyAsync(&t.host_stats, t.stats.p, sizeof(Stats), hipMemcpyDeviceToHost, st));
    BT_HIP(hipStreamSynchronize(st));
    if (flag) fail(BTREE_EINVAL, "btree_find_neighbors: h must be finite and >= 0");
    return total;
}

void find_pass2(Tree& t, const double* h, const int64_t* offsets, int32_t* nbrs, hipStream_t st) {
    const bool f32 = t.prm.precision == BTREE_FP32_FILTER;
    if (f32) launch_find<true, kFill>(t, h, nullptr, offsets, nbrs, st);
    else launch_find<false, kFill>(t, h, nullptr, offsets, nbrs, st);
}

}  // namespace bt

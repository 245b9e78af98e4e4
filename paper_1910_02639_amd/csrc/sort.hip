// Stable LSD radix sort of (uint32 key, int32 value) pairs, 8 bits a pass.
// Used to order particles along a Morton curve of the root box before the
// level-synchronous build (particles reordered along the walk curve, as the
// paper does for locality; here it also lets a wavefront's particles share
// histogram bins so their atomics can be combined).
//
// Per pass: (1) per-tile digit histograms in LDS, written digit-major;
// (2) exclusive scan of the digit-major counts; (3) each tile ranks its keys
// stably (within a wavefront, lanes with equal digits are found with 8
// ballots), reorders them by digit in LDS and writes each digit's run to
// consecutive addresses.
#include "prim.h"

namespace bt {

namespace {

constexpr int kT = 256;
constexpr int kW = kT / 64;
constexpr int kRounds = 16;
constexpr int kTile = kT * kRounds;
constexpr int kDigits = 256;

__global__ __launch_bounds__(kT) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                   int shift, int32_t* __restrict__ cnt,
                                                   int64_t ntiles) {
    __shared__ int32_t h[kDigits];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        int64_t i = base + r * kT + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xff], 1);
    }
    __syncthreads();
    cnt[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kT) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                      const int32_t* __restrict__ vin,
                                                      uint32_t* __restrict__ kout,
                                                      int32_t* __restrict__ vout, int64_t n,
                                                      int shift,
                                                      const int64_t* __restrict__ off,
                                                      int64_t ntiles) {
    __shared__ uint32_t sk[kTile];
    __shared__ int32_t sv[kTile];
    __shared__ int32_t cnt[kDigits];  // keys of each digit ranked so far, then digit starts
    __shared__ int32_t wc[kW][kDigits];
    __shared__ int64_t scan_tmp[kW + 1];
    const int t = threadIdx.x, w = t >> 6;
    cnt[t] = 0;
    for (int k = 0; k < kW; ++k) wc[k][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    // Rank every key of the tile among the tile's keys of its digit, in
    // index order (stable): earlier rounds, then lower wavefronts, then
    // lower lanes.
    uint32_t key[kRounds];
    int32_t val[kRounds], rank[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + r * kT + t;
        const bool v = i < n;
        key[r] = v ? kin[i] : 0xffffffffu;
        val[r] = v ? vin[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const bool v = base + r * kT + t < n;
        const uint32_t d = (key[r] >> shift) & 0xffu;
        uint64_t peers = __ballot(v);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const int below = lanes_below(peers);
        if (v && below == 0) wc[w][d] = __popcll(peers);
        __syncthreads();
        int rk = cnt[d] + below;
        for (int k = 0; k < w; ++k) rk += wc[k][d];
        rank[r] = v ? rk : -1;
        __syncthreads();
        cnt[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
        for (int k = 0; k < kW; ++k) wc[k][t] = 0;
        __syncthreads();
    }
    // Digit starts inside the tile; keys move to their place in LDS.
    int64_t tot;
    const int32_t start = (int32_t)block_excl_scan<kT>(cnt[t], scan_tmp, &tot);
    cnt[t] = start;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        if (rank[r] < 0) continue;
        const int p = cnt[(key[r] >> shift) & 0xffu] + rank[r];
        sk[p] = key[r];
        sv[p] = val[r];
    }
    __syncthreads();
    // Out in tile order: keys of one digit are consecutive here and land on
    // consecutive addresses of their digit's output range.
    const int m = (int)min<int64_t>(kTile, n - base);
    for (int p = t; p < m; p += kT) {
        const uint32_t k = sk[p];
        const uint32_t d = (k >> shift) & 0xffu;
        const int64_t g = off[(int64_t)d * ntiles + blockIdx.x] + (p - cnt[d]);
        kout[g] = k;
        vout[g] = sv[p];
    }
}

}  // namespace

// Sorts (keys, vals) by the low `bits` bits of the keys (bits multiple of 8).
// k0/v0 hold the input and receive the output; k1/v1 are scratch of n.
void radix_sort_pairs(uint32_t* k0, int32_t* v0, uint32_t* k1, int32_t* v1, int64_t n, int bits,
                      Tree& t, DBuf& cnt, DBuf& off, hipStream_t st) {
    const int64_t ntiles = (n + kTile - 1) / kTile;
    cnt.reserve(sizeof(int32_t) * kDigits * ntiles);
    off.reserve(sizeof(int64_t) * (kDigits * ntiles + 1));
    uint32_t* ka = k0;
    int32_t* va = v0;
    uint32_t* kb = k1;
    int32_t* vb = v1;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kT), 0, st, ka, n, shift,
                           cnt.as<int32_t>(), ntiles);
        BT_LAUNCH();
        scan_exclusive_i32(cnt.as<int32_t>(), off.as<int64_t>(), kDigits * ntiles, t, st);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kT), 0, st, ka, va, kb, vb,
                           n, shift, off.as<int64_t>(), ntiles);
        BT_LAUNCH();
        uint32_t* tk = ka; ka = kb; kb = tk;
        int32_t* tv = va; va = vb; vb = tv;
    }
    if (ka != k0) {
        BT_HIP(hipMemcpyAsync(k0, ka, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
        BT_HIP(hipMemcpyAsync(v0, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    }
}

}  // namespace bt

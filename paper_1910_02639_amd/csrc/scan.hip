// Exclusive prefix sums into int64 (CSR offsets, node and leaf numbering).
// Three launches: per-tile sums, one workgroup scanning the tile sums, then
// per-tile scans that add the tile's base.  out has n+1 entries; out[n] is
// the total.
#include "prim.h"

namespace bt {

namespace {

constexpr int kT = 256;
constexpr int kItems = 8;
constexpr int kTile = kT * kItems;

template <class In>
__global__ __launch_bounds__(kT) void k_tile_sum(const In* __restrict__ in, int64_t n,
                                                 int64_t* __restrict__ tsum) {
    __shared__ int64_t sh[kT / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int64_t k = base + i * kT + threadIdx.x;
        if (k < n) s += (int64_t)in[k];
    }
    s = block_sum<kT>(s, sh);
    if (threadIdx.x == 0) tsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(kT) void k_scan_tiles(int64_t* __restrict__ tsum, int64_t ntiles) {
    __shared__ int64_t sh[kT / 64 + 1];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < ntiles; b0 += kT) {
        int64_t k = b0 + threadIdx.x;
        int64_t v = k < ntiles ? tsum[k] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan<kT>(v, sh, &tot);
        if (k < ntiles) tsum[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) tsum[ntiles] = carry;
}

template <class In>
__global__ __launch_bounds__(kT) void k_tile_scan(const In* __restrict__ in, int64_t n,
                                                  const int64_t* __restrict__ tsum,
                                                  int64_t ntiles, int64_t* __restrict__ out,
                                                  const int* __restrict__ guard) {
    __shared__ int64_t sh[kT / 64 + 1];
    if (guard && *guard) return;  // invalid input detected upstream: write nothing
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int64_t v[kItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int64_t k = base + i;
        v[i] = k < n ? (int64_t)in[k] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_excl_scan<kT>(s, sh, &tot) + tsum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int64_t k = base + i;
        if (k < n) out[k] = ex;
        ex += v[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tsum[ntiles];
}

template <class In>
void scan_impl(const In* in, int64_t* out, int64_t n, Tree& t, hipStream_t st,
               const int* guard) {
    int64_t ntiles = (n + kTile - 1) / kTile;
    if (ntiles < 1) ntiles = 1;
    t.scan_tmp.reserve(sizeof(int64_t) * (size_t)(ntiles + 1));
    int64_t* ts = t.scan_tmp.as<int64_t>();
    hipLaunchKernelGGL(k_tile_sum<In>, dim3((unsigned)ntiles), dim3(kT), 0, st, in, n, ts);
    BT_LAUNCH();
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kT), 0, st, ts, ntiles);
    BT_LAUNCH();
    hipLaunchKernelGGL(k_tile_scan<In>, dim3((unsigned)ntiles), dim3(kT), 0, st, in, n, ts,
                       ntiles, out, guard);
    BT_LAUNCH();
}

// Variants whose length lives in device memory (*nptr <= ncap): launched for
// the capacity, tiles past the length do nothing.  No host read is needed, so
// they can run inside a captured graph.
template <class In>
__global__ __launch_bounds__(kT) void k_tile_sum_dev(const In* __restrict__ in,
                                                     const int32_t* __restrict__ nptr,
                                                     int64_t* __restrict__ tsum) {
    __shared__ int64_t sh[kT / 64 + 1];
    const int64_t n = *nptr;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base >= n) {
        if (threadIdx.x == 0) tsum[blockIdx.x] = 0;
        return;
    }
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int64_t k = base + i * kT + threadIdx.x;
        if (k < n) s += (int64_t)in[k];
    }
    s = block_sum<kT>(s, sh);
    if (threadIdx.x == 0) tsum[blockIdx.x] = s;
}

template <class In>
__global__ __launch_bounds__(kT) void k_tile_scan_dev(const In* __restrict__ in,
                                                      const int32_t* __restrict__ nptr,
                                                      const int64_t* __restrict__ tsum,
                                                      int64_t ntiles, int64_t* __restrict__ out) {
    __shared__ int64_t sh[kT / 64 + 1];
    const int64_t n = *nptr;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tsum[ntiles];
    if ((int64_t)blockIdx.x * kTile >= n) return;
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int64_t v[kItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int64_t k = base + i;
        v[i] = k < n ? (int64_t)in[k] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_excl_scan<kT>(s, sh, &tot) + tsum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int64_t k = base + i;
        if (k < n) out[k] = ex;
        ex += v[i];
    }
}

template <class In>
void scan_dev_impl(const In* in, int64_t* out, const int32_t* nptr, int64_t ncap, Tree& t,
                   hipStream_t st) {
    int64_t ntiles = (ncap + kTile - 1) / kTile;
    if (ntiles < 1) ntiles = 1;
    if (t.scan_tmp.bytes < sizeof(int64_t) * (size_t)(ntiles + 1))
        fail(BTREE_EDEVICE, "scan workspace not reserved");
    int64_t* ts = t.scan_tmp.as<int64_t>();
    hipLaunchKernelGGL(k_tile_sum_dev<In>, dim3((unsigned)ntiles), dim3(kT), 0, st, in, nptr, ts);
    BT_LAUNCH();
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kT), 0, st, ts, ntiles);
    BT_LAUNCH();
    hipLaunchKernelGGL(k_tile_scan_dev<In>, dim3((unsigned)ntiles), dim3(kT), 0, st, in, nptr, ts,
                       ntiles, out);
    BT_LAUNCH();
}

// K arrays of one device length scanned together (two launches for all
// K): tile sums and tile scans of array q go to tsum[q * (ntiles+1)].
template <int K>
struct ScanK {
    const int64_t* in[K];
    int64_t* out[K];
};

template <int K>
__global__ __launch_bounds__(kT) void k_tile_sum_devk(ScanK<K> a, const int32_t* __restrict__ nptr,
                                                      int64_t* __restrict__ tsum, int64_t ntiles) {
    __shared__ int64_t sh[kT / 64 + 1];
    const int64_t n = *nptr;
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        int64_t s = 0;
        if (base < n) {
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const int64_t k = base + i * kT + threadIdx.x;
                if (k < n) s += a.in[q][k];
            }
            s = block_sum<kT>(s, sh);
        }
        if (threadIdx.x == 0) tsum[q * (ntiles + 1) + blockIdx.x] = s;
    }
}

// Each workgroup adds the sums of the tiles before its own (a short loop:
// these scans run over per-cell arrays, a few tiles long), and the one that
// holds the last element writes the total, so no separate pass scans the
// tile sums.
template <int K>
__global__ __launch_bounds__(kT) void k_tile_scan_devk(ScanK<K> a, const int32_t* __restrict__ nptr,
                                                       const int64_t* __restrict__ tsum,
                                                       int64_t ntiles) {
    __shared__ int64_t sh[kT / 64 + 1];
    const int64_t n = *nptr;
    const int64_t b = blockIdx.x;
    if (n <= 0) {
        if (b == 0 && threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q < K; ++q) a.out[q][0] = 0;
        }
        return;
    }
    if (b * kTile >= n) return;  // uniform over the workgroup
    const bool last = (b + 1) * kTile >= n;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int64_t* ts = tsum + q * (ntiles + 1);
        int64_t pre = 0;
        for (int64_t j = threadIdx.x; j < b; j += kT) pre += ts[j];
        pre = block_sum<kT>(pre, sh);
        const int64_t base = b * kTile + (int64_t)threadIdx.x * kItems;
        int64_t v[kItems];
        int64_t s = 0;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int64_t k = base + i;
            v[i] = k < n ? a.in[q][k] : 0;
            s += v[i];
        }
        int64_t tot;
        int64_t ex = block_excl_scan<kT>(s, sh, &tot) + pre;
        if (last && threadIdx.x == 0) a.out[q][n] = pre + tot;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int64_t k = base + i;
            if (k < n) a.out[q][k] = ex;
            ex += v[i];
        }
    }
}

template <int K>
void scank_dev_i64(const ScanK<K>& a, const int32_t* nptr, int64_t ncap, Tree& t, hipStream_t st) {
    int64_t ntiles = (ncap + kTile - 1) / kTile;
    if (ntiles < 1) ntiles = 1;
    if (t.scan_tmp.bytes < sizeof(int64_t) * (size_t)(K * (ntiles + 1)))
        fail(BTREE_EDEVICE, "scan workspace not reserved");
    int64_t* ts = t.scan_tmp.as<int64_t>();
    hipLaunchKernelGGL(k_tile_sum_devk<K>, dim3((unsigned)ntiles), dim3(kT), 0, st, a, nptr, ts,
                       ntiles);
    BT_LAUNCH();
    hipLaunchKernelGGL(k_tile_scan_devk<K>, dim3((unsigned)ntiles), dim3(kT), 0, st, a, nptr, ts,
                       ntiles);
    BT_LAUNCH();
}

}  // namespace

void scan2_dev_i64(const int64_t* in0, int64_t* out0, const int64_t* in1, int64_t* out1,
                   const int32_t* nptr, int64_t ncap, Tree& t, hipStream_t st) {
    scank_dev_i64<2>(ScanK<2>{{in0, in1}, {out0, out1}}, nptr, ncap, t, st);
}

void scan3_dev_i64(const int64_t* in0, int64_t* out0, const int64_t* in1, int64_t* out1,
                   const int64_t* in2, int64_t* out2, const int32_t* nptr, int64_t ncap,
                   Tree& t, hipStream_t st) {
    scank_dev_i64<3>(ScanK<3>{{in0, in1, in2}, {out0, out1, out2}}, nptr, ncap, t, st);
}

void scan_reserve(Tree& t, int64_t ncap) {
    int64_t ntiles = (ncap + kTile - 1) / kTile;
    if (ntiles < 1) ntiles = 1;
    t.scan_tmp.reserve(sizeof(int64_t) * (size_t)(ntiles + 1));
}

void scan_dev_i32(const int32_t* in, int64_t* out, const int32_t* nptr, int64_t ncap, Tree& t,
                  hipStream_t st) {
    scan_dev_impl<int32_t>(in, out, nptr, ncap, t, st);
}

void scan_dev_i64(const int64_t* in, int64_t* out, const int32_t* nptr, int64_t ncap, Tree& t,
                  hipStream_t st) {
    scan_dev_impl<int64_t>(in, out, nptr, ncap, t, st);
}

void scan_exclusive_i32(const int32_t* in, int64_t* out, int64_t n, Tree& t, hipStream_t st,
                        const int* guard) {
    scan_impl<int32_t>(in, out, n, t, st, guard);
}

void scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, Tree& t, hipStream_t st,
                        const int* guard) {
    scan_impl<int64_t>(in, out, n, t, st, guard);
}

}  // namespace bt

// Wavefront and workgroup primitives for gfx950 (wave64).
#pragma once

#include "common.h"

namespace bt {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane (v_mbcnt_lo/hi).
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Adds, for every active lane, 1 to counter[idx] with one atomic per distinct
// idx in the wavefront.  Cheap when neighbouring lanes share idx (particles
// sorted along a space-filling curve).
__device__ __forceinline__ void wave_agg_inc(int32_t* counter, int64_t idx, bool active) {
    uint64_t rem = __ballot(active);
    while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int64_t li = __shfl(idx, leader, 64);
        const uint64_t peers = __ballot(active && idx == li);
        if (lane_id() == leader) atomicAdd(&counter[li], (int32_t)__popcll(peers));
        rem &= ~peers;
    }
}

// Like wave_agg_inc, and returns the old value of counter[idx] plus the
// number of lower lanes with the same idx (a unique slot per lane).  The
// groups of equal idx are found first (register work only), then every
// group's first lane issues its atomic in one instruction, so the wavefront
// waits for one atomic round trip however many groups it has.
__device__ __forceinline__ int32_t wave_agg_slot(int32_t* counter, int64_t idx, bool active) {
    uint64_t rem = __ballot(active);
    int leader_of_mine = 0, rank = 0, group = 0;
    while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int64_t li = __shfl(idx, leader, 64);
        const bool mine = active && idx == li;
        const uint64_t peers = __ballot(mine);
        if (mine) {
            leader_of_mine = leader;
            rank = lanes_below(peers);
        }
        if (lane_id() == leader) group = __popcll(peers);
        rem &= ~peers;
    }
    int32_t base = 0;
    if (group) base = atomicAdd(&counter[idx], (int32_t)group);
    base = __shfl(base, leader_of_mine, 64);
    return base + rank;
}

// Orders a wavefront's shared-memory accesses: what its lanes stored before
// the call is what its lanes load after it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T t = __shfl_up(v, d, 64);
        if (l >= d) v += t;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
    return v;
}

// Exclusive scan over a workgroup of NT threads (NT multiple of 64).
// `scratch` must hold NT/64 + 1 int64 values in LDS.  Returns the exclusive
// prefix of v; *total receives the workgroup sum.  Contains barriers.
template <int NT>
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* scratch, int64_t* total) {
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(v);
    if (lane_id() == 63) scratch[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int k = 0; k < NW; ++k) {
            int64_t c = scratch[k];
            scratch[k] = run;
            run += c;
        }
        scratch[NW] = run;
    }
    __syncthreads();
    int64_t ex = inc - v + scratch[w];
    *total = scratch[NW];
    __syncthreads();
    return ex;
}

template <int NT>
__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* scratch) {
    constexpr int NW = NT / 64;
    v = wave_sum(v);
    if (lane_id() == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t s = 0;
    for (int k = 0; k < NW; ++k) s += scratch[k];
    __syncthreads();
    return s;
}

}  // namespace bt

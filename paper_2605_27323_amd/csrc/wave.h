// Wave- and block-level helpers of the GPU kernels (device code only):
// lane ranks within a 64-lane ballot, the per-wave queue chunk of the
// persistent traversal kernels, and block-aggregated queue reservation.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ptmi {

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// position of this lane among the set lanes of a 64-bit ballot below it
__device__ __forceinline__ uint32_t rank_in(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// one atomic per wave reserves room for the wave's set lanes; every set
// lane gets base + its rank among them
__device__ __forceinline__ uint32_t wave_reserve(uint32_t* ctr, uint64_t m) {
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(ctr, (uint32_t)__popcll(m));
    base = __builtin_amdgcn_readfirstlane(base);
    return base + rank_in(m);
}

// Sum v over the 64 lanes of the wave (every lane calls this) and add the
// sum to *dst with one atomic.
__device__ __forceinline__ void wave_add_u64(unsigned long long* dst, uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane_id() == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

// lane 0's value, in every lane
__device__ __forceinline__ unsigned long long wave_broadcast_u64(unsigned long long v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Workgroup order in which consecutive parts of a queue are handed out.
// The dispatcher places workgroup b on XCD b mod 8 (each XCD has its own
// L2); with xcd_local the order b' = (b mod 8) * (G / 8) + b / 8 gives every
// XCD one contiguous eighth of the queue, so that neighbouring rays (close
// pixels, similar directions) share an L2 instead of being spread over all
// eight.  Grids that are not a multiple of 8 keep launch order.
__device__ __forceinline__ uint32_t block_order(int xcd_local) {
    const uint32_t b = blockIdx.x;
    if (!xcd_local || (gridDim.x & 7u) != 0u) return b;
    return (b & 7u) * (gridDim.x >> 3) + (b >> 3);
}

// The contiguous chunk [next, end) of a queue of `count` entries owned by
// this wave in a persistent kernel (waves in block_order).
__device__ __forceinline__ void wave_chunk(uint32_t count, uint32_t& next, uint32_t& end, int xcd_local = 0) {
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t wave = (block_order(xcd_local) * blockDim.x + threadIdx.x) >> 6;
    const uint32_t chunk = (uint32_t)(((uint64_t)count + nwaves - 1) / nwaves);
    next = (uint32_t)min((uint64_t)wave * chunk, (uint64_t)count);
    end = (uint32_t)min((uint64_t)next + chunk, (uint64_t)count);
    // the same for every lane of the wave: keep them in scalar registers
    next = __builtin_amdgcn_readfirstlane(next);
    end = __builtin_amdgcn_readfirstlane(end);
}

// Block-aggregated reservation on two queue counters: every thread of the
// block calls this once per trip (it synchronises the block) with its
// wave's ballots m0, m1; one atomic per counter and block.  Returns the
// slots of this lane (valid where its bit is set).  `par` alternates
// between trips: the counts are double-buffered so that two barriers per
// trip suffice.  Blocks of at most 256 threads.
struct BlockReserve {
    uint32_t cnt[2][2][4];
    uint32_t base[2][2];
};

__device__ __forceinline__ void block_reserve2(BlockReserve& br, int par, uint32_t* c0, uint64_t m0, uint32_t* c1,
                                               uint64_t m1, uint32_t& j0, uint32_t& j1) {
    const uint32_t w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane_id() == 0) {
        br.cnt[par][0][w] = (uint32_t)__popcll(m0);
        br.cnt[par][1][w] = (uint32_t)__popcll(m1);
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint32_t tot = 0;
        for (uint32_t k = 0; k < nw; ++k) tot += br.cnt[par][threadIdx.x][k];
        br.base[par][threadIdx.x] = tot ? atomicAdd(threadIdx.x == 0 ? c0 : c1, tot) : 0u;
    }
    __syncthreads();
    uint32_t o0 = br.base[par][0], o1 = br.base[par][1];
    for (uint32_t k = 0; k < w; ++k) {
        o0 += br.cnt[par][0][k];
        o1 += br.cnt[par][1][k];
    }
    j0 = o0 + rank_in(m0);
    j1 = o1 + rank_in(m1);
}

}  // namespace ptmi

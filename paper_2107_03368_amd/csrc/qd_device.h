// Wavefront-level helpers for gfx950 (64-lane waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qd {

typedef unsigned long long u64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ u64 ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Set bits of mask in the lanes below this one (a lane's rank among the set lanes).
__device__ __forceinline__ uint32_t lanes_below(u64 mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ u64 readlane64(u64 v, int l) {
    return (u64)readlane((uint32_t)v, l) | ((u64)readlane((uint32_t)(v >> 32), l) << 32);
}
__device__ __forceinline__ uint32_t readfirst(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// v from lane (lane - 1); lane 0 keeps its own value.
__device__ __forceinline__ u64 shift_up64(u64 v) {
    int l = lane_id();
    int src = (l > 0 ? l - 1 : 0) << 2;
    uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)v);
    uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(v >> 32));
    return (u64)lo | ((u64)hi << 32);
}

// Sum over each aligned group of 8 lanes; every lane of the group gets the sum.
// DPP: quad_perm [1,0,3,2], quad_perm [2,3,0,1], then row_half_mirror
// (lane i <-> 7-i inside 8 lanes, which pairs the two quads).
__device__ __forceinline__ uint32_t sum8(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);
    return v;
}

// Sum over each 32-lane half of the wave; every lane gets its half's sum.
__device__ __forceinline__ uint32_t sum32_half(uint32_t v) {
    v = sum8(v);
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);  // row_mirror (16 lanes)
    v += (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);             // xor 16 within 32
    return v;
}

// Float sum over the wave in a fixed butterfly order (every lane gets it).
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ uint32_t popc4(uint4 a) {
    return __popc(a.x) + __popc(a.y) + __popc(a.z) + __popc(a.w);
}
__device__ __forceinline__ uint32_t popc_and4(uint4 a, uint4 b) {
    return __popc(a.x & b.x) + __popc(a.y & b.y) + __popc(a.z & b.z) + __popc(a.w & b.w);
}

// Insert candidate c into a sorted k-list held one entry per lane (lane r has
// the r-th smallest; unused slots and lanes >= k hold KEY_NONE).  Requires c
// to be smaller than the k-th entry.
__device__ __forceinline__ u64 list_insert(u64 e, u64 c, uint32_t k) {
    const u64 none = ~0ull;
    int l = lane_id();
    int pos = __popcll(ballot(e < c));
    u64 up = shift_up64(e);
    u64 r = l < pos ? e : (l == pos ? c : up);
    return l < (int)k ? r : none;
}

// Ascending bitonic sort of n (a power of two) keys in LDS by the whole block.
// Must be entered by every thread after the keys are written and synced.
__device__ inline void block_bitonic_sort(u64 *a, uint32_t n) {
    for (uint32_t size = 2; size <= n; size <<= 1)
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = threadIdx.x; t < n / 2; t += blockDim.x) {
                uint32_t lo = 2 * t - (t & (stride - 1));
                uint32_t hi = lo + stride;
                bool up = (lo & size) == 0;
                u64 x = a[lo], y = a[hi];
                if ((x > y) == up) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
            __syncthreads();
        }
}

__device__ __forceinline__ uint32_t next_pow2(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace qd

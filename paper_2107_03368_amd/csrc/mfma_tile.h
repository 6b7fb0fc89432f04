// Overlap counts on the matrix cores: for a tile of 256 "A" rows (queries)
// and 256 "B" rows (database rows or bit summaries) of 4096 bits each,
// C[i][j] = popcount(A_i AND B_j), the term every weighted distance and every
// node bound of Eq. 1 is built from.  Over the 4096 bit positions this is a
// dense {0,1} matrix product, computed with v_mfma_i32_16x16x64_i8 on bits
// unpacked to bytes (exact: counts stay below 2^13).
//
// A block of 8 waves owns the 256 x 256 tile.  The K dimension is streamed in
// chunks of 512 bits: packed chunks go global -> registers -> LDS (the next
// chunk's loads are in flight while the current one is used), and for each
// 64-bit step the whole block unpacks the step to bytes in LDS (one bit per
// byte; double-buffered, so the unpack of step s+1 follows the MFMAs of step
// s with one barrier per step).  Every wave multiplies its 128 x 64 eighth as
// 8 x 4 MFMA tiles.  Lane l supplies A rows (l % 16) at k = 16*(l/16) .. +15
// and B columns likewise, and receives C rows 4*(l/16) .. +3 of column l % 16.
//
// Rows are given per load slot: thread t reads 16 bytes of row (t/4 + 128 u)
// for u = 0..3 (rows 0..255 are A, 256..511 are B); a null row reads zeros.
// The tile is the same whether rows are contiguous (sequential search) or
// gathered through a list (the blocked tree search).
#pragma once

#include "qd_device.h"

namespace qd {
namespace mt {

constexpr int kThreads = 512;  // 8 waves
constexpr int MA = 256;        // A rows (queries) per tile
constexpr int MB = 256;        // B rows per tile
constexpr int KCH = 512;       // bits per packed chunk (8 steps of 64)
constexpr int CHB = KCH / 8;   // bytes per row per chunk (64)
constexpr int UST = 80;        // unpacked row stride in LDS (64 bytes + 16 pad)
constexpr int kLoads = (MA + MB) * 4 / kThreads;  // 16-byte loads per thread per chunk

typedef int v4i __attribute__((ext_vector_type(4)));

struct Smem {
    uint8_t pk[2][(MA + MB) * CHB];  // packed chunk (A rows then B rows), double-buffered
    uint8_t uk[2][(MA + MB) * UST];  // unpacked 64-bit step, double-buffered
};

// 4 bits -> 4 bytes of 0/1 (bit e -> byte e): the multiplier places bit e at
// bit 8e with no two terms overlapping, so no carries occur.
__device__ __forceinline__ uint32_t spread4(uint32_t x) { return ((x & 0xFu) * 0x00204081u) & 0x01010101u; }

// Row handled by load slot u of this thread (0..511; < 256 is an A row).
__device__ __forceinline__ int slot_row(int u) { return (int)(threadIdx.x >> 2) + u * (kThreads / 4); }

// Tile coordinates of the accumulator entry acc[a][b][r] of this lane.
__device__ __forceinline__ int acc_arow(int a, int r) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    return (w >> 2) * 128 + a * 16 + (lane >> 4) * 4 + r;
}
__device__ __forceinline__ int acc_brow(int b) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    return (w & 3) * 64 + b * 16 + (lane & 15);
}

__device__ __forceinline__ void overlap_tile(const uint4 *const (&src)[kLoads], Smem &sm, v4i (&acc)[8][4]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wq = w >> 2, wr = w & 3;  // 2 x 4 waves, each 128 A rows x 64 B rows
    const int li = lane & 15, lg = lane >> 4;
    const int j = tid & 3;  // 16-byte piece of the 64-byte chunk row

#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = v4i{0, 0, 0, 0};

    uint4 pre[kLoads];
    auto load_chunk = [&](int c) {
#pragma unroll
        for (int u = 0; u < kLoads; u++) pre[u] = src[u] ? src[u][c * 4 + j] : make_uint4(0, 0, 0, 0);
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int u = 0; u < kLoads; u++) {
            const int i = tid + u * kThreads;
            *reinterpret_cast<uint4 *>(&sm.pk[buf][(i >> 2) * CHB + (i & 3) * 16]) = pre[u];
        }
    };
    // unpack 64-bit step s of the packed chunk in pk[pb] into uk[ub]
    auto unpack = [&](int pb, int s, int ub) {
        for (int i = tid; i < (MA + MB) * 4; i += kThreads) {
            const int r = i >> 2, g = i & 3;
            const uint32_t bits = *reinterpret_cast<const uint16_t *>(&sm.pk[pb][r * CHB + s * 8 + g * 2]);
            *reinterpret_cast<uint4 *>(&sm.uk[ub][r * UST + g * 16]) =
                make_uint4(spread4(bits), spread4(bits >> 4), spread4(bits >> 8), spread4(bits >> 12));
        }
    };

    constexpr int kSteps = 4096 / 64, kPerChunk = KCH / 64;
    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    unpack(0, 0, 0);
    __syncthreads();
    for (int g = 0; g < kSteps; g++) {
        const int c = g / kPerChunk, s = g % kPerChunk;
        if (s == 0 && c + 1 < kSteps / kPerChunk) load_chunk(c + 1);  // in flight during this chunk
        const uint8_t *ua = sm.uk[g & 1];
        const uint8_t *ubp = sm.uk[g & 1] + MA * UST;
        v4i af[8], bf[4];
#pragma unroll
        for (int a = 0; a < 8; a++) af[a] = *reinterpret_cast<const v4i *>(ua + (wq * 128 + a * 16 + li) * UST + lg * 16);
#pragma unroll
        for (int b = 0; b < 4; b++) bf[b] = *reinterpret_cast<const v4i *>(ubp + (wr * 64 + b * 16 + li) * UST + lg * 16);
#pragma unroll
        for (int a = 0; a < 8; a++)
#pragma unroll
            for (int b = 0; b < 4; b++)
                acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[b], acc[a][b], 0, 0, 0);
        if (g + 1 < kSteps) {
            const int c1 = (g + 1) / kPerChunk, s1 = (g + 1) % kPerChunk;
            if (s1 == 0) {
                store_chunk(c1 & 1);  // the other packed buffer: nobody reads it now
                __syncthreads();
            }
            unpack(c1 & 1, s1, (g + 1) & 1);
        }
        __syncthreads();
    }
}

}  // namespace mt
}  // namespace qd

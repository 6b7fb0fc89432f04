// Overlap counts on the matrix cores: for a tile of 256 "A" rows (queries)
// and 256 "B" rows (database rows or bit summaries) of 4096 bits each,
// C[i][j] = popcount(A_i AND B_j), the term every weighted distance and every
// node bound of Eq. 1 is built from.  Over the 4096 bit positions this is a
// dense {0,1} matrix product, computed with v_mfma_i32_16x16x64_i8 on bits
// unpacked to bytes (exact: counts stay below 2^13).
//
// A block of 8 waves owns the 256 x 256 tile, and thread t owns row t (A rows
// 0..255, then B rows).  The K dimension is streamed in windows of 128 bits:
// each thread keeps its row's current 512-bit chunk in registers (the next
// chunk's loads are in flight meanwhile) and unpacks one 128-bit window of it
// to 128 bytes of 0/1 in LDS (rows 144 bytes apart, so 16 consecutive rows
// fall on distinct banks).  Windows are double-buffered: while the matrix
// cores consume window w, the threads unpack window w+1 into the other
// buffer, with one barrier per window.  Every wave multiplies its 128 x 64
// eighth as 8 x 4 MFMA tiles per 64-bit step.  Lane l supplies A rows (l % 16)
// at k = 16*(l/16) .. +15 and B columns likewise, and receives C rows
// 4*(l/16) .. +3 of column l % 16.
//
// A null row reads zeros.  The tile is the same whether rows are contiguous
// (sequential search) or gathered through a list (the blocked tree search).
#pragma once

#include "qd_device.h"

namespace qd {
namespace mt {

constexpr int kThreads = 512;  // 8 waves, one row per thread
constexpr int MA = 256;        // A rows (queries) per tile
constexpr int MB = 256;        // B rows per tile
constexpr int WIN = 128;       // bits per window (two 64-bit MFMA steps)
constexpr int UST = 144;       // unpacked row stride in LDS (128 bytes + 16 pad)

typedef int v4i __attribute__((ext_vector_type(4)));

struct Smem {
    uint8_t uk[2][(MA + MB) * UST];  // unpacked window, double-buffered
};

// 4 bits -> 4 bytes of 0/1 (bit e -> byte e): the multiplier places bit e at
// bit 8e with no two terms overlapping, so no carries occur.
__device__ __forceinline__ uint32_t spread4(uint32_t x) { return ((x & 0xFu) * 0x00204081u) & 0x01010101u; }

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup x runs on
// XCD x % 8), and each XCD has its own L2.  xcd_tile maps workgroup x to a
// tile index so that every XCD gets one contiguous range of the n tiles: tiles
// that share B rows (consecutive indices) then share one L2.  Returns false
// for the padding workgroups of a grid of xcd_grid(n) workgroups.
constexpr uint32_t kXcds = 8;
__host__ __device__ inline uint64_t xcd_grid(uint64_t n) { return (n + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ bool xcd_tile(uint64_t x, uint64_t n, uint64_t &tile) {
    const uint64_t per = (n + kXcds - 1) / kXcds;
    tile = (x % kXcds) * per + x / kXcds;
    return tile < n;
}

// Row owned by this thread (0..511; < 256 is an A row).
__device__ __forceinline__ int own_row() { return (int)threadIdx.x; }

// Tile coordinates of the accumulator entry acc[a][b][r] of this lane.
__device__ __forceinline__ int acc_arow(int a, int r) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    return (w >> 2) * 128 + a * 16 + (lane >> 4) * 4 + r;
}
__device__ __forceinline__ int acc_brow(int b) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    return (w & 3) * 64 + b * 16 + (lane & 15);
}

// 128 bits -> 128 bytes of 0/1 at dst (16-byte aligned)
__device__ __forceinline__ void unpack_window(uint4 v, uint8_t *dst) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int h = 0; h < 8; h++) {
        const uint32_t x = w[h >> 1] >> ((h & 1) * 16);
        *reinterpret_cast<uint4 *>(dst + h * 16) =
            make_uint4(spread4(x), spread4(x >> 4), spread4(x >> 8), spread4(x >> 12));
    }
}

// row: this thread's row (32 x 16 bytes) or null
__device__ __forceinline__ void overlap_tile(const uint4 *row, Smem &sm, v4i (&acc)[8][4]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wq = w >> 2, wr = w & 3;  // 2 x 4 waves, each 128 A rows x 64 B rows
    const int li = lane & 15, lg = lane >> 4;

#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = v4i{0, 0, 0, 0};

    // 16-byte piece i of 512-bit chunk c of this thread's row
    auto piece = [&](int c, int i) { return row ? row[c * 4 + i] : make_uint4(0, 0, 0, 0); };
    uint4 cur[4], nxt[4];
#pragma unroll
    for (int i = 0; i < 4; i++) cur[i] = piece(0, i);
    unpack_window(cur[0], sm.uk[0] + tid * UST);
    __syncthreads();
    constexpr int kChunks = 4096 / (4 * WIN);
    for (int c = 0; c < kChunks; c++) {
        const bool more = c + 1 < kChunks;
#pragma unroll
        for (int wi = 0; wi < 4; wi++) {  // window 4c + wi, in buffer wi & 1
            if (more) nxt[wi] = piece(c + 1, wi);  // the next chunk, one piece per window
            const uint8_t *ua = sm.uk[wi & 1];
            const uint8_t *ubp = sm.uk[wi & 1] + MA * UST;
#pragma unroll
            for (int ks = 0; ks < 2; ks++) {
                v4i af[8], bf[4];
#pragma unroll
                for (int a = 0; a < 8; a++)
                    af[a] = *reinterpret_cast<const v4i *>(ua + (wq * 128 + a * 16 + li) * UST + ks * 64 + lg * 16);
#pragma unroll
                for (int b = 0; b < 4; b++)
                    bf[b] = *reinterpret_cast<const v4i *>(ubp + (wr * 64 + b * 16 + li) * UST + ks * 64 + lg * 16);
#pragma unroll
                for (int a = 0; a < 8; a++)
#pragma unroll
                    for (int b = 0; b < 4; b++)
                        acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[b], acc[a][b], 0, 0, 0);
                // keep one step's fragments live at a time (register budget of two waves per SIMD)
                __builtin_amdgcn_sched_barrier(0);
            }
            // window 4c + wi + 1 into the other buffer, last read before the previous barrier
            if (wi < 3)
                unpack_window(cur[wi + 1], sm.uk[(wi + 1) & 1] + tid * UST);
            else if (more)
                unpack_window(nxt[0], sm.uk[0] + tid * UST);
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; i++) cur[i] = nxt[i];
    }
}

}  // namespace mt
}  // namespace qd

// Overlap counts on the matrix cores: for a tile of 256 "A" rows (queries)
// and 256 "B" rows (database rows or bit summaries) of 4096 bits each,
// C[i][j] = popcount(A_i AND B_j), the term every weighted distance and every
// node bound of Eq. 1 is built from.  Over the 4096 bit positions this is a
// dense {0,1} matrix product.  It runs as the FP4 (e2m1) matrix instruction
// v_mfma_scale_f32_16x16x128_f8f6f4: every bit becomes one 4-bit element
// (0 or 0.5), both operands carry the block scale 2, so every product is 0
// or 1 and the fp32 accumulator holds the exact count (at most 4096 < 2^24).
// The order in which bits become elements only has to be the same for both
// operands, since the sum over K does not depend on it.
//
// A block of 8 waves owns the 256 x 256 tile, and thread t owns row t (A rows
// 0..255, then B rows).  The K dimension is streamed in windows of 256 bits:
// each thread loads its row's next window into registers while the current
// one is multiplied, then unpacks it to 128 bytes of elements in LDS (rows 144
// bytes apart, so 16 consecutive rows fall on distinct banks).  Windows are
// double-buffered: while the matrix cores consume window w, the threads
// unpack window w+1 into the other buffer, with one barrier per window.
// Every wave multiplies its 128 x 64 eighth as 8 x 4 tiles per 128-bit step.
// Lane l supplies A rows (l % 16) at k = 32*(l/16) .. +31 (16 bytes) and B
// columns likewise, and receives C rows 4*(l/16) .. +3 of column l % 16.
//
// A missing row reads as zeros.  The tile is the same whether rows are contiguous
// (sequential search) or gathered through a list (the blocked tree search).
#pragma once

#include "qd_device.h"

namespace qd {
namespace mt {

constexpr int kThreads = 512;  // 8 waves, one row per thread
constexpr int MA = 256;        // A rows (queries) per tile
constexpr int MB = 256;        // B rows per tile
constexpr int WIN = 256;       // bits per window (two 128-bit matrix steps)
constexpr int UST = 144;       // unpacked row stride in LDS (128 bytes + 16 pad)

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct Smem {
    uint8_t uk[2][(MA + MB) * UST];  // unpacked window, double-buffered
};

// 8 bits -> 8 elements of 0/1 (e2m1 0x1 = 0.5) in the nibbles of a word,
// nibble 2i holding bit i and nibble 2i+1 bit i+4.  The multiply copies the
// low 7 bits to offsets 0, 7, 14, 21 without overlap (so without carries); the
// mask keeps bits 0, 4, 1, 5, 2, 6, 3 at nibbles 0..6; bit 7 goes to nibble 7.
__device__ __forceinline__ uint32_t nib8(uint32_t y) {
    return (((y & 0x7Fu) * 0x00204081u) & 0x11111111u) | ((y & 0x80u) << 21);
}

// 128 bits -> 64 bytes of elements at dst (16-byte aligned); input word j
// becomes bytes 16j .. 16j+15
__device__ __forceinline__ void unpack_half(uint4 p, uint8_t *dst) {
    const uint32_t w[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
    for (int j = 0; j < 4; j++)
        *reinterpret_cast<uint4 *>(dst + j * 16) =
            make_uint4(nib8(w[j] & 0xFF), nib8((w[j] >> 8) & 0xFF), nib8((w[j] >> 16) & 0xFF), nib8(w[j] >> 24));
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup x runs on
// XCD x % 8), and each XCD has its own L2.  xcd_tile maps workgroup x to a
// tile index so that every XCD gets one contiguous range of the n tiles: tiles
// that share B rows (consecutive indices) then share one L2.  Returns false
// for the padding workgroups of a grid of xcd_grid(n) workgroups.
constexpr uint32_t kXcds = 8;
// A dispatch packet holds the grid size in work-items as a 32-bit number, so a
// launch of kThreads-thread workgroups stays below 2^32 / kThreads of them;
// kernels take their tiles in a workgroup-stride loop over a grid of at most
// kMaxGrid workgroups (a multiple of kXcds, so a workgroup keeps its XCD).
constexpr uint64_t kMaxGrid = 1ull << 22;
__host__ __device__ inline uint64_t tile_grid(uint64_t n) { return n < kMaxGrid ? n : kMaxGrid; }
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

// Exact count held by an accumulator entry.
__device__ __forceinline__ uint32_t count(float c) { return (uint32_t)c; }

// row: this thread's row (32 x 16 bytes), always a readable global row; when
// zero is set its bits count as 0 (a missing row past the end of the input)
__device__ __forceinline__ void overlap_tile(const uint4 *row, bool zero, Smem &sm, v4f (&acc)[8][4]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wq = w >> 2, wr = w & 3;  // 2 x 4 waves, each 128 A rows x 64 B rows
    const int li = lane & 15, lg = lane >> 4;

#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    // window v of this thread's row is its 16-byte pieces 2v, 2v+1 (global
    // loads: a generic pointer would make them flat loads, which also hold
    // the LDS counter the fragment reads wait on)
    auto piece = [&](int i) {
        const uint4 v = row[i];
        return zero ? make_uint4(0, 0, 0, 0) : v;
    };
    constexpr int kWins = 4096 / WIN;
    unpack_half(piece(0), sm.uk[0] + tid * UST);
    unpack_half(piece(1), sm.uk[0] + tid * UST + 64);
    __syncthreads();
    for (int win = 0; win < kWins; win++) {  // window win is in buffer win & 1
        const int h = win & 1;
        const bool more = win + 1 < kWins;
        // the next window: in flight during this one's matrix steps
        const uint4 n0 = piece(more ? 2 * win + 2 : 0), n1 = piece(more ? 2 * win + 3 : 1);
        const uint8_t *ua = sm.uk[h];
        const uint8_t *ubp = sm.uk[h] + MA * UST;
        uint8_t *nx = sm.uk[h ^ 1] + tid * UST;  // last read before the previous barrier
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
                for (int b = 0; b < 4; b++) {
                    const v8i av = {af[a][0], af[a][1], af[a][2], af[a][3], 0, 0, 0, 0};
                    const v8i bv = {bf[b][0], bf[b][1], bf[b][2], bf[b][3], 0, 0, 0, 0};
                    // formats 4 = e2m1 for both operands; scales 128 = 2^1
                    acc[a][b] =
                        __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc[a][b], 4, 4, 0, 128, 0, 128);
                }
            // one step's fragments live at a time (register budget of two waves per SIMD)
            __builtin_amdgcn_sched_barrier(0);
            // half ks of the next window, into the other buffer
            if (more) unpack_half(ks == 0 ? n0 : n1, nx + ks * 64);
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
    }
}

}  // namespace mt
}  // namespace qd

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
// 0..255, then B rows).  The K dimension is streamed in windows of 512 bits:
// each thread copies its row's window, still packed, into LDS (rows 72 bytes
// apart), three windows deep: window w + 2 is loaded into registers at the
// start of window w and stored at its end, before the one barrier per window,
// so the reads of window w + 1 never wait for a barrier.  Every wave
// multiplies its 128 x 64 eighth as 8 x 4 tiles per 128-bit matrix step.  In
// step s of a window, lane l reads one 32-bit word of a row, word 4s + l/16
// of row l % 16 of each fragment, and expands it in registers to the 32
// elements the instruction takes from it (k = 32*(l/16) .. +31): element
// 8j + i holds bit 4i + j, so four shift-and-mask operations make the 16
// bytes.  With rows 18 words apart the 64 lanes of such a read fall on
// distinct banks in each half.  The words of the next step are read while
// the current one runs.  Lane l receives C rows 4*(l/16) .. +3 of column
// l % 16.
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
constexpr int WIN = 512;       // bits per window (four 128-bit matrix steps)
constexpr int RST = 72;        // packed row stride in LDS (64 bytes + 8 pad)
constexpr int NBUF = 3;        // windows held in LDS

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct Smem {
    uint8_t rw[NBUF][(MA + MB) * RST];  // packed windows
};

// 32 bits -> the 32 e2m1 elements (0 or 0.5) of one lane's operand: element
// 8j + i (nibble i of word j) holds bit 4i + j
__device__ __forceinline__ v8i expand(uint32_t w) {
    constexpr uint32_t M = 0x11111111u;
    return v8i{(int)(w & M), (int)((w >> 1) & M), (int)((w >> 2) & M), (int)((w >> 3) & M), 0, 0, 0, 0};
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

    // window v of this thread's row is its 16-byte pieces 4v .. 4v+3 (global
    // loads: a generic pointer would make them flat loads, which also hold
    // the LDS counter the fragment reads wait on)
    // Loaded as they are; a missing row is masked to zeros only when stored, so
    // nothing waits for the loads before then (and no branch skips them).
    const uint32_t keep = zero ? 0u : ~0u;
    auto piece = [&](int i) { return row[i]; };
    auto stage = [&](uint8_t *dst, uint4 p0, uint4 p1, uint4 p2, uint4 p3) {
        uint2 *d = reinterpret_cast<uint2 *>(dst + tid * RST);  // 8-byte aligned
        d[0] = make_uint2(p0.x & keep, p0.y & keep);
        d[1] = make_uint2(p0.z & keep, p0.w & keep);
        d[2] = make_uint2(p1.x & keep, p1.y & keep);
        d[3] = make_uint2(p1.z & keep, p1.w & keep);
        d[4] = make_uint2(p2.x & keep, p2.y & keep);
        d[5] = make_uint2(p2.z & keep, p2.w & keep);
        d[6] = make_uint2(p3.x & keep, p3.y & keep);
        d[7] = make_uint2(p3.z & keep, p3.w & keep);
    };
    constexpr int kWins = 4096 / WIN;
    stage(sm.rw[0], piece(0), piece(1), piece(2), piece(3));
    stage(sm.rw[1], piece(4), piece(5), piece(6), piece(7));
    __syncthreads();
    // fragment f < 8: A rows wq*128 + 16f + li; f >= 8: B rows wr*64 + 16(f-8) + li
    int roff[12];
#pragma unroll
    for (int f = 0; f < 12; f++)
        roff[f] = (f < 8 ? wq * 128 + f * 16 + li : MA + wr * 64 + (f - 8) * 16 + li) * RST + lg * 4;
    uint32_t r[2][12];  // the words of this step and of the next
#pragma unroll
    for (int f = 0; f < 12; f++) r[0][f] = *reinterpret_cast<const uint32_t *>(sm.rw[0] + roff[f]);
    auto step = [&](const uint32_t (&x)[12]) {
        v8i bv[4];
#pragma unroll
        for (int b = 0; b < 4; b++) bv[b] = expand(x[8 + b]);
#pragma unroll
        for (int a = 0; a < 8; a++) {
            const v8i av = expand(x[a]);
#pragma unroll
            for (int b = 0; b < 4; b++)
                // formats 4 = e2m1 for both operands; scales 128 = 2^1
                acc[a][b] =
                    __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv[b], acc[a][b], 4, 4, 0, 128, 0, 128);
        }
    };
    // Every window runs the same code: the last two load pieces of window 0
    // and 1 again (in bounds) and store them into buffers no later window of
    // this tile reads, and the last reads words it does not use, so the
    // compiler keeps one loop instead of peeling its end.
    int cur = 0;  // buffer of window win; window win + 1 is in the next, win + 2 goes to the one after
    for (int win = 0; win < kWins; win++) {
        const int nxt = cur == NBUF - 1 ? 0 : cur + 1, stg = nxt == NBUF - 1 ? 0 : nxt + 1;
        const uint8_t *buf = sm.rw[cur];
        const int nb = (4 * win + 8) & 31;
        const uint4 n0 = piece(nb), n1 = piece(nb + 1), n2 = piece(nb + 2), n3 = piece(nb + 3);
#pragma unroll
        for (int s = 0; s < 4; s++) {
            // the next step's words: from this window, or the first of the next
            // window (published by the previous window's barrier)
            const uint8_t *src = s < 3 ? buf + (s + 1) * 16 : sm.rw[nxt];
#pragma unroll
            for (int f = 0; f < 12; f++) r[(s + 1) & 1][f] = *reinterpret_cast<const uint32_t *>(src + roff[f]);
            // one step at a time: the next step's reads go out before this step's work
            __builtin_amdgcn_sched_barrier(0);
            step(r[s & 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // the buffer of window win - 1: every wave finished reading it before
        // the previous barrier
        __builtin_amdgcn_sched_barrier(0);
        stage(sm.rw[stg], n0, n1, n2, n3);
        __syncthreads();
        cur = nxt;
    }
}

}  // namespace mt
}  // namespace qd

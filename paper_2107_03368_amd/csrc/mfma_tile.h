// Overlap counts on the matrix cores: for a tile of 256 "A" rows (queries)
// and 256 "B" rows (database rows or bit summaries) of 4096 bits each,
// C[i][j] = popcount(A_i AND B_j), the term every weighted distance and every
// node bound of Eq. 1 is built from.  Over the 4096 bit positions this is a
// dense {0,1} matrix product.  It runs as the FP4 (e2m1) matrix instruction
// v_mfma_scale_f32_16x16x128_f8f6f4: every bit becomes one 4-bit element,
// zero or a power of two whose value on the A side is the reciprocal of its
// value on the B side, so every product is 0 or 1 and the fp32 accumulator
// holds the exact count (at most 4096 < 2^24).  The order in which bits
// become elements only has to be the same for both operands, since the sum
// over K does not depend on it.
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
// 8j + i holds bit 4i + j, so a few shift-and-mask operations make the 16
// bytes (expand_a, expand_b; in the tile two words at a time, their shifts
// as 64-bit shifts of the pair).  With rows 18 words apart the 64 lanes of such a read fall on
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

// 32 bits -> the 32 e2m1 elements of one lane's operand: element 8j + i
// (nibble i of word j) comes from bit 4i + j.  The A side keeps bits 0..2 of
// each nibble where they are (values 0.5, 1 and 2); the B side gives the same
// bits the reciprocal values (2, 1 and 0.5).  Bit 3, the e2m1 sign bit, moves
// to bit 1 (value 1) on both sides, so the product of two set bits is exactly
// 1, three of the A side's four words need no shift, and the B side's last
// two words come from one shift right by 2.
__device__ __forceinline__ v8i expand_a(uint32_t w) {
    constexpr uint32_t M = 0x11111111u;
    return v8i{(int)(w & M), (int)(w & (M << 1)), (int)(w & (M << 2)), (int)((w >> 2) & (M << 1)), 0, 0, 0, 0};
}
__device__ __forceinline__ v8i expand_b(uint32_t w) {
    constexpr uint32_t M = 0x11111111u;
    const uint32_t r2 = w >> 2;
    return v8i{(int)((w << 2) & (M << 2)), (int)(w & (M << 1)), (int)(r2 & M), (int)(r2 & (M << 1)), 0, 0, 0, 0};
}

// The same expansions for two words at once: their shifts run as one 64-bit
// shift of the pair (one instruction that costs about 1.3 times a 32-bit
// shift; the bits that cross between the two words fall outside the masks).
// Written as instructions because the compiler splits a 64-bit shift whose
// halves are masked back into two 32-bit shifts.
__device__ __forceinline__ uint64_t shr64_2(uint64_t w) {
    uint64_t r;
    asm("v_lshrrev_b64 %0, 2, %1" : "=v"(r) : "v"(w));
    return r;
}
__device__ __forceinline__ uint64_t shl64_2(uint64_t w) {
    uint64_t r;
    asm("v_lshlrev_b64 %0, 2, %1" : "=v"(r) : "v"(w));
    return r;
}
__device__ __forceinline__ void expand_a2(uint32_t w0, uint32_t w1, v8i &o0, v8i &o1) {
    constexpr uint32_t M = 0x11111111u;
    const uint64_t r2 = shr64_2(((uint64_t)w1 << 32) | w0);
    o0 = v8i{(int)(w0 & M), (int)(w0 & (M << 1)), (int)(w0 & (M << 2)), (int)((uint32_t)r2 & (M << 1)), 0, 0, 0, 0};
    o1 = v8i{(int)(w1 & M), (int)(w1 & (M << 1)), (int)(w1 & (M << 2)), (int)((uint32_t)(r2 >> 32) & (M << 1)),
             0, 0, 0, 0};
}
__device__ __forceinline__ void expand_b2(uint32_t w0, uint32_t w1, v8i &o0, v8i &o1) {
    constexpr uint32_t M = 0x11111111u;
    const uint64_t w = ((uint64_t)w1 << 32) | w0;
    const uint64_t l2 = shl64_2(w), r2 = shr64_2(w);
    const uint32_t r2lo = (uint32_t)r2, r2hi = (uint32_t)(r2 >> 32);
    o0 = v8i{(int)((uint32_t)l2 & (M << 2)), (int)(w0 & (M << 1)), (int)(r2lo & M), (int)(r2lo & (M << 1)), 0, 0,
             0, 0};
    o1 = v8i{(int)((uint32_t)(l2 >> 32) & (M << 2)), (int)(w1 & (M << 1)), (int)(r2hi & M), (int)(r2hi & (M << 1)),
             0, 0, 0, 0};
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

// Tiles in a row, streamed: while a tile's last two windows run, the next
// tile's first two windows are loaded and stored, and the words of its first
// step are read, so a tile that follows another starts without waiting for
// its loads.  `Stream` carries that state from one tile to the next.
struct Stream {
    int cur;           // buffer holding window 0 of the next tile to run
    uint32_t r0[12];   // the words of that tile's first step
};

// Rows: this thread's row (32 x 16 bytes), always a readable global row; when
// the zero flag is set its bits count as 0 (a missing row past the end of
// the input), read from a row of zeros, so the loaded words need no mask.  A
// global-memory pointer: a generic one would make the window loads flat
// loads, which also hold the LDS counter the fragment reads wait on (the row
// of zeros is a global variable, so a choice between it and a row stays
// global).
static __device__ uint4 kZeroRow[32];  // never written: zero-initialised

__device__ __forceinline__ const uint4 *row_or_zero(const uint4 *row, bool zero) { return zero ? kZeroRow : row; }

// Stage the first two windows of a stream's first tile.
__device__ __forceinline__ void stream_begin(const uint4 *row, bool zero, Smem &sm, Stream &st) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wq = w >> 2, wr = w & 3, li = lane & 15, lg = lane >> 4;
    const uint4 *src = row_or_zero(row, zero);
#pragma unroll
    for (int v = 0; v < 2; v++) {
        uint2 *d = reinterpret_cast<uint2 *>(sm.rw[v] + tid * RST);
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const uint4 p = src[4 * v + c];
            d[2 * c] = make_uint2(p.x, p.y);
            d[2 * c + 1] = make_uint2(p.z, p.w);
        }
    }
    __syncthreads();
    st.cur = 0;
#pragma unroll
    for (int f = 0; f < 12; f++)
        st.r0[f] = *reinterpret_cast<const uint32_t *>(
            sm.rw[0] + (f < 8 ? wq * 128 + f * 16 + li : MA + wr * 64 + (f - 8) * 16 + li) * RST + lg * 4);
}

// Multiply the stream's current tile (rows `row`) while staging the first two
// windows of the next one (rows `next`, read when windows 6 and 7 load them,
// so the hook may still set them; the current rows again after the last
// tile: in bounds, never used).  idle (the same in a whole wave): the wave
// stages its rows as always but multiplies nothing, its accumulators stay
// zero (a wave whose A rows hold no listed query).  hook(win) runs after window win's barrier,
// win = 0..7, for the kernel's own work on the next tile (such as a chain of
// dependent metadata loads, one link per window, which then never stalls a
// wave: a whole window passes between a load and its use).
template <class Hook>
__device__ __forceinline__ void stream_tile(const uint4 *row, bool zero, const uint4 *const &next,
                                            const bool &next_zero, Smem &sm, Stream &st, v4f (&acc)[8][4],
                                            Hook &&hook, bool idle = false) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wq = w >> 2, wr = w & 3;  // 2 x 4 waves, each 128 A rows x 64 B rows
    const int li = lane & 15, lg = lane >> 4;

#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    // window v of a row is its 16-byte pieces 4v .. 4v+3, loaded as they
    // are (a missing row from the row of zeros) and stored unchanged, so
    // nothing waits for the loads before then (and no branch skips them).
    const uint4 *const own_src = row_or_zero(row, zero);
    auto stage = [&](uint8_t *dst, uint4 p0, uint4 p1, uint4 p2, uint4 p3) {
        uint2 *d = reinterpret_cast<uint2 *>(dst + tid * RST);  // 8-byte aligned
        d[0] = make_uint2(p0.x, p0.y);
        d[1] = make_uint2(p0.z, p0.w);
        d[2] = make_uint2(p1.x, p1.y);
        d[3] = make_uint2(p1.z, p1.w);
        d[4] = make_uint2(p2.x, p2.y);
        d[5] = make_uint2(p2.z, p2.w);
        d[6] = make_uint2(p3.x, p3.y);
        d[7] = make_uint2(p3.z, p3.w);
    };
    constexpr int kWins = 4096 / WIN;
    // fragment f < 8: A rows wq*128 + 16f + li; f >= 8: B rows wr*64 + 16(f-8) + li
    int roff[12];
#pragma unroll
    for (int f = 0; f < 12; f++)
        roff[f] = (f < 8 ? wq * 128 + f * 16 + li : MA + wr * 64 + (f - 8) * 16 + li) * RST + lg * 4;
    uint32_t r[2][12];  // the words of this step and of the next
#pragma unroll
    for (int f = 0; f < 12; f++) r[0][f] = st.r0[f];
    auto step = [&](const uint32_t (&x)[12]) {
        v8i bv[4], avs[8];
        expand_b2(x[8], x[9], bv[0], bv[1]);
        expand_b2(x[10], x[11], bv[2], bv[3]);
#pragma unroll
        for (int a = 0; a < 8; a += 2) expand_a2(x[a], x[a + 1], avs[a], avs[a + 1]);
#pragma unroll
        for (int a = 0; a < 8; a++) {
            const v8i av = avs[a];
#pragma unroll
            for (int b = 0; b < 4; b++)
                // formats 4 = e2m1 for both operands; scales 127 = 2^0
                acc[a][b] =
                    __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv[b], acc[a][b], 4, 4, 0, 127, 0, 127);
        }
    };
    // Every window runs the same code, so the compiler keeps one loop instead
    // of peeling its end (a peeled end spilled registers in the kernels).
    int cur = st.cur;  // buffer of window win; window win + 1 is in the next, win + 2 goes to the one after
    for (int win = 0; win < kWins; win++) {
        const int nxt = cur == NBUF - 1 ? 0 : cur + 1, stg = nxt == NBUF - 1 ? 0 : nxt + 1;
        const uint8_t *buf = sm.rw[cur];
        // window win + 2 of this tile, or window win - 6 of the next
        const bool own = win + 2 < kWins;
        const uint4 *src = own ? own_src : row_or_zero(next, next_zero);
        const int nb = (4 * win + 8) & 31;
        const uint4 n0 = src[nb], n1 = src[nb + 1], n2 = src[nb + 2], n3 = src[nb + 3];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            // the next step's words: from this window, or the first of the next
            // window (published by the previous window's barrier)
            const uint8_t *from = s < 3 ? buf + (s + 1) * 16 : sm.rw[nxt];
#pragma unroll
            for (int f = 0; f < 12; f++) r[(s + 1) & 1][f] = *reinterpret_cast<const uint32_t *>(from + roff[f]);
            // one step at a time: the next step's reads go out before this step's work
            __builtin_amdgcn_sched_barrier(0);
            if (!idle) step(r[s & 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // the buffer of window win - 1: every wave finished reading it before
        // the previous barrier
        stage(sm.rw[stg], n0, n1, n2, n3);
        __syncthreads();
        hook(win);
        cur = nxt;
    }
    st.cur = cur;
#pragma unroll
    for (int f = 0; f < 12; f++) st.r0[f] = r[0][f];
}

// One tile on its own.
__device__ __forceinline__ void overlap_tile(const uint4 *row, bool zero, Smem &sm, v4f (&acc)[8][4]) {
    Stream st;
    stream_begin(row, zero, sm, st);
    stream_tile(row, zero, row, zero, sm, st, acc, [](int) {});
}

}  // namespace mt
}  // namespace qd

// Batched Dissimilarity Tree search on the matrix cores (QD_ORDER_BLOCKED).
//
// The per-query traversal (tree_knn.hip) expands nodes one query at a time on
// the vector ALUs.  This order searches a whole batch of queries at once over
// the tree's leaf order cut into blocks of 256 consecutive rows.  Block b
// holds leaf-order rows 256b .. 256b+255 and carries the sum (OR) image of
// those rows, so every row t in it has K(q, t) >= A_lb(q, b) * wB with
// A_lb = |q| - popcount(q AND OR_b): the node bound of Section 4.2 applied to
// the block's rows.  Leaf order keeps each subtree's rows together, so a
// block's image is about as tight as the image of a subtree of that size.
//
//  1. Bounds: A_lb for every (query, block) pair, on the matrix cores (the
//     shared overlap tile, with the block images as B rows).
//  2. Plan, per query: sorting the blocks by (A_lb, b) defines the rounds.
//     Round 1 takes the first m1 blocks (default 16); round r >= 2 extends
//     the covered prefix to about T2 * g^(r-2) blocks (default g = 4), rounded
//     down to whole bound levels (at least one more level), and the last round
//     takes everything left.
//  3. Round 1 (vector ALUs, one wave per query): the exact top k over the
//     rows of those blocks, which gives the first k-th key.
//  4. Rounds r >= 2 (matrix cores): block b takes part for query q when its
//     (A_lb, b) lies in q's range for the round and A_lb * wB <= q's k-th
//     key.  Every block lists its queries in query order; each tile of 256
//     listed queries x the block's 256 rows is one overlap tile, and every row
//     with K <= the query's k-th key is appended to the query's candidate
//     buffer.  Each query then merges its candidates into its top k.  A query
//     stops when no remaining block can hold a key <= its k-th key.
//     A query whose candidate buffer overflows repeats the round with the
//     k-th key of the candidates it stored.
//  5. Results; a query whose key cannot tighten that way (more than a buffer
//     of rows tie at its k-th key), or that still runs after the last pass,
//     is searched again by the per-query depth-first traversal.
//
// Driving the rounds: a direct call checks on the host after each pass
// whether any query still runs.  A captured plan runs a fixed number of
// passes instead; every kernel reads its work (running queries, tile and
// pair counts, the batch size) from device memory, so a pass with nothing
// to do only costs its launches, and nothing waits for the host.
//
// Exactness: a row with K <= the final k-th key lies in a block whose bound
// is at most that key, hence at most the query's k-th key in every round (it
// only decreases), so the block is evaluated in the round that covers its
// (A_lb, b) and the row is appended.  The top k of the appended rows under
// (K, row) are therefore the sequential-search result.
#include <algorithm>
#include <vector>

#include "mfma_tile.h"
#include "qd_device.h"
#include "qd_internal.h"
#include "qd_launch.h"
#include "qd_tree.h"

namespace qd {

int popcount_rows_launch(const uint64_t *d_db, uint64_t n, uint16_t *d_pop, hipStream_t s);

namespace {

constexpr uint32_t kBlk = mt::MB;          // rows per block
constexpr uint32_t kM1 = 64;               // most blocks in round 1 (default 16)
constexpr int kRounds = 24;                // rounds 1 .. kRounds; the last takes every remaining block
constexpr int kMaxPasses = 64;             // matrix-core passes (rounds and repeats) per batch
// Passes of a batch that runs without the host (captured graphs).  The
// searches measured here finish in 5 to 6 passes (rounds plus overflow
// repeats); a query still running after them takes the exact fallback.
constexpr int kGraphPasses = 10;
constexpr uint32_t kCap = 8128;            // candidate slots per query per round (kCap + k <= 8192)
constexpr int kGroup = 8;                  // blocks per wave when building the lists (more waves hide the loads' latency)
static_assert(32 % kGroup == 0, "a wave's blocks share one word of done bits");
constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr uint32_t kLevels = QD_BITS + 1;  // A_lb in 0 .. 4096
constexpr uint32_t kMaxBatch = 16384;      // queries per batch (list entries are 16-bit)
// A block list (or the rest of one past its full 256-query tiles) shorter
// than this is evaluated on the vector ALUs, one wave per (query, block)
// pair, instead of in a matrix-core tile that costs the same for 1 or 256
// listed queries (measured at 10M rows x 8,192 queries: 12 and 16 fastest,
// 24 0.4%, 32 0.9% and 48 2% slower).
constexpr uint32_t kShortList = 16;

// Position of block b of bound level L in the per-query block order; a round
// covers the keys in (lo, hi].  Key 0 is below every block.
__device__ __forceinline__ u64 range_key(uint32_t level, uint32_t b) { return ((u64)(level + 1) << 32) | b; }
// Largest key of a block whose bound A_lb * wB does not exceed K.
__device__ __forceinline__ u64 cap_key(uint32_t K, uint32_t wb) {
    return K == kInf ? ~0ull : range_key(K / wb, kInf);
}

__device__ __forceinline__ uint32_t weight_a(uint32_t pq) { return pq > 1 ? pq : 1; }

// The keys a query running round r may evaluate early, to fill a tile of
// round r: those of round r + 1, (c[r], min(c[r+1], cap)]; none after the
// last round.  Stored as (lo, hi) with hi <= lo meaning none.
__device__ __forceinline__ void set_fill_range(u64 *fr, const u64 *c, uint32_t r, u64 cap) {
    fr[0] = r < (uint32_t)kRounds ? c[r] : 0;
    fr[1] = r < (uint32_t)kRounds ? (c[r + 1] < cap ? c[r + 1] : cap) : 0;
}
__device__ __forceinline__ uint32_t weight_b(uint32_t pq) { return (QD_BITS - pq) > 1 ? QD_BITS - pq : 1; }

// OR image of each block of 256 leaf-order rows; one 64-thread block per
// image, thread w owns word w.  With bpop, also the smallest and largest
// popcount of the block's rows.
__global__ __launch_bounds__(64) void block_image_kernel(const uint64_t *__restrict__ sorted, uint64_t n,
                                                         uint64_t *__restrict__ img, const uint16_t *__restrict__ pop,
                                                         uint16_t *__restrict__ bpop) {
    const uint64_t b = blockIdx.x;
    const int w = threadIdx.x;
    const uint64_t r0 = b * kBlk, r1 = r0 + kBlk < n ? r0 + kBlk : n;
    uint64_t acc = 0;
    for (uint64_t r = r0; r < r1; r++) acc |= sorted[r * QD_WORDS + w];
    img[b * QD_WORDS + w] = acc;
    if (bpop) {
        uint32_t mn = 0xFFFFu, mx = 0;
        for (uint64_t r = r0 + w; r < r1; r += 64) {
            const uint32_t v = pop[r];
            mn = v < mn ? v : mn;
            mx = v > mx ? v : mx;
        }
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) {
            const uint32_t a = (uint32_t)__shfl_xor((int)mn, sh), c = (uint32_t)__shfl_xor((int)mx, sh);
            mn = a < mn ? a : mn;
            mx = c > mx ? c : mx;
        }
        if (w == 0) {
            bpop[2 * b] = (uint16_t)mn;
            bpop[2 * b + 1] = (uint16_t)mx;
        }
    }
}

// Bound level L of every (query, block) pair in a tile of 256 queries x 256
// blocks: every row of the block has key >= L * wB.  With the sum image
// alone L = A_lb = |q| - ov (ov = popcount(q AND image)); with the block's
// popcount range [pmin, pmax], A_lb = |q| - min(ov, pmax), B_lb =
// max(pmin - ov, 0) and L = min(A_lb + floor(B_lb * wA / wB), 4096).  Stored
// query-major (lbq[q][b], for the per-query plan) and block-major
// (lbb[b][q], for the per-block lists).  Queries q >= nqb get level 0xFFFF
// in lbb.
__global__ __launch_bounds__(mt::kThreads) void bound_kernel(const uint4 *__restrict__ q, uint32_t nqb, uint32_t nqp,
                                                             const uint4 *__restrict__ img, uint64_t nblk,
                                                             const uint16_t *__restrict__ bpop,
                                                             const uint16_t *__restrict__ qpop, uint32_t n_qtiles,
                                                             uint16_t *__restrict__ lbq, uint16_t *__restrict__ lbb,
                                                             const uint32_t *__restrict__ nq_dev) {
    __shared__ mt::Smem sm;
    __shared__ uint32_t s_pq[mt::MA], s_dm[mt::MA], s_pmin[mt::MB], s_pmax[mt::MB];
    if (nq_dev) nqb = min(nqb, *nq_dev);  // the batch's size on the device (captured graphs)
    const uint64_t n_tiles = (uint64_t)n_qtiles * ((nblk + mt::MB - 1) / mt::MB);
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint32_t q0 = (uint32_t)(tile % n_qtiles) * mt::MA;
        if (q0 >= nqb) continue;  // whole workgroup: no query of this tile is in the batch
        const uint64_t b0 = (tile / n_qtiles) * mt::MB;
        const int own = mt::own_row();
        const uint4 *row;
        bool ok;
        if (own < mt::MA) {
            ok = q0 + own < nqb;
            row = ok ? q + (uint64_t)(q0 + own) * 32 : q;
            const uint32_t pq = ok ? qpop[q0 + own] : 0;
            s_pq[own] = pq;
            // floor(x / wB) for every x < 2^25 as (x * m) >> (25 + l), with
            // l = ceil(log2 wB) and m = ceil(2^(25 + l) / wB) < 2^26
            // (division by an invariant integer; checked for every wB and
            // at both sides of every multiple of it); m | l << 26
            const uint32_t wb = weight_b(pq), l = 32u - (uint32_t)__builtin_clz(wb | 1u) - ((wb & (wb - 1)) == 0);
            s_dm[own] = (uint32_t)((((uint64_t)1 << (25 + l)) + wb - 1) / wb) | (l << 26);
        } else {
            ok = b0 + (own - mt::MA) < nblk;
            row = ok ? img + (b0 + (own - mt::MA)) * 32 : img;
            // without ranges: pmin = 0 and pmax = 4096 leave the plain bound
            s_pmin[own - mt::MA] = ok && bpop ? bpop[2 * (b0 + (own - mt::MA))] : 0;
            s_pmax[own - mt::MA] = ok && bpop ? bpop[2 * (b0 + (own - mt::MA)) + 1] : QD_BITS;
        }
        mt::v4f acc[8][4];
        mt::overlap_tile(row, !ok, sm, acc);  // its barriers also publish s_pq, s_pmin, s_pmax
#pragma unroll
        for (int a = 0; a < 8; a++) {
            // one group of queries at a time, so their metadata loads stay next to their use
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int bb = 0; bb < 4; bb++) {
                const uint64_t blk = b0 + mt::acc_brow(bb);
                if (blk >= nblk) continue;
                const uint32_t pmin = s_pmin[mt::acc_brow(bb)], pmax = s_pmax[mt::acc_brow(bb)];
                const uint32_t qa = q0 + mt::acc_arow(a, 0);  // this lane's 4 consecutive queries
                u64 packed = 0;
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const uint32_t qi = qa + r;
                    uint32_t v = 0xFFFFu;
                    if (qi < nqb) {
                        const uint32_t pq = s_pq[qi - q0], dm = s_dm[qi - q0], ov = mt::count(acc[a][bb][r]);
                        const uint32_t al = pq - (ov < pmax ? ov : pmax);
                        const uint32_t bl = pmin > ov ? pmin - ov : 0;
                        // floor(bl * wA / wB); bl * wA <= 2^24
                        const uint32_t x = __umul24(bl, weight_a(pq));
                        v = al + (uint32_t)(((uint64_t)x * (dm & 0x3FFFFFFu)) >> (25 + (dm >> 26)));
                        v = v < QD_BITS ? v : QD_BITS;
                        lbq[(uint64_t)qi * nblk + blk] = (uint16_t)v;
                    }
                    packed |= (u64)v << (16 * r);
                }
                *reinterpret_cast<u64 *>(lbb + blk * nqp + qa) = packed;
            }
        }
        __syncthreads();  // the next tile rewrites s_pq
    }
}

// Per query: histogram of A_lb over the blocks, round 1's blocks (the first
// min(m1, nblk) in (A_lb, b) order, listed in block order) and the range end
// of every round.  One 256-thread block per query.
__global__ __launch_bounds__(256) void plan_kernel(const uint16_t *__restrict__ lbq, uint64_t nblk, uint32_t m1,
                                                   uint64_t t2, uint32_t growth, u64 *__restrict__ cuts,
                                                   uint32_t *__restrict__ r1list, const uint32_t *__restrict__ nq_dev) {
    __shared__ uint32_t cum[kLevels];
    __shared__ uint32_t part[256];
    __shared__ uint32_t s_bcut;
    const uint32_t qi = blockIdx.x, tid = threadIdx.x;
    const uint32_t nqb = nq_dev ? min(gridDim.x, *nq_dev) : gridDim.x;
    if (qi >= nqb) return;  // whole block
    // t2 = 0: round 2 covers enough blocks that a block's list holds ~128
    // queries on average
    if (t2 == 0) t2 = (128 * nblk + nqb - 1) / nqb;
    if (t2 < 2 * (uint64_t)m1) t2 = 2 * (uint64_t)m1;
    const uint16_t *row = lbq + (uint64_t)qi * nblk;
    for (uint32_t i = tid; i < kLevels; i += 256) cum[i] = 0;
    if (tid == 0) s_bcut = kInf;
    __syncthreads();
    // eight loads in flight per thread, then their counts
    for (uint64_t b0 = tid; b0 < nblk; b0 += 256 * 8) {
        uint32_t v[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint64_t b = b0 + 256 * i;
            v[i] = b < nblk ? row[b] : kLevels;
        }
#pragma unroll
        for (int i = 0; i < 8; i++)
            if (v[i] < kLevels) atomicAdd(&cum[v[i]], 1u);
    }
    __syncthreads();
    // inclusive prefix over the levels; thread t owns levels [t*per, t*per+per)
    constexpr uint32_t per = (kLevels + 255) / 256;
    uint32_t s = 0;
    for (uint32_t i = 0; i < per; i++) {
        const uint32_t L = tid * per + i;
        if (L < kLevels) s += cum[L];
    }
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int t = 0; t < 256; t++) {
            const uint32_t v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    {
        uint32_t run = part[tid];
        for (uint32_t i = 0; i < per; i++) {
            const uint32_t L = tid * per + i;
            if (L < kLevels) {
                run += cum[L];
                cum[L] = run;
            }
        }
    }
    __syncthreads();
    // round 1: all blocks below level L1 and the first r1 blocks of level L1
    const uint32_t T1 = (uint32_t)(nblk < m1 ? nblk : m1);
    uint32_t lo = 0, hi = kLevels - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if (cum[mid] >= T1)
            hi = mid;
        else
            lo = mid + 1;
    }
    const uint32_t L1 = lo;
    const uint32_t before = L1 ? cum[L1 - 1] : 0;
    const uint32_t r1 = T1 - before, at_level = cum[L1] - before;
    // Round 1's blocks, listed in block order: the 4 waves take a quarter of
    // the blocks each; they first count the blocks below level L1 and at L1
    // in their quarter, so each knows how many of each come before it, then
    // list their quarter's blocks and find the last block of level L1 taken.
    // The levels of 8 steps are loaded at once, so their latencies overlap.
    __shared__ uint32_t s_lt[4], s_eq[4];
    const int lane = (int)(tid & 63), wv = (int)(tid >> 6);
    const uint64_t quarter = (nblk + 3) / 4;
    const uint64_t w0 = quarter * wv, w1 = w0 + quarter < nblk ? w0 + quarter : nblk;
    {
        uint32_t lt = 0, eq = 0;
        for (uint64_t base = w0; base < w1; base += 512) {
            uint32_t vs[8];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint64_t b = base + 64 * i + lane;
                vs[i] = b < w1 ? row[b] : 0xFFFFu;
            }
#pragma unroll
            for (int i = 0; i < 8; i++) {
                lt += (uint32_t)__popcll(ballot(vs[i] < L1));
                eq += (uint32_t)__popcll(ballot(vs[i] == L1));
            }
        }
        if (lane == 0) {
            s_lt[wv] = lt;
            s_eq[wv] = eq;
        }
    }
    __syncthreads();
    {
        uint32_t lt_before = 0, eq_seen = 0;
        for (int v = 0; v < wv; v++) {
            lt_before += s_lt[v];
            eq_seen += s_eq[v];
        }
        uint32_t pos = lt_before + (eq_seen < r1 ? eq_seen : r1);
        for (uint64_t base = w0; base < w1; base += 512) {
            uint32_t vs[8];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint64_t b = base + 64 * i + lane;
                vs[i] = b < w1 ? row[b] : 0xFFFFu;
            }
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint64_t b = base + 64 * i + lane;
                const uint32_t v = vs[i];
                const bool eq = v == L1;
                const u64 meq = ballot(eq);
                const uint32_t rank = eq_seen + lanes_below(meq);
                const bool in = v < L1 || (eq && rank < r1);
                if (eq && rank + 1 == r1 && r1 < at_level) s_bcut = (uint32_t)b;
                const u64 min_ = ballot(in);
                if (in) r1list[(uint64_t)qi * kM1 + pos + lanes_below(min_)] = (uint32_t)b;
                pos += (uint32_t)__popcll(min_);
                eq_seen += (uint32_t)__popcll(meq);
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        u64 *c = cuts + (uint64_t)qi * (kRounds + 1);
        c[0] = 0;
        c[1] = range_key(L1, s_bcut);
        uint32_t Lp = L1;
        bool whole = s_bcut == kInf;
        uint64_t T = t2;
        for (int r = 2; r <= kRounds; r++) {
            uint32_t L = kLevels - 1;
            if (r < kRounds) {
                // largest level whose cumulative count is <= T (or none)
                int best = -1;
                uint32_t a = 0, b = kLevels;  // search in [a, b)
                while (a < b) {
                    const uint32_t mid = (a + b) / 2;
                    if ((uint64_t)cum[mid] <= T) {
                        best = (int)mid;
                        a = mid + 1;
                    } else {
                        b = mid;
                    }
                }
                const uint32_t need = Lp + (whole ? 1u : 0u);
                L = best >= (int)need ? (uint32_t)best : need;
                if (L > kLevels - 1) L = kLevels - 1;
            }
            c[r] = range_key(L, kInf);
            Lp = L;
            whole = true;
            T = T < (1ull << 40) ? growth * T : T;
        }
    }
}

// Round 1 on the vector ALUs: one wave per query keeps the exact top k over
// the rows of its round-1 blocks (8 lanes per row, 8 rows per step), then
// sets the k-th key and the range of round 2.
__global__ __launch_bounds__(256) void round1_kernel(const uint4 *__restrict__ q, uint32_t nqb, uint32_t k,
                                                     const uint4 *__restrict__ sorted,
                                                     const uint16_t *__restrict__ tpop,
                                                     const uint32_t *__restrict__ perm, uint64_t n, uint64_t nblk,
                                                     const uint32_t *__restrict__ r1list, uint32_t n1,
                                                     const u64 *__restrict__ cuts, const uint16_t *__restrict__ qpop,
                                                     u64 *__restrict__ top, uint32_t *__restrict__ ntop,
                                                     uint32_t *__restrict__ thrk, u64 *__restrict__ rec,
                                                     u64 *__restrict__ frange, uint32_t *__restrict__ qround,
                                                     uint32_t *__restrict__ counters, uint32_t *__restrict__ qst,
                                                     const uint32_t *__restrict__ nq_dev) {
    const int lane = lane_id();
    const uint32_t qi = readfirst(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (qi >= nqb) return;
    if (nq_dev && qi >= *nq_dev) {  // beyond the batch on the device: never runs
        if (lane == 0) {
            rec[2 * qi] = rec[2 * qi + 1] = 0;
            ntop[qi] = 0;
        }
        return;
    }
    const int g = lane >> 3, j = lane & 7;
    uint4 qv[4];
#pragma unroll
    for (int i = 0; i < 4; i++) qv[i] = q[(uint64_t)qi * 32 + j + 8 * i];
    const uint32_t pq = readfirst(qpop[qi]);
    const uint32_t wa = weight_a(pq), wb = weight_b(pq);
    u64 list = KEY_NONE;  // lane r holds the r-th best key (K << 32 | row)
    uint32_t kworst = kInf;
    uint32_t rows = 0;
    for (uint32_t i = 0; i < n1; i++) {
        const uint32_t b = readfirst(r1list[(uint64_t)qi * kM1 + i]);
        const uint64_t r0 = (uint64_t)b * kBlk;
        const uint32_t m = readfirst((uint32_t)(n - r0 < kBlk ? n - r0 : kBlk));
        rows += m;
        for (uint32_t base = 0; base < m; base += 8) {
            const uint32_t r = base + (uint32_t)g;
            const bool valid = r < m;
            const uint64_t pos = r0 + (valid ? r : 0);
            uint4 tv[4];
#pragma unroll
            for (int i2 = 0; i2 < 4; i2++) tv[i2] = sorted[pos * 32 + j + 8 * i2];
            const uint32_t c = sum8(popc_and4(tv[0], qv[0]) + popc_and4(tv[1], qv[1]) + popc_and4(tv[2], qv[2]) +
                                    popc_and4(tv[3], qv[3]));
            const uint32_t K = (pq - c) * wb + ((uint32_t)tpop[pos] - c) * wa;
            const u64 key = valid ? ((u64)K << 32) | perm[pos] : KEY_NONE;
            const u64 lim = readlane64(list, (int)k - 1);
            u64 mk = ballot(j == 0 && key < lim);
            while (mk) {
                const int L = __builtin_ctzll(mk);
                mk &= mk - 1;
                const u64 cand = readlane64(key, L);
                if (cand < readlane64(list, (int)k - 1)) list = list_insert(list, cand, k);
            }
        }
    }
    kworst = readfirst((uint32_t)(readlane64(list, (int)k - 1) >> 32));
    if (lane < (int)k) top[(uint64_t)qi * k + lane] = list;
    const uint32_t have = (uint32_t)__popcll(ballot(list != KEY_NONE));
    if (lane == 0) {
        ntop[qi] = have;
        thrk[qi] = kworst;
        const u64 *c = cuts + (uint64_t)qi * (kRounds + 1);
        const u64 lo = c[1];
        u64 hi = c[2];
        const u64 cap = cap_key(kworst, wb);
        hi = hi < cap ? hi : cap;
        const bool active = hi > lo;
        rec[2 * qi] = lo;
        rec[2 * qi + 1] = active ? hi : 0;
        set_fill_range(frange + 2 * qi, c, 2, cap);
        qround[qi] = 2;
        if (active) atomicAdd(&counters[0], 1u);
        if (qst) {
            qst[(uint64_t)qi * 4 + 0] = n1;
            qst[(uint64_t)qi * 4 + 1] = 1;
            qst[(uint64_t)qi * 4 + 2] = (uint32_t)nblk;
            qst[(uint64_t)qi * 4 + 3] = rows;
        }
    }
}

// Bound-led start: from the root, enter at every inner node holding more than
// max_rows rows the child with the lower bound (the node bound of Section
// 4.2 with the popcount range when stored; ties: the similar child), as the
// depth-first traversal's first descent does.  One wave per query, a
// half-wave per child (its 32 image chunks).
__global__ __launch_bounds__(256) void bound_descend_kernel(const uint4 *__restrict__ q, uint32_t nqb,
                                                            const uint16_t *__restrict__ qpop,
                                                            const uint4 *__restrict__ orimg,
                                                            const int32_t *__restrict__ child,
                                                            const uint32_t *__restrict__ count,
                                                            const uint16_t *__restrict__ pmin,
                                                            const uint16_t *__restrict__ pmax, uint32_t max_rows,
                                                            uint32_t *__restrict__ node_out,
                                                            const uint32_t *__restrict__ nq_dev) {
    const int lane = lane_id();
    const uint32_t qi = readfirst(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (qi >= nqb || (nq_dev && qi >= *nq_dev)) return;
    const uint4 qn = q[(uint64_t)qi * 32 + (lane & 31)];
    const uint32_t pq = readfirst(qpop[qi]);
    const uint32_t wa = weight_a(pq), wb = weight_b(pq);
    uint32_t node = 0;
    for (;;) {
        const int32_t c0 = child[2 * (uint64_t)node];
        if (c0 < 0 || count[node] <= max_rows) break;
        const int32_t c1 = child[2 * (uint64_t)node + 1];
        const int32_t c = lane < 32 ? c0 : c1;
        const uint4 o = orimg[(uint64_t)c * 32 + (lane & 31)];
        uint32_t ov = popc_and4(qn, o);
#pragma unroll
        for (int sh = 1; sh < 32; sh <<= 1) ov += (uint32_t)__shfl_xor((int)ov, sh);
        uint32_t al = pq - ov, bl = 0;
        if (pmin) {
            const uint32_t lo = pmin[c], hi = pmax[c];
            al = pq - (ov < hi ? ov : hi);
            bl = lo > ov ? lo - ov : 0;
        }
        const uint32_t kb = al * wb + bl * wa;
        const uint32_t k0 = readlane(kb, 0), k1 = readlane(kb, 32);
        node = readfirst((uint32_t)(k1 < k0 ? c1 : c0));
    }
    if (lane == 0) node_out[qi] = node;
}

// Start at a descent's node (the model's or the bound's): round 1 takes the
// n1 consecutive blocks of the leaf order that begin with the first block of
// the node the descent reached
// (moved back so they stay inside the rows).  Those pairs are marked done, and
// round 2's range starts at the lowest key (cuts[1] = 0), so every other block
// is still covered by the bound-ordered rounds and no block is evaluated twice.
// One thread per query.
__global__ void learned_start_kernel(const uint32_t *__restrict__ node, uint32_t nqb,
                                     const uint32_t *__restrict__ begin, uint64_t nblk, uint32_t n1,
                                     uint32_t *__restrict__ r1list, u64 *__restrict__ cuts, uint32_t *__restrict__ done,
                                     uint32_t nqp, const uint32_t *__restrict__ nq_dev) {
    const uint32_t qi = blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= nqb || (nq_dev && qi >= *nq_dev)) return;
    uint64_t b0 = begin[node[qi]] / kBlk;
    if (b0 + n1 > nblk) b0 = nblk - n1;
    for (uint32_t i = 0; i < n1; i++) {
        const uint64_t b = b0 + i;
        r1list[(uint64_t)qi * kM1 + i] = (uint32_t)b;
        done[(b / 32) * nqp + qi] |= 1u << (b % 32);  // this thread owns query qi's bits
    }
    cuts[(uint64_t)qi * (kRounds + 1) + 1] = 0;
}

// The queries running this round (rec[2q + 1] > rec[2q]), in query order:
// act[0 .. *nact).  One block of 1024 threads.
__global__ __launch_bounds__(1024) void active_kernel(const u64 *__restrict__ rec, uint32_t nqb,
                                                      uint32_t *__restrict__ act, uint32_t *__restrict__ nact) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t base;
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) base = 0;
    __syncthreads();
    for (uint32_t q0 = 0; q0 < nqb; q0 += 1024) {
        const uint32_t qi = q0 + tid;
        const bool run = qi < nqb && rec[2 * qi + 1] > rec[2 * qi];
        const u64 m = ballot(run);
        if (lane == 0) wsum[w] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = base;
        for (uint32_t v = 0; v < w; v++) before += wsum[v];
        if (run) act[before + lanes_below(m)] = qi;
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
            for (uint32_t v = 0; v < 16; v++) t += wsum[v];
            base += t;
        }
        __syncthreads();
    }
    if (tid == 0) *nact = base;
}

// Per-block query lists for one round: wave w of block x handles the
// kGroup blocks starting at (4x + w) * kGroup and walks the running queries
// (act, in query order), 256 at a time: each thread of the workgroup fetches
// one query's record, fill range and done word into LDS for all four waves
// (the next 256 are fetched while these are walked).
// A query is listed for a block whose key lies in its range of this round,
// unless an earlier round already evaluated the pair (done bit).  The same
// walk collects, per block, up to 255 queries whose next round covers the
// block (fill range); the first of them fill the free query slots of the
// block's last tile and are marked done, so the next round skips them.
// Filling uses the tile the round runs anyway; such a pair is evaluated once,
// against a k-th key at least as large as the next round's, so no row is lost.
static_assert(4 * kGroup == 32, "a workgroup's blocks share one word of done bits");
__global__ __launch_bounds__(256) void list_kernel(const uint16_t *__restrict__ lbb, uint64_t nblk, uint64_t n,
                                                   uint32_t nqb, uint32_t nqp, const uint32_t *__restrict__ act,
                                                   const uint32_t *__restrict__ nact, const u64 *__restrict__ rec,
                                                   const u64 *__restrict__ frange, uint32_t *__restrict__ done,
                                                   uint16_t *__restrict__ list,
                                                   uint32_t *__restrict__ cnt, uint32_t *__restrict__ qst) {
    __shared__ uint16_t s_fill[4][kGroup][mt::MA - 1];  // per wave and block: fill candidates
    __shared__ u64 s_r[2][4][256];                       // per query: round range lo, hi; fill range lo, hi
    __shared__ uint32_t s_q[2][256], s_d[2][256];        // per query: its id, its done word
    const int lane = lane_id(), t = (int)threadIdx.x;
    uint16_t(*fillq)[mt::MA - 1] = s_fill[t >> 6];
    const uint64_t b0 = ((uint64_t)blockIdx.x * 4 + (t >> 6)) * kGroup;
    const bool have = b0 < nblk;  // the same in a whole wave; every wave takes part in the staging
    const uint32_t nb = have ? readfirst((uint32_t)(nblk - b0 < (uint64_t)kGroup ? nblk - b0 : kGroup)) : 0;
    const uint64_t dword = blockIdx.x;  // the workgroup's 32 blocks share one word of done bits
    const uint32_t dshift = (uint32_t)(b0 % 32);
    uint32_t c[kGroup], f[kGroup];
#pragma unroll
    for (int jj = 0; jj < kGroup; jj++) c[jj] = f[jj] = 0;
    const uint32_t na = readfirst(*nact);
    // when every query runs the list is the identity and is not read
    const bool all = na == nqb;
    uint32_t fq = 0, fd = 0;  // this thread's fetch for the next 256: query, done word, ranges
    u64 fr[4] = {0, 0, 0, 0};
    auto fetch = [&](uint32_t i0) {  // unconditional and in bounds (na >= 1)
        const uint32_t ia = i0 + (uint32_t)t < na ? i0 + (uint32_t)t : na - 1;
        fq = all ? ia : act[ia];
        fr[0] = rec[2 * (uint64_t)fq];
        fr[1] = rec[2 * (uint64_t)fq + 1];
        fr[2] = frange[2 * (uint64_t)fq];
        fr[3] = frange[2 * (uint64_t)fq + 1];
        fd = done[dword * nqp + fq];
    };
    if (na) fetch(0);
    int sb = 0;
    for (uint32_t i00 = 0; i00 < na; i00 += 256) {
        s_q[sb][t] = fq;
        s_d[sb][t] = fd;
#pragma unroll
        for (int x = 0; x < 4; x++) s_r[sb][x][t] = fr[x];
        // also: every wave finished reading this buffer two batches ago
        __syncthreads();
        if (i00 + 256 < na) fetch(i00 + 256);
        // two groups of 64 queries at a time: their bounds are loaded before any is used
        for (int h = 0; have && h < 2; h++) {
            uint16_t rlv[2][kGroup];
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const uint32_t qc = s_q[sb][128 * h + 64 * u + lane];
#pragma unroll
                for (int jj = 0; jj < kGroup; jj++)
                    rlv[u][jj] = lbb[(b0 + ((uint32_t)jj < nb ? jj : 0)) * nqp + qc];
            }
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int e = 128 * h + 64 * u + lane;
                const uint32_t qi = s_q[sb][e];
                const bool in = i00 + (uint32_t)e < na;
                const u64 lo = in ? s_r[sb][0][e] : 0, hi = in ? s_r[sb][1][e] : 0;
                const bool run = hi > lo;  // only a query running this round has its candidates merged
                const u64 flo = run ? s_r[sb][2][e] : 0, fhi = run ? s_r[sb][3][e] : 0;
                if (ballot(run) == 0) continue;
                const uint32_t dbits = run ? s_d[sb][e] >> dshift : 0;
                uint32_t mb = 0, mr = 0;
#pragma unroll
                for (int jj = 0; jj < kGroup; jj++) {
                    if ((uint32_t)jj < nb) {
                        const uint64_t b = b0 + jj;
                        const u64 key = range_key(rlv[u][jj], (uint32_t)b);
                        const bool d = (dbits >> jj) & 1u;
                        const bool m = key > lo && key <= hi && !d;
                        const u64 mask = ballot(m);
                        if (m) list[b * nqp + c[jj] + lanes_below(mask)] = (uint16_t)qi;
                        c[jj] += (uint32_t)__popcll(mask);
                        if (m) {
                            mb++;
                            mr += b + 1 < nblk ? (uint32_t)kBlk : (uint32_t)(n - b * kBlk);
                        }
                        if (f[jj] < mt::MA - 1) {  // fill candidates, in query order
                            const bool mf = key > flo && key <= fhi && !d;
                            const u64 fmask = ballot(mf);
                            const uint32_t at = f[jj] + lanes_below(fmask);
                            if (mf && at < mt::MA - 1) fillq[jj][at] = (uint16_t)qi;
                            const uint32_t t2 = f[jj] + (uint32_t)__popcll(fmask);
                            f[jj] = t2 < mt::MA - 1 ? t2 : mt::MA - 1;
                        }
                    }
                }
                if (qst && mb) {
                    atomicAdd(&qst[(uint64_t)qi * 4 + 0], mb);
                    atomicAdd(&qst[(uint64_t)qi * 4 + 3], mr);
                }
            }
        }
        sb ^= 1;
    }
    if (!have) return;
    // the first candidates fill the last tile's free slots
    for (uint32_t jj = 0; jj < nb; jj++) {
        const uint64_t b = b0 + jj;
        const uint32_t free_slots = c[jj] % mt::MA ? mt::MA - c[jj] % mt::MA : 0;
        const uint32_t take = f[jj] < free_slots ? f[jj] : free_slots;
        for (uint32_t i = (uint32_t)lane; i < take; i += 64) {
            const uint32_t qi = fillq[jj][i];  // written by this wave above (LDS keeps its order)
            list[b * nqp + c[jj] + i] = (uint16_t)qi;
            atomicOr(&done[dword * nqp + qi], 1u << (dshift + jj));
            if (qst) {
                atomicAdd(&qst[(uint64_t)qi * 4 + 0], 1u);
                atomicAdd(&qst[(uint64_t)qi * 4 + 3], b + 1 < nblk ? (uint32_t)kBlk : (uint32_t)(n - b * kBlk));
            }
        }
        if (lane == 0) cnt[b] = c[jj] + take;
    }
}

// A block listed for c queries: full tiles of 256 queries on the matrix
// cores, the rest of the list as one more tile if it holds at least
// kShortList queries, else as (query, block) pairs for the vector ALUs (the
// last short_pairs(c) entries of the list).
__device__ __forceinline__ uint32_t short_pairs(uint32_t c) { return c % mt::MA >= kShortList ? 0 : c % mt::MA; }
__device__ __forceinline__ uint32_t mfma_tiles(uint32_t c) { return (c - short_pairs(c) + mt::MA - 1) / mt::MA; }

// Exclusive prefixes over the blocks of the matrix-core tiles (off) and of
// the short-list pairs (voff); off[nblk], voff[nblk], total[0] and total[1]
// receive the sums.  One workgroup: each of its 16 waves takes a contiguous
// segment of the blocks, 64 consecutive blocks at a time (one per lane, so
// the loads and stores are coalesced), sums it, and after one exchange of the
// segment sums writes the prefixes with a scan across its lanes.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)v, d);
        v += lane >= d ? t : 0u;
    }
    return v;
}

__global__ __launch_bounds__(1024) void tile_scan_kernel(const uint32_t *__restrict__ cnt, uint64_t nblk,
                                                         uint32_t *__restrict__ off, uint32_t *__restrict__ voff,
                                                         uint32_t *__restrict__ total) {
    constexpr int kW = 16;  // waves
    __shared__ uint32_t wsum[kW], wvsum[kW];
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const uint64_t seg = ((nblk + kW - 1) / kW + 63) / 64 * 64;  // blocks per wave, whole rounds of 64
    const uint64_t s0 = (uint64_t)w * seg;
    const uint64_t s1 = s0 + seg < nblk ? s0 + seg : nblk;
    // eight rounds' loads in flight at a time
    constexpr int kU = 8;
    uint32_t st = 0, sv = 0;
    for (uint64_t r0 = s0; r0 < s1; r0 += 64 * kU) {
        uint32_t cv[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const uint64_t b = r0 + 64 * u + (uint32_t)lane;
            cv[u] = b < s1 ? cnt[b] : 0;  // 0: no tiles, no pairs
        }
#pragma unroll
        for (int u = 0; u < kU; u++) {
            st += mfma_tiles(cv[u]);
            sv += short_pairs(cv[u]);
        }
    }
    st = readlane(wave_incl_scan(st), 63);
    sv = readlane(wave_incl_scan(sv), 63);
    if (lane == 0) {
        wsum[w] = st;
        wvsum[w] = sv;
    }
    __syncthreads();
    uint32_t run = 0, vrun = 0, all = 0, vall = 0;  // this segment's start; the totals
    for (int i = 0; i < kW; i++) {
        run += i < w ? wsum[i] : 0u;
        vrun += i < w ? wvsum[i] : 0u;
        all += wsum[i];
        vall += wvsum[i];
    }
    for (uint64_t r0 = s0; r0 < s1; r0 += 64 * kU) {
        uint32_t cv[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const uint64_t b = r0 + 64 * u + (uint32_t)lane;
            cv[u] = b < s1 ? cnt[b] : 0;
        }
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const uint64_t b = r0 + 64 * u + (uint32_t)lane;
            const uint32_t t = mfma_tiles(cv[u]), v = short_pairs(cv[u]);
            const uint32_t it = wave_incl_scan(t), iv = wave_incl_scan(v);
            if (b < s1) {
                off[b] = run + it - t;
                voff[b] = vrun + iv - v;
            }
            run += readlane(it, 63);
            vrun += readlane(iv, 63);
        }
    }
    if (threadIdx.x == 0) {
        off[nblk] = all;
        voff[nblk] = vall;
        total[0] = all;
        total[1] = vall;
    }
}

// The tile records, one thread per tile: tile x lies in the block b with
// off[b] <= x < off[b + 1] (the last block whose prefix is at most x: a
// block without tiles has the same prefix as the next one), found by
// bisection; tinfo[x] = (block, offset of the tile's first query in the
// block's list, queries in the tile, the block's smallest popcount).  The
// grid strides over the tiles the prefix counted.
__global__ __launch_bounds__(256) void tile_info_kernel(const uint32_t *__restrict__ cnt,
                                                        const uint32_t *__restrict__ off, uint64_t nblk,
                                                        const uint16_t *__restrict__ bpop,
                                                        const uint32_t *__restrict__ ntiles,
                                                        uint4 *__restrict__ tinfo) {
    const uint32_t total = *ntiles;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t lo = 0, hi = nblk;  // off[lo] <= x < off[hi] (off[0] = 0, off[nblk] = total)
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) / 2;
            if (off[mid] <= x)
                lo = mid;
            else
                hi = mid;
        }
        const uint32_t c = cnt[lo];
        const uint32_t listed = c - short_pairs(c);  // the list's short rest is not in a tile
        const uint32_t t0 = ((uint32_t)x - off[lo]) * mt::MA;
        const uint32_t m = listed - t0 < (uint32_t)mt::MA ? listed - t0 : (uint32_t)mt::MA;
        tinfo[x] = make_uint4((uint32_t)lo, t0, m, bpop ? bpop[2 * lo] : 0u);
    }
}

// The (query, block) pairs of short lists on the vector ALUs: one wave per
// pair, 8 lanes per row and 8 rows per step over the block's rows; rows with
// K <= the query's k-th key join its candidates, as in eval_kernel.
__global__ __launch_bounds__(256) void eval_short_kernel(const uint4 *__restrict__ q, const uint4 *__restrict__ sorted,
                                                         uint64_t n, uint64_t nblk, uint32_t nqp,
                                                         const uint16_t *__restrict__ list,
                                                         const uint32_t *__restrict__ cnt,
                                                         const uint32_t *__restrict__ voff,
                                                         const uint16_t *__restrict__ tpop,
                                                         const uint32_t *__restrict__ perm,
                                                         const uint16_t *__restrict__ qpop,
                                                         const uint32_t *__restrict__ thrk, uint32_t *__restrict__ ccnt,
                                                         u64 *__restrict__ cand) {
    const int lane = lane_id(), g = lane >> 3, j = lane & 7;
    const uint64_t total = voff[nblk];
    const uint64_t groups = (total + 3) / 4;  // four consecutive pairs per workgroup
    // workgroup v of the virtual grid runs on XCD v % 8 (gridDim.x is a multiple of 8): each XCD
    // takes a contiguous range of pairs, so a block's rows are fetched into one L2
    for (uint64_t v = blockIdx.x; v < mt::xcd_grid(groups); v += gridDim.x) {
        uint64_t grp;
        if (!mt::xcd_tile(v, groups, grp)) continue;
        const uint64_t i = readfirst((uint32_t)(grp * 4 + (threadIdx.x >> 6)));
        if (i >= total) continue;
        uint64_t lo = 0, hi = nblk;  // voff[lo] <= i < voff[hi]
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) / 2;
            if (voff[mid] <= i)
                lo = mid;
            else
                hi = mid;
        }
        const uint64_t b = lo;
        const uint32_t c = cnt[b];
        const uint32_t qi = readfirst((uint32_t)list[b * nqp + (c - short_pairs(c)) + (i - voff[b])]);
        uint4 qv[4];
#pragma unroll
        for (int ii = 0; ii < 4; ii++) qv[ii] = q[(uint64_t)qi * 32 + j + 8 * ii];
        const uint32_t pq = readfirst(qpop[qi]);
        const uint32_t wa = weight_a(pq), wb = weight_b(pq);
        const uint32_t th = readfirst(thrk[qi]);
        const uint64_t r0 = b * kBlk;
        const uint32_t m = (uint32_t)(n - r0 < kBlk ? n - r0 : kBlk);
        for (uint32_t base = 0; base < m; base += 8) {
            const uint32_t r = base + (uint32_t)g;
            const bool valid = r < m;
            const uint64_t pos = r0 + (valid ? r : 0);
            uint4 tv[4];
#pragma unroll
            for (int ii = 0; ii < 4; ii++) tv[ii] = sorted[pos * 32 + j + 8 * ii];
            const uint32_t c = sum8(popc_and4(tv[0], qv[0]) + popc_and4(tv[1], qv[1]) + popc_and4(tv[2], qv[2]) +
                                    popc_and4(tv[3], qv[3]));
            const uint32_t K = (pq - c) * wb + ((uint32_t)tpop[pos] - c) * wa;
            if (valid && j == 0 && K <= th) {
                const uint32_t at = atomicAdd(&ccnt[qi], 1u);
                if (at < kCap) cand[(uint64_t)qi * kCap + at] = ((u64)K << 32) | perm[pos];
            }
        }
    }
}

// Tiles of 256 listed queries of a block x the block's rows, in a persistent
// grid: workgroup x takes tiles x, x + G, x + 2G, ... of the virtual tile
// order (G = gridDim.x, a multiple of 8, so the workgroup stays on one XCD and
// the XCD's tiles form one contiguous range of the tile list).  The tiles are
// streamed: the next tile's first two windows are staged during the current
// tile's last two, and its metadata is fetched during the current tile, one
// dependent load per window, so the matrix cores do not wait for a tile to
// start.  The metadata of consecutive tiles alternates between two LDS
// copies, so no barrier closes a tile: a wave that finishes its epilogue
// goes on to the next tile's first window while others still test their
// pairs (the window buffers are free: every wave read them before the last
// window's barrier).  A wave's passing pairs claim their candidate slots
// (the atomics) at the end of its epilogue and are written during the next
// tile's first window, once the slots have come back.
__global__ __launch_bounds__(mt::kThreads) void eval_kernel(const uint4 *__restrict__ q, const uint4 *__restrict__ sorted,
                                                            uint64_t n, uint32_t nqp, const uint32_t *__restrict__ ntiles,
                                                            const uint16_t *__restrict__ list,
                                                            const uint4 *__restrict__ tinfo,
                                                            const uint16_t *__restrict__ tpop,
                                                            const uint32_t *__restrict__ perm,
                                                            const uint16_t *__restrict__ qpop,
                                                            const uint32_t *__restrict__ thrk,
                                                            uint32_t *__restrict__ ccnt, u64 *__restrict__ cand) {
    __shared__ mt::Smem sm;
    // two copies (tiles alternate): query slot's query, |q|, k-th key; row's |t|
    __shared__ uint32_t s_qi[2][mt::MA], s_pq[2][mt::MA], s_th[2][mt::MA], s_tp[2][mt::MB];
    __shared__ __align__(16) float s_cmin[2][mt::MA];  // per query slot: the least overlap that can reach its k-th key
    // per wave: the tile's passing (query, key, row) entries, appended in order
    // and written out together, so the candidate slots' atomics overlap
    // instead of waiting one after another
    constexpr uint32_t kQueue = 320;  // room for one (a, rr) group's 256 entries past the flush mark
    __shared__ uint32_t s_cq[mt::kThreads / 64][kQueue][3];
    const uint32_t total = *ntiles;  // written by the tile prefix
    const uint64_t vend = mt::xcd_grid(total);
    const int r = mt::own_row();
    const bool arow = r < mt::MA;  // the same in a whole wave
    // a lane-varying zero: keeps the per-tile record load a vector load (a
    // scalar load shares its completion counter with the LDS reads)
    const uint32_t vz = __builtin_amdgcn_mbcnt_lo(0u, 0u);
    // A tile's fetch is three dependent loads: its record (block b, list
    // offset t0, queries m, the block's smallest popcount), then this thread's
    // list entry (A rows) or row popcount (B rows), then the query's |q| and
    // k-th key.  Every load is unconditional and in bounds (a row past m or n
    // reads a valid entry and is masked when used).
    uint4 info;          // the record
    uint32_t pb, pc, pd; // loads in flight: list entry or |t|; |q|; k-th key
    uint32_t qi = 0, tp = 0, pq = 0, th = 0;
    bool ok = false;
    auto issue_b = [&](const uint4 &in) {
        const uint64_t r0 = (uint64_t)in.x * kBlk;
        pb = arow ? list[(uint64_t)in.x * nqp + in.y + r]  // t0 + 256 <= nqp: the entry exists
                  : tpop[r0 + (r - mt::MA) < n ? r0 + (r - mt::MA) : n - 1];
    };
    auto take_b = [&](const uint4 &in) {
        const uint64_t r0 = (uint64_t)in.x * kBlk;
        ok = arow ? (uint32_t)r < in.z : r0 + (r - mt::MA) < n;
        qi = arow && ok ? pb : 0;
        tp = !arow && ok ? pb : 0;
    };
    auto issue_c = [&]() {
        pc = qpop[qi];
        pd = thrk[qi];
    };
    auto take_c = [&]() {
        pq = arow && ok ? pc : 0;
        th = arow && ok ? pd : 0;
    };
    // K = |q|*wB + |t|*wA - C*(wA + wB) with |t| >= the block's smallest
    // popcount: a row with C*(wA + wB) below X = |q|*wB + min|t|*wA - (the
    // k-th key) has K above the k-th key.  wA + wB is 4096, or 4097 when |q|
    // is 0 or 4096, so a row can only pass with C >= ceil(X / 4097) = cmin
    // (a division by a constant; the exact key test follows)
    auto cmin_of = [&](const uint4 &in) -> float {
        const uint32_t wa = weight_a(pq), wb = weight_b(pq);
        const uint32_t S = __umul24(pq, wb) + __umul24(in.w, wa);  // |q|*wB + min|t|*wA < 2^25
        const uint32_t X = S - (S < th ? S : th);                    // max(S - k-th key, 0)
        const uint32_t cmin = (X + 4096u) / 4097u;
        return arow && ok ? (float)cmin : 1e30f;
    };
    auto row_of = [&](const uint4 &in) -> const uint4 * {
        const uint64_t r0 = (uint64_t)in.x * kBlk;
        return arow ? q + (uint64_t)qi * 32 : sorted + (ok ? r0 + (r - mt::MA) : 0) * 32;
    };
    auto publish = [&](float cmin, int pb) {  // read after the next barrier
        if (arow) {
            s_qi[pb][r] = qi;
            s_pq[pb][r] = pq;
            s_th[pb][r] = th;
            s_cmin[pb][r] = cmin;
        } else {
            s_tp[pb][r - mt::MA] = tp;
        }
    };

    uint64_t v = blockIdx.x, xt;
    if (!(v < vend && mt::xcd_tile(v, total, xt))) return;  // whole workgroup: no tile
    // the first tile: fetched here, waiting for each load
    info = tinfo[xt + vz];
    issue_b(info);
    take_b(info);
    issue_c();
    take_c();
    uint4 cur = info;
    const uint4 *row = row_of(cur);
    bool cur_ok = ok;
    int par = 0;  // metadata copy of the current tile
    publish(cmin_of(cur), par);
    mt::Stream st;
    mt::stream_begin(row, !cur_ok, sm, st);  // its barrier also publishes the metadata
    const int wv = r >> 6, lane = r & 63;
    uint32_t (*cq)[3] = s_cq[wv];
    // the previous tile's passing pairs still to be written: entry `lane` of
    // this wave's queue, its claimed slot and its row's original index
    uint32_t dn = 0, dpos = 0, dperm = 0;
    auto store_claimed = [&]() {
        if ((uint32_t)lane < dn && dpos < kCap)
            cand[(uint64_t)cq[lane][0] * kCap + dpos] = ((u64)cq[lane][1] << 32) | dperm;
        dn = 0;
    };
    for (;;) {
        // tiles of this workgroup only run out at the end of its XCD's range
        const uint64_t vn = v + gridDim.x;
        const bool more = vn < vend && mt::xcd_tile(vn, total, xt);
        const uint64_t xn = more ? xt : 0;
        uint4 pa = info;      // the next tile's record, in flight
        const uint4 *nrow = row;
        bool nok = false;
        float ncmin = 0.f;
        mt::v4f acc[8][4];
        // after window w: take what window w - 1 loaded (the window's own store
        // waited for every earlier load), then issue the next loads
        bool nzero = true;
        // the waves of A rows 128..255 have nothing to multiply when the tile
        // lists at most 128 queries
        const bool idle = (r >> 8) == 1 && cur.z <= (uint32_t)(mt::MA / 2);
        mt::stream_tile(row, !cur_ok, nrow, nzero, sm, st, acc, [&](int win) {
            if (win == 0) store_claimed();
            if (win == 1) info = pa;
            if (win == 2) take_b(info);
            if (win == 3) {
                take_c();
                ncmin = cmin_of(info);
                nrow = row_of(info);
                nok = ok;
                nzero = !more || !ok;
            }
            pa = tinfo[xn + vz];
            issue_b(info);
            issue_c();
        }, idle);
        const uint64_t r0 = (uint64_t)cur.x * kBlk;
        const uint32_t *t_qi = s_qi[par], *t_pq = s_pq[par], *t_th = s_th[par], *t_tp = s_tp[par];
        const float *t_cmin = s_cmin[par];
        // this lane's four rows: their popcounts and whether they exist, the
        // same for every query group of the tile
        uint32_t tpv[4];
        bool rv[4];
#pragma unroll
        for (int bb = 0; bb < 4; bb++) {
            tpv[bb] = t_tp[mt::acc_brow(bb)];
            rv[bb] = r0 + (uint64_t)mt::acc_brow(bb) < n;
        }
        // a group's four query slots are consecutive: their least overlaps
        // are one 16-byte read, issued a group ahead of the test
        float4 cm_next = *reinterpret_cast<const float4 *>(t_cmin + mt::acc_arow(0, 0));
        uint32_t nq = 0;  // entries in this wave's queue (the same in every lane)
        auto flush = [&]() {
            for (uint32_t e = lane; e < nq; e += 64) {
                const uint32_t qk = cq[e][0], K = cq[e][1], rw = cq[e][2];
                const uint32_t pos = atomicAdd(&ccnt[qk], 1u);
                if (pos < kCap) cand[(uint64_t)qk * kCap + pos] = ((u64)K << 32) | perm[rw];
            }
            nq = 0;
        };
#pragma unroll
        for (int a = 0; a < 8; a++) {
            // one group of queries at a time, so their metadata loads stay next to their use
            __builtin_amdgcn_sched_barrier(0);
            const float4 cm = cm_next;
            if (a < 7) cm_next = *reinterpret_cast<const float4 *>(t_cmin + mt::acc_arow(a + 1, 0));
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                const uint32_t i = (uint32_t)mt::acc_arow(a, rr);
                // most (query, row) pairs miss the k-th key by far: test this
                // lane's 4 rows at once against the least useful overlap
                const float mx = fmaxf(fmaxf(acc[a][0][rr], acc[a][1][rr]), fmaxf(acc[a][2][rr], acc[a][3][rr]));
                // (a slot past the tile's queries has least overlap 1e30)
                const bool act = mx >= (rr == 0 ? cm.x : rr == 1 ? cm.y : rr == 2 ? cm.z : cm.w);
                if (ballot(act) == 0) continue;
                const uint32_t qk = t_qi[i];
                const uint32_t pk = t_pq[i];
                const uint32_t wa = weight_a(pk), wb = weight_b(pk);
                const uint32_t tk = t_th[i];
                // K = |q|*wB + |t|*wA - C*(wA + wB): the first two terms per
                // row once per group, then one 24-bit multiply-add per pair
                // (C <= 4096 and wA + wB <= 4097; every term below 2^26)
                const uint32_t P = __umul24(pk, wb);
                const int nsw = -(int)(wa + wb);
                uint32_t PT[4];
#pragma unroll
                for (int bb = 0; bb < 4; bb++) PT[bb] = P + __umul24(tpv[bb], wa);
#pragma unroll
                for (int bb = 0; bb < 4; bb++) {
                    const uint64_t rw = r0 + mt::acc_brow(bb);
                    const uint32_t C = mt::count(acc[a][bb][rr]);
                    const uint32_t K = (uint32_t)((int)PT[bb] + __mul24((int)C, nsw));
                    const bool pass = act & rv[bb] & (K <= tk);  // no short-circuit: no branch per test
                    const u64 pm = ballot(pass);
                    if (pass) {
                        const uint32_t e = nq + lanes_below(pm);
                        cq[e][0] = qk;
                        cq[e][1] = K;
                        cq[e][2] = (uint32_t)rw;
                    }
                    nq += (uint32_t)__popcll(pm);
                }
                if (nq > kQueue - 256) flush();  // the next group adds at most 4 x 64
            }
        }
        if (nq > 64) {
            flush();
        } else {  // claim the slots now, write them during the next tile
            if ((uint32_t)lane < nq) {
                dpos = atomicAdd(&ccnt[cq[lane][0]], 1u);
                dperm = perm[cq[lane][2]];
            }
            dn = nq;
            nq = 0;
        }
        if (!more) {
            store_claimed();
            break;
        }
        par ^= 1;
        publish(ncmin, par);  // the other copy: this tile's may still be read
        cur = info;
        row = nrow;
        cur_ok = nok;
        v = vn;
    }
}

// After a round: merge each running query's candidates into its top k,
// update its k-th key and set its next range.  A query whose candidates
// overflowed the buffer repeats the round: the k best of the candidates it
// did store (real rows, as is its top k) bound its final k-th key, so the
// repeat keeps fewer rows; when that bound does not tighten the key, the
// query goes to the per-query fallback.  Either way the next-round pairs
// filled into this round are forgotten (their done bits cleared).  One block
// per query.
__global__ __launch_bounds__(256) void select_kernel(uint32_t k, const uint16_t *__restrict__ qpop,
                                                     const u64 *__restrict__ cuts, u64 *__restrict__ rec,
                                                     uint32_t *__restrict__ qround, uint32_t *__restrict__ ccnt,
                                                     const u64 *__restrict__ cand, u64 *__restrict__ top,
                                                     uint32_t *__restrict__ ntop, uint32_t *__restrict__ thrk,
                                                     uint32_t *__restrict__ counters, uint32_t *__restrict__ redo,
                                                     uint32_t *__restrict__ qst, const uint16_t *__restrict__ lbq,
                                                     uint64_t nblk, uint32_t *__restrict__ done, uint64_t dw, uint32_t nqp,
                                                     u64 *__restrict__ frange, const uint32_t *__restrict__ r1list,
                                                     uint32_t n1_marked) {
    __shared__ u64 keys[8192];
    const uint32_t qi = blockIdx.x;
    const u64 lo = rec[2 * qi], hi = rec[2 * qi + 1];
    if (!(hi > lo)) return;  // not running
    const uint32_t m = ccnt[qi];
    const bool over = m > kCap;
    const uint32_t stored = over ? kCap : m;
    const uint32_t nt = ntop[qi];
    const uint32_t th = thrk[qi];
    uint32_t have = nt, th_new = th;
    if (stored > 0) {
        const uint32_t total = nt + stored;  // <= k + kCap <= 8192
        auto key_at = [&](uint32_t i) {
            return i < nt ? top[(uint64_t)qi * k + i] : cand[(uint64_t)qi * kCap + (i - nt)];
        };
        uint32_t np = 0;  // sort keys[0 .. np), which holds the k smallest keys
        if (total > 1024) {
            // Large sets: the k-th smallest K by bisection over this thread's
            // (at most 32) key values, then only the keys with K up to it
            // are sorted.  Every key's K is at most the query's k-th key
            // (candidates are written only below it), so K* lies in [0, th].
            uint32_t kv[32];
#pragma unroll
            for (int j = 0; j < 32; j++) {
                const uint32_t i = threadIdx.x + 256u * j;
                kv[j] = i < total ? (uint32_t)(key_at(i) >> 32) : 0xFFFFFFFFu;
            }
            __shared__ uint32_t s_part[4];
            auto count_le = [&](uint32_t v) {  // keys with K <= v, in every thread
                uint32_t c = 0;
#pragma unroll
                for (int j = 0; j < 32; j++) c += kv[j] <= v;
                c = (uint32_t)wave_sum_f((float)c);  // <= 8192: exact in fp32
                __syncthreads();  // the previous count's partial sums were read
                if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = c;
                __syncthreads();
                return s_part[0] + s_part[1] + s_part[2] + s_part[3];
            };
            uint32_t lo = 0, hi = th;  // count_le(th) = total >= k
            while (lo < hi) {
                const uint32_t mid = lo + (hi - lo) / 2;
                if (count_le(mid) >= k) hi = mid;
                else lo = mid + 1;
            }
            const uint32_t c = count_le(lo);
            if (c <= 1024) {
                // keys with K <= K*, compacted into keys[0 .. c) in key-index order
                __shared__ uint32_t s_base;
                if (threadIdx.x == 0) s_base = 0;
                __syncthreads();
#pragma unroll
                for (int j = 0; j < 32; j++) {
                    const uint32_t i = threadIdx.x + 256u * j;
                    const bool in = kv[j] <= lo;
                    const u64 bm = ballot(in);
                    uint32_t base = 0;
                    if ((threadIdx.x & 63) == 0 && bm) base = atomicAdd(&s_base, (uint32_t)__popcll(bm));
                    base = readlane(base, 0);
                    if (in) keys[base + lanes_below(bm)] = key_at(i);
                }
                np = next_pow2(c < 2 ? 2 : c);
                __syncthreads();
                for (uint32_t i = c + threadIdx.x; i < np; i += 256) keys[i] = KEY_NONE;
            }
        }
        if (np == 0) {  // small sets, or a K* shared by more than 1,024 keys: sort them all
            np = next_pow2(total < 2 ? 2 : total);
            for (uint32_t i = threadIdx.x; i < np; i += 256) keys[i] = i < total ? key_at(i) : KEY_NONE;
        }
        __syncthreads();
        block_bitonic_sort(keys, np);
        const uint32_t kth = total >= k ? (uint32_t)(keys[k - 1] >> 32) : kInf;
        th_new = kth < th ? kth : th;
        if (!over) {
            have = total < k ? total : k;
            for (uint32_t i = threadIdx.x; i < have; i += 256) top[(uint64_t)qi * k + i] = keys[i];
        }
    }
    if (over) {
        // the pairs this round filled in from the next one lost candidates too:
        // clear their done bits (keys past this round's end), so they are listed again
        const u64 end = cuts[(uint64_t)qi * (kRounds + 1) + qround[qi]];
        for (uint64_t wd = threadIdx.x; wd < dw; wd += 256) {
            uint32_t clear = 0;
            for (uint32_t j = 0; j < 32; j++) {
                const uint64_t b = wd * 32 + j;
                if (b < nblk && range_key(lbq[(uint64_t)qi * nblk + b], (uint32_t)b) > end) clear |= 1u << j;
            }
            done[(uint64_t)wd * nqp + qi] &= ~clear;
        }
        if (n1_marked) {
            // a learned round 1 evaluated blocks anywhere in the key order: they stay done
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < n1_marked; i += 256) {
                const uint32_t b = r1list[(uint64_t)qi * kM1 + i];
                atomicOr(&done[(uint64_t)(b / 32) * nqp + qi], 1u << (b % 32));
            }
        }
    }
    if (threadIdx.x != 0) return;
    ccnt[qi] = 0;
    if (qst) qst[(uint64_t)qi * 4 + 1] += 1;
    const u64 *c = cuts + (uint64_t)qi * (kRounds + 1);
    const uint32_t r = qround[qi];
    const uint32_t wb = weight_b(qpop[qi]);
    if (over) {
        const u64 cap = cap_key(th_new, wb);
        const u64 nhi = c[r] < cap ? c[r] : cap;
        if (th_new < th && nhi > lo) {  // repeat round r with the tighter key
            thrk[qi] = th_new;
            rec[2 * qi + 1] = nhi;
            set_fill_range(frange + 2 * qi, c, r, cap);
            atomicAdd(&counters[0], 1u);
        } else {
            redo[atomicAdd(&counters[1], 1u)] = qi;
            rec[2 * qi + 1] = 0;
        }
        return;
    }
    ntop[qi] = have;
    thrk[qi] = th_new;
    qround[qi] = r + 1;
    const u64 nlo = c[r];
    const u64 cap = cap_key(th_new, wb);
    u64 nhi = 0;
    if (r < (uint32_t)kRounds) nhi = c[r + 1] < cap ? c[r + 1] : cap;
    const bool active = nhi > nlo;
    rec[2 * qi] = nlo;
    rec[2 * qi + 1] = active ? nhi : 0;
    set_fill_range(frange + 2 * qi, c, r + 1, cap);
    if (active) atomicAdd(&counters[0], 1u);
}

// Queries still running after the last pass go to the per-query fallback.
__global__ void leftover_kernel(uint32_t nqb, u64 *__restrict__ rec, uint32_t *__restrict__ counters,
                                uint32_t *__restrict__ redo) {
    const uint32_t qi = blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= nqb) return;
    if (rec[2 * qi + 1] > rec[2 * qi]) {
        redo[atomicAdd(&counters[1], 1u)] = qi;
        rec[2 * qi + 1] = 0;
    }
}

// Results from the top-k keys: one wave per query, lane r writes rank r.
__global__ __launch_bounds__(256) void emit_kernel(const uint64_t *__restrict__ q, uint32_t nqb, uint32_t k,
                                                   const u64 *__restrict__ top, const uint32_t *__restrict__ ntop,
                                                   const uint64_t *__restrict__ sorted,
                                                   const uint32_t *__restrict__ iperm, uint32_t *idx, int32_t *missed,
                                                   int32_t *extra, float *dist, const uint32_t *__restrict__ qst,
                                                   uint32_t *d_qstats, unsigned long long *gstats,
                                                   const uint32_t *__restrict__ nq_dev) {
    const int lane = lane_id();
    const uint32_t qi = readfirst(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (qi >= nqb || (nq_dev && qi >= *nq_dev)) return;
    const uint32_t nt = ntop[qi];
    if (lane < (int)k) {
        const uint64_t o = (uint64_t)qi * k + lane;
        if ((uint32_t)lane >= nt) {
            idx[o] = QD_PAD_IDX;
            missed[o] = -1;
            extra[o] = -1;
            dist[o] = __builtin_inff();
        } else {
            const u64 e = top[o];
            const uint32_t row = (uint32_t)e;
            const uint64_t *qq = q + (uint64_t)qi * QD_WORDS;
            const uint64_t *tt = sorted + (uint64_t)iperm[row] * QD_WORDS;
            uint32_t a = 0, b = 0, pq = 0;
            for (int w = 0; w < QD_WORDS; w++) {
                const uint64_t x = qq[w], y = tt[w];
                a += __popcll(x & ~y);
                b += __popcll(~x & y);
                pq += __popcll(x);
            }
            const uint32_t wa = weight_a(pq), wb = weight_b(pq);
            idx[o] = row;
            missed[o] = (int32_t)a;
            extra[o] = (int32_t)b;
            dist[o] = (float)((double)(a * wb + b * wa) / ((double)wa * (double)wb));
        }
    }
    if (qst && lane < 4) {
        const uint32_t v = qst[(uint64_t)qi * 4 + lane];
        if (d_qstats) d_qstats[(uint64_t)qi * 4 + lane] = v;
        if (gstats) atomicAdd(&gstats[lane], (unsigned long long)v);
    }
}

// The fallback's queries (list[0 .. *m)) gathered into consecutive rows.
__global__ void gather_kernel(const uint4 *__restrict__ q, const uint32_t *__restrict__ list,
                              const uint32_t *__restrict__ m, uint4 *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *m * 32) out[i] = q[(uint64_t)list[i >> 5] * 32 + (i & 31)];
}

// The fallback's results back to their queries' rows.
template <class T>
__global__ void scatter_kernel(const T *__restrict__ src, const uint32_t *__restrict__ list,
                               const uint32_t *__restrict__ m, uint32_t k, T *__restrict__ dst) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *m * k) dst[(uint64_t)list[i / k] * k + (i % k)] = src[i];
}

// Clears n words (a kernel, not a memset node, so a captured graph replays it
// reliably).
__global__ void zero_kernel(uint32_t *__restrict__ p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

inline size_t up256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

int tree_block_images(qd_tree_s *t, hipStream_t s) {
    t->n_blk = (t->n + kBlk - 1) / kBlk;
    QD_HIP_CHECK(hipMalloc((void **)&t->d_blk, t->n_blk * 512));
    if (t->d_pmin) QD_HIP_CHECK(hipMalloc((void **)&t->d_bpop, t->n_blk * 4));
    hipLaunchKernelGGL(block_image_kernel, dim3((uint32_t)t->n_blk), dim3(64), 0, s, t->d_sorted, t->n, t->d_blk,
                       t->d_pop, t->d_bpop);
    QD_HIP_CHECK(hipGetLastError());
    return QD_OK;
}

// Workspace of one batch of up to qb queries (offsets into one allocation).
BlockedLayout blocked_layout(qd_tree_t t, uint32_t nq, uint32_t k, bool model) {
    BlockedLayout L;
    const uint64_t nblk = t->n_blk;
    // batch: up to kMaxBatch queries, bound and list matrices within about 12 GiB
    uint32_t qb = nq < kMaxBatch ? nq : kMaxBatch;
    if (qb == 0) qb = 1;
    auto batch_bytes = [&](uint32_t b) {
        return (uint64_t)up256(b) * (nblk * 6 + (nblk + 31) / 32 * 4 + kCap * 8 + (uint64_t)k * 8 + 512);
    };
    while (qb > 256 && batch_bytes(qb) > (12ull << 30)) qb = (qb + 1) / 2;
    L.qb = qb;
    const size_t P = up256(qb);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += up256(bytes);
        return at;
    };
    L.qpop = take(P * 2);
    L.lbq = take(P * nblk * 2);
    L.lbb = take(P * nblk * 2);
    L.list = take(P * nblk * 2);
    L.cuts = take(P * (kRounds + 1) * 8);
    L.r1 = take(P * kM1 * 4);
    L.rec = take(P * 16);
    L.thr = take(P * 4);
    L.ntop = take(P * 4);
    L.top = take(P * k * 8);
    L.ccnt = take(P * 4);
    L.cand = take(P * kCap * 8);
    L.cnt = take(nblk * 4);
    L.qr = take(P * 4);
    L.act = take(P * 4 + 4);
    L.off = take((nblk + 1) * 4);
    L.voff = take((nblk + 1) * 4);
    L.ctr = take(64);
    L.done = take(P * ((nblk + 31) / 32) * 4);
    L.fr = take(P * 16);
    L.tinfo = take(nblk * (P / mt::MA) * 16);  // tile records: at most ceil(nqb / 256) per block
    L.redo = take(P * 4);
    L.qst = take(P * 16);
    L.lnode = take(P * 4);
    L.gst = take(32);
    // the per-query fallback for queries whose key cannot tighten: gathered
    // queries, their results, and a depth-first traversal's workspace (a
    // best-first one at one wave per CU for a tree deeper than the
    // depth-first stack: its bucket pools are large, and the fallback is rare)
    L.fb_order = depth_first_fits(t) ? QD_ORDER_DEPTH_FIRST : QD_ORDER_BEST_FIRST;
    L.fb = tree_launch_shape(t, qb, k, L.fb_order, L.fb_order == QD_ORDER_DEPTH_FIRST ? 0 : 1, 1);
    L.fbq = take(P * 512);
    L.fbr = take(P * k * 16);
    L.fbws = take(L.fb.total());
    L.model = model;
    if (model) L.mdesc = take(model_descend_bytes(qb));  // the learned start's descent
    L.bytes = o;
    return L;
}

// Five counts of a direct call's blocked search, in pinned host memory: one
// small buffer per host thread, allocated on its first use and kept until the
// process ends (a thread runs one call at a time).
static uint32_t *pinned_counts() {
    static thread_local uint32_t *p = nullptr;
    if (!p && hipHostMalloc((void **)&p, 64, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    return p;
}

// One batch of nqb queries (nqb <= L.qb) at qq; nq_dev (nullable): the
// batch's size on the device, at most nqb.  With graph, nothing waits for
// the host: the rounds run as kGraphPasses fixed passes whose kernels read
// their work from device memory (a pass with no running query does nothing),
// queries still running after them take the fallback, and the launches can
// be captured.  Otherwise the same passes run until the host, one pass late,
// sees that no query runs any more.  gst (nullable): totals of the per-query
// stats.
int blocked_batch(qd_tree_t t, const BlockedLayout &L, char *ws, const uint64_t *qq, uint32_t nqb,
                  const uint32_t *nq_dev, uint32_t k, const qd_search_params *p, uint32_t *oi, int32_t *om,
                  int32_t *ox, float *od, uint32_t *d_qstats, unsigned long long *gst, bool graph, hipStream_t s) {
    const uint64_t n = t->n, nblk = t->n_blk;
    const uint32_t m1 = p && p->round1_blocks ? p->round1_blocks : 16;
    const uint32_t growth = p && p->round_growth ? p->round_growth : 4;
    const uint64_t t2 = p ? p->round2_blocks : 0;
    qd_model_t model = p ? p->model : nullptr;
    const size_t P = up256(L.qb);
    uint16_t *qpop = (uint16_t *)(ws + L.qpop), *lbq = (uint16_t *)(ws + L.lbq), *lbb = (uint16_t *)(ws + L.lbb),
             *list = (uint16_t *)(ws + L.list);
    u64 *cuts = (u64 *)(ws + L.cuts), *rec = (u64 *)(ws + L.rec), *top = (u64 *)(ws + L.top),
        *cand = (u64 *)(ws + L.cand), *frange = (u64 *)(ws + L.fr);
    uint32_t *r1list = (uint32_t *)(ws + L.r1), *thr = (uint32_t *)(ws + L.thr), *ntop = (uint32_t *)(ws + L.ntop),
             *ccnt = (uint32_t *)(ws + L.ccnt), *cnt = (uint32_t *)(ws + L.cnt), *off = (uint32_t *)(ws + L.off),
             *voff = (uint32_t *)(ws + L.voff), *ctr = (uint32_t *)(ws + L.ctr), *donebits = (uint32_t *)(ws + L.done),
             *redo = (uint32_t *)(ws + L.redo), *qst = (uint32_t *)(ws + L.qst), *qround = (uint32_t *)(ws + L.qr),
             *lnode = (uint32_t *)(ws + L.lnode);
    uint4 *tinfo = (uint4 *)(ws + L.tinfo);
    uint32_t *act = (uint32_t *)(ws + L.act), *nact = act + P;
    const bool want_stats = d_qstats || gst;
    const uint32_t nqp = (uint32_t)up256(nqb);
    const uint4 *q4 = reinterpret_cast<const uint4 *>(qq);
    const uint64_t dw = (nblk + 31) / 32;  // done-bit words per query, stored word-major (word, query)
    int rc = popcount_rows_launch(qq, nqb, qpop, s);
    if (rc != QD_OK) return rc;
    // counters: [0] running (round 1 and select), [1] fallback queries, [2] tiles, [3] short pairs
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, ctr, (uint64_t)16);
    hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)std::min<uint64_t>((nqb + 255) / 256, 1024)), dim3(256), 0, s, ccnt,
                       (uint64_t)nqb);
    hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)std::min<uint64_t>((nqp * dw + 255) / 256, 4096)), dim3(256), 0, s,
                       donebits, (uint64_t)nqp * dw);
    const uint32_t n_qtiles = nqp / mt::MA;
    const uint64_t n_btiles = (nblk + mt::MB - 1) / mt::MB;
    {
        KernelTimer timer("tree_block_bounds", s);
        hipLaunchKernelGGL(bound_kernel, dim3((uint32_t)mt::tile_grid(n_qtiles * n_btiles)), dim3(mt::kThreads), 0, s,
                           q4, nqb, nqp, reinterpret_cast<const uint4 *>(t->d_blk), nblk, t->d_bpop, qpop, n_qtiles,
                           lbq, lbb, nq_dev);
    }
    {
        KernelTimer timer("tree_block_plan", s);
        hipLaunchKernelGGL(plan_kernel, dim3(nqb), dim3(256), 0, s, lbq, nblk, m1, t2, growth, cuts, r1list, nq_dev);
    }
    const uint32_t n1 = (uint32_t)(nblk < m1 ? nblk : m1);
    // round 1 at consecutive blocks where a descent from the root leads: the
    // model's (learned order) or the bound's
    const bool descend = model || (p && p->round1_start == QD_START_BOUND_DESCENT);
    if (model) {
        rc = model_descend(model, t, qq, nqb, n1 * kBlk, lnode, L.model ? ws + L.mdesc : nullptr, s);
        if (rc != QD_OK) return rc;
    } else if (descend) {
        KernelTimer timer("tree_block_descend", s);
        hipLaunchKernelGGL(bound_descend_kernel, dim3((nqb + 3) / 4), dim3(256), 0, s, q4, nqb, qpop,
                           reinterpret_cast<const uint4 *>(t->d_or), t->d_child, t->d_count, t->d_pmin, t->d_pmax,
                           n1 * kBlk, lnode, nq_dev);
    }
    if (descend)
        hipLaunchKernelGGL(learned_start_kernel, dim3((nqb + 255) / 256), dim3(256), 0, s, lnode, nqb, t->d_begin,
                           nblk, n1, r1list, cuts, donebits, nqp, nq_dev);
    {
        KernelTimer timer("tree_block_round1", s);
        hipLaunchKernelGGL(round1_kernel, dim3((nqb + 3) / 4), dim3(256), 0, s, q4, nqb, k,
                           reinterpret_cast<const uint4 *>(t->d_sorted), t->d_pop, t->d_perm, n, nblk, r1list, n1,
                           cuts, qpop, top, ntop, thr, rec, frange, qround, ctr, want_stats ? qst : nullptr, nq_dev);
    }
    if (hipGetLastError() != hipSuccess) return fail(QD_ERR_DEVICE, "blocked search: launch failed");
    // persistent matrix-core tiles: one workgroup per CU (the tile's LDS and
    // registers leave room for one), a multiple of the 8 XCDs
    const uint64_t eval_grid = mt::xcd_grid((uint64_t)device_cus());
    const uint64_t short_grid = mt::xcd_grid((uint64_t)device_cus() * 8);
    // tile records: at most ceil(nqb / 256) tiles per block
    const uint64_t info_grid = std::min<uint64_t>((nblk * (nqp / mt::MA) + 255) / 256, (uint64_t)device_cus() * 8);
    const int passes = graph ? kGraphPasses : kMaxPasses;
    bool running = true;
    // Direct calls: the host learns whether any query still runs one pass
    // late.  Every pass's kernels read their work from device memory (as in
    // a graph), the counts after each pass's lists are copied to pinned host
    // memory, and the host waits for that copy only while the pass's
    // evaluation runs, so the device never idles waiting for the host; once
    // a pass listed no running query the loop stops (that pass's launches
    // found no work).
    uint32_t *hb = nullptr;  // running queries, counters (tiles, short pairs at 3, 4)
    hipEvent_t ev = nullptr;
    if (!graph) {
        hb = pinned_counts();
        if (!hb) return fail(QD_ERR_OOM, "blocked search: pinned host memory");
        QD_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    for (int pass = 0; pass < passes; pass++) {
        if (!graph && pass > 0) {
            const hipError_t e = hipEventSynchronize(ev);
            if (e != hipSuccess) {
                (void)hipEventDestroy(ev);
                return fail(QD_ERR_DEVICE, "blocked search: %s", hipGetErrorString(e));
            }
            if (hb[0] == 0) {
                running = false;
                break;  // no query ran in the previous pass
            }
            profile_count("tree_block_tiles", hb[3]);
            profile_count("tree_block_short_pairs", hb[4]);
        }
        {
            KernelTimer timer("tree_block_lists", s);
            const uint64_t waves = (nblk + kGroup - 1) / kGroup;
            hipLaunchKernelGGL(active_kernel, dim3(1), dim3(1024), 0, s, rec, nqb, act, nact);
            hipLaunchKernelGGL(list_kernel, dim3((uint32_t)((waves + 3) / 4)), dim3(256), 0, s, lbb, nblk, n, nqb,
                               nqp, act, nact, rec, frange, donebits, list, cnt, want_stats ? qst : nullptr);
            hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(1024), 0, s, cnt, nblk, off, voff, ctr + 2);
            hipLaunchKernelGGL(tile_info_kernel, dim3((uint32_t)info_grid), dim3(256), 0, s, cnt, off, nblk,
                               t->d_bpop, ctr + 2, tinfo);
        }
        if (!graph) {
            hipError_t e = hipMemcpyAsync(hb, nact, 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipMemcpyAsync(hb + 1, ctr, 16, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipEventRecord(ev, s);
            if (e != hipSuccess) {
                (void)hipEventDestroy(ev);
                return fail(QD_ERR_DEVICE, "blocked search: %s", hipGetErrorString(e));
            }
        }
        {
            KernelTimer timer("tree_block_eval", s);
            hipLaunchKernelGGL(eval_kernel, dim3((uint32_t)eval_grid), dim3(mt::kThreads), 0, s, q4,
                               reinterpret_cast<const uint4 *>(t->d_sorted), n, nqp, ctr + 2, list, tinfo, t->d_pop,
                               t->d_perm, qpop, thr, ccnt, cand);
        }
        {
            KernelTimer timer("tree_block_eval_short", s);
            hipLaunchKernelGGL(eval_short_kernel, dim3((uint32_t)short_grid), dim3(256), 0, s, q4,
                               reinterpret_cast<const uint4 *>(t->d_sorted), n, nblk, nqp, list, cnt, voff, t->d_pop,
                               t->d_perm, qpop, thr, ccnt, cand);
        }
        {
            KernelTimer timer("tree_block_select", s);
            hipLaunchKernelGGL(select_kernel, dim3(nqb), dim3(256), 0, s, k, qpop, cuts, rec, qround, ccnt, cand,
                               top, ntop, thr, ctr, redo, want_stats ? qst : nullptr, lbq, nblk, donebits, dw, nqp,
                               frange, r1list, descend ? n1 : 0u);
        }
        if (hipGetLastError() != hipSuccess) {
            if (ev) (void)hipEventDestroy(ev);
            return fail(QD_ERR_DEVICE, "blocked search: launch failed");
        }
    }
    if (ev) (void)hipEventDestroy(ev);
    // queries still running after the last pass join the fallback
    if (running)
        hipLaunchKernelGGL(leftover_kernel, dim3((nqb + 255) / 256), dim3(256), 0, s, nqb, rec, ctr, redo);
    hipLaunchKernelGGL(emit_kernel, dim3((nqb + 3) / 4), dim3(256), 0, s, qq, nqb, k, top, ntop, t->d_sorted,
                       t->d_iperm, oi, om, ox, od, want_stats ? qst : nullptr, d_qstats, gst, nq_dev);
    // The fallback: queries whose candidate buffer overflowed with a key that
    // could not tighten (more rows tie at it than a buffer holds), searched
    // one by one depth-first; their count (ctr[1]) stays on the device, so an
    // empty fallback only costs launches that find no work.
    uint4 *gq = reinterpret_cast<uint4 *>(ws + L.fbq);
    uint32_t *ri = reinterpret_cast<uint32_t *>(ws + L.fbr);
    int32_t *rm = reinterpret_cast<int32_t *>(ri + P * k), *rx = rm + P * k;
    float *rd = reinterpret_cast<float *>(rx + P * k);
    hipLaunchKernelGGL(gather_kernel, dim3((nqb * 32 + 255) / 256), dim3(256), 0, s, q4, redo, ctr + 1, gq);
    rc = tree_launch(t, L.fb, ws + L.fbws, reinterpret_cast<const uint64_t *>(gq), nqb, ctr + 1, k, L.fb_order,
                     nullptr, 0, ri, rm, rx, rd, nullptr, nullptr, 0, s);
    if (rc != QD_OK) return rc;
    const dim3 g((nqb * k + 255) / 256);
    hipLaunchKernelGGL(scatter_kernel<uint32_t>, g, dim3(256), 0, s, ri, redo, ctr + 1, k, oi);
    hipLaunchKernelGGL(scatter_kernel<int32_t>, g, dim3(256), 0, s, rm, redo, ctr + 1, k, om);
    hipLaunchKernelGGL(scatter_kernel<int32_t>, g, dim3(256), 0, s, rx, redo, ctr + 1, k, ox);
    hipLaunchKernelGGL(scatter_kernel<float>, g, dim3(256), 0, s, rd, redo, ctr + 1, k, od);
    if (hipGetLastError() != hipSuccess) return fail(QD_ERR_DEVICE, "blocked search: fallback launch failed");
    return QD_OK;
}

int knn_tree_blocked(qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k, const qd_search_params *p,
                     uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, uint32_t *d_qstats,
                     qd_stats *h_stats, hipStream_t s) {
    int rc = blocked_check(t, p);
    if (rc != QD_OK) return rc;
    if (h_stats) *h_stats = qd_stats{0, 0, 0, 0};
    const BlockedLayout L = blocked_layout(t, nq, k, p && p->model);
    char *ws = nullptr;
    QD_HIP_CHECK(hipMallocAsync((void **)&ws, L.bytes, s));
    unsigned long long *gst = h_stats ? (unsigned long long *)(ws + L.gst) : nullptr;
    if (gst) hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, (uint32_t *)gst, (uint64_t)8);
    for (uint32_t qb0 = 0; qb0 < nq && rc == QD_OK; qb0 += L.qb) {
        const uint32_t nqb = nq - qb0 < L.qb ? nq - qb0 : L.qb;
        const uint64_t o = (uint64_t)qb0 * k;
        rc = blocked_batch(t, L, ws, d_q + (uint64_t)qb0 * QD_WORDS, nqb, nullptr, k, p, d_idx + o, d_missed + o,
                           d_extra + o, d_dist + o, d_qstats ? d_qstats + (uint64_t)qb0 * 4 : nullptr, gst, false, s);
    }
    if (rc == QD_OK && h_stats) {
        unsigned long long hs[4];
        hipError_t e = hipMemcpyAsync(hs, gst, sizeof hs, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = fail(QD_ERR_DEVICE, "stats: %s", hipGetErrorString(e));
        else *h_stats = qd_stats{hs[0], hs[1], hs[2], hs[3]};
    }
    (void)hipFreeAsync(ws, s);
    return rc;
}

int blocked_check(qd_tree_t t, const qd_search_params *p) {
    if (!t->d_blk || t->n_blk == 0) return fail(QD_ERR_INVALID, "tree has no block images");
    if (t->n_blk > 0x7FFFFFFFull) return fail(QD_ERR_UNSUPPORTED, "too many blocks");
    const uint32_t m1 = p && p->round1_blocks ? p->round1_blocks : 16;
    const uint32_t growth = p && p->round_growth ? p->round_growth : 4;
    if (m1 > kM1) return fail(QD_ERR_INVALID, "round1_blocks=%u above %u", m1, kM1);
    if (growth < 2 || growth > 64) return fail(QD_ERR_INVALID, "round_growth=%u outside 2..64", growth);
    if (p && p->round1_start > QD_START_BOUND_DESCENT)
        return fail(QD_ERR_INVALID, "round1_start=%u unknown", p->round1_start);
    return QD_OK;
}

}  // namespace qd

// Sequential-search k-NN under the Weighted Hamming distance (Eq. 1) and the
// per-row popcount, for gfx950.
//
// Scan kernel: a block of 4 waves serves one tile of QT queries over a slice of
// the database.  Each wave streams its own contiguous run of rows; a row
// (512 B) is spread over 8 lanes, lane j of a group holding the 16-byte
// chunks j, j+8, j+16, j+24, so one load instruction reads 8 whole 128-byte
// lines.  The query tile sits in registers as the same slices.  Per pair only
// the overlap C = popcount(q AND t) is counted (AND + BCNT per dword); with
// |q| and |t| it gives A = |q| - C, B = |t| - C and the key
// K = A*wB + B*wA.  Each wave keeps, per query, its k best (K, row) keys in
// one register across the 64 lanes and inserts only candidates below the
// current k-th key.  A merge kernel then reduces the per-wave lists of every
// query to the exact top k and writes the results.
//
// Batches of a few queries take the same slices on the matrix cores instead
// (scan_small_mfma_kernel): a wave holds 16 queries and counts 16 rows
// against them at a time as one FP4 matrix product (the encoding of
// mfma_tile.h), so its vector work per row no longer grows with the number
// of queries.
#include <mutex>

#include "mfma_tile.h"
#include "qd_device.h"
#include "qd_internal.h"
#include "qd_launch.h"

namespace qd {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kRowsPerStep = 8;  // rows per wave per step (8 lanes per row)
constexpr uint32_t kMaxParts = 4096;
constexpr uint32_t kMaxCand = QD_MAX_K * QD_MAX_K;

template <int QT>
__global__ __launch_bounds__(kBlock) void scan_topk_kernel(const uint4 *__restrict__ db, uint64_t n,
                                                           const uint4 *__restrict__ q, uint32_t nq, uint32_t k,
                                                           uint32_t n_qtiles, uint32_t n_parts,
                                                           uint64_t rows_per_part, u64 *__restrict__ part,
                                                           const uint32_t *__restrict__ nq_dev) {
    if (nq_dev) {
        nq = *nq_dev;  // size given on the device (captured graphs)
        if ((blockIdx.x % n_qtiles) * QT >= nq) return;  // whole block
    }
    const int lane = lane_id();
    const int g = lane >> 3, j = lane & 7;
    const uint32_t qtile = blockIdx.x % n_qtiles;
    // wave-uniform (readfirstlane) so the row loop compiles as a uniform loop
    const uint32_t p = readfirst((blockIdx.x / n_qtiles) * kWavesPerBlock + (threadIdx.x >> 6));
    if (p >= n_parts) return;  // whole wave
    const uint64_t r0 = (uint64_t)p * rows_per_part;
    const uint64_t r1 = r0 + rows_per_part < n ? r0 + rows_per_part : n;

    uint4 qv[QT][4];
    uint32_t wa[QT], wb[QT], pq[QT];
    u64 list[QT], thr[QT];
#pragma unroll
    for (int t = 0; t < QT; t++) {
        const uint32_t qi = qtile * QT + t;
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            qv[t][i] = qi < nq ? q[(uint64_t)qi * 32 + j + 8 * i] : make_uint4(0, 0, 0, 0);
            s += popc4(qv[t][i]);
        }
        pq[t] = readfirst(sum8(s));
        wa[t] = pq[t] > 1 ? pq[t] : 1;
        wb[t] = (QD_BITS - pq[t]) > 1 ? QD_BITS - pq[t] : 1;
        list[t] = KEY_NONE;
        thr[t] = qi < nq ? KEY_NONE : 0;  // padding queries never insert
    }

    // rows of the next step are loaded before this step's work, so a wave
    // always has a step's loads in flight while it counts
    uint4 tn[4];
    {
        const uint64_t row = r0 + g;
#pragma unroll
        for (int i = 0; i < 4; i++) tn[i] = row < r1 ? db[row * 32 + j + 8 * i] : make_uint4(0, 0, 0, 0);
    }
    for (uint64_t base = r0; base < r1; base += kRowsPerStep) {
        const uint64_t row = base + g;
        const bool valid = row < r1;
        uint4 tv[4];
#pragma unroll
        for (int i = 0; i < 4; i++) tv[i] = tn[i];
        const uint64_t nrow = row + kRowsPerStep;
#pragma unroll
        for (int i = 0; i < 4; i++) tn[i] = nrow < r1 ? db[nrow * 32 + j + 8 * i] : make_uint4(0, 0, 0, 0);
        const uint32_t tp = sum8(popc4(tv[0]) + popc4(tv[1]) + popc4(tv[2]) + popc4(tv[3]));
#pragma unroll
        for (int t = 0; t < QT; t++) {
            uint32_t c = popc_and4(tv[0], qv[t][0]) + popc_and4(tv[1], qv[t][1]) + popc_and4(tv[2], qv[t][2]) +
                         popc_and4(tv[3], qv[t][3]);
            c = sum8(c);
            const uint32_t K = (pq[t] - c) * wb[t] + (tp - c) * wa[t];
            const u64 key = valid ? ((u64)K << 32) | (uint32_t)row : KEY_NONE;
            u64 m = ballot(j == 0 && key < thr[t]);
            while (m) {
                const int L = __builtin_ctzll(m);
                m &= m - 1;
                const u64 c2 = readlane64(key, L);
                if (c2 < thr[t]) {
                    list[t] = list_insert(list[t], c2, k);
                    thr[t] = readlane64(list[t], (int)k - 1);
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < QT; t++) {
        const uint32_t qi = qtile * QT + t;
        if (qi < nq && lane < (int)k) part[((uint64_t)qi * n_parts + p) * k + lane] = list[t];
    }
}

// Tiles of 16 queries on the matrix cores.  A wave keeps the 16 queries of
// its tile in registers and streams its slice of rows 16 at a time.  The
// 16 x 16 overlap counts of a group are one chain of 32 FP4 matrix steps
// (expand_a / expand_b of mfma_tile.h): lane l (row or query l % 16, lane
// group g = l / 16) loads the 16-byte pieces 4i + g, i = 0..7, of its row,
// and step 4i + c takes word c of piece i, so the four lane groups of a step
// cover four different words and the 32 steps cover all 128.  One load
// instruction reads 64 contiguous bytes of each of the 16 rows.  Lane l then
// holds the counts of queries 4g .. 4g + 3 against row l % 16; the row's
// popcount is summed over its four lanes.  The per-query k-lists are kept in
// LDS and taken into a register (one entry per lane) only to insert, while
// every lane filters with the current k-th key of its four queries.  Rows
// past the slice's end are read as the slice's last row and never listed.
constexpr int kSmallQ = 16;     // queries per wave (one matrix tile)
constexpr int kSmallRows = 16;  // rows per matrix product

__global__ __launch_bounds__(kBlock) void scan_small_mfma_kernel(const uint4 *__restrict__ db, uint64_t n,
                                                                 const uint4 *__restrict__ q, uint32_t nq,
                                                                 uint32_t k, uint32_t n_qtiles, uint32_t n_parts,
                                                                 uint64_t rows_per_part, u64 *__restrict__ part,
                                                                 const uint32_t *__restrict__ nq_dev) {
    extern __shared__ u64 lists_lds[];  // kWavesPerBlock x kSmallQ x k keys
    const int lane = lane_id();
    const int li = lane & 15, lg = lane >> 4;
    // wave w serves query tile w % n_qtiles over row slice w / n_qtiles, so
    // the waves of a workgroup share their rows when there are several tiles
    const uint32_t wv = threadIdx.x >> 6;
    const uint64_t w = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    const uint32_t qtile = readfirst((uint32_t)(w % n_qtiles));
    const uint32_t p = readfirst((uint32_t)(w / n_qtiles));
    if (p >= n_parts) return;  // whole wave
    if (nq_dev) {
        nq = *nq_dev;  // size given on the device (captured graphs)
        if (qtile * kSmallQ >= nq) return;  // whole wave
    }
    const uint64_t r0 = (uint64_t)p * rows_per_part;
    const uint64_t r1 = r0 + rows_per_part < n ? r0 + rows_per_part : n;
    u64 *wl = lists_lds + (size_t)wv * kSmallQ * k;

    // words of query li taken by this lane's group, and its popcount
    uint32_t qw[32];
    uint32_t s = 0;
    {
        const uint32_t qi = qtile * kSmallQ + li;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint4 v = qi < nq ? q[(uint64_t)qi * 32 + 4 * i + lg] : make_uint4(0, 0, 0, 0);
            qw[4 * i] = v.x;
            qw[4 * i + 1] = v.y;
            qw[4 * i + 2] = v.z;
            qw[4 * i + 3] = v.w;
            s += popc4(v);
        }
    }
    s += (uint32_t)__shfl_xor((int)s, 16);
    s += (uint32_t)__shfl_xor((int)s, 32);  // every lane of column li: |query li|
    // constants of this lane's accumulator rows, queries 4 lg + r
    uint32_t pq[4], wa[4], wb[4];
    u64 thr[4];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        pq[r] = (uint32_t)__shfl((int)s, 4 * lg + r);
        wa[r] = pq[r] > 1 ? pq[r] : 1;
        wb[r] = (QD_BITS - pq[r]) > 1 ? QD_BITS - pq[r] : 1;
        thr[r] = qtile * kSmallQ + 4 * lg + r < nq ? KEY_NONE : 0;  // padding queries never list
    }
    for (int t = 0; t < kSmallQ; t++)
        if (lane < (int)k) wl[t * k + lane] = KEY_NONE;

    auto load = [&](uint64_t base, uint4 (&t)[8]) {
        const uint64_t row = base + li < r1 ? base + li : r1 - 1;
        const uint4 *src = db + row * 32 + lg;
#pragma unroll
        for (int i = 0; i < 8; i++) t[i] = src[4 * i];
    };
    // the next group's rows are loaded before this group's work
    uint4 tn[8];
    load(r0, tn);
    for (uint64_t base = r0; base < r1; base += kSmallRows) {
        uint4 tv[8];
#pragma unroll
        for (int i = 0; i < 8; i++) tv[i] = tn[i];
        if (base + kSmallRows < r1) load(base + kSmallRows, tn);
        mt::v4f acc = {0.f, 0.f, 0.f, 0.f};
        uint32_t tp = 0;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint32_t w4[4] = {tv[i].x, tv[i].y, tv[i].z, tv[i].w};
#pragma unroll
            for (int c = 0; c < 4; c++) {
                tp += __popc(w4[c]);
                // formats 4 = e2m1 for both operands; scales 127 = 2^0
                acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(mt::expand_a(qw[4 * i + c]),
                                                                       mt::expand_b(w4[c]), acc, 4, 4, 0, 127, 0,
                                                                       127);
            }
        }
        tp += (uint32_t)__shfl_xor((int)tp, 16);
        tp += (uint32_t)__shfl_xor((int)tp, 32);  // |row li|
        const uint64_t row = base + li;
        const bool valid = row < r1;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint32_t c = mt::count(acc[r]);
            const uint32_t K = (pq[r] - c) * wb[r] + (tp - c) * wa[r];
            const u64 key = valid ? ((u64)K << 32) | (uint32_t)row : KEY_NONE;
            u64 m = ballot(key < thr[r]);
            while (m) {
                const int L = __builtin_ctzll(m);
                m &= m - 1;
                const uint32_t t = 4 * (L >> 4) + r;  // the query of lane L's row r
                const u64 c2 = readlane64(key, L);
                u64 lst = lane < (int)k ? wl[t * k + lane] : KEY_NONE;
                if (c2 < readlane64(lst, (int)k - 1)) {
                    lst = list_insert(lst, c2, k);
                    if (lane < (int)k) wl[t * k + lane] = lst;
                    const u64 nk = readlane64(lst, (int)k - 1);
                    if (lg == (L >> 4)) thr[r] = nk;  // the lanes whose row r is query t
                }
            }
        }
    }
    for (int t = 0; t < kSmallQ; t++) {
        const uint32_t qi = qtile * kSmallQ + t;
        if (qi < nq && lane < (int)k) part[((uint64_t)qi * n_parts + p) * k + lane] = wl[t * k + lane];
    }
}

// One block per query: exact top k from n_parts sorted lists of k keys, then
// the result rows.  U = the k-th smallest list head bounds the k-th key from
// above (those k heads are k distinct candidates), and only lists whose head
// is <= U (at most k of them: keys are distinct) can hold keys <= U, so at
// most k*k candidates are gathered and sorted.  The lists are first read
// only at their heads, then the qualifying lists' entries all at once.
__global__ __launch_bounds__(kBlock) void merge_emit_kernel(const u64 *__restrict__ part, uint32_t n_parts,
                                                            uint32_t k, const uint64_t *__restrict__ q,
                                                            const uint64_t *__restrict__ db, uint32_t *idx,
                                                            int32_t *missed, int32_t *extra, float *dist,
                                                            const uint32_t *__restrict__ nq_dev) {
    if (nq_dev && blockIdx.x >= *nq_dev) return;  // whole block
    __shared__ u64 heads[kMaxParts];
    __shared__ u64 cand[kMaxCand];
    __shared__ uint32_t qual[QD_MAX_K];
    __shared__ uint32_t ncand, nqual;
    const uint32_t qi = blockIdx.x;
    const u64 *lists = part + (uint64_t)qi * n_parts * k;
    const uint32_t hp = next_pow2(n_parts < 2 ? 2 : n_parts);
    for (uint32_t i = threadIdx.x; i < hp; i += blockDim.x) heads[i] = i < n_parts ? lists[(uint64_t)i * k] : KEY_NONE;
    if (threadIdx.x == 0) ncand = nqual = 0;
    __syncthreads();
    block_bitonic_sort(heads, hp);
    const u64 U = k <= n_parts ? heads[k - 1] : KEY_NONE;
    for (uint32_t p = threadIdx.x; p < n_parts; p += blockDim.x) {
        const u64 h = lists[(uint64_t)p * k];
        if (h != KEY_NONE && h <= U) {
            const uint32_t at = atomicAdd(&nqual, 1u);
            if (at < QD_MAX_K) qual[at] = p;
        }
    }
    __syncthreads();
    const uint32_t nl = nqual < (uint32_t)QD_MAX_K ? nqual : (uint32_t)QD_MAX_K;
    for (uint32_t i = threadIdx.x; i < nl * k; i += blockDim.x) {
        const u64 e = lists[(uint64_t)qual[i / k] * k + i % k];
        if (e != KEY_NONE && e <= U) cand[atomicAdd(&ncand, 1u)] = e;  // a prefix of each list
    }
    __syncthreads();
    const uint32_t nc = ncand;
    const uint32_t cp = next_pow2(nc < 2 ? 2 : nc);
    for (uint32_t i = nc + threadIdx.x; i < cp; i += blockDim.x) cand[i] = KEY_NONE;
    __syncthreads();
    block_bitonic_sort(cand, cp);
    if (threadIdx.x < k) {
        const uint32_t r = threadIdx.x;
        const uint64_t o = (uint64_t)qi * k + r;
        const u64 e = r < nc ? cand[r] : KEY_NONE;
        if (e == KEY_NONE) {
            idx[o] = QD_PAD_IDX;
            missed[o] = -1;
            extra[o] = -1;
            dist[o] = __builtin_inff();
        } else {
            const uint32_t row = (uint32_t)e;
            const uint64_t *qq = q + (uint64_t)qi * QD_WORDS;
            const uint64_t *tt = db + (uint64_t)row * QD_WORDS;
            uint32_t a = 0, b = 0, pqv = 0;
            for (int w = 0; w < QD_WORDS; w++) {
                const uint64_t x = qq[w], y = tt[w];
                a += __popcll(x & ~y);
                b += __popcll(~x & y);
                pqv += __popcll(x);
            }
            const uint32_t wav = pqv > 1 ? pqv : 1;
            const uint32_t wbv = (QD_BITS - pqv) > 1 ? QD_BITS - pqv : 1;
            const uint32_t K = a * wbv + b * wav;
            idx[o] = row;
            missed[o] = (int32_t)a;
            extra[o] = (int32_t)b;
            dist[o] = (float)((double)K / ((double)wav * (double)wbv));
        }
    }
}

__global__ __launch_bounds__(kBlock) void popcount_rows_kernel(const uint4 *__restrict__ db, uint64_t n,
                                                               uint16_t *__restrict__ pop) {
    const int lane = lane_id();
    const int g = lane >> 3, j = lane & 7;
    const uint64_t wave = readfirst((uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t base = wave * kRowsPerStep; base < n; base += nwaves * kRowsPerStep) {
        const uint64_t row = base + g;
        const bool valid = row < n;
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < 4; i++) s += valid ? popc4(db[row * 32 + j + 8 * i]) : 0;
        s = sum8(s);
        if (valid && j == 0) pop[row] = (uint16_t)s;
    }
}

size_t small_lds_bytes(uint32_t k) { return (size_t)kWavesPerBlock * kSmallQ * k * sizeof(u64); }

// Waves of scan_small_mfma_kernel the whole device holds at once, for lists of k.
uint64_t small_mfma_resident_waves(uint32_t k) {
    static std::mutex mu;
    static uint32_t cache[64][QD_MAX_K + 1] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (cache[dev][k] == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, scan_small_mfma_kernel, kBlock, small_lds_bytes(k)) !=
                hipSuccess ||
            nb < 1) {
            (void)hipGetLastError();
            nb = 2;
        }
        cache[dev][k] = (uint32_t)nb * kWavesPerBlock;
    }
    return (uint64_t)cache[dev][k] * device_cus();
}

template <int QT>
void launch_scan(dim3 grid, hipStream_t s, const uint4 *db, uint64_t n, const uint4 *q, uint32_t nq, uint32_t k,
                 uint32_t n_qtiles, uint32_t n_parts, uint64_t rpp, u64 *part, const uint32_t *nq_dev) {
    hipLaunchKernelGGL(scan_topk_kernel<QT>, grid, dim3(kBlock), 0, s, db, n, q, nq, k, n_qtiles, n_parts, rpp, part,
                       nq_dev);
}

}  // namespace

BruteLaunch brute_launch_shape(uint64_t n, uint32_t nq, uint32_t k, uint32_t qt_force, uint32_t parts_force) {
    BruteLaunch sh;
    uint32_t qt = qt_force;
    if (qt == 0)
        qt = nq >= kSmallMfmaMinQueries ? QD_QUERY_TILE_MATRIX
             : nq <= 1                  ? 1
             : nq <= 2                  ? 2
             : nq <= 4                  ? 4
             : nq <= 8                  ? 8
                                        : 16;
    sh.qt = qt;
    const bool matrix = qt == QD_QUERY_TILE_MATRIX;
    const uint32_t per_tile = matrix ? (uint32_t)kSmallQ : qt;
    sh.n_qtiles = (nq + per_tile - 1) / per_tile;
    if (sh.n_qtiles == 0) sh.n_qtiles = 1;
    uint64_t parts = parts_force;
    if (parts == 0) {
        if (matrix) {
            // one wave per resident slot: every wave runs from start to end
            const uint64_t slots = small_mfma_resident_waves(k);
            parts = slots / sh.n_qtiles;
        } else {
            const uint64_t want_waves = (uint64_t)device_cus() * 16;
            parts = (want_waves + sh.n_qtiles - 1) / sh.n_qtiles;
        }
    }
    const uint64_t max_by_rows = (n + 255) / 256;  // at least 256 rows per wave
    if (parts > max_by_rows) parts = max_by_rows;
    if (parts > kMaxParts) parts = kMaxParts;
    if (parts < 1) parts = 1;
    const uint64_t step = matrix ? (uint64_t)kSmallRows : (uint64_t)kRowsPerStep;
    uint64_t rpp = (n + parts - 1) / parts;
    rpp = (rpp + step - 1) / step * step;
    sh.rows_per_part = rpp;
    sh.n_parts = (uint32_t)((n + rpp - 1) / rpp);
    sh.blocks = matrix ? ((uint64_t)sh.n_parts * sh.n_qtiles + kWavesPerBlock - 1) / kWavesPerBlock
                       : (uint64_t)((sh.n_parts + kWavesPerBlock - 1) / kWavesPerBlock) * sh.n_qtiles;
    sh.part_bytes = (size_t)(nq ? nq : 1) * sh.n_parts * k * sizeof(u64);
    return sh;
}

int brute_launch(const BruteLaunch &sh, u64 *part, const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq,
                 const uint32_t *nq_dev, uint32_t k, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra,
                 float *d_dist, hipStream_t s, bool timed) {
    // the dispatch packet holds the grid size in work-items as a 32-bit number
    if (sh.blocks * kBlock > 0xFFFFFFFFull) return fail(QD_ERR_UNSUPPORTED, "launch too large");
    const uint4 *db4 = reinterpret_cast<const uint4 *>(d_db);
    const uint4 *q4 = reinterpret_cast<const uint4 *>(d_q);
    dim3 grid((uint32_t)sh.blocks);
    if (sh.qt == QD_QUERY_TILE_MATRIX) {
        KernelTimer timer(timed ? "wh_scan_small_mfma" : nullptr, s);
        hipLaunchKernelGGL(scan_small_mfma_kernel, grid, dim3(kBlock), small_lds_bytes(k), s, db4, n, q4, nq, k,
                           sh.n_qtiles, sh.n_parts, sh.rows_per_part, part, nq_dev);
    } else {
        KernelTimer timer(timed ? "wh_scan_topk" : nullptr, s);
        switch (sh.qt) {
            case 1: launch_scan<1>(grid, s, db4, n, q4, nq, k, sh.n_qtiles, sh.n_parts, sh.rows_per_part, part, nq_dev); break;
            case 2: launch_scan<2>(grid, s, db4, n, q4, nq, k, sh.n_qtiles, sh.n_parts, sh.rows_per_part, part, nq_dev); break;
            case 4: launch_scan<4>(grid, s, db4, n, q4, nq, k, sh.n_qtiles, sh.n_parts, sh.rows_per_part, part, nq_dev); break;
            case 8: launch_scan<8>(grid, s, db4, n, q4, nq, k, sh.n_qtiles, sh.n_parts, sh.rows_per_part, part, nq_dev); break;
            default: launch_scan<16>(grid, s, db4, n, q4, nq, k, sh.n_qtiles, sh.n_parts, sh.rows_per_part, part, nq_dev); break;
        }
    }
    QD_HIP_CHECK(hipGetLastError());
    {
        KernelTimer timer(timed ? "topk_merge" : nullptr, s);
        hipLaunchKernelGGL(merge_emit_kernel, dim3(nq), dim3(kBlock), 0, s, part, sh.n_parts, k, d_q, d_db, d_idx,
                           d_missed, d_extra, d_dist, nq_dev);
    }
    QD_HIP_CHECK(hipGetLastError());
    return QD_OK;
}

int merge_launch(const u64 *part, uint32_t n_parts, uint32_t k, const uint64_t *d_q, const uint64_t *d_db,
                 uint32_t nq, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, hipStream_t s) {
    if (n_parts < 1 || n_parts > kMaxParts) return fail(QD_ERR_INVALID, "%u lists per query outside 1..%u", n_parts,
                                                        kMaxParts);
    KernelTimer timer("topk_merge", s);
    hipLaunchKernelGGL(merge_emit_kernel, dim3(nq), dim3(kBlock), 0, s, part, n_parts, k, d_q, d_db, d_idx, d_missed,
                       d_extra, d_dist, nullptr);
    QD_HIP_CHECK(hipGetLastError());
    return QD_OK;
}

int knn_bruteforce_mfma(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                        uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream);

int popcount_rows_launch(const uint64_t *d_db, uint64_t n, uint16_t *d_pop, hipStream_t s) {
    if (n == 0) return QD_OK;
    uint64_t waves = (n + kRowsPerStep - 1) / kRowsPerStep;
    uint64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    const uint64_t cap = (uint64_t)device_cus() * 32;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(popcount_rows_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, s,
                       reinterpret_cast<const uint4 *>(d_db), n, d_pop);
    QD_HIP_CHECK(hipGetLastError());
    return QD_OK;
}

// Batches of at least kMfmaMinQueries queries over at least kMfmaMinRows
// rows use the matrix-core path (the overlap counts are then a dense
// contraction).

int knn_bruteforce_impl(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                        uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream,
                        uint32_t qt_force, uint32_t parts_force) {
    if (k < 1 || k > QD_MAX_K) return fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
    if (n < 1 || n > QD_MAX_ROWS) return fail(QD_ERR_INVALID, "n=%llu outside 1..%llu", (u64)n, (u64)QD_MAX_ROWS);
    if (nq == 0) return QD_OK;
    if (!d_db || !d_q || !d_idx || !d_missed || !d_extra || !d_dist) return fail(QD_ERR_INVALID, "null pointer");
    if (!aligned16(d_db) || !aligned16(d_q)) return fail(QD_ERR_INVALID, "descriptor arrays must be 16-byte aligned");
    if (qt_force && qt_force != 1 && qt_force != 2 && qt_force != 4 && qt_force != 8 && qt_force != 16 &&
        qt_force != QD_QUERY_TILE_MATRIX)
        return fail(QD_ERR_INVALID, "query tile %u not in {1,2,4,8,16,QD_QUERY_TILE_MATRIX}", qt_force);
    if (qt_force == 0 && parts_force == 0 && nq >= kMfmaMinQueries && n >= kMfmaMinRows) {
        const int rc = knn_bruteforce_mfma(d_db, n, d_q, nq, k, d_idx, d_missed, d_extra, d_dist, stream);
        if (rc != QD_ERR_UNSUPPORTED) return rc;
        clear_error();
    }
    hipStream_t s = (hipStream_t)stream;
    const BruteLaunch sh = brute_launch_shape(n, nq, k, qt_force, parts_force);
    u64 *part = nullptr;
    QD_HIP_CHECK(hipMallocAsync((void **)&part, sh.part_bytes, s));
    const int rc = brute_launch(sh, part, d_db, n, d_q, nq, nullptr, k, d_idx, d_missed, d_extra, d_dist, s);
    hipError_t e2 = hipFreeAsync(part, s);
    if (rc != QD_OK) return rc;
    if (e2 != hipSuccess) return fail(QD_ERR_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e2));
    return QD_OK;
}

}  // namespace qd

extern "C" int qd_popcount_rows(const uint64_t *d_db, uint64_t n, uint16_t *d_pop, void *stream) {
    using namespace qd;
    if (n == 0) return QD_OK;
    if (!d_db || !d_pop) return fail(QD_ERR_INVALID, "null pointer");
    if (!aligned16(d_db)) return fail(QD_ERR_INVALID, "descriptor array must be 16-byte aligned");
    return popcount_rows_launch(d_db, n, d_pop, (hipStream_t)stream);
}

extern "C" int qd_knn_bruteforce(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                                 uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist,
                                 void *stream) {
    return qd::knn_bruteforce_impl(d_db, n, d_q, nq, k, d_idx, d_missed, d_extra, d_dist, stream, 0, 0);
}

// Same search with an explicit launch shape: query tile (1,2,4,8,16; 0 =
// automatic) and number of row slices per tile (0 = automatic).  Used by the
// autotuner and by tests that check results do not depend on the shape.
extern "C" int qd_knn_bruteforce_shaped(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq,
                                        uint32_t k, uint32_t query_tile, uint32_t row_parts, uint32_t *d_idx,
                                        int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream) {
    return qd::knn_bruteforce_impl(d_db, n, d_q, nq, k, d_idx, d_missed, d_extra, d_dist, stream, query_tile,
                                   row_parts);
}

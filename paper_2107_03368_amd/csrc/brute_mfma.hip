// Large-batch sequential search on the matrix cores.
//
// For many queries the overlap counts C[q][t] = popcount(q AND t) of Eq. 1
// form a dense {0,1} matrix product C = Q T^T over the 4096 bit positions;
// they are computed by the shared 256 x 256 tile (mfma_tile.h), one block per
// (query tile, row tile).
//
// Selection: a first sequential search over a sample of the rows gives each
// query an upper bound U_q on its k-th key (the sample's k-th key: those k
// rows are candidates too); for a large sample that search runs on the
// matrix cores as well, with its own smaller sample.  The matrix pass keeps every (row, key) with
// key <= U_q in a per-query candidate buffer; the exact top k are all among
// them.  A final kernel sorts each query's candidates and writes the
// results; queries whose buffer overflowed are searched again by the
// register-tiled scan, so the result is exact in every case.
#include <algorithm>
#include <vector>

#include "mfma_tile.h"
#include "qd_device.h"
#include "qd_internal.h"
#include "qd_launch.h"

namespace qd {

int knn_bruteforce_impl(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                        uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream,
                        uint32_t qt_force, uint32_t parts_force);
int popcount_rows_launch(const uint64_t *d_db, uint64_t n, uint16_t *d_pop, hipStream_t s);

namespace {

constexpr int kBlock = 256;
constexpr int MQ = mt::MA;        // queries per block
constexpr int MR = mt::MB;        // rows per block
constexpr uint32_t kCap = 8192;   // candidate slots per query

// Tiles of 256 queries x 256 rows in a persistent grid of G workgroups.
// When the query tiles and G split evenly over the 8 XCDs, the workgroups of
// XCD c (x % 8 == c) run the query tiles c, c + 8, ... against every row
// tile, taking (row tile, query tile) pairs in order from a counter of their
// own; otherwise all workgroups share one counter over all tiles.  Claimed in
// order, as the hardware would dispatch one workgroup per tile, the few
// tiles of a row tile run at about the same time, so each L2 fetches a row
// tile once and keeps its XCD's queries.  The tiles are streamed: the next
// tile's first two windows are staged during the current tile's last two and
// its metadata is loaded during the current tile, so the matrix cores do not
// wait for a tile to start.
__global__ __launch_bounds__(mt::kThreads) void scan_mfma_kernel(const uint4 *__restrict__ db, uint64_t n,
                                                                 const uint4 *__restrict__ q, uint32_t nq,
                                                                 const uint16_t *__restrict__ tpop,
                                                                 const uint16_t *__restrict__ qpop,
                                                                 const u64 *__restrict__ thr, uint32_t n_qtiles,
                                                                 uint32_t *__restrict__ tctr,
                                                                 uint32_t *__restrict__ cnt, u64 *__restrict__ cand,
                                                                 const uint32_t *__restrict__ nq_dev) {
    __shared__ mt::Smem sm;
    if (nq_dev) {  // the batch's size on the device (captured graphs): fewer query tiles
        nq = min(nq, *nq_dev);
        n_qtiles = (nq + MQ - 1) / MQ;
    }
    // Per tile row (queries 0..255, then rows): |q| or |t|, and for queries the
    // candidate bound and the least overlap that can reach it (the row half of
    // these two is written but not read, so every thread stores alike).  Two
    // sets: the current tile's, and the next tile's, written during the current tile.
    __shared__ uint32_t s_p[2][MQ + MR];
    __shared__ u64 s_th[2][MQ + MR];
    __shared__ __align__(16) float s_cmin[2][MQ + MR];
    // per wave: the tile's passing (query, key, row) entries, appended in order
    // and written out together, so the candidate slots' atomics overlap
    // instead of waiting one after another
    constexpr uint32_t kQueue = 320;  // room for one (a, rr) group's 256 entries past the flush mark
    __shared__ uint32_t s_cq[mt::kThreads / 64][kQueue][3];
    const int r = mt::own_row();
    const bool arow = r < MQ;  // the same in a whole wave
    // this thread's row of tile `tile` and the index of its metadata (always in bounds)
    struct Part {
        const uint4 *row;
        bool ok;
        uint64_t at;  // query or row index whose |q| / bound or |t| this thread loads
    };
    // the claimable tiles: j = 0 .. count - 1 -> (query tile, row tile)
    const uint64_t n_rtiles = (n + MR - 1) / MR, G = gridDim.x, x = blockIdx.x;
    const bool by_xcd = n_qtiles % mt::kXcds == 0 && G % mt::kXcds == 0;
    const uint32_t qper = by_xcd ? n_qtiles / mt::kXcds : n_qtiles;  // query tiles per row tile of a counter
    const uint32_t cx = by_xcd ? (uint32_t)(x % mt::kXcds) : 0;
    const uint64_t count = n_rtiles * qper;
    uint32_t *ctr = tctr + cx;
    auto coords = [&](uint64_t j, uint32_t &qt, uint64_t &rt) {
        rt = j / qper;
        qt = (by_xcd ? cx : 0) + (by_xcd ? mt::kXcds : 1) * (uint32_t)(j % qper);
    };
    auto part_of = [&](uint64_t j) {
        uint32_t qt;
        uint64_t rt;
        coords(j, qt, rt);
        const uint32_t q0 = qt * MQ;
        const uint64_t t0 = rt * MR;
        Part p;
        if (arow) {
            p.ok = q0 + r < nq;
            p.at = p.ok ? q0 + r : 0;
            p.row = q + p.at * 32;
        } else {
            p.ok = t0 + (r - MQ) < n;
            p.at = p.ok ? t0 + (r - MQ) : 0;
            p.row = db + p.at * 32;
        }
        return p;
    };
    // loads of a part's metadata: issued one window before they are used
    uint32_t lp;  // |q| or |t|
    u64 lt;       // the query's bound
    auto issue = [&](const Part &p) {
        lp = arow ? qpop[p.at] : tpop[p.at];
        lt = thr[arow ? p.at : 0];
    };
    auto publish = [&](const Part &p, int h) {  // read after the next barrier; no branch
        const uint32_t pv = p.ok ? lp : 0;
        const u64 th = p.ok && arow ? lt : 0;
        // K = |q|*wB + |t|*wA - C*(wA + wB) >= |q|*wB - C*(wA + wB): a row
        // with C*(wA + wB) below X = |q|*wB - (the bound's key) has K above
        // it.  wA + wB is 4096, or 4097 when |q| is 0 or 4096, so a row can
        // only pass with C >= ceil(X / 4097) = cmin (a division by a
        // constant, a multiply and a shift; the exact key test follows)
        const uint32_t wb = (QD_BITS - pv) > 1 ? QD_BITS - pv : 1;
        const uint32_t P = __umul24(pv, wb), Kb = (uint32_t)(th >> 32);  // |q|*wB <= 2^22
        const uint32_t X = P - (P < Kb ? P : Kb);                          // max(P - Kb, 0)
        const uint32_t cmin = (X + 4096u) / 4097u;
        s_p[h][r] = pv;
        s_th[h][r] = th;
        s_cmin[h][r] = p.ok ? (float)cmin : 1e30f;
    };
    __shared__ uint32_t s_claim[2];
    if (r == 0) {
        s_claim[0] = atomicAdd(ctr, 1u);
        s_claim[1] = atomicAdd(ctr, 1u);
    }
    __syncthreads();
    uint64_t tile = s_claim[0], tn = s_claim[1];  // this tile, the next
    if (tile >= count) return;  // whole workgroup
    Part cur = part_of(tile);
    issue(cur);
    int h = 0;  // the current tile's metadata set
    publish(cur, h);
    mt::Stream st;
    mt::stream_begin(cur.row, !cur.ok, sm, st);  // its barrier also publishes the metadata
    for (;;) {
        const bool more = tn < count;
        const Part nx = part_of(more ? tn : tile);
        // the tile after next: claimed now, taken after this tile
        uint32_t claim = 0;
        if (r == 0 && more) claim = atomicAdd(ctr, 1u);
        const bool nzero = !more || !nx.ok;
        mt::v4f acc[8][4];
        // the next tile's metadata: loaded after every window and stored after
        // the next one (a window later, so no store waits for its load) into
        // the other set, which the previous tile's epilogue finished reading;
        // the same code after every window keeps the window loop one block
        // (after window 0 the set receives this tile's metadata, overwritten
        // after window 1)
        mt::stream_tile(cur.row, !cur.ok, nx.row, nzero, sm, st, acc, [&](int) {
            publish(nx, h ^ 1);
            issue(nx);
        });
        uint32_t qt;
        uint64_t rt;
        coords(tile, qt, rt);
        const uint32_t q0 = qt * MQ;
        const uint64_t t0 = rt * MR;

        // epilogue: keys of this lane's 32 queries x 4 rows
        const int lane = r & 63;
        uint32_t (*cq)[3] = s_cq[r >> 6];
        uint32_t nqe = 0;  // entries in this wave's queue (the same in every lane)
        auto flush = [&]() {
            for (uint32_t e = lane; e < nqe; e += 64) {
                const uint32_t qi = cq[e][0];
                const uint32_t pos = atomicAdd(&cnt[qi], 1u);
                if (pos < kCap) cand[(uint64_t)qi * kCap + pos] = ((u64)cq[e][1] << 32) | cq[e][2];
            }
            nqe = 0;
        };
        // this lane's four rows: their popcounts and whether they exist, the
        // same for every query group of the tile
        uint32_t tpv[4];
        bool rv[4];
#pragma unroll
        for (int b = 0; b < 4; b++) {
            tpv[b] = s_p[h][MQ + mt::acc_brow(b)];
            rv[b] = t0 + (uint64_t)mt::acc_brow(b) < n;
        }
        // a group's four query slots are consecutive: their least overlaps
        // are one 16-byte read, issued a group ahead of the test
        float4 cm_next = *reinterpret_cast<const float4 *>(&s_cmin[h][mt::acc_arow(0, 0)]);
#pragma unroll
        for (int a = 0; a < 8; a++) {
            // one group of queries at a time, so their metadata loads stay next to their use
            __builtin_amdgcn_sched_barrier(0);
            const float4 cm = cm_next;
            if (a < 7) cm_next = *reinterpret_cast<const float4 *>(&s_cmin[h][mt::acc_arow(a + 1, 0)]);
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                const int ai = mt::acc_arow(a, rr);
                // test this lane's 4 rows of the query at once (most miss by far)
                const float mx = fmaxf(fmaxf(acc[a][0][rr], acc[a][1][rr]), fmaxf(acc[a][2][rr], acc[a][3][rr]));
                const uint32_t qi = q0 + ai;
                // (a slot past the last query has least overlap 1e30)
                const bool act = mx >= (rr == 0 ? cm.x : rr == 1 ? cm.y : rr == 2 ? cm.z : cm.w);
                if (ballot(act) == 0) continue;
                const uint32_t pq = s_p[h][ai];
                const uint32_t wa = pq > 1 ? pq : 1, wb = (QD_BITS - pq) > 1 ? QD_BITS - pq : 1;
                const u64 th = s_th[h][ai];
                // K = |q|*wB + |t|*wA - C*(wA + wB): the first two terms per
                // row once per group, then one 24-bit multiply-add per pair
                // (C <= 4096 and wA + wB <= 4097; every term below 2^26)
                const uint32_t P = __umul24(pq, wb);
                const int nsw = -(int)(wa + wb);
                uint32_t PT[4];
#pragma unroll
                for (int b = 0; b < 4; b++) PT[b] = P + __umul24(tpv[b], wa);
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const uint64_t t = t0 + mt::acc_brow(b);
                    const uint32_t C = mt::count(acc[a][b][rr]);
                    const uint32_t K = (uint32_t)((int)PT[b] + __mul24((int)C, nsw));
                    const u64 key = ((u64)K << 32) | (uint32_t)t;
                    const bool pass = act & rv[b] & (key <= th);  // no short-circuit: no branch per test
                    const u64 pm = ballot(pass);
                    if (pass) {
                        const uint32_t e = nqe + lanes_below(pm);
                        cq[e][0] = qi;
                        cq[e][1] = K;
                        cq[e][2] = (uint32_t)t;
                    }
                    nqe += (uint32_t)__popcll(pm);
                }
                if (nqe > kQueue - 256) flush();  // the next group adds at most 4 x 64
            }
        }
        flush();
        if (r == 0) s_claim[0] = claim;
        __syncthreads();  // this set is rewritten during the next tile
        if (!more) break;
        h ^= 1;
        cur = nx;
        tile = tn;
        tn = s_claim[0];
    }
}

// One block per query: sort the candidates (<= kCap), write the first k.
// Overflowed queries are left for the fallback and flagged in `redo`.
__global__ __launch_bounds__(kBlock) void select_emit_kernel(const uint32_t *__restrict__ cnt,
                                                             const u64 *__restrict__ cand, uint32_t k,
                                                             const uint64_t *__restrict__ q,
                                                             const uint64_t *__restrict__ db, uint32_t *idx,
                                                             int32_t *missed, int32_t *extra, float *dist,
                                                             uint32_t *redo, uint32_t *n_redo,
                                                             const uint32_t *__restrict__ nq_dev) {
    __shared__ u64 keys[kCap];
    const uint32_t qi = blockIdx.x;
    if (nq_dev && qi >= *nq_dev) return;  // whole block
    const uint32_t m = cnt[qi];
    if (m > kCap) {
        if (threadIdx.x == 0) redo[atomicAdd(n_redo, 1u)] = qi;
        return;
    }
    const uint32_t np = next_pow2(m < 2 ? 2 : m);
    for (uint32_t i = threadIdx.x; i < np; i += kBlock) keys[i] = i < m ? cand[(uint64_t)qi * kCap + i] : KEY_NONE;
    __syncthreads();
    block_bitonic_sort(keys, np);
    if (threadIdx.x < k) {
        const uint32_t r = threadIdx.x;
        const uint64_t o = (uint64_t)qi * k + r;
        const u64 e = r < m ? keys[r] : KEY_NONE;
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
            idx[o] = row;
            missed[o] = (int32_t)a;
            extra[o] = (int32_t)b;
            dist[o] = (float)((double)(a * wbv + b * wav) / ((double)wav * (double)wbv));
        }
    }
}

// thr[q] = the k-th sample key, from the sample search's outputs
__global__ void sample_threshold_kernel(const uint32_t *__restrict__ idx, const int32_t *__restrict__ missed,
                                        const int32_t *__restrict__ extra, const uint16_t *__restrict__ qpop,
                                        uint32_t nq, uint32_t k, u64 *__restrict__ thr) {
    const uint32_t qi = blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    const uint64_t o = (uint64_t)qi * k + (k - 1);
    const uint32_t pq = qpop[qi];
    const uint32_t wa = pq > 1 ? pq : 1, wb = (QD_BITS - pq) > 1 ? QD_BITS - pq : 1;
    thr[qi] = idx[o] == QD_PAD_IDX ? KEY_NONE
                                   : ((u64)((uint32_t)missed[o] * wb + (uint32_t)extra[o] * wa) << 32) | idx[o];
}

// The overflowed queries (list[0 .. *m)) gathered into consecutive rows.
__global__ void gather_queries_kernel(const uint4 *__restrict__ q, const uint32_t *__restrict__ list,
                                      const uint32_t *__restrict__ m, uint4 *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *m * 32) out[i] = q[(uint64_t)list[i >> 5] * 32 + (i & 31)];
}

// Their results back to their queries' rows.
template <class T>
__global__ void scatter_rows_kernel(const T *__restrict__ src, const uint32_t *__restrict__ list,
                                    const uint32_t *__restrict__ m, uint32_t k, T *__restrict__ dst) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *m * k) dst[(uint64_t)list[i / k] * k + (i % k)] = src[i];
}

// Clears n words (a kernel, not a memset node, so a captured graph replays it reliably).
__global__ void zero_words_kernel(uint32_t *__restrict__ p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}


// Rows of the threshold sample of a matrix-core pass over n rows: about
// k*n/1024, so about 1,024 candidates per query are expected.
inline uint64_t sample_rows(uint64_t n, uint32_t k) { return std::max<uint64_t>((uint64_t)k * 64, (n * k + 1023) / 1024); }
inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

// Level l searches rows [0, rows[l]) for the batch; every level but the last
// is a matrix-core pass whose thresholds come from level l + 1 over its
// sample (a prefix of the rows); the last level is the register-tiled scan.
MfmaLayout mfma_layout(uint64_t n, uint32_t nq, uint32_t k) {
    MfmaLayout L;
    uint64_t rows = n;
    // level 0 is a matrix-core pass (the caller checked); deeper ones when big enough
    for (;;) {
        L.rows.push_back(rows);
        const uint64_t smp = sample_rows(rows, k);
        const bool mfma = L.rows.size() == 1 ? smp * 4 <= rows
                                             : nq >= kMfmaMinQueries && rows >= kMfmaMinRows && smp * 4 <= rows;
        if (!mfma || L.rows.size() == kMaxLevels) break;
        rows = smp;
    }
    const size_t levels = L.rows.size();
    L.base = brute_launch_shape(L.rows.back(), nq, k, 0, 0);
    size_t fb_part = 0;
    for (size_t l = 0; l + 1 < levels; l++) {
        L.fb[l] = brute_launch_shape(L.rows[l], nq, k, 16, 0);
        fb_part = std::max(fb_part, L.fb[l].part_bytes);
    }
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o += al256(b);
        return at;
    };
    L.tpop = take(n * 2);
    L.qpop = take((size_t)nq * 2);
    L.cnt = take((size_t)nq * 4);
    L.cand = take((size_t)nq * kCap * 8);
    L.redo = take((size_t)nq * 4);
    L.ctr = take(4 * (1 + mt::kXcds));
    for (size_t l = 0; l + 1 < levels; l++) {
        L.thr[l] = take((size_t)nq * 8);
        L.smp[l] = take((size_t)nq * k * 16);  // the sample's results: level l + 1's outputs
    }
    L.base_part = take(L.base.part_bytes);
    L.gq = take((size_t)nq * 512);
    L.fbr = take((size_t)nq * k * 16);
    L.fb_part = take(fb_part);
    L.bytes = o;
    return L;
}

// Level l of the search of nq queries (nq_dev: their count on the device,
// nullable) into the four result arrays; nothing waits for the host.
static int mfma_level(const MfmaLayout &L, size_t l, char *ws, const uint64_t *d_db, const uint64_t *d_q, uint32_t nq,
                      const uint32_t *nq_dev, uint32_t k, uint32_t *idx, int32_t *mis, int32_t *ext, float *dist,
                      hipStream_t s) {
    const uint64_t n = L.rows[l];
    const bool top = l == 0;
    if (l + 1 == L.rows.size())  // the register-tiled scan
        return brute_launch(L.base, reinterpret_cast<u64 *>(ws + L.base_part), d_db, n, d_q, nq, nq_dev, k, idx, mis,
                            ext, dist, s);
    // thresholds from the sample: level l + 1 over the first rows
    uint32_t *sidx = (uint32_t *)(ws + L.smp[l]);
    int32_t *smis = (int32_t *)(sidx + (size_t)nq * k), *sext = smis + (size_t)nq * k;
    float *sdist = (float *)(sext + (size_t)nq * k);
    int rc = mfma_level(L, l + 1, ws, d_db, d_q, nq, nq_dev, k, sidx, smis, sext, sdist, s);
    if (rc != QD_OK) return rc;
    const uint16_t *tpop = (const uint16_t *)(ws + L.tpop), *qpop = (const uint16_t *)(ws + L.qpop);
    u64 *thr = (u64 *)(ws + L.thr[l]);
    uint32_t *cnt = (uint32_t *)(ws + L.cnt), *redo = (uint32_t *)(ws + L.redo), *ctr = (uint32_t *)(ws + L.ctr);
    uint32_t *n_redo = ctr, *tctr = ctr + 1;  // overflow count, one tile counter per XCD
    u64 *cand = (u64 *)(ws + L.cand);
    hipLaunchKernelGGL(sample_threshold_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, sidx, smis, sext, qpop, nq, k,
                       thr);
    hipLaunchKernelGGL(zero_words_kernel, dim3((uint32_t)std::min<uint64_t>((nq + 255) / 256, 1024)), dim3(256), 0, s,
                       cnt, (uint64_t)nq);
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, ctr, (uint64_t)(1 + mt::kXcds));
    const uint32_t n_qtiles = (nq + MQ - 1) / MQ;
    const uint64_t n_rtiles = (n + MR - 1) / MR;
    {
        KernelTimer timer(top ? "wh_scan_mfma" : "wh_scan_mfma_sample", s);
        // persistent: one workgroup per CU (the tile's LDS and registers leave room for one)
        const uint64_t grid = std::min<uint64_t>(n_qtiles * n_rtiles, (uint64_t)device_cus());
        hipLaunchKernelGGL(scan_mfma_kernel, dim3((uint32_t)grid), dim3(mt::kThreads), 0, s,
                           reinterpret_cast<const uint4 *>(d_db), n, reinterpret_cast<const uint4 *>(d_q), nq, tpop,
                           qpop, thr, n_qtiles, tctr, cnt, cand, nq_dev);
    }
    {
        KernelTimer timer(top ? "topk_select" : "topk_select_sample", s);
        hipLaunchKernelGGL(select_emit_kernel, dim3(nq), dim3(kBlock), 0, s, cnt, cand, k, d_q, d_db, idx, mis, ext,
                           dist, redo, n_redo, nq_dev);
    }
    // queries whose candidate buffer overflowed: searched again by the
    // register-tiled scan over this level's rows; their count stays on the
    // device, so an empty fallback only costs launches that find no work
    uint4 *gq = (uint4 *)(ws + L.gq);
    uint32_t *ri = (uint32_t *)(ws + L.fbr);
    int32_t *rm = (int32_t *)(ri + (size_t)nq * k), *rx = rm + (size_t)nq * k;
    float *rd = (float *)(rx + (size_t)nq * k);
    hipLaunchKernelGGL(gather_queries_kernel, dim3((nq * 32 + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<const uint4 *>(d_q), redo, n_redo, gq);
    rc = brute_launch(L.fb[l], reinterpret_cast<u64 *>(ws + L.fb_part), d_db, n, reinterpret_cast<const uint64_t *>(gq),
                      nq, n_redo, k, ri, rm, rx, rd, s, /*timed=*/false);
    if (rc != QD_OK) return rc;
    const dim3 g((nq * k + 255) / 256);
    hipLaunchKernelGGL(scatter_rows_kernel<uint32_t>, g, dim3(256), 0, s, ri, redo, n_redo, k, idx);
    hipLaunchKernelGGL(scatter_rows_kernel<int32_t>, g, dim3(256), 0, s, rm, redo, n_redo, k, mis);
    hipLaunchKernelGGL(scatter_rows_kernel<int32_t>, g, dim3(256), 0, s, rx, redo, n_redo, k, ext);
    hipLaunchKernelGGL(scatter_rows_kernel<float>, g, dim3(256), 0, s, rd, redo, n_redo, k, dist);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QD_ERR_DEVICE, "matrix-core scan: %s", hipGetErrorString(e));
    return QD_OK;
}

int mfma_run(const MfmaLayout &L, char *ws, const uint64_t *d_db, const uint64_t *d_q, uint32_t nq,
             const uint32_t *nq_dev, uint32_t k, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist,
             hipStream_t s) {
    int rc = popcount_rows_launch(d_db, L.rows[0], (uint16_t *)(ws + L.tpop), s);
    if (rc == QD_OK) rc = popcount_rows_launch(d_q, nq, (uint16_t *)(ws + L.qpop), s);
    if (rc != QD_OK) return rc;
    return mfma_level(L, 0, ws, d_db, d_q, nq, nq_dev, k, d_idx, d_missed, d_extra, d_dist, s);
}

bool mfma_eligible(uint64_t n, uint32_t nq, uint32_t k) {
    return nq >= kMfmaMinQueries && n >= kMfmaMinRows && sample_rows(n, k) * 4 <= n;
}

// Matrix-core path for large batches; returns QD_ERR_UNSUPPORTED when the
// shape is not worth it (the caller then uses the register-tiled scan).
int knn_bruteforce_mfma(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                        uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (sample_rows(n, k) * 4 > n) return QD_ERR_UNSUPPORTED;
    const MfmaLayout L = mfma_layout(n, nq, k);
    char *ws = nullptr;
    QD_HIP_CHECK(hipMallocAsync((void **)&ws, L.bytes, s));
    const int rc = mfma_run(L, ws, d_db, d_q, nq, nullptr, k, d_idx, d_missed, d_extra, d_dist, s);
    (void)hipFreeAsync(ws, s);
    return rc;
}

}  // namespace qd

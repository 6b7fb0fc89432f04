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
thread_local int g_sample_depth = 0;  // > 0 inside the search of a threshold sample

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
                                                                 uint32_t *__restrict__ cnt, u64 *__restrict__ cand) {
    __shared__ mt::Smem sm;
    // Per tile row (queries 0..255, then rows): |q| or |t|, and for queries the
    // candidate bound and the least overlap that can reach it (the row half of
    // these two is written but not read, so every thread stores alike).  Two
    // sets: the current tile's, and the next tile's, written during the current tile.
    __shared__ uint32_t s_p[2][MQ + MR];
    __shared__ u64 s_th[2][MQ + MR];
    __shared__ float s_cmin[2][MQ + MR];
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
#pragma unroll
        for (int a = 0; a < 8; a++) {
            // one group of queries at a time, so their metadata loads stay next to their use
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                const int ai = mt::acc_arow(a, rr);
                // test this lane's 4 rows of the query at once (most miss by far)
                const float mx = fmaxf(fmaxf(acc[a][0][rr], acc[a][1][rr]), fmaxf(acc[a][2][rr], acc[a][3][rr]));
                const uint32_t qi = q0 + ai;
                const bool act = mx >= s_cmin[h][ai] && qi < nq;
                if (ballot(act) == 0) continue;
                const uint32_t pq = s_p[h][ai];
                const uint32_t wa = pq > 1 ? pq : 1, wb = (QD_BITS - pq) > 1 ? QD_BITS - pq : 1;
                const u64 th = s_th[h][ai];
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const int bi = mt::acc_brow(b);
                    const uint64_t t = t0 + bi;
                    const uint32_t C = mt::count(acc[a][b][rr]);
                    const uint32_t K = (pq - C) * wb + (s_p[h][MQ + bi] - C) * wa;
                    const u64 key = ((u64)K << 32) | (uint32_t)t;
                    const bool pass = act && t < n && key <= th;
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
                                                             uint32_t *redo, uint32_t *n_redo) {
    __shared__ u64 keys[kCap];
    const uint32_t qi = blockIdx.x;
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

__global__ void gather_queries_kernel(const uint4 *__restrict__ q, const uint32_t *__restrict__ list, uint32_t m,
                                      uint4 *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m * 32) out[i] = q[(uint64_t)list[i >> 5] * 32 + (i & 31)];
}

template <class T>
__global__ void scatter_rows_kernel(const T *__restrict__ src, const uint32_t *__restrict__ list, uint32_t m,
                                    uint32_t k, T *__restrict__ dst) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m * k) dst[(uint64_t)list[i / k] * k + (i % k)] = src[i];
}

}  // namespace

// Matrix-core path for large batches; returns QD_ERR_UNSUPPORTED when the
// shape is not worth it (the caller then uses the register-tiled scan).
int knn_bruteforce_mfma(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                        uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    // sample: about k*n/1024 rows, so about 1,024 candidates per query are expected
    uint64_t sample = std::max<uint64_t>((uint64_t)k * 64, (n * k + 1023) / 1024);
    if (sample * 4 > n) return QD_ERR_UNSUPPORTED;
    const uint32_t n_qtiles = (nq + MQ - 1) / MQ;
    const uint64_t n_rtiles = (n + MR - 1) / MR;
    // scratch: tpop n*2 | qpop nq*2 | thr nq*8 | cnt nq*4 | cand nq*cap*8 | sample outputs nq*k*16 | redo nq*4+4
    const size_t a_tpop = 0, a_qpop = a_tpop + (n * 2 + 255) / 256 * 256;
    const size_t a_thr = a_qpop + ((size_t)nq * 2 + 255) / 256 * 256;
    const size_t a_cnt = a_thr + (size_t)nq * 8;
    const size_t a_cand = a_cnt + ((size_t)nq * 4 + 255) / 256 * 256;
    const size_t a_smp = a_cand + (size_t)nq * kCap * 8;
    const size_t a_redo = a_smp + (size_t)nq * k * 16;
    const size_t bytes = a_redo + (size_t)nq * 4 + 256;
    char *ws = nullptr;
    QD_HIP_CHECK(hipMallocAsync((void **)&ws, bytes, s));
    uint16_t *tpop = (uint16_t *)(ws + a_tpop), *qpop = (uint16_t *)(ws + a_qpop);
    u64 *thr = (u64 *)(ws + a_thr);
    uint32_t *cnt = (uint32_t *)(ws + a_cnt);
    u64 *cand = (u64 *)(ws + a_cand);
    uint32_t *sidx = (uint32_t *)(ws + a_smp);
    int32_t *smis = (int32_t *)(sidx + (size_t)nq * k), *sext = smis + (size_t)nq * k;
    float *sdist = (float *)(sext + (size_t)nq * k);
    uint32_t *redo = (uint32_t *)(ws + a_redo);
    uint32_t *n_redo = redo + nq;
    auto done = [&](int rc) {
        (void)hipFreeAsync(ws, s);
        return rc;
    };
    int rc = popcount_rows_launch(d_db, n, tpop, s);
    if (rc == QD_OK) rc = popcount_rows_launch(d_q, nq, qpop, s);
    if (rc != QD_OK) return done(rc);
    // thresholds from the first `sample` rows (large samples take this same
    // path, with a sample of their own; its launches are timed apart)
    ++g_sample_depth;
    rc = knn_bruteforce_impl(d_db, sample, d_q, nq, k, sidx, smis, sext, sdist, stream, 0, 0);
    --g_sample_depth;
    if (rc != QD_OK) return done(rc);
    hipLaunchKernelGGL(sample_threshold_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, sidx, smis, sext, qpop, nq, k,
                       thr);
    uint32_t *tctr = n_redo + 1;  // one tile counter per XCD (in the last 256 bytes)
    if (hipMemsetAsync(cnt, 0, (size_t)nq * 4, s) != hipSuccess ||
        hipMemsetAsync(n_redo, 0, 4 * (1 + mt::kXcds), s) != hipSuccess)
        return done(fail(QD_ERR_DEVICE, "memset"));
    {
        KernelTimer timer(g_sample_depth ? "wh_scan_mfma_sample" : "wh_scan_mfma", s);
        // persistent: one workgroup per CU (the tile's LDS and registers leave room for one)
        const uint64_t grid = std::min<uint64_t>(n_qtiles * n_rtiles, (uint64_t)device_cus());
        hipLaunchKernelGGL(scan_mfma_kernel, dim3((uint32_t)grid), dim3(mt::kThreads), 0, s,
                           reinterpret_cast<const uint4 *>(d_db), n, reinterpret_cast<const uint4 *>(d_q), nq, tpop,
                           qpop, thr, n_qtiles, tctr, cnt, cand);
    }
    {
        KernelTimer timer(g_sample_depth ? "topk_select_sample" : "topk_select", s);
        hipLaunchKernelGGL(select_emit_kernel, dim3(nq), dim3(kBlock), 0, s, cnt, cand, k, d_q, d_db, d_idx, d_missed,
                           d_extra, d_dist, redo, n_redo);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return done(fail(QD_ERR_DEVICE, "matrix-core scan: %s", hipGetErrorString(e)));
    // queries whose candidate buffer overflowed: search them again with the scan
    uint32_t h_redo = 0;
    e = hipMemcpyAsync(&h_redo, n_redo, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(fail(QD_ERR_DEVICE, "overflow check: %s", hipGetErrorString(e)));
    if (h_redo > 0) {
        uint4 *gq = nullptr;
        char *ro = nullptr;
        if (hipMallocAsync((void **)&gq, (size_t)h_redo * 512, s) != hipSuccess ||
            hipMallocAsync((void **)&ro, (size_t)h_redo * k * 16, s) != hipSuccess)
            return done(fail(QD_ERR_OOM, "fallback scratch"));
        hipLaunchKernelGGL(gather_queries_kernel, dim3((h_redo * 32 + 255) / 256), dim3(256), 0, s,
                           reinterpret_cast<const uint4 *>(d_q), redo, h_redo, gq);
        uint32_t *ri = (uint32_t *)ro;
        int32_t *rm = (int32_t *)(ri + (size_t)h_redo * k), *rx = rm + (size_t)h_redo * k;
        float *rd = (float *)(rx + (size_t)h_redo * k);
        rc = knn_bruteforce_impl(d_db, n, reinterpret_cast<const uint64_t *>(gq), h_redo, k, ri, rm, rx, rd, stream, 16,
                                 0);
        if (rc == QD_OK) {
            const dim3 g((h_redo * k + 255) / 256);
            hipLaunchKernelGGL(scatter_rows_kernel<uint32_t>, g, dim3(256), 0, s, ri, redo, h_redo, k, d_idx);
            hipLaunchKernelGGL(scatter_rows_kernel<int32_t>, g, dim3(256), 0, s, rm, redo, h_redo, k, d_missed);
            hipLaunchKernelGGL(scatter_rows_kernel<int32_t>, g, dim3(256), 0, s, rx, redo, h_redo, k, d_extra);
            hipLaunchKernelGGL(scatter_rows_kernel<float>, g, dim3(256), 0, s, rd, redo, h_redo, k, d_dist);
            if (hipGetLastError() != hipSuccess) rc = fail(QD_ERR_DEVICE, "fallback scatter");
        }
        (void)hipFreeAsync(gq, s);
        (void)hipFreeAsync(ro, s);
    }
    return done(rc);
}

}  // namespace qd

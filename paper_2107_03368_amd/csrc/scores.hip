// Object-level distance scores (Section 6.4, the object matching behind
// Table 1 and the confusion matrices): the score of query object g against
// database object o is the sum, over g's descriptors in their given order, of
// each descriptor's distance (Eq. 1) to its nearest descriptor of o.
//
// Stage 1 groups the database rows by object (a counting sort of row ids: one
// histogram, one scan that also numbers each object's 256-row tiles, one
// scatter).  Stage 2 is a sequential search in which every row tile belongs
// to one object: work item (256-descriptor tile, row tile) runs the shared
// overlap tile (mfma_tile.h) on the gathered rows, takes each descriptor's
// smallest key over the tile, reduces it over the tile's lanes and waves, and
// folds it into minK[descriptor][object] with one atomic minimum per
// descriptor; the minimum does not depend on the order of the tiles.  Stage 3
// gives every (query object, object) pair one thread, which adds the terms
// minK / (wA wB) in float64, descriptor after descriptor.  Query descriptors
// are taken in batches that bound minK; each batch continues the running sums.
// qd_score_rows ranks the objects of each query object and rescales its row
// to [0, 1], the confusion-matrix row.
#include "mfma_tile.h"
#include "qd_device.h"
#include "qd_internal.h"

namespace qd {

int popcount_rows_launch(const uint64_t *d_db, uint64_t n, uint16_t *d_pop, hipStream_t s);

namespace {

constexpr int kBlock = 256;
constexpr int MQ = mt::MA;  // descriptors per tile
constexpr int MR = mt::MB;  // rows per tile
constexpr uint32_t kNoKey = 0xFFFFFFFFu;       // above every key (keys are < 2^24)
constexpr uint64_t kMinKBytes = 1ull << 30;    // minK of one batch
constexpr uint64_t kMaxBatch = 1ull << 18;     // query descriptors per batch
constexpr uint32_t kMaxObjects = 65536;        // object ids are uint16

// Smallest of the 16 values of a row of lanes (every lane of the row gets it).
__device__ __forceinline__ uint32_t min16(uint32_t v) {
    uint32_t t = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
    v = t < v ? t : v;
    t = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
    v = t < v ? t : v;
    t = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v = t < v ? t : v;
    t = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);  // row_mirror
    return t < v ? t : v;
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_f64_kernel(double *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void obj_count_kernel(const uint16_t *__restrict__ obj_of, uint64_t n, uint32_t n_obj,
                                 uint32_t *__restrict__ cnt) {
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t o = obj_of[t];
        if (o < n_obj) atomicAdd(&cnt[o], 1u);  // ids >= n_obj belong to no object
    }
}

// One block: roff = exclusive prefix of the row counts, toff = exclusive
// prefix of the tile counts ceil(cnt / 256); both with the total at n_obj.
// Also clears the scatter cursors.
__global__ __launch_bounds__(1024) void obj_offsets_kernel(const uint32_t *__restrict__ cnt, uint32_t n_obj,
                                                           uint64_t *__restrict__ roff, uint32_t *__restrict__ toff,
                                                           uint32_t *__restrict__ cursor) {
    __shared__ uint64_t prow[1024];
    __shared__ uint32_t ptile[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t chunk = (n_obj + 1023) / 1024;
    const uint32_t c0 = tid * chunk < n_obj ? tid * chunk : n_obj;
    const uint32_t c1 = c0 + chunk < n_obj ? c0 + chunk : n_obj;
    uint64_t sr = 0;
    uint32_t st = 0;
    for (uint32_t o = c0; o < c1; o++) {
        sr += cnt[o];
        st += (cnt[o] + MR - 1) / MR;
    }
    prow[tid] = sr;
    ptile[tid] = st;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
        const uint64_t vr = tid >= d ? prow[tid - d] : 0;
        const uint32_t vt = tid >= d ? ptile[tid - d] : 0;
        __syncthreads();
        prow[tid] += vr;
        ptile[tid] += vt;
        __syncthreads();
    }
    uint64_t rr = prow[tid] - sr;
    uint32_t rt = ptile[tid] - st;
    for (uint32_t o = c0; o < c1; o++) {
        roff[o] = rr;
        toff[o] = rt;
        cursor[o] = 0;
        rr += cnt[o];
        rt += (cnt[o] + MR - 1) / MR;
    }
    if (tid == 1023) {
        roff[n_obj] = prow[1023];
        toff[n_obj] = ptile[1023];
    }
}

// Row ids grouped by object; within an object in any order (a minimum over
// the object's rows does not depend on it).
__global__ void obj_scatter_kernel(const uint16_t *__restrict__ obj_of, uint64_t n, uint32_t n_obj,
                                   const uint64_t *__restrict__ roff, uint32_t *__restrict__ cursor,
                                   uint32_t *__restrict__ order) {
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t o = obj_of[t];
        if (o < n_obj) order[roff[o] + atomicAdd(&cursor[o], 1u)] = (uint32_t)t;
    }
}

// Tile (qt, rt) for tile = rt * n_qtiles + qt; row tile rt lies in the object
// o with toff[o] <= rt < toff[o + 1] (binary search; objects without rows
// have no tiles).  Consecutive work items share a row tile.
__global__ __launch_bounds__(mt::kThreads) void objscan_kernel(
    const uint4 *__restrict__ db, const uint32_t *__restrict__ order, const uint16_t *__restrict__ tpop,
    const uint64_t *__restrict__ roff, const uint32_t *__restrict__ toff, uint32_t n_obj, const uint4 *__restrict__ q,
    uint32_t nq, const uint16_t *__restrict__ qpop, uint32_t n_qtiles, uint32_t *__restrict__ minK) {
    __shared__ mt::Smem sm;
    __shared__ uint32_t s_pq[MQ], s_tp[MR], s_min[MQ];
    const uint64_t n_tiles = (uint64_t)n_qtiles * toff[n_obj];
    const int lane = threadIdx.x & 63;
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint32_t qt = (uint32_t)(tile % n_qtiles);
        const uint32_t rt = (uint32_t)(tile / n_qtiles);
        uint32_t lo = 0, hi = n_obj;  // toff[lo] <= rt < toff[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (toff[mid] <= rt)
                lo = mid;
            else
                hi = mid;
        }
        const uint32_t o = lo;
        const uint64_t r0 = roff[o] + (uint64_t)(rt - toff[o]) * MR, r1 = roff[o + 1];
        const uint32_t nb = r1 - r0 < (uint64_t)MR ? (uint32_t)(r1 - r0) : (uint32_t)MR;  // rows in this tile
        const uint32_t q0 = qt * MQ;
        const int r = mt::own_row();
        const uint4 *row;
        bool ok;
        if (r < MQ) {
            ok = q0 + r < nq;
            row = ok ? q + (uint64_t)(q0 + r) * 32 : q;
            s_pq[r] = ok ? qpop[q0 + r] : 0;
            s_min[r] = kNoKey;
        } else {
            ok = (uint32_t)(r - MQ) < nb;
            const uint32_t t = ok ? order[r0 + (r - MQ)] : order[r0];
            row = db + (uint64_t)t * 32;
            s_tp[r - MQ] = ok ? tpop[t] : 0;
        }
        mt::v4f acc[8][4];
        mt::overlap_tile(row, !ok, sm, acc);  // its barriers also publish the metadata above

        // this lane's 32 descriptors x 4 rows: smallest key per descriptor.
        // K = |q|*wB - (C*(wA + wB) - |t|*wA), so the smallest K is |q|*wB
        // minus the largest C*(wA + wB) - |t|*wA; rows past the tile's end
        // get |t| = 32767, which no real row's value can lose to.
        int32_t tpv[4];
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const int bi = mt::acc_brow(b);
            tpv[b] = (uint32_t)bi < nb ? (int32_t)s_tp[bi] : 32767;
        }
#pragma unroll
        for (int a = 0; a < 8; a++) {
            // one group of queries at a time, so their metadata loads stay next to their use
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                const int ai = mt::acc_arow(a, rr);
                const uint32_t pq = s_pq[ai];
                const int32_t wa = pq > 1 ? (int32_t)pq : 1, wb = (QD_BITS - pq) > 1 ? (int32_t)(QD_BITS - pq) : 1;
                int32_t vmax = (int32_t)mt::count(acc[a][0][rr]) * (wa + wb) - tpv[0] * wa;
#pragma unroll
                for (int b = 1; b < 4; b++) {
                    const int32_t v = (int32_t)mt::count(acc[a][b][rr]) * (wa + wb) - tpv[b] * wa;
                    vmax = v > vmax ? v : vmax;
                }
                uint32_t m = (uint32_t)((int32_t)pq * wb - vmax);
                // the 16 lanes of a row hold the same descriptors, 16 rows each
                m = min16(m);
                if ((lane & 15) == 0) atomicMin(&s_min[ai], m);  // the 4 waves of this descriptor half
            }
        }
        __syncthreads();
        if (r < MQ && q0 + r < nq) atomicMin(&minK[(uint64_t)(q0 + r) * n_obj + o], s_min[r]);
        // the next tile rewrites s_pq / s_tp only after every lane has read them (above);
        // s_min[r] is read and rewritten by thread r alone
    }
}

// Thread (g, o) for the query objects that overlap this batch, descriptors
// [d0, d0 + nb): adds the batch's terms of g's descriptors, in order, to the
// running score.  g_lo .. g_hi is found per thread by binary search on qoff.
__global__ __launch_bounds__(kBlock) void score_sum_kernel(const uint32_t *__restrict__ minK,
                                                           const uint16_t *__restrict__ qpop, uint64_t d0,
                                                           uint32_t nb, const uint64_t *__restrict__ qoff,
                                                           uint32_t nqo, const uint64_t *__restrict__ roff,
                                                           uint32_t n_obj, double *__restrict__ scores) {
    const uint64_t d1 = d0 + nb;
    // first g whose descriptors end after d0; first g whose descriptors start at or after d1
    uint32_t lo = 0, hi = nqo;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (qoff[mid + 1] <= d0)
            lo = mid + 1;
        else
            hi = mid;
    }
    const uint32_t g_lo = lo;
    hi = nqo;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (qoff[mid] < d1)
            lo = mid + 1;
        else
            hi = mid;
    }
    const uint32_t g_hi = lo;
    const uint64_t total = (uint64_t)(g_hi - g_lo) * n_obj;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t g = g_lo + (uint32_t)(i / n_obj), o = (uint32_t)(i % n_obj);
        const uint64_t a = qoff[g] > d0 ? qoff[g] : d0, b = qoff[g + 1] < d1 ? qoff[g + 1] : d1;
        if (a >= b) continue;
        const bool empty = roff[o + 1] == roff[o];  // the minimum over no rows is +infinity
        double s = scores[(uint64_t)g * n_obj + o];
#pragma unroll 8
        for (uint64_t d = a; d < b; d++) {
            const uint32_t P = qpop[d - d0];
            const uint32_t wa = P > 1 ? P : 1, wb = (QD_BITS - P) > 1 ? QD_BITS - P : 1;
            const double term =
                empty ? __builtin_inf() : (double)minK[(d - d0) * n_obj + o] / ((double)wa * (double)wb);
            s += term;
        }
        scores[(uint64_t)g * n_obj + o] = s;
    }
}

// One block per row of scores: the lowest finite score (ties to the lower
// object id) and the highest, by a block reduction; then, with normalize, the
// row rescaled in place.
__global__ __launch_bounds__(kBlock) void score_rows_kernel(double *__restrict__ scores, uint32_t nqo, uint32_t n_obj,
                                                            int normalize, int32_t *__restrict__ best) {
    __shared__ double s_mn[kBlock], s_mx[kBlock];
    __shared__ int32_t s_arg[kBlock];
    const uint32_t tid = threadIdx.x;
    for (uint32_t g = blockIdx.x; g < nqo; g += gridDim.x) {
        double *row = scores + (uint64_t)g * n_obj;
        double mn = __builtin_inf(), mx = -__builtin_inf();
        int32_t arg = -1;
        for (uint32_t o = tid; o < n_obj; o += kBlock) {  // increasing o: a tie keeps the first
            const double v = row[o];
            if (!__builtin_isfinite(v)) continue;
            if (v < mn) {
                mn = v;
                arg = (int32_t)o;
            }
            mx = v > mx ? v : mx;
        }
        s_mn[tid] = mn;
        s_mx[tid] = mx;
        s_arg[tid] = arg;
        __syncthreads();
        for (uint32_t h = kBlock / 2; h > 0; h >>= 1) {
            if (tid < h) {
                const double m2 = s_mn[tid + h];
                const int32_t a2 = s_arg[tid + h];
                if (a2 >= 0 && (s_arg[tid] < 0 || m2 < s_mn[tid] || (m2 == s_mn[tid] && a2 < s_arg[tid]))) {
                    s_mn[tid] = m2;
                    s_arg[tid] = a2;
                }
                s_mx[tid] = s_mx[tid + h] > s_mx[tid] ? s_mx[tid + h] : s_mx[tid];
            }
            __syncthreads();
        }
        const double lo = s_mn[0], hi = s_mx[0];
        if (tid == 0) best[g] = s_arg[0];
        if (normalize) {
            for (uint32_t o = tid; o < n_obj; o += kBlock) {
                const double v = row[o];
                row[o] = !__builtin_isfinite(v) ? 1.0 : hi > lo ? (v - lo) / (hi - lo) : 0.0;
            }
        }
        __syncthreads();  // the next row reuses the reduction arrays
    }
}

uint32_t blocks_for(uint64_t n, uint64_t cap) {
    const uint64_t b = (n + kBlock - 1) / kBlock;
    return (uint32_t)(b < 1 ? 1 : b > cap ? cap : b);
}

}  // namespace
}  // namespace qd

extern "C" int qd_object_scores(const uint64_t *d_db, uint64_t n, const uint16_t *d_obj_of, uint32_t n_obj,
                                const uint64_t *d_qdesc, uint64_t n_qdesc, const uint64_t *d_qoff, uint32_t nqo,
                                double *d_scores, void *stream) {
    using namespace qd;
    clear_error();
    if (n_obj < 1 || n_obj > kMaxObjects) return fail(QD_ERR_INVALID, "n_obj=%u outside 1..65536", n_obj);
    if (nqo == 0) return QD_OK;
    if (!d_qoff || !d_scores || (n && (!d_db || !d_obj_of)) || (n_qdesc && !d_qdesc))
        return fail(QD_ERR_INVALID, "null pointer");
    if ((n && !aligned16(d_db)) || (n_qdesc && !aligned16(d_qdesc)))
        return fail(QD_ERR_INVALID, "descriptor arrays must be 16-byte aligned");
    if (n > 0xFFFFFFFFull) return fail(QD_ERR_INVALID, "more than 2^32 - 1 database rows");
    hipStream_t s = (hipStream_t)stream;
    const uint64_t n_scores = (uint64_t)nqo * n_obj;
    const uint32_t cap = (uint32_t)device_cus() * 16;
    hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks_for(n_scores, cap)), dim3(kBlock), 0, s, d_scores, n_scores);
    QD_HIP_CHECK(hipGetLastError());
    if (n_qdesc == 0) return QD_OK;

    uint64_t nb_max = kMinKBytes / 4 / n_obj / MQ * MQ;
    if (nb_max < (uint64_t)MQ) nb_max = MQ;
    if (nb_max > kMaxBatch) nb_max = kMaxBatch;
    if (nb_max > n_qdesc) nb_max = n_qdesc;
    // scratch: row order, row popcounts, counts / cursors, offsets, batch popcounts, minK
    const size_t o_order = 0, o_tpop = o_order + ((n * 4 + 255) & ~255ull);
    const size_t o_cnt = o_tpop + ((n * 2 + 255) & ~255ull);
    const size_t o_cur = o_cnt + (((size_t)n_obj * 4 + 255) & ~255ull);
    const size_t o_roff = o_cur + (((size_t)n_obj * 4 + 255) & ~255ull);
    const size_t o_toff = o_roff + ((((size_t)n_obj + 1) * 8 + 255) & ~255ull);
    const size_t o_qpop = o_toff + ((((size_t)n_obj + 1) * 4 + 255) & ~255ull);
    const size_t o_mink = o_qpop + ((nb_max * 2 + 255) & ~255ull);
    const size_t bytes = o_mink + nb_max * n_obj * 4;
    char *ws = nullptr;
    QD_HIP_CHECK(hipMallocAsync((void **)&ws, bytes, s));
    uint32_t *order = reinterpret_cast<uint32_t *>(ws + o_order);
    uint16_t *tpop = reinterpret_cast<uint16_t *>(ws + o_tpop);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + o_cnt);
    uint32_t *cursor = reinterpret_cast<uint32_t *>(ws + o_cur);
    uint64_t *roff = reinterpret_cast<uint64_t *>(ws + o_roff);
    uint32_t *toff = reinterpret_cast<uint32_t *>(ws + o_toff);
    uint16_t *qpop = reinterpret_cast<uint16_t *>(ws + o_qpop);
    uint32_t *minK = reinterpret_cast<uint32_t *>(ws + o_mink);
    auto done = [&](int rc) {
        (void)hipFreeAsync(ws, s);
        return rc;
    };

    {
        KernelTimer timer("object_group", s);
        hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n_obj, cap)), dim3(kBlock), 0, s, cnt, (uint64_t)n_obj,
                           0u);
        if (n) {
            hipLaunchKernelGGL(obj_count_kernel, dim3(blocks_for(n, cap)), dim3(kBlock), 0, s, d_obj_of, n, n_obj, cnt);
        }
        hipLaunchKernelGGL(obj_offsets_kernel, dim3(1), dim3(1024), 0, s, cnt, n_obj, roff, toff, cursor);
        if (n) {
            hipLaunchKernelGGL(obj_scatter_kernel, dim3(blocks_for(n, cap)), dim3(kBlock), 0, s, d_obj_of, n, n_obj,
                               roff, cursor, order);
        }
        if (hipGetLastError() != hipSuccess) return done(fail(QD_ERR_DEVICE, "object grouping launch failed"));
        const int rc = popcount_rows_launch(d_db, n, tpop, s);
        if (rc != QD_OK) return done(rc);
    }
    // row tiles: at most one ragged tile per object that has rows
    const uint64_t row_tiles_max = (n + MR - 1) / MR + (n < n_obj ? n : n_obj);
    for (uint64_t d0 = 0; d0 < n_qdesc; d0 += nb_max) {
        const uint32_t nb = (uint32_t)(n_qdesc - d0 < nb_max ? n_qdesc - d0 : nb_max);
        const uint64_t *qb = d_qdesc + d0 * QD_WORDS;
        int rc = popcount_rows_launch(qb, nb, qpop, s);
        if (rc != QD_OK) return done(rc);
        if (n) {
            const uint64_t m = (uint64_t)nb * n_obj;
            hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(m, cap)), dim3(kBlock), 0, s, minK, m, kNoKey);
            KernelTimer timer("object_scan", s);
            const uint32_t n_qtiles = (nb + MQ - 1) / MQ;
            const uint64_t grid = mt::tile_grid((uint64_t)n_qtiles * row_tiles_max);
            hipLaunchKernelGGL(objscan_kernel, dim3((uint32_t)grid), dim3(mt::kThreads), 0, s,
                               reinterpret_cast<const uint4 *>(d_db), order, tpop, roff, toff, n_obj,
                               reinterpret_cast<const uint4 *>(qb), nb, qpop, n_qtiles, minK);
            if (hipGetLastError() != hipSuccess) return done(fail(QD_ERR_DEVICE, "object scan launch failed"));
        }
        {
            KernelTimer timer("object_sum", s);
            const uint64_t pairs = (uint64_t)(nqo < nb ? nqo : nb + 1) * n_obj;  // query objects overlapping the batch
            hipLaunchKernelGGL(score_sum_kernel, dim3(blocks_for(pairs, cap * 4)), dim3(kBlock), 0, s, minK, qpop, d0,
                               nb, d_qoff, nqo, roff, n_obj, d_scores);
            if (hipGetLastError() != hipSuccess) return done(fail(QD_ERR_DEVICE, "score sum launch failed"));
        }
    }
    return done(QD_OK);
}

extern "C" int qd_score_rows(double *d_scores, uint32_t nqo, uint32_t n_obj, int normalize, int32_t *d_best,
                             void *stream) {
    using namespace qd;
    clear_error();
    if (nqo == 0) return QD_OK;
    if (n_obj < 1) return fail(QD_ERR_INVALID, "n_obj=0");
    if (!d_scores || !d_best) return fail(QD_ERR_INVALID, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t cap = (uint32_t)device_cus() * 16;
    KernelTimer timer("score_rows", s);
    hipLaunchKernelGGL(score_rows_kernel, dim3(nqo < cap ? nqo : cap), dim3(kBlock), 0, s, d_scores, nqo, n_obj,
                       normalize ? 1 : 0, d_best);
    QD_HIP_CHECK(hipGetLastError());
    return QD_OK;
}


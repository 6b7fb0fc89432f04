// Sequential search over a bit-plane index, for small query batches.
//
// A query only ever asks whether a database row has the bits the query has:
// the overlap C = popcount(q AND t) is the number of the query's set bits that
// are set in t.  The index stores the database transposed: plane b holds bit
// b of every row (row i at bit i % 64 of word i / 64), so a query reads only
// its |q| planes (|q| is 2-8% of 4096 bits here) instead of every 512-byte
// row.  This is the same sequential search of Section 6.2, reorganised for
// latency-bound batches of a few queries.
//
// A wave serves one query over a range of plane words; lane l owns word w
// (64 rows) per step.  Counting: the |q| plane words of w are added as 1-bit
// numbers into bit-sliced counters with carry-save adders, 16 at a time
// (ones, twos, fours, eights hold the low 4 binary digits of C for all 64
// rows; each group's carry-out of weight 16 ripples into the higher digits).
// Filtering: every row with key K <= the wave's current k-th key has
//   C >= T = ceil((|q|*wB + pmin_w*wA - K_k) / (wA + wB)),
// pmin_w the smallest popcount among the word's 64 rows, because K =
// |q|*wB + |t|*wA - C*(wA + wB); C >= T is compared bit-sliced for all 64 rows
// at once.  Only rows that pass get their C extracted, their exact key
// computed with |t|, and are offered to the wave's top-k list (one 64-bit key
// per lane, as in the row scan).  The four waves of a block take consecutive
// word ranges of one query and merge their lists in LDS; the per-block lists
// are merged by the row scan's merge kernel, which also writes A, B and the
// distance.
#include "qd_device.h"
#include "qd_internal.h"

struct qd_planes_s {
    int device = 0;
    uint64_t n = 0;                  // database rows
    uint64_t words = 0;              // plane words holding rows: ceil(n / 64)
    uint64_t stride = 0;             // plane length in words (words rounded up to 8)
    uint64_t *d_planes = nullptr;    // 4096 x stride words
    uint16_t *d_pop = nullptr;       // n: popcount of each row
    uint16_t *d_wmin = nullptr;      // stride: smallest popcount of each word's rows
    const uint64_t *d_db = nullptr;  // the caller's rows (read by the final merge)
};

namespace qd {

int popcount_rows_launch(const uint64_t *d_db, uint64_t n, uint16_t *d_pop, hipStream_t s);
int merge_launch(const u64 *part, uint32_t n_parts, uint32_t k, const uint64_t *d_q, const uint64_t *d_db,
                 uint32_t nq, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, hipStream_t s);

namespace {

constexpr int kTBlock = 512;           // transpose: 8 waves, one plane word each
constexpr int kSBlock = 256;           // search: 4 waves
constexpr int kSWaves = kSBlock / 64;
constexpr uint32_t kMaxParts = 4096;   // lists per query (the merge kernel's limit)
constexpr int kDigits = 13;            // binary digits of C <= 4096 (with room for T < 8192)
constexpr uint64_t kMaxGrid = 1u << 20;

// Block x transposes the 512 rows of plane words 8x .. 8x+7: wave v takes
// word 8x+v, lane i row 64(8x+v)+i; for each descriptor word r the 64 ballots
// of its bits give the 64 plane words of bits 64r .. 64r+63, which are staged
// in LDS so that each plane receives 8 consecutive words (64 bytes) at once.
__global__ __launch_bounds__(kTBlock) void planes_transpose_kernel(const uint64_t *__restrict__ db, uint64_t n,
                                                                   uint64_t stride, uint64_t *__restrict__ planes) {
    __shared__ uint64_t buf[64][8];
    const int lane = threadIdx.x & 63, v = threadIdx.x >> 6;
    const int c = threadIdx.x >> 3, vv = threadIdx.x & 7;
    for (uint64_t x0 = blockIdx.x; x0 * 8 < stride; x0 += gridDim.x) {
        const uint64_t w0 = x0 * 8;
        const uint64_t row = (w0 + v) * 64 + lane;
        const bool ok = row < n;
        for (int r = 0; r < 64; r++) {
            const uint64_t x = ok ? db[row * QD_WORDS + r] : 0;
            uint64_t mine = 0;
#pragma unroll 8
            for (int b = 0; b < 64; b++) {
                const uint64_t bal = ballot((x >> b) & 1);
                mine = lane == b ? bal : mine;
            }
            buf[lane][v] = mine;  // plane 64r + lane, word w0 + v
            __syncthreads();
            planes[(uint64_t)(64 * r + c) * stride + w0 + vv] = buf[c][vv];
            __syncthreads();
        }
    }
}

__global__ void word_min_kernel(const uint16_t *__restrict__ pop, uint64_t n, uint64_t stride,
                                uint16_t *__restrict__ wmin) {
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < stride;
         w += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t m = 0xFFFFu;
        for (uint64_t r = w * 64; r < w * 64 + 64 && r < n; r++) m = pop[r] < m ? pop[r] : m;
        wmin[w] = (uint16_t)(m == 0xFFFFu ? 0 : m);  // a word past the rows: no row passes anyway
    }
}

// carry-save adder: (h, l) = the two binary digits of a + b + c
__device__ __forceinline__ void csa(uint64_t &h, uint64_t &l, uint64_t a, uint64_t b, uint64_t c) {
    const uint64_t u = a ^ b;
    h = (a & b) | (u & c);
    l = u ^ c;
}

// Block (query qi, group g): wave v scans plane words [p*wpp, (p+1)*wpp) of
// the first `words`, p = 4g + v; the block's four top-k lists are merged and
// its k best keys (K << 32 | row) written to part[(qi*n_groups+g)*k ..].
__global__ __launch_bounds__(kSBlock) void planes_scan_kernel(const uint64_t *__restrict__ planes, uint64_t stride,
                                                              uint64_t words, uint64_t n,
                                                              const uint16_t *__restrict__ tpop,
                                                              const uint16_t *__restrict__ wmin,
                                                              const uint64_t *__restrict__ q, uint32_t nq, uint32_t k,
                                                              uint32_t n_groups, uint64_t wpp, u64 *__restrict__ part) {
    __shared__ uint16_t bits_all[kSWaves][QD_BITS + 16];
    __shared__ u64 lists[kSWaves][64];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const uint32_t qi = blockIdx.x / n_groups, grp = blockIdx.x % n_groups;
    const uint32_t p = grp * kSWaves + wv;
    if (qi >= nq) return;  // the whole block
    uint16_t *bits = bits_all[wv];
    uint32_t P = 0;
    {
        // the query's set bits, ascending: lane l lists those of word l
        const uint64_t qw = q[(uint64_t)qi * QD_WORDS + lane];
        const uint32_t c = (uint32_t)__popcll(qw);
        uint32_t incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, d);
            if (lane >= d) incl += t;
        }
        uint32_t off = incl - c;
        for (uint64_t m = qw; m; m &= m - 1) bits[off++] = (uint16_t)(64 * lane + __builtin_ctzll(m));
        P = readlane(incl, 63);
    }
    __syncthreads();  // the bit lists are complete
    const uint32_t wa = P > 1 ? P : 1, wb = (QD_BITS - P) > 1 ? QD_BITS - P : 1;
    const uint32_t groups = (P + 15) / 16;
    // binary digits of the number of 16-groups: the high counter's width
    const uint32_t hi_digits = groups ? 32 - __builtin_clz(groups) : 0;
    const uint64_t w0 = (uint64_t)p * wpp, w1 = w0 + wpp < words ? w0 + wpp : words;

    u64 list = KEY_NONE, thr = KEY_NONE;
    for (uint64_t base = w0; base < w1; base += 64) {
        const uint64_t w = base + lane;
        const bool valid = w < w1;
        uint64_t ones = 0, twos = 0, fours = 0, eights = 0;
        uint64_t hi[kDigits - 4];
#pragma unroll
        for (int l = 0; l < kDigits - 4; l++) hi[l] = 0;
        for (uint32_t g = 0; g < groups; g++) {
            uint64_t x[16];
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const uint32_t j = g * 16 + i;
                const uint32_t b = j < P ? readfirst((uint32_t)bits[j]) : 0;  // the same plane for every lane
                x[i] = (valid && j < P) ? planes[(uint64_t)b * stride + w] : 0;
            }
            uint64_t twosA, twosB, foursA, foursB, eightsA, eightsB, sixteens;
            csa(twosA, ones, ones, x[0], x[1]);
            csa(twosB, ones, ones, x[2], x[3]);
            csa(foursA, twos, twos, twosA, twosB);
            csa(twosA, ones, ones, x[4], x[5]);
            csa(twosB, ones, ones, x[6], x[7]);
            csa(foursB, twos, twos, twosA, twosB);
            csa(eightsA, fours, fours, foursA, foursB);
            csa(twosA, ones, ones, x[8], x[9]);
            csa(twosB, ones, ones, x[10], x[11]);
            csa(foursA, twos, twos, twosA, twosB);
            csa(twosA, ones, ones, x[12], x[13]);
            csa(twosB, ones, ones, x[14], x[15]);
            csa(foursB, twos, twos, twosA, twosB);
            csa(eightsB, fours, fours, foursA, foursB);
            csa(sixteens, eights, eights, eightsA, eightsB);
            // add the carry-out of weight 16 into the higher digits
            uint64_t carry = sixteens;
#pragma unroll
            for (int l = 0; l < kDigits - 4; l++) {
                if ((uint32_t)l < hi_digits) {
                    const uint64_t t = hi[l] & carry;
                    hi[l] ^= carry;
                    carry = t;
                }
            }
        }
        // rows that may have K <= the current k-th key: C >= T, bit-sliced
        uint64_t pass = 0;
        if (valid) {
            uint32_t T = 0;
            if (thr != KEY_NONE) {
                const int64_t X = (int64_t)P * wb + (int64_t)wmin[w] * wa - (int64_t)(thr >> 32);
                T = X <= 0 ? 0u : (uint32_t)((X + wa + wb - 1) / (wa + wb));
            }
            if (T < (1u << kDigits)) {
                const uint64_t dig[kDigits] = {ones,  twos,  fours, eights, hi[0], hi[1], hi[2],
                                               hi[3], hi[4], hi[5], hi[6],  hi[7], hi[8]};
                uint64_t gt = 0, eq = ~0ull;
#pragma unroll
                for (int l = kDigits - 1; l >= 0; l--) {
                    const uint64_t tl = (T >> l) & 1 ? ~0ull : 0ull;
                    gt |= eq & dig[l] & ~tl;
                    eq &= ~(dig[l] ^ tl);
                }
                pass = gt | eq;
                const uint64_t r0 = w * 64;
                if (r0 + 64 > n) pass &= (1ull << (n - r0)) - 1;  // rows past the end
            }
        }
        // offer the passing rows, one per lane per round
        while (ballot(pass != 0)) {
            u64 key = KEY_NONE;
            if (pass) {
                const int i = __builtin_ctzll(pass);
                pass &= pass - 1;
                const uint32_t C = (uint32_t)((ones >> i) & 1) | (uint32_t)((twos >> i) & 1) << 1 |
                                   (uint32_t)((fours >> i) & 1) << 2 | (uint32_t)((eights >> i) & 1) << 3 |
                                   (uint32_t)((hi[0] >> i) & 1) << 4 | (uint32_t)((hi[1] >> i) & 1) << 5 |
                                   (uint32_t)((hi[2] >> i) & 1) << 6 | (uint32_t)((hi[3] >> i) & 1) << 7 |
                                   (uint32_t)((hi[4] >> i) & 1) << 8 | (uint32_t)((hi[5] >> i) & 1) << 9 |
                                   (uint32_t)((hi[6] >> i) & 1) << 10 | (uint32_t)((hi[7] >> i) & 1) << 11 |
                                   (uint32_t)((hi[8] >> i) & 1) << 12;
                const uint64_t row = w * 64 + (uint64_t)i;
                const uint32_t K = (P - C) * wb + (tpop[row] - C) * wa;
                key = ((u64)K << 32) | (uint32_t)row;
            }
            u64 m = ballot(key < thr);
            while (m) {
                const int L = __builtin_ctzll(m);
                m &= m - 1;
                const u64 c2 = readlane64(key, L);
                if (c2 < thr) {
                    list = list_insert(list, c2, k);
                    thr = readlane64(list, (int)k - 1);
                }
            }
        }
    }
    // merge the block's lists into wave 0's
    lists[wv][lane] = list;
    __syncthreads();
    if (wv != 0) return;
    for (int v = 1; v < kSWaves; v++) {
        const u64 key = lists[v][lane];
        u64 m = ballot(key < thr);
        while (m) {
            const int L = __builtin_ctzll(m);
            m &= m - 1;
            const u64 c2 = readlane64(key, L);
            if (c2 < thr) {
                list = list_insert(list, c2, k);
                thr = readlane64(list, (int)k - 1);
            }
        }
    }
    if (lane < (int)k) part[((uint64_t)qi * n_groups + grp) * k + lane] = list;
}

}  // namespace
}  // namespace qd

extern "C" int qd_planes_build(const uint64_t *d_db, uint64_t n, void *stream, qd_planes_t *out) {
    using namespace qd;
    clear_error();
    if (!out) return fail(QD_ERR_INVALID, "null output handle");
    *out = nullptr;
    if (!d_db) return fail(QD_ERR_INVALID, "null database");
    if (n < 1 || n > QD_MAX_ROWS) return fail(QD_ERR_INVALID, "n=%llu outside 1..%llu", (u64)n, (u64)QD_MAX_ROWS);
    if (!aligned16(d_db)) return fail(QD_ERR_INVALID, "database must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    qd_planes_s *P = new qd_planes_s();
    P->n = n;
    P->words = (n + 63) / 64;
    P->stride = (P->words + 7) / 8 * 8;
    P->d_db = d_db;
    auto release = [&](int code) {
        qd_planes_free(P);
        return code;
    };
    if (hipMalloc((void **)&P->d_planes, (size_t)QD_BITS * P->stride * 8) != hipSuccess ||
        hipMalloc((void **)&P->d_pop, n * 2) != hipSuccess || hipMalloc((void **)&P->d_wmin, P->stride * 2) != hipSuccess)
        return release(fail(QD_ERR_OOM, "bit-plane allocation failed"));
    {
        KernelTimer timer("planes_transpose", s);
        const uint64_t blocks = P->stride / 8 < kMaxGrid ? P->stride / 8 : kMaxGrid;
        hipLaunchKernelGGL(planes_transpose_kernel, dim3((uint32_t)blocks), dim3(kTBlock), 0, s, d_db, n, P->stride,
                           P->d_planes);
    }
    int rc = popcount_rows_launch(d_db, n, P->d_pop, s);
    if (rc != QD_OK) return release(rc);
    const uint64_t wb = (P->stride + 255) / 256;
    hipLaunchKernelGGL(word_min_kernel, dim3((uint32_t)(wb < kMaxGrid ? wb : kMaxGrid)), dim3(256), 0, s, P->d_pop, n,
                       P->stride, P->d_wmin);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return release(fail(QD_ERR_DEVICE, "bit-plane build kernels failed"));
    (void)hipGetDevice(&P->device);
    *out = P;
    return QD_OK;
}

extern "C" int qd_planes_free(qd_planes_t p) {
    if (!p) return QD_OK;
    void *ptrs[] = {p->d_planes, p->d_pop, p->d_wmin};
    for (void *x : ptrs)
        if (x) (void)hipFree(x);
    delete p;
    return QD_OK;
}

extern "C" int qd_knn_planes(qd_planes_t pl, const uint64_t *d_q, uint32_t nq, uint32_t k, uint32_t *d_idx,
                             int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream) {
    using namespace qd;
    clear_error();
    if (!pl) return fail(QD_ERR_INVALID, "null bit-plane index");
    if (k < 1 || k > QD_MAX_K) return fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
    if (nq == 0) return QD_OK;
    if (!d_q || !d_idx || !d_missed || !d_extra || !d_dist) return fail(QD_ERR_INVALID, "null pointer");
    if (!aligned16(d_q)) return fail(QD_ERR_INVALID, "queries must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    // lists per query: enough waves to fill the chip, at least 64 words (4,096 rows) each
    const uint64_t want = ((uint64_t)device_cus() * 16 + nq - 1) / nq;
    uint64_t parts = (pl->words + 63) / 64;
    if (parts > want) parts = want;
    if (parts > kMaxParts) parts = kMaxParts;
    if (parts < 1) parts = 1;
    uint64_t wpp = (pl->words + parts - 1) / parts;
    wpp = (wpp + 63) / 64 * 64;
    // four waves (consecutive parts) per block, one merged list per block
    const uint32_t groups = (uint32_t)((pl->words + wpp * kSWaves - 1) / (wpp * kSWaves));
    const uint64_t blocks = (uint64_t)nq * groups;
    if (blocks * kSBlock > 0xFFFFFFFFull) return fail(QD_ERR_UNSUPPORTED, "launch too large");
    u64 *part = nullptr;
    QD_HIP_CHECK(hipMallocAsync((void **)&part, (size_t)blocks * k * 8, s));
    {
        KernelTimer timer("planes_scan", s);
        hipLaunchKernelGGL(planes_scan_kernel, dim3((uint32_t)blocks), dim3(kSBlock), 0, s, pl->d_planes, pl->stride,
                           pl->words, pl->n, pl->d_pop, pl->d_wmin, d_q, nq, k, groups, wpp, part);
    }
    int rc = hipGetLastError() == hipSuccess ? QD_OK : fail(QD_ERR_DEVICE, "bit-plane scan launch failed");
    if (rc == QD_OK) rc = merge_launch(part, groups, k, d_q, pl->d_db, nq, d_idx, d_missed, d_extra, d_dist, s);
    const hipError_t e = hipFreeAsync(part, s);
    if (rc != QD_OK) return rc;
    if (e != hipSuccess) return fail(QD_ERR_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
    return QD_OK;
}

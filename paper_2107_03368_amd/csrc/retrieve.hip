// Partial-object retrieval by voting (Section 3): every descriptor of a query
// object finds its k nearest database descriptors, each neighbour casts one
// vote for the object it belongs to, and the first object to reach the vote
// threshold, counted in the order the descriptors are given (and within a
// descriptor in neighbour rank order), is the match.
//
// All descriptors of all query objects are searched in one launch (the
// persistent tree kernel or the batched scan).  The vote kernel gives every
// query object one block: the full histogram is built with LDS atomics, and
// one wave replays the votes in order, 64 at a time, to find the winner: for
// each distinct object among the 64 votes, a ballot gives its lanes, the
// running count says whether its threshold-th vote falls in this group, and
// the earliest such vote wins.  Objects beyond 8192 keep their histogram in
// global memory; the replay counts stay in LDS as bytes.
#include "qd_device.h"
#include "qd_internal.h"
#include "qd_launch.h"
#include "qd_tree.h"

namespace qd {

int knn_bruteforce_impl(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                        uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream,
                        uint32_t qt_force, uint32_t parts_force);
int knn_tree_impl(qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k, int order, const float *d_scores,
                  uint32_t n_scored, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist,
                  uint32_t *d_qstats, qd_stats *h_stats, void *stream, uint32_t waves_per_cu, uint32_t *d_trace,
                  uint32_t n_traced);

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kLdsBins = 8192;      // histogram bins kept in LDS (more go to global atomics)
constexpr uint32_t kMaxObjects = 65536;  // object ids are uint16

__global__ __launch_bounds__(kBlock) void vote_kernel(const uint32_t *__restrict__ nn, uint32_t k,
                                                      const uint16_t *__restrict__ obj_of, uint64_t n_db,
                                                      uint32_t n_obj, const uint64_t *__restrict__ qoff,
                                                      uint32_t threshold, uint32_t *__restrict__ votes,
                                                      int32_t *__restrict__ winner, uint32_t *__restrict__ used,
                                                      const uint32_t *__restrict__ nqo_dev) {
    if (nqo_dev && blockIdx.x >= *nqo_dev) return;  // whole block (size given on the device)
    __shared__ uint32_t hist[kLdsBins];
    __shared__ uint8_t running[kMaxObjects];  // votes so far per object, saturating at the threshold
    const uint32_t g = blockIdx.x;
    const uint64_t d0 = qoff[g], d1 = qoff[g + 1];
    const uint64_t nv = (d1 - d0) * k;  // votes of this query object, in order
    const uint32_t *v = nn + d0 * k;
    const bool in_lds = n_obj <= kLdsBins;
    uint32_t *out = votes + (uint64_t)g * n_obj;
    for (uint32_t i = threadIdx.x; i < n_obj; i += kBlock) {
        if (in_lds)
            hist[i] = 0;
        else
            out[i] = 0;
        running[i] = 0;
    }
    __syncthreads();
    uint32_t *h = in_lds ? hist : out;
    for (uint64_t i = threadIdx.x; i < nv; i += kBlock) {
        const uint32_t row = v[i];
        if (row < n_db) {
            const uint32_t o = obj_of[row];
            if (o < n_obj) atomicAdd(&h[o], 1u);  // ids >= n_obj cast no vote
        }
    }
    __syncthreads();
    if (in_lds)
        for (uint32_t i = threadIdx.x; i < n_obj; i += kBlock) out[i] = hist[i];
    if (threadIdx.x >= 64) return;
    // ordered replay by wave 0
    const int lane = lane_id();
    uint64_t win_pos = ~0ull;
    int32_t win_obj = -1;
    for (uint64_t base = 0; base < nv && win_obj < 0 && threshold > 0; base += 64) {
        const uint64_t i = base + lane;
        const uint32_t row = i < nv ? v[i] : QD_PAD_IDX;
        uint32_t o = row < n_db ? obj_of[row] : 0xFFFFFFFFu;
        if (o >= n_obj) o = 0xFFFFFFFFu;
        u64 pending = ballot(o != 0xFFFFFFFFu);
        while (pending) {
            const int L = __builtin_ctzll(pending);
            const uint32_t ov = readlane(o, L);
            const u64 same = ballot(o == ov);
            pending &= ~same;
            const uint32_t before = readfirst(running[ov]);
            const uint32_t add = (uint32_t)__popcll(same);
            if (before < threshold && before + add >= threshold) {
                // the (threshold - before)-th lane of `same` holds the crossing vote
                u64 mk = same;
                for (uint32_t c = 1; c < threshold - before; c++) mk &= mk - 1;
                const uint64_t pos = base + (uint64_t)__builtin_ctzll(mk);
                if (pos < win_pos) {
                    win_pos = pos;
                    win_obj = (int32_t)ov;
                }
            }
            if (lane == 0) running[ov] = (uint8_t)(before + add < threshold ? before + add : threshold);
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (lane == 0) {
        winner[g] = win_obj;
        used[g] = win_obj >= 0 ? (uint32_t)(win_pos / k + 1) : (uint32_t)(d1 - d0);
    }
}

}  // namespace

int vote_launch(const uint32_t *nn, uint32_t k, const uint16_t *obj_of, uint64_t n_db, uint32_t n_obj,
                const uint64_t *qoff, uint32_t nqo, const uint32_t *nqo_dev, uint32_t threshold, uint32_t *votes,
                int32_t *winner, uint32_t *used, hipStream_t s) {
    KernelTimer timer("vote", s);
    hipLaunchKernelGGL(vote_kernel, dim3(nqo), dim3(kBlock), 0, s, nn, k, obj_of, n_db, n_obj, qoff, threshold, votes,
                       winner, used, nqo_dev);
    QD_HIP_CHECK(hipGetLastError());
    return QD_OK;
}

}  // namespace qd

extern "C" int qd_retrieve_objects(qd_tree_t t, const uint64_t *d_db, uint64_t n, const uint16_t *d_obj_of,
                                   uint32_t n_obj, const uint64_t *d_qdesc, uint64_t n_qdesc,
                                   const uint64_t *d_qoff, uint32_t nqo, uint32_t k, uint32_t vote_threshold,
                                   const qd_search_params *params, uint32_t *d_votes, int32_t *d_winner,
                                   uint32_t *d_used, uint32_t *d_nn_idx, void *stream) {
    using namespace qd;
    if (k < 1 || k > QD_MAX_K) return fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
    if (n_obj < 1 || n_obj > 65536) return fail(QD_ERR_INVALID, "n_obj=%u outside 1..65536", n_obj);
    if (vote_threshold > 255) return fail(QD_ERR_INVALID, "vote threshold %u above 255", vote_threshold);
    if (nqo == 0) return QD_OK;
    if (!d_obj_of || !d_qoff || !d_votes || !d_winner || !d_used || (n_qdesc && !d_qdesc))
        return fail(QD_ERR_INVALID, "null pointer");
    if (n_qdesc > 0xFFFFFFFFull) return fail(QD_ERR_INVALID, "too many query descriptors");
    const uint64_t n_db = t ? t->n : n;
    if (!t && (!d_db || n < 1)) return fail(QD_ERR_INVALID, "no tree and no database");
    if (params && (params->d_scores || params->d_visited))
        return fail(QD_ERR_INVALID, "scores and traces are per call of qd_knn_tree only");
    hipStream_t s = (hipStream_t)stream;
    const size_t m = (size_t)n_qdesc * k;
    uint32_t *nn = d_nn_idx;
    char *ws = nullptr;
    if (n_qdesc) {
        // scratch: neighbour rows (unless the caller keeps them) + the other k-NN outputs
        const size_t bytes = (nn ? 0 : m * 4) + m * 12;
        QD_HIP_CHECK(hipMallocAsync((void **)&ws, bytes, s));
        char *p = ws;
        if (!nn) {
            nn = reinterpret_cast<uint32_t *>(p);
            p += m * 4;
        }
        int32_t *missed = reinterpret_cast<int32_t *>(p);
        int32_t *extra = missed + m;
        float *dist = reinterpret_cast<float *>(extra + m);
        int rc;
        if (t)
            rc = knn_tree_impl(t, d_qdesc, (uint32_t)n_qdesc, k, params ? (int)params->order : QD_ORDER_BEST_FIRST,
                               nullptr, 0, nn, missed, extra, dist, nullptr, nullptr, stream,
                               params ? params->waves_per_cu : 0, nullptr, 0);
        else
            rc = knn_bruteforce_impl(d_db, n, d_qdesc, (uint32_t)n_qdesc, k, nn, missed, extra, dist, stream, 0, 0);
        if (rc != QD_OK) {
            (void)hipFreeAsync(ws, s);
            return rc;
        }
    }
    const int rc = vote_launch(nn, k, d_obj_of, n_db, n_obj, d_qoff, nqo, nullptr, vote_threshold, d_votes, d_winner,
                               d_used, s);
    if (ws) (void)hipFreeAsync(ws, s);
    return rc;
}

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
#include <algorithm>
#include <vector>

#include "qd_device.h"
#include "qd_internal.h"
#include "qd_launch.h"
#include "qd_tree.h"

namespace qd {

int knn_bruteforce_impl(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                        uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream,
                        uint32_t qt_force, uint32_t parts_force);

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kLdsBins = 8192;      // histogram bins kept in LDS (more go to global atomics)
constexpr uint32_t kMaxObjects = 65536;  // object ids are uint16

__global__ __launch_bounds__(kBlock) void vote_kernel(const uint32_t *__restrict__ nn, uint32_t k,
                                                      const uint16_t *__restrict__ obj_of, uint64_t n_db,
                                                      uint32_t n_obj, const uint64_t *__restrict__ qoff,
                                                      const uint64_t *__restrict__ qend,
                                                      uint32_t threshold, uint32_t *__restrict__ votes,
                                                      int32_t *__restrict__ winner, uint32_t *__restrict__ used,
                                                      const uint32_t *__restrict__ nqo_dev) {
    if (nqo_dev && blockIdx.x >= *nqo_dev) return;  // whole block (size given on the device)
    __shared__ uint32_t hist[kLdsBins];
    __shared__ uint8_t running[kMaxObjects];  // votes so far per object, saturating at the threshold
    const uint32_t g = blockIdx.x;
    const uint64_t d0 = qoff[g], d1 = qend ? qend[g] : qoff[g + 1];  // a prefix when qend is given
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
                int32_t *winner, uint32_t *used, hipStream_t s, const uint64_t *qend) {
    KernelTimer timer("vote", s);
    hipLaunchKernelGGL(vote_kernel, dim3(nqo), dim3(kBlock), 0, s, nn, k, obj_of, n_db, n_obj, qoff, qend, threshold,
                       votes, winner, used, nqo_dev);
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
                               params ? params->waves_per_cu : 0, nullptr, 0, params ? params->query_split : 0);
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

// ---- retrieval that stops at the vote threshold ------------------------------
//
// The paper processes a query object's descriptors one at a time and stops as
// soon as an object reaches the threshold, so most descriptors of a query
// object are never searched.  Here every round takes, for every query object
// still undecided, its next chunk of descriptors (16 in the first round, twice
// as many each round), searches all of them in one batched k-NN call, and
// replays the votes of each object's searched prefix; an object whose replay
// finds a winner stops.  Since the replay counts the same votes in the same
// order, winner and used equal qd_retrieve_objects' exactly.

namespace qd {
namespace {

__global__ void gather_desc_kernel(const uint4 *__restrict__ q, const uint32_t *__restrict__ ids, uint32_t m,
                                   uint4 *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (uint64_t)m * 32) out[i] = q[(uint64_t)ids[i >> 5] * 32 + (i & 31)];
}

__global__ void scatter_nn_kernel(const uint32_t *__restrict__ src, const uint32_t *__restrict__ ids, uint32_t m,
                                  uint32_t k, uint32_t *__restrict__ nn) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (uint64_t)m * k) nn[(uint64_t)ids[i / k] * k + (i % k)] = src[i];
}

}  // namespace
}  // namespace qd

extern "C" int qd_retrieve_objects_early(qd_tree_t t, const uint64_t *d_db, uint64_t n, const uint16_t *d_obj_of,
                                         uint32_t n_obj, const uint64_t *d_qdesc, uint64_t n_qdesc,
                                         const uint64_t *d_qoff, uint32_t nqo, uint32_t k, uint32_t vote_threshold,
                                         const qd_search_params *params, uint32_t *d_votes, int32_t *d_winner,
                                         uint32_t *d_used, uint64_t *h_searched, void *stream) {
    using namespace qd;
    if (h_searched) *h_searched = 0;
    if (k < 1 || k > QD_MAX_K) return fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
    if (n_obj < 1 || n_obj > 65536) return fail(QD_ERR_INVALID, "n_obj=%u outside 1..65536", n_obj);
    if (vote_threshold < 1 || vote_threshold > 255)
        return fail(QD_ERR_INVALID, "vote threshold %u outside 1..255", vote_threshold);
    if (nqo == 0) return QD_OK;
    if (!d_obj_of || !d_qoff || !d_votes || !d_winner || !d_used || (n_qdesc && !d_qdesc))
        return fail(QD_ERR_INVALID, "null pointer");
    if (n_qdesc > 0xFFFFFFFFull) return fail(QD_ERR_INVALID, "too many query descriptors");
    if (n_qdesc && !aligned16(d_qdesc)) return fail(QD_ERR_INVALID, "query descriptors must be 16-byte aligned");
    const uint64_t n_db = t ? t->n : n;
    if (!t && (!d_db || n < 1)) return fail(QD_ERR_INVALID, "no tree and no database");
    if (params && (params->d_scores || params->d_visited))
        return fail(QD_ERR_INVALID, "scores and traces are per call of qd_knn_tree only");
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint64_t> off(nqo + 1);
    QD_HIP_CHECK(hipMemcpyAsync(off.data(), d_qoff, (nqo + 1) * 8, hipMemcpyDeviceToHost, s));
    QD_HIP_CHECK(hipStreamSynchronize(s));
    if (off[0] != 0 || off[nqo] != n_qdesc) return fail(QD_ERR_INVALID, "d_qoff must run from 0 to n_qdesc");
    for (uint32_t g = 0; g < nqo; g++)
        if (off[g + 1] < off[g]) return fail(QD_ERR_INVALID, "d_qoff must not decrease");
    // scratch: neighbours (n_qdesc x k), per-object prefix ends, one round's
    // descriptor ids, gathered descriptors and k-NN outputs (at most n_qdesc)
    const uint64_t nd = n_qdesc ? n_qdesc : 1;
    const size_t b_nn = nd * k * 4, b_end = (size_t)nqo * 8, b_ids = nd * 4, b_q = nd * 512, b_out = nd * k * 16;
    char *ws = nullptr;
    QD_HIP_CHECK(hipMallocAsync((void **)&ws, b_nn + b_end + b_ids + b_q + b_out + 5 * 256, s));
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    uint32_t *nn = reinterpret_cast<uint32_t *>(ws);
    uint64_t *qend = reinterpret_cast<uint64_t *>(ws + up(b_nn));
    uint32_t *ids = reinterpret_cast<uint32_t *>(ws + up(b_nn) + up(b_end));
    uint4 *gq = reinterpret_cast<uint4 *>(ws + up(b_nn) + up(b_end) + up(b_ids));
    uint32_t *oi = reinterpret_cast<uint32_t *>(ws + up(b_nn) + up(b_end) + up(b_ids) + up(b_q));
    int32_t *om = reinterpret_cast<int32_t *>(oi + nd * k);
    int32_t *ox = om + nd * k;
    float *od = reinterpret_cast<float *>(ox + nd * k);
    auto done = [&](int code) {
        (void)hipFreeAsync(ws, s);
        return code;
    };
    std::vector<uint64_t> done_n(nqo, 0), end(nqo);
    std::vector<char> decided(nqo, 0);
    std::vector<int32_t> h_win(nqo);
    std::vector<uint32_t> h_used(nqo), h_ids;
    uint64_t searched = 0;
    for (uint64_t chunk = 16;; chunk *= 2) {
        if (abort_requested()) {  // between rounds
            (void)hipStreamSynchronize(s);
            return done(fail(QD_ERR_ABORTED, "retrieval aborted"));
        }
        h_ids.clear();
        for (uint32_t g = 0; g < nqo; g++) {
            if (decided[g]) continue;
            const uint64_t total = off[g + 1] - off[g];
            const uint64_t take = std::min<uint64_t>(chunk, total - done_n[g]);
            for (uint64_t i = 0; i < take; i++) h_ids.push_back((uint32_t)(off[g] + done_n[g] + i));
            done_n[g] += take;
        }
        if (h_ids.empty()) break;
        const uint32_t m = (uint32_t)h_ids.size();
        searched += m;
        if (hipMemcpyAsync(ids, h_ids.data(), (size_t)m * 4, hipMemcpyHostToDevice, s) != hipSuccess)
            return done(fail(QD_ERR_DEVICE, "upload"));
        hipLaunchKernelGGL(gather_desc_kernel, dim3((uint32_t)(((uint64_t)m * 32 + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<const uint4 *>(d_qdesc), ids, m, gq);
        const uint64_t *gq64 = reinterpret_cast<const uint64_t *>(gq);
        int rc;
        if (t)
            rc = knn_tree_impl(t, gq64, m, k, params ? (int)params->order : QD_ORDER_BEST_FIRST, nullptr, 0, oi, om,
                               ox, od, nullptr, nullptr, stream, params ? params->waves_per_cu : 0, nullptr, 0,
                               params ? params->query_split : 0);
        else
            rc = knn_bruteforce_impl(d_db, n, gq64, m, k, oi, om, ox, od, stream, 0, 0);
        if (rc != QD_OK) return done(rc);
        hipLaunchKernelGGL(scatter_nn_kernel, dim3((uint32_t)(((uint64_t)m * k + 255) / 256)), dim3(256), 0, s, oi,
                           ids, m, k, nn);
        for (uint32_t g = 0; g < nqo; g++) end[g] = off[g] + done_n[g];
        if (hipMemcpyAsync(qend, end.data(), (size_t)nqo * 8, hipMemcpyHostToDevice, s) != hipSuccess)
            return done(fail(QD_ERR_DEVICE, "upload"));
        rc = vote_launch(nn, k, d_obj_of, n_db, n_obj, d_qoff, nqo, nullptr, vote_threshold, d_votes, d_winner,
                         d_used, s, qend);
        if (rc != QD_OK) return done(rc);
        if (hipMemcpyAsync(h_win.data(), d_winner, (size_t)nqo * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(h_used.data(), d_used, (size_t)nqo * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return done(fail(QD_ERR_DEVICE, "early-exit round"));
        for (uint32_t g = 0; g < nqo; g++)
            if (h_win[g] >= 0) decided[g] = 1;
    }
    // final replay over exactly the descriptors each object used: the votes
    // of the searched prefix up to the decision
    for (uint32_t g = 0; g < nqo; g++) end[g] = off[g] + (decided[g] ? h_used[g] : off[g + 1] - off[g]);
    if (hipMemcpyAsync(qend, end.data(), (size_t)nqo * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return done(fail(QD_ERR_DEVICE, "upload"));
    const int rc = vote_launch(nn, k, d_obj_of, n_db, n_obj, d_qoff, nqo, nullptr, vote_threshold, d_votes, d_winner,
                               d_used, s, qend);
    if (rc == QD_OK && hipStreamSynchronize(s) != hipSuccess) return done(fail(QD_ERR_DEVICE, "final replay"));
    if (h_searched) *h_searched = searched;
    return done(rc);
}

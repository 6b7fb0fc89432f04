// Batched retrieval plans captured in a hipGraph, and the launch autotuner.
//
// A plan fixes the search (tree or sequential), k, the vote threshold and the
// largest batch it will serve, allocates every buffer once, and records the
// whole batch (k-NN of every query descriptor in one persistent launch, then
// the votes) into a hipGraph whose kernels read the batch sizes from device
// memory.  Running a batch copies the inputs into the plan's buffers, sets the
// sizes with a one-thread kernel, replays the graph and copies the outputs
// out, so no allocation and no host synchronisation happens per batch.
//
// The autotuner times every launch configuration that gives exact results
// (all of them do) on a caller's sample batch and keeps the fastest.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "qd_internal.h"
#include "qd_launch.h"
#include "qd_tree.h"

struct qd_plan_s {
    int device = 0;
    qd_tree_t tree = nullptr;
    const uint64_t *db = nullptr;
    uint64_t n = 0;
    const uint16_t *obj_of = nullptr;
    uint32_t n_obj = 0;
    uint64_t max_qdesc = 0;
    uint32_t max_qobj = 0, k = 0, threshold = 0;
    char *mem = nullptr;
    uint64_t *q = nullptr;
    uint64_t *qoff = nullptr;
    uint32_t *sizes = nullptr;
    uint32_t *nn = nullptr;
    int32_t *mi = nullptr, *ex = nullptr;
    float *di = nullptr;
    char *ws = nullptr;
    uint32_t *votes = nullptr;
    int32_t *winner = nullptr;
    uint32_t *used = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace qd {
namespace {

__global__ void set_sizes_kernel(uint32_t *sizes, uint32_t n_qdesc, uint32_t nqo) {
    sizes[0] = n_qdesc;
    sizes[1] = nqo;
}

// Blocked order: the descriptors of batch i of qb each, sizes[2 + i].
__global__ void batch_sizes_kernel(uint32_t *sizes, uint32_t n_batches, uint32_t qb) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_batches) return;
    const uint64_t b0 = (uint64_t)i * qb, nd = sizes[0];
    sizes[2 + i] = nd > b0 ? (uint32_t)(nd - b0 < qb ? nd - b0 : qb) : 0u;
}

void plan_release(qd_plan_s *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->mem) (void)hipFree(p->mem);
    delete p;
}

}  // namespace
}  // namespace qd

extern "C" int qd_plan_create(qd_tree_t t, const uint64_t *d_db, uint64_t n, const uint16_t *d_obj_of,
                              uint32_t n_obj, uint64_t max_qdesc, uint32_t max_qobj, uint32_t k,
                              uint32_t vote_threshold, const qd_search_params *params, uint32_t query_tile,
                              qd_plan_t *out) {
    using namespace qd;
    if (!out) return fail(QD_ERR_INVALID, "null output handle");
    *out = nullptr;
    if (k < 1 || k > QD_MAX_K) return fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
    if (n_obj < 1 || n_obj > 65536) return fail(QD_ERR_INVALID, "n_obj=%u outside 1..65536", n_obj);
    if (vote_threshold > 255) return fail(QD_ERR_INVALID, "vote threshold %u above 255", vote_threshold);
    if (max_qdesc < 1 || max_qdesc > 0xFFFFFFFFull || max_qobj < 1)
        return fail(QD_ERR_INVALID, "plan capacities must be positive (and max_qdesc < 2^32)");
    if (!d_obj_of || (!t && (!d_db || n < 1))) return fail(QD_ERR_INVALID, "null pointer");
    if (params && (params->d_scores || params->d_visited))
        return fail(QD_ERR_INVALID, "scores and traces are per call of qd_knn_tree only");
    const int order = params ? (int)params->order : QD_ORDER_BEST_FIRST;
    if (t && order != QD_ORDER_BEST_FIRST && order != QD_ORDER_DEPTH_FIRST && order != QD_ORDER_BLOCKED)
        return fail(QD_ERR_INVALID, "unknown frontier order");
    // a model sets where the blocked order's first round starts (its descent
    // runs on the plan's workspace); the depth-first order's scoring
    // allocates per call
    if (params && params->model && !(t && order == QD_ORDER_BLOCKED))
        return fail(QD_ERR_UNSUPPORTED, "a plan takes a model for the blocked order only");
    if (query_tile != 0 && query_tile != 1 && query_tile != 2 && query_tile != 4 && query_tile != 8 &&
        query_tile != 16 && query_tile != QD_QUERY_TILE_MATRIX)
        return fail(QD_ERR_INVALID, "query tile %u not in {0,1,2,4,8,16,QD_QUERY_TILE_MATRIX}", query_tile);
    const bool blocked = t && order == QD_ORDER_BLOCKED;
    if (blocked) {
        const int rc = blocked_check(t, params);
        if (rc != QD_OK) return rc;
    }
    if (params && !split_ok(params->query_split))
        return fail(QD_ERR_INVALID, "query_split %u: 0 or a power of two up to 16", params->query_split);
    qd_plan_s *p = new qd_plan_s();
    p->tree = t;
    p->db = d_db;
    p->n = t ? t->n : n;
    p->obj_of = d_obj_of;
    p->n_obj = n_obj;
    p->max_qdesc = max_qdesc;
    p->max_qobj = max_qobj;
    p->k = k;
    p->threshold = vote_threshold;
    (void)hipGetDevice(&p->device);
    const uint32_t nqmax = (uint32_t)max_qdesc;
    TreeLaunch TL;
    BruteLaunch BL;
    BlockedLayout KL;
    MfmaLayout ML;
    uint32_t n_batches = 1;
    size_t ws_bytes;
    // sequential search: the large-batch matrix-core path when the largest
    // batch is big enough (query_tile 0), else the row scan with that tile
    // (0: chosen for the largest batch as qd_knn_bruteforce would)
    const bool mfma = !t && query_tile == 0 && mfma_eligible(n, nqmax, k);
    if (blocked) {
        KL = blocked_layout(t, nqmax, k, params && params->model);
        n_batches = (uint32_t)((nqmax + KL.qb - 1) / KL.qb);
        ws_bytes = KL.bytes;
    } else if (mfma) {
        ML = mfma_layout(n, nqmax, k);
        ws_bytes = ML.bytes;
    } else if (t) {
        TL = tree_launch_shape(t, nqmax, k, order, params ? params->waves_per_cu : 0, params ? params->query_split : 0);
        ws_bytes = TL.total();
    } else {
        BL = brute_launch_shape(n, nqmax, k, query_tile, 0);
        ws_bytes = BL.part_bytes;
    }
    // one allocation: q | qoff | sizes | nn mi ex di | votes winner used | ws
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_q = 0, o_off = o_q + al(max_qdesc * 512), o_sz = o_off + al(((size_t)max_qobj + 1) * 8);
    const size_t o_nn = o_sz + al(((size_t)n_batches + 2) * 4), m = (size_t)max_qdesc * k;
    const size_t o_mi = o_nn + al(m * 4), o_ex = o_mi + al(m * 4), o_di = o_ex + al(m * 4);
    const size_t o_vo = o_di + al(m * 4), o_wi = o_vo + al((size_t)max_qobj * n_obj * 4);
    const size_t o_us = o_wi + al((size_t)max_qobj * 4), o_ws = o_us + al((size_t)max_qobj * 4);
    const size_t total = o_ws + al(ws_bytes);
    if (hipMalloc((void **)&p->mem, total) != hipSuccess) {
        plan_release(p);
        return fail(QD_ERR_OOM, "plan allocation of %zu bytes failed", total);
    }
    p->q = (uint64_t *)(p->mem + o_q);
    p->qoff = (uint64_t *)(p->mem + o_off);
    p->sizes = (uint32_t *)(p->mem + o_sz);
    p->nn = (uint32_t *)(p->mem + o_nn);
    p->mi = (int32_t *)(p->mem + o_mi);
    p->ex = (int32_t *)(p->mem + o_ex);
    p->di = (float *)(p->mem + o_di);
    p->votes = (uint32_t *)(p->mem + o_vo);
    p->winner = (int32_t *)(p->mem + o_wi);
    p->used = (uint32_t *)(p->mem + o_us);
    p->ws = p->mem + o_ws;
    // record the batch into a graph on a private stream (default priority)
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        plan_release(p);
        return fail(QD_ERR_DEVICE, "stream creation failed");
    }
    int rc = QD_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        if (blocked) {
            // batches of KL.qb descriptors, each with its size on the device
            hipLaunchKernelGGL(batch_sizes_kernel, dim3((n_batches + 255) / 256), dim3(256), 0, cs, p->sizes,
                               n_batches, KL.qb);
            for (uint32_t i = 0; i < n_batches && rc == QD_OK; i++) {
                const uint64_t b0 = (uint64_t)i * KL.qb;
                const uint32_t nqb = (uint32_t)std::min<uint64_t>(KL.qb, nqmax - b0);
                const uint64_t o = b0 * k;
                rc = blocked_batch(t, KL, p->ws, p->q + b0 * QD_WORDS, nqb, p->sizes + 2 + i, k, params, p->nn + o,
                                   p->mi + o, p->ex + o, p->di + o, nullptr, nullptr, /*graph=*/true, cs);
            }
        } else if (mfma) {
            rc = mfma_run(ML, p->ws, d_db, p->q, nqmax, p->sizes, k, p->nn, p->mi, p->ex, p->di, cs);
        } else if (t)
            rc = tree_launch(t, TL, p->ws, p->q, nqmax, p->sizes, k, order, nullptr, 0, p->nn, p->mi, p->ex, p->di,
                             nullptr, nullptr, 0, cs);
        else
            rc = brute_launch(BL, reinterpret_cast<u64 *>(p->ws), d_db, n, p->q, nqmax, p->sizes, k, p->nn, p->mi,
                              p->ex, p->di, cs);
        if (rc == QD_OK)
            rc = vote_launch(p->nn, k, d_obj_of, p->n, n_obj, p->qoff, max_qobj, p->sizes + 1, vote_threshold,
                             p->votes, p->winner, p->used, cs);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        p->graph = g;
        if (rc == QD_OK && e2 != hipSuccess) rc = fail(QD_ERR_DEVICE, "graph capture: %s", hipGetErrorString(e2));
    } else {
        rc = fail(QD_ERR_DEVICE, "begin capture: %s", hipGetErrorString(e));
    }
    if (rc == QD_OK) {
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(QD_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
    (void)hipStreamDestroy(cs);
    if (rc != QD_OK) {
        plan_release(p);
        return rc;
    }
    *out = p;
    return QD_OK;
}

extern "C" int qd_plan_run(qd_plan_t p, const uint64_t *d_qdesc, uint64_t n_qdesc, const uint64_t *d_qoff,
                           uint32_t nqo, uint32_t *d_votes, int32_t *d_winner, uint32_t *d_used, void *stream) {
    using namespace qd;
    if (!p) return fail(QD_ERR_INVALID, "null plan");
    if (n_qdesc > p->max_qdesc || nqo > p->max_qobj)
        return fail(QD_ERR_INVALID, "batch (%llu descriptors, %u objects) above the plan's capacity", (u64)n_qdesc,
                    nqo);
    if (nqo == 0) return QD_OK;
    if (!d_qoff || !d_votes || !d_winner || !d_used || (n_qdesc && !d_qdesc)) return fail(QD_ERR_INVALID, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    if (n_qdesc) QD_HIP_CHECK(hipMemcpyAsync(p->q, d_qdesc, n_qdesc * 512, hipMemcpyDeviceToDevice, s));
    QD_HIP_CHECK(hipMemcpyAsync(p->qoff, d_qoff, ((size_t)nqo + 1) * 8, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(set_sizes_kernel, dim3(1), dim3(1), 0, s, p->sizes, (uint32_t)n_qdesc, nqo);
    QD_HIP_CHECK(hipGetLastError());
    {
        KernelTimer timer("plan_graph", s);
        QD_HIP_CHECK(hipGraphLaunch(p->exec, s));
    }
    QD_HIP_CHECK(hipMemcpyAsync(d_votes, p->votes, (size_t)nqo * p->n_obj * 4, hipMemcpyDeviceToDevice, s));
    QD_HIP_CHECK(hipMemcpyAsync(d_winner, p->winner, (size_t)nqo * 4, hipMemcpyDeviceToDevice, s));
    QD_HIP_CHECK(hipMemcpyAsync(d_used, p->used, (size_t)nqo * 4, hipMemcpyDeviceToDevice, s));
    return QD_OK;
}

extern "C" int qd_plan_free(qd_plan_t p) {
    qd::plan_release(p);
    return QD_OK;
}

// ---- autotuner ------------------------------------------------------------

namespace qd {
int knn_bruteforce_impl(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                        uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream,
                        uint32_t qt_force, uint32_t parts_force);

namespace {
using TuneKey = std::tuple<int, uint64_t, uint64_t, uint32_t, uint32_t, uint32_t>;  // device, n, nodes, nq, k, mask
std::mutex g_tune_mu;
std::map<TuneKey, qd_tuning> g_tune;
bool g_tune_loaded = false;

// Optional file cache: one line per entry,
// "dev n nodes nq k mask path order wpc qt ms round1 round2 growth start".
void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = getenv("QD_TUNE_CACHE");
    if (!f) return;
    FILE *fp = fopen(f, "r");
    if (!fp) return;
    int dev, path, order;
    unsigned long long n, nodes;
    unsigned nq, k, mask, wpc, qt, r1, r2, gr, st;
    float ms;
    while (fscanf(fp, "%d %llu %llu %u %u %u %d %d %u %u %f %u %u %u %u", &dev, &n, &nodes, &nq, &k, &mask, &path,
                  &order, &wpc, &qt, &ms, &r1, &r2, &gr, &st) == 15) {
        qd_tuning t{path, (qd_order)order, wpc, qt, ms, r1, r2, gr, st};
        g_tune[TuneKey{dev, n, nodes, nq, k, mask}] = t;
    }
    fclose(fp);
}

void tune_store(const TuneKey &key, const qd_tuning &t) {
    g_tune[key] = t;
    const char *f = getenv("QD_TUNE_CACHE");
    if (!f) return;
    FILE *fp = fopen(f, "a");
    if (!fp) return;
    fprintf(fp, "%d %llu %llu %u %u %u %d %d %u %u %.6f %u %u %u %u\n", std::get<0>(key),
            (unsigned long long)std::get<1>(key), (unsigned long long)std::get<2>(key), std::get<3>(key),
            std::get<4>(key), std::get<5>(key), t.path, (int)t.order, t.waves_per_cu, t.query_tile, t.ms,
            t.round1_blocks, t.round2_blocks, t.round_growth, t.round1_start);
    fclose(fp);
}
}  // namespace
}  // namespace qd

extern "C" int qd_autotune(qd_tree_t t, const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq,
                           uint32_t k, uint32_t reps, uint32_t order_mask, qd_tuning *best, qd_tuning *all,
                           uint32_t max_all, uint32_t *n_all, void *stream) {
    using namespace qd;
    if (!best || (!t && (!d_db || n < 1)) || !d_q || nq == 0) return fail(QD_ERR_INVALID, "bad autotune arguments");
    if (k < 1 || k > QD_MAX_K) return fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
    if (reps == 0) reps = 3;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const uint32_t all_orders = (1u << QD_ORDER_BEST_FIRST) | (1u << QD_ORDER_DEPTH_FIRST) | (1u << QD_ORDER_BLOCKED);
    const uint32_t mask = t ? (order_mask ? order_mask & all_orders : all_orders) : 0;
    if (t && mask == 0) return fail(QD_ERR_INVALID, "order_mask 0x%x names no frontier order", order_mask);
    const TuneKey key{dev, t ? t->n : n, t ? t->n_nodes : 0, nq, k, mask};
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_load();
        auto it = g_tune.find(key);
        if (it != g_tune.end() && !all) {
            *best = it->second;
            if (n_all) *n_all = 0;
            return QD_OK;
        }
    }
    std::vector<qd_tuning> cand;
    if (t) {
        for (int order : {QD_ORDER_BEST_FIRST, QD_ORDER_DEPTH_FIRST})
            for (uint32_t wpc : {4u, 8u, 12u, 16u, 32u}) {
                if (!(mask & (1u << order))) continue;
                // best-first: registers hold 12 waves per CU; depth-first: 16
                if (order == QD_ORDER_BEST_FIRST ? wpc > 12 : wpc == 12) continue;
                cand.push_back({1, (qd_order)order, wpc, 0, 0.f, 0, 0, 0, 0});
            }
        // the blocked order's round schedule around its default (16 blocks in
        // round 1, round 2 at ~128 queries per block list, growth 4)
        const uint64_t t2 = std::max<uint64_t>(32, (128 * t->n_blk + nq - 1) / nq);
        const uint32_t half = (uint32_t)std::min<uint64_t>(t2 / 2, 0xFFFFFFFFull);
        const uint32_t dbl = (uint32_t)std::min<uint64_t>(t2 * 2, 0xFFFFFFFFull);
        const uint32_t sched[][4] = {{16, 0, 4, 0}, {8, 0, 4, 0}, {32, 0, 4, 0}, {16, 0, 2, 0}, {16, 0, 8, 0},
                                     {16, half, 4, 0}, {16, dbl, 4, 0}, {16, 0, 4, 1}, {8, 0, 4, 1}};
        if (mask & (1u << QD_ORDER_BLOCKED))
            for (auto &sc : sched) cand.push_back({1, QD_ORDER_BLOCKED, 0, 0, 0.f, sc[0], sc[1], sc[2], sc[3]});
    } else {
        for (uint32_t qt : {0u, 4u, 8u, 16u, QD_QUERY_TILE_MATRIX})
            cand.push_back({0, QD_ORDER_BEST_FIRST, 0, qt, 0.f, 0, 0, 0, 0});
    }
    char *ws = nullptr;
    const size_t m = (size_t)nq * k;
    QD_HIP_CHECK(hipMallocAsync((void **)&ws, m * 16, s));
    uint32_t *idx = (uint32_t *)ws;
    int32_t *mi = (int32_t *)(ws + m * 4), *ex = (int32_t *)(ws + m * 8);
    float *di = (float *)(ws + m * 12);
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    int rc = QD_OK;
    for (auto &c : cand) {
        if (abort_requested()) {  // between candidates
            rc = fail(QD_ERR_ABORTED, "autotune aborted");
            break;
        }
        auto run = [&]() {
            if (c.path && c.order == QD_ORDER_BLOCKED) {
                qd_search_params sp{};
                sp.order = QD_ORDER_BLOCKED;
                sp.round1_blocks = c.round1_blocks;
                sp.round2_blocks = c.round2_blocks;
                sp.round_growth = c.round_growth;
                sp.round1_start = c.round1_start;
                return knn_tree_blocked(t, d_q, nq, k, &sp, idx, mi, ex, di, nullptr, nullptr, s);
            }
            return c.path ? knn_tree_impl(t, d_q, nq, k, (int)c.order, nullptr, 0, idx, mi, ex, di, nullptr, nullptr,
                                          stream, c.waves_per_cu, nullptr, 0)
                          : knn_bruteforce_impl(d_db, n, d_q, nq, k, idx, mi, ex, di, stream, c.query_tile, 0);
        };
        rc = run();  // warm-up
        if (rc != QD_OK) break;
        (void)hipEventRecord(a, s);
        for (uint32_t r = 0; r < reps && rc == QD_OK; r++) rc = run();
        (void)hipEventRecord(b, s);
        if (rc != QD_OK) break;
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        c.ms = ms / reps;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFreeAsync(ws, s);
    if (rc != QD_OK) return rc;
    size_t bi = 0;
    for (size_t i = 1; i < cand.size(); i++)
        if (cand[i].ms < cand[bi].ms) bi = i;
    *best = cand[bi];
    if (all) {
        const uint32_t na = (uint32_t)std::min<size_t>(cand.size(), max_all);
        for (uint32_t i = 0; i < na; i++) all[i] = cand[i];
        if (n_all) *n_all = na;
    } else if (n_all) {
        *n_all = 0;
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_store(key, *best);
    return QD_OK;
}

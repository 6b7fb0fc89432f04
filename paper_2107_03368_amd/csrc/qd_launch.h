// Launch helpers shared by the search entry points and the captured plans:
// every launch takes its scratch from the caller and may read its batch size
// from device memory, so a plan can record it once in a hipGraph.
#pragma once

#include <vector>

#include "qd_internal.h"

namespace qd {

struct TreeLaunch {
    uint64_t blocks = 0, slots = 0, pool_chunks = 0;
    uint32_t split = 1;  // concurrent subtree searches per query
    size_t head = 0, prev_bytes = 0, pool_bytes = 0;
    size_t split_bytes = 0;  // after the pool: the searches' lists and statistics, merged into the results
    size_t total() const { return head + prev_bytes + pool_bytes + split_bytes; }
};
// Per-query orders on up to nq_max queries with k neighbours; split = 0
// picks the default number of subtree searches per query (1: none).
TreeLaunch tree_launch_shape(qd_tree_t t, uint32_t nq_max, uint32_t k, int order, uint32_t waves_per_cu,
                             uint32_t split);
bool split_ok(uint32_t split);  // 0 or a power of two up to 16
// The per-query and blocked orders behind qd_knn_tree (split: as in
// tree_launch_shape; a traced search runs unsplit).
int knn_tree_impl(qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k, int order, const float *d_scores,
                  uint32_t n_scored, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist,
                  uint32_t *d_qstats, qd_stats *h_stats, void *stream, uint32_t waves_per_cu, uint32_t *d_trace,
                  uint32_t n_traced, uint32_t split = 0);
// The depth-first order's LDS stack holds the tree's depth.
bool depth_first_fits(qd_tree_t t);
int tree_launch(qd_tree_t t, const TreeLaunch &L, char *ws, const uint64_t *d_q, uint32_t nq,
                const uint32_t *nq_dev, uint32_t k, int order, const float *d_scores, uint32_t n_scored,
                uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, uint32_t *d_qstats,
                uint32_t *d_trace, uint32_t n_traced, hipStream_t s);

// The blocked tree search (QD_ORDER_BLOCKED) on a workspace the caller
// owns: batches of up to qb queries, byte offsets of every buffer in it.
struct BlockedLayout {
    uint32_t qb = 0;
    size_t qpop = 0, lbq = 0, lbb = 0, list = 0, cuts = 0, r1 = 0, rec = 0, thr = 0, ntop = 0, top = 0, ccnt = 0,
           cand = 0, cnt = 0, qr = 0, act = 0, off = 0, voff = 0, ctr = 0, done = 0, fr = 0, tinfo = 0, redo = 0,
           qst = 0, lnode = 0, gst = 0, fbq = 0, fbr = 0, fbws = 0, mdesc = 0, bytes = 0;
    bool model = false;  // the layout holds a learned start's descent workspace (at mdesc)
    TreeLaunch fb;       // the per-query fallback's launch
    int fb_order = QD_ORDER_DEPTH_FIRST;
};
int blocked_check(qd_tree_t t, const qd_search_params *p);
BlockedLayout blocked_layout(qd_tree_t t, uint32_t nq_max, uint32_t k, bool model = false);
// One batch of nqb queries (at most L.qb); nq_dev (nullable): the batch's
// size on the device.  graph: no host synchronisation (capturable).
int blocked_batch(qd_tree_t t, const BlockedLayout &L, char *ws, const uint64_t *d_q, uint32_t nqb,
                  const uint32_t *nq_dev, uint32_t k, const qd_search_params *p, uint32_t *d_idx, int32_t *d_missed,
                  int32_t *d_extra, float *d_dist, uint32_t *d_qstats, unsigned long long *gst, bool graph,
                  hipStream_t s);

// Batches of at least this many queries scan in tiles of 16 queries on the
// matrix cores (QD_QUERY_TILE_MATRIX), smaller ones on the vector ALUs.
constexpr uint32_t kSmallMfmaMinQueries = 3;
struct BruteLaunch {
    uint32_t qt = 0, n_qtiles = 0, n_parts = 0;
    uint64_t rows_per_part = 0, blocks = 0;
    size_t part_bytes = 0;
};
BruteLaunch brute_launch_shape(uint64_t n, uint32_t nq_max, uint32_t k, uint32_t qt_force, uint32_t parts_force);
int brute_launch(const BruteLaunch &L, u64 *part, const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq,
                 const uint32_t *nq_dev, uint32_t k, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra,
                 float *d_dist, hipStream_t s, bool timed = true);

// The matrix-core sequential search on a workspace the caller owns.  Level
// l searches the first rows[l] rows; every level but the last is a
// matrix-core pass whose candidate bounds come from the next level (a
// sample), the last level is the row scan.  Smaller batches take the row
// scan alone: its 16-query matrix tiles make one pass over the rows per tile,
// while the 256 x 256 tiles here cost the same for 1 to 256 queries; the two
// break even at about 160 queries.
constexpr uint32_t kMfmaMinQueries = 160;
constexpr uint64_t kMfmaMinRows = 1u << 16;
constexpr int kMaxLevels = 4;
struct MfmaLayout {
    std::vector<uint64_t> rows;
    BruteLaunch base, fb[kMaxLevels];
    size_t tpop = 0, qpop = 0, cnt = 0, cand = 0, redo = 0, ctr = 0, thr[kMaxLevels] = {}, smp[kMaxLevels] = {},
           base_part = 0, gq = 0, fbr = 0, fb_part = 0, bytes = 0;
};
// Whether a batch of nq queries over n rows takes the matrix cores.
bool mfma_eligible(uint64_t n, uint32_t nq, uint32_t k);
MfmaLayout mfma_layout(uint64_t n, uint32_t nq_max, uint32_t k);
// nq_dev (nullable): the batch's size on the device (<= nq).  Never waits for the host.
int mfma_run(const MfmaLayout &L, char *ws, const uint64_t *d_db, const uint64_t *d_q, uint32_t nq,
             const uint32_t *nq_dev, uint32_t k, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist,
             hipStream_t s);

int vote_launch(const uint32_t *nn, uint32_t k, const uint16_t *obj_of, uint64_t n_db, uint32_t n_obj,
                const uint64_t *qoff, uint32_t nqo, const uint32_t *nqo_dev, uint32_t threshold, uint32_t *votes,
                int32_t *winner, uint32_t *used, hipStream_t s, const uint64_t *qend = nullptr);

}  // namespace qd

// Launch helpers shared by the search entry points and the captured plans:
// every launch takes its scratch from the caller and may read its batch size
// from device memory, so a plan can record it once in a hipGraph.
#pragma once

#include "qd_internal.h"

namespace qd {

struct TreeLaunch {
    uint64_t blocks = 0, slots = 0, pool_chunks = 0;
    size_t head = 0, prev_bytes = 0, pool_bytes = 0;
    size_t total() const { return head + prev_bytes + pool_bytes; }
};
TreeLaunch tree_launch_shape(qd_tree_t t, uint32_t nq_max, int order, uint32_t waves_per_cu);
int tree_launch(qd_tree_t t, const TreeLaunch &L, char *ws, const uint64_t *d_q, uint32_t nq,
                const uint32_t *nq_dev, uint32_t k, int order, const float *d_scores, uint32_t n_scored,
                uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, uint32_t *d_qstats,
                uint32_t *d_trace, uint32_t n_traced, hipStream_t s);

struct BruteLaunch {
    uint32_t qt = 0, n_qtiles = 0, n_parts = 0;
    uint64_t rows_per_part = 0, blocks = 0;
    size_t part_bytes = 0;
};
BruteLaunch brute_launch_shape(uint64_t n, uint32_t nq_max, uint32_t k, uint32_t qt_force, uint32_t parts_force);
int brute_launch(const BruteLaunch &L, u64 *part, const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq,
                 const uint32_t *nq_dev, uint32_t k, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra,
                 float *d_dist, hipStream_t s, bool timed = true);

int vote_launch(const uint32_t *nn, uint32_t k, const uint16_t *obj_of, uint64_t n_db, uint32_t n_obj,
                const uint64_t *qoff, uint32_t nqo, const uint32_t *nqo_dev, uint32_t threshold, uint32_t *votes,
                int32_t *winner, uint32_t *used, hipStream_t s, const uint64_t *qend = nullptr);

}  // namespace qd

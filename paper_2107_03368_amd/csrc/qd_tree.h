// Library-owned Dissimilarity Tree (opaque to callers as qd_tree_t).
#pragma once

#include <vector>

#include "qd_internal.h"

struct qd_tree_s {
    int device = 0;
    uint64_t n = 0;         // database rows
    uint64_t n_nodes = 0;   // breadth-first numbered, root 0
    uint64_t n_leaves = 0;
    uint32_t depth = 0;     // number of levels
    uint32_t max_leaf = 32;
    bool has_and = false;
    uint64_t *d_sorted = nullptr;  // n x 64 words: rows in leaf order
    uint32_t *d_perm = nullptr;    // n: database row of each leaf-order position
    uint64_t *d_or = nullptr;      // n_nodes x 64 words: sum (OR) image
    uint64_t *d_and = nullptr;     // n_nodes x 64 words: product (AND) image, optional
    int32_t *d_child = nullptr;    // n_nodes x 2: similar, dissimilar (-1 for a leaf)
    uint32_t *d_begin = nullptr;   // n_nodes: first leaf-order position
    uint32_t *d_count = nullptr;   // n_nodes: rows under the node
    uint16_t *d_pop = nullptr;     // n: popcount of each leaf-order row
    int32_t *d_parent = nullptr;   // n_nodes: parent node (-1 for the root)
    uint8_t *d_depth = nullptr;    // n_nodes: level of the node (root 0)
    uint32_t *d_iperm = nullptr;   // n: leaf-order position of each database row
    uint16_t *d_pmin = nullptr;    // n_nodes: smallest row popcount under the node (null: plain bound)
    uint16_t *d_pmax = nullptr;    // n_nodes: largest row popcount under the node
    uint64_t n_blk = 0;            // blocks of 256 leaf-order rows
    uint64_t *d_blk = nullptr;     // n_blk x 64 words: OR image of each block's rows
    uint16_t *d_bpop = nullptr;    // n_blk x 2: smallest, largest row popcount of each block (null: plain)
    std::vector<uint32_t> level_max;  // host: most rows of any node of each level (root level 0)
    // The per-query search split into n = 2^e subtree searches (e = 0..4):
    // d_split_roots[n - 1 .. 2n - 2] are the n subtree roots (-1: none) and
    // split_nodes[e] the most nodes any of them holds.
    int32_t *d_split_roots = nullptr;  // 31 entries
    uint64_t split_nodes[5] = {};
};

namespace qd {
struct TreeLaunch;  // qd_launch.h
void tree_release(qd_tree_s *t);
// Completes a tree whose n, n_nodes, max_leaf, has_and, d_sorted (rows in
// leaf order) and d_perm are set, from its breadth-first structure (child
// pairs, begin, count): uploads the structure, derives parents, levels,
// popcounts, images, popcount ranges (want_pop), the inverse permutation and
// the block images.  Synchronous; on failure it releases t.
// Learned start of the blocked search: d_node[i] = the node reached from the
// root by entering, at every inner node holding more than max_rows rows, the
// child the model scores higher for query i (ties: the similar child).
// ws (nullable): a workspace of model_descend_bytes(nq) the caller owns
// (nothing is allocated then, so the launches can be captured); without it
// the call allocates one.
size_t model_descend_bytes(uint32_t nq);
int model_descend(qd_model_t m, qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t max_rows, uint32_t *d_node,
                  char *ws, hipStream_t s);
int tree_finish(qd_tree_s *t, const std::vector<int32_t> &child, const std::vector<uint32_t> &begin,
                const std::vector<uint32_t> &count, bool want_pop, hipStream_t s);
// Block images for the batched search (tree_blocked.hip).
int tree_block_images(qd_tree_s *t, hipStream_t s);
int knn_tree_blocked(qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k, const qd_search_params *p,
                     uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, uint32_t *d_qstats,
                     qd_stats *h_stats, hipStream_t s);
}

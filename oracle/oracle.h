/* CPU oracle for Weighted Hamming search over 64x64-bit QUICCI descriptors.
 * Test infrastructure only (see oracle.c); not part of the GPU library. */
#ifndef QD_ORACLE_H
#define QD_ORACLE_H
#include <stdint.h>

void or_wh_literal(const uint64_t *q, const uint64_t *t, int64_t *A, int64_t *B, int64_t *P);
double or_wh_eq1(int64_t A, int64_t B, int64_t P);
int64_t or_wh_key(int64_t A, int64_t B, int64_t P);
float or_wh_dist(int64_t A, int64_t B, int64_t P);
int or_knn_brute(const uint64_t *db, int64_t n, const uint64_t *q, int64_t nq, int k, uint32_t *idx,
                 int32_t *missed, int32_t *extra, float *dist);
int64_t or_split_node(const uint64_t *db, const uint32_t *mem, int64_t n, uint8_t *side);
int64_t or_tree_build(const uint64_t *db, int64_t n, int max_leaf, int64_t cap, int32_t *child, int64_t *begin,
                      int64_t *count, uint64_t *or_img, uint64_t *and_img, uint32_t *perm);
int64_t or_node_bound(const uint64_t *q, const uint64_t *or_img, const uint64_t *and_img);
int64_t or_node_bound_pop(const uint64_t *q, const uint64_t *or_img, const uint64_t *and_img, int64_t pmin,
                          int64_t pmax);
int or_tree_knn(const uint64_t *db, const int32_t *child, const int64_t *begin, const int64_t *count,
                const uint64_t *or_img, const uint64_t *and_img, const int64_t *pmin, const int64_t *pmax,
                const uint32_t *perm, int64_t n_nodes,
                const uint64_t *q, int64_t nq, int k, const int64_t *score, uint32_t *idx, int32_t *missed,
                int32_t *extra, float *dist, int64_t *stats);
void or_votes(const uint32_t *nn_idx, int k, const uint16_t *obj_of, int64_t n_db, int64_t n_obj,
              const uint64_t *qoff, int64_t nqo, int64_t threshold, uint32_t *votes, int32_t *winner,
              uint32_t *used);
void or_object_scores(const uint64_t *db, int64_t n, const uint16_t *obj_of, int64_t n_obj, const uint64_t *q,
                      const uint64_t *qoff, int64_t nqo, double *scores);
void or_score_rows(double *scores, int64_t nqo, int64_t n_obj, int normalize, int32_t *best);
#endif

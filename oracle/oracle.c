/*
 * CPU ORACLE for Weighted Hamming search over 64x64-bit QUICCI descriptors.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product library never
 * calls it and shares no code with it.
 *
 * Paper: van Blokland & Theoharis, "Partial 3D Object Retrieval using Local
 * Binary QUICCI Descriptors and Dissimilarity Tree Indexing" (2021).
 *
 * Descriptor: uint64[64]; word r is image row r, bit c of it is column c.
 * The image is N x N = 64 x 64 bits (Section 6).  Bit positions enter the
 * distance only pairwise, so the row/column convention matters only for the
 * tie order of equally popular bits in the tree build (reading: ascending
 * b = 64*r + c).
 *
 * Readings of the paper that this file fixes (each is also listed in the
 * design notes):
 *  - Eq. 1's second denominator is max(N*N - |q|, 1): the number of type B
 *    errors that can occur (Section 2.3 prose; the query listing uses
 *    len(query) - popcnt(query)).
 *  - Ranking uses the exact integer key K = A*wB + B*wA = d*wA*wB with
 *    wA = max(|q|,1), wB = max(4096-|q|,1); ties in K are broken by ascending
 *    database index.  The reported distance is the double quotient K/(wA*wB)
 *    rounded to float.
 *  - Tree build (Listing 1): bit popularity is computed once per node; bits
 *    are taken in ascending (popularity, bit index); after each bit's move the
 *    split stops once the dissimilar side holds at least half the node; a move
 *    that would empty the similar side is not applied and ends the split; a
 *    node is a leaf when it holds at most max_leaf descriptors or when no
 *    split is possible.  Sum (OR) and product (AND) images are stored for
 *    every node, leaves included.
 *  - Tree query (Listing 2): best-first on the lower bound; a node is pushed
 *    and processed when fewer than k results exist or its bound is <= the
 *    current k-th key (tie-inclusive, so index tie-breaks match the brute
 *    force); the search stops at the first popped node whose bound exceeds
 *    the k-th key.  The bound uses the sum image (the product-image term is
 *    optional; the paper omits the product image for sparse QUICCI).
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define OR_WORDS 64
#define OR_NBITS 4096 /* N*N with N = 64 */

static inline int bit_of(const uint64_t *d, int r, int c) { return (int)((d[r] >> c) & 1ULL); }

/* ---------------------------------------------------------------------------
 * Eq. 1, written out over rows r and columns c.
 *   A = sum q[r,c] * (1 - t[r,c])      type A errors (Section 2.3)
 *   B = sum (1 - q[r,c]) * t[r,c]      type B errors
 *   P = sum q[r,c]                     |q|
 * ------------------------------------------------------------------------- */
void or_wh_literal(const uint64_t *q, const uint64_t *t, int64_t *A, int64_t *B, int64_t *P) {
    int64_t a = 0, b = 0, p = 0;
    for (int r = 0; r < 64; r++)
        for (int c = 0; c < 64; c++) {
            int qb = bit_of(q, r, c), tb = bit_of(t, r, c);
            a += qb * (1 - tb);
            b += (1 - qb) * tb;
            p += qb;
        }
    *A = a;
    *B = b;
    *P = p;
}

/* Eq. 1 as printed, in double: A / max(|q|,1) + B / max(N*N - |q|, 1). */
double or_wh_eq1(int64_t A, int64_t B, int64_t P) {
    double wa = P > 1 ? (double)P : 1.0;
    double wb = (OR_NBITS - P) > 1 ? (double)(OR_NBITS - P) : 1.0;
    return (double)A / wa + (double)B / wb;
}

static inline int64_t w_a(int64_t P) { return P > 1 ? P : 1; }
static inline int64_t w_b(int64_t P) { return (OR_NBITS - P) > 1 ? (OR_NBITS - P) : 1; }

/* Integer rank key: d * wA * wB exactly. */
int64_t or_wh_key(int64_t A, int64_t B, int64_t P) { return A * w_b(P) + B * w_a(P); }

/* Reported distance: the key over wA*wB as one double division, then float. */
float or_wh_dist(int64_t A, int64_t B, int64_t P) {
    return (float)((double)or_wh_key(A, B, P) / ((double)w_a(P) * (double)w_b(P)));
}

/* Type A / type B counts by whole words: a bit of (q AND NOT t) is exactly a
 * position with q = 1, t = 0; a bit of (NOT q AND t) one with q = 0, t = 1. */
static inline void wh_counts(const uint64_t *q, const uint64_t *t, int64_t *A, int64_t *B) {
    int64_t a = 0, b = 0;
    for (int w = 0; w < OR_WORDS; w++) {
        a += __builtin_popcountll(q[w] & ~t[w]);
        b += __builtin_popcountll(~q[w] & t[w]);
    }
    *A = a;
    *B = b;
}

static inline int64_t popcount_desc(const uint64_t *d) {
    int64_t p = 0;
    for (int w = 0; w < OR_WORDS; w++) p += __builtin_popcountll(d[w]);
    return p;
}

typedef struct {
    int64_t key;
    int64_t idx;
    int64_t A, B;
} or_cand;

static int cand_cmp(const void *x, const void *y) {
    const or_cand *a = (const or_cand *)x, *b = (const or_cand *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

static void emit(const or_cand *R, int64_t nr, int64_t P, int k, uint32_t *idx, int32_t *missed, int32_t *extra,
                 float *dist) {
    for (int r = 0; r < k; r++) {
        if (r < nr) {
            idx[r] = (uint32_t)R[r].idx;
            missed[r] = (int32_t)R[r].A;
            extra[r] = (int32_t)R[r].B;
            dist[r] = or_wh_dist(R[r].A, R[r].B, P);
        } else {
            idx[r] = 0xFFFFFFFFu;
            missed[r] = -1;
            extra[r] = -1;
            dist[r] = __builtin_inff();
        }
    }
}

/* ---------------------------------------------------------------------------
 * Sequential (brute-force) k-nearest-neighbour search: every database row is
 * scored, all are sorted by (K, index), the first k are returned.  This is
 * the paper's reference "sequential search" (Section 6.2).
 * ------------------------------------------------------------------------- */
int or_knn_brute(const uint64_t *db, int64_t n, const uint64_t *q, int64_t nq, int k, uint32_t *idx,
                 int32_t *missed, int32_t *extra, float *dist) {
    if (k <= 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < nq; j++) {
        const uint64_t *qj = q + j * OR_WORDS;
        int64_t P = popcount_desc(qj);
        or_cand *all = (or_cand *)malloc((size_t)(n > 0 ? n : 1) * sizeof(or_cand));
        for (int64_t i = 0; i < n; i++) {
            int64_t A, B;
            wh_counts(qj, db + i * OR_WORDS, &A, &B);
            all[i].key = or_wh_key(A, B, P);
            all[i].idx = i;
            all[i].A = A;
            all[i].B = B;
        }
        qsort(all, (size_t)n, sizeof(or_cand), cand_cmp);
        emit(all, n < k ? n : k, P, k, idx + j * k, missed + j * k, extra + j * k, dist + j * k);
        free(all);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Dissimilarity Tree construction (Section 4.1, Listing 1).
 * ------------------------------------------------------------------------- */

typedef struct {
    uint32_t cnt;
    uint32_t bit;
} bitpop;

static int bitpop_cmp(const void *x, const void *y) {
    const bitpop *a = (const bitpop *)x, *b = (const bitpop *)y;
    if (a->cnt != b->cnt) return a->cnt < b->cnt ? -1 : 1;
    return a->bit < b->bit ? -1 : (a->bit > b->bit);
}

/* Split one node holding members mem[0..n-1] (database rows, in the node's
 * order).  side[j] becomes 1 when member j goes to the dissimilar subset.
 * Returns the size of the dissimilar subset.
 *   1. popularity of every bit over the node's descriptors;
 *   2. bit positions in ascending popularity (ties: ascending bit index);
 *   3. for each bit in that order, every descriptor still in the similar set
 *      that has the bit set moves to the dissimilar set, keeping order;
 *      stop once the dissimilar set holds at least half of the node, and do
 *      not apply a move that would leave the similar set empty. */
int64_t or_split_node(const uint64_t *db, const uint32_t *mem, int64_t n, uint8_t *side) {
    bitpop order[OR_NBITS];
    for (int b = 0; b < OR_NBITS; b++) {
        order[b].cnt = 0;
        order[b].bit = (uint32_t)b;
    }
    for (int64_t j = 0; j < n; j++) {
        const uint64_t *d = db + (uint64_t)mem[j] * OR_WORDS;
        for (int r = 0; r < 64; r++)
            for (int c = 0; c < 64; c++) order[64 * r + c].cnt += (uint32_t)bit_of(d, r, c);
    }
    qsort(order, OR_NBITS, sizeof(bitpop), bitpop_cmp);

    int64_t *S = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t nS = n, nD = 0;
    for (int64_t j = 0; j < n; j++) {
        S[j] = j;
        side[j] = 0;
    }
    for (int o = 0; o < OR_NBITS; o++) {
        int b = (int)order[o].bit, r = b >> 6, c = b & 63;
        int64_t moving = 0;
        for (int64_t j = 0; j < nS; j++) moving += bit_of(db + (uint64_t)mem[S[j]] * OR_WORDS, r, c);
        if (moving == 0) continue;
        if (moving == nS) break; /* would leave the similar set empty */
        int64_t keep = 0;
        for (int64_t j = 0; j < nS; j++) {
            if (bit_of(db + (uint64_t)mem[S[j]] * OR_WORDS, r, c))
                side[S[j]] = 1;
            else
                S[keep++] = S[j];
        }
        nS = keep;
        nD += moving;
        if (2 * nD >= n) break;
    }
    free(S);
    return nD;
}

/* Build the whole tree.  Nodes are numbered breadth first (root 0; within a
 * level, similar child before dissimilar child, parents in order), which is
 * the order a FIFO of pending nodes produces.  Node i holds the rows
 * perm[begin[i] .. begin[i]+count[i]-1]; a split writes the similar rows
 * first, then the dissimilar rows, each in their previous relative order.
 * child[2i], child[2i+1] = similar, dissimilar child, or -1 for a leaf.
 * Returns the number of nodes, or -1 if cap is too small. */
int64_t or_tree_build(const uint64_t *db, int64_t n, int max_leaf, int64_t cap, int32_t *child, int64_t *begin,
                      int64_t *count, uint64_t *or_img, uint64_t *and_img, uint32_t *perm) {
    if (n <= 0 || cap < 1) return -1;
    for (int64_t i = 0; i < n; i++) perm[i] = (uint32_t)i;
    int64_t nn = 1;
    begin[0] = 0;
    count[0] = n;
    uint8_t *side = (uint8_t *)malloc((size_t)n);
    uint32_t *tmp = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    for (int64_t i = 0; i < nn; i++) {
        child[2 * i] = child[2 * i + 1] = -1;
        int64_t b0 = begin[i], m = count[i];
        if (m <= max_leaf) continue;
        int64_t nD = or_split_node(db, perm + b0, m, side);
        if (nD == 0 || nD == m) continue; /* no split possible: oversized leaf */
        if (nn + 2 > cap) {
            free(side);
            free(tmp);
            return -1;
        }
        int64_t s = 0, d = m - nD;
        for (int64_t j = 0; j < m; j++) {
            if (side[j])
                tmp[d++] = perm[b0 + j];
            else
                tmp[s++] = perm[b0 + j];
        }
        memcpy(perm + b0, tmp, (size_t)m * sizeof(uint32_t));
        child[2 * i] = (int32_t)nn;
        begin[nn] = b0;
        count[nn] = m - nD;
        nn++;
        child[2 * i + 1] = (int32_t)nn;
        begin[nn] = b0 + m - nD;
        count[nn] = nD;
        nn++;
    }
    free(side);
    free(tmp);
    for (int64_t i = 0; i < nn; i++) {
        uint64_t *o = or_img + i * OR_WORDS;
        uint64_t *a = and_img ? and_img + i * OR_WORDS : NULL;
        for (int w = 0; w < OR_WORDS; w++) {
            o[w] = 0;
            if (a) a[w] = ~0ULL;
        }
        for (int64_t j = begin[i]; j < begin[i] + count[i]; j++) {
            const uint64_t *d = db + (uint64_t)perm[j] * OR_WORDS;
            for (int w = 0; w < OR_WORDS; w++) {
                o[w] |= d[w];
                if (a) a[w] &= d[w];
            }
        }
    }
    return nn;
}

/* ---------------------------------------------------------------------------
 * Dissimilarity Tree query (Section 4.2, Listing 2).
 * ------------------------------------------------------------------------- */

/* Lower bound on the key K over every descriptor of a node.  A query bit that
 * is 0 in the node's sum image is a type A error for every descriptor in the
 * node; a query 0-bit that is 1 in the product image is a type B error for
 * every descriptor.  K = A*wB + B*wA is monotone in A and B. */
int64_t or_node_bound(const uint64_t *q, const uint64_t *or_img, const uint64_t *and_img) {
    int64_t P = popcount_desc(q);
    int64_t a = 0, b = 0;
    for (int w = 0; w < OR_WORDS; w++) {
        a += __builtin_popcountll(q[w] & ~or_img[w]);
        if (and_img) b += __builtin_popcountll(~q[w] & and_img[w]);
    }
    return a * w_b(P) + b * w_a(P);
}

/* The same bound tightened by the popcount range [pmin, pmax] of the node's
 * rows.  A row t under the node shares at most min(ov, |t|) bits with q,
 * where ov = popcount(q AND OR): so A >= |q| - min(ov, pmax), and
 * B = |t| - C >= pmin - ov.  Together with the product-image term, B is at
 * least the larger of the two (and of 0). */
int64_t or_node_bound_pop(const uint64_t *q, const uint64_t *or_img, const uint64_t *and_img, int64_t pmin,
                          int64_t pmax) {
    int64_t P = popcount_desc(q);
    int64_t ov = 0, b_and = 0;
    for (int w = 0; w < OR_WORDS; w++) {
        ov += __builtin_popcountll(q[w] & or_img[w]);
        if (and_img) b_and += __builtin_popcountll(~q[w] & and_img[w]);
    }
    int64_t a = P - (ov < pmax ? ov : pmax);
    int64_t b = pmin - ov;
    if (b < b_and) b = b_and;
    if (b < 0) b = 0;
    return a * w_b(P) + b * w_a(P);
}

typedef struct {
    int64_t key;  /* priority (bound, or caller-given score) */
    int64_t node;
    int64_t bound;
} or_open;

typedef struct {
    or_open *h;
    int64_t n, cap;
} or_heap;

static int open_less(const or_open *a, const or_open *b) {
    return a->key < b->key || (a->key == b->key && a->node < b->node);
}
static void heap_push(or_heap *H, or_open v) {
    if (H->n == H->cap) {
        H->cap = H->cap ? 2 * H->cap : 64;
        H->h = (or_open *)realloc(H->h, (size_t)H->cap * sizeof(or_open));
    }
    int64_t i = H->n++;
    H->h[i] = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!open_less(&H->h[i], &H->h[p])) break;
        or_open t = H->h[i];
        H->h[i] = H->h[p];
        H->h[p] = t;
        i = p;
    }
}
static or_open heap_pop(or_heap *H) {
    or_open top = H->h[0];
    H->h[0] = H->h[--H->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < H->n && open_less(&H->h[l], &H->h[m])) m = l;
        if (r < H->n && open_less(&H->h[r], &H->h[m])) m = r;
        if (m == i) break;
        or_open t = H->h[i];
        H->h[i] = H->h[m];
        H->h[m] = t;
        i = m;
    }
    return top;
}

/* Insert a candidate into the result list R (sorted by (key, idx), at most k). */
static void results_insert(or_cand *R, int64_t *nr, int k, or_cand c) {
    if (*nr == k && cand_cmp(&c, &R[k - 1]) >= 0) return;
    int64_t i = *nr < k ? (*nr)++ : k - 1;
    while (i > 0 && cand_cmp(&c, &R[i - 1]) < 0) {
        R[i] = R[i - 1];
        i--;
    }
    R[i] = c;
}

/* One query.  score == NULL: plain best-first order on the bound, with the
 * early stop.  score != NULL: frontier ordered by score[node] (ascending),
 * every popped node re-checked against the current k-th key and skipped if it
 * cannot improve the results; the loop runs until the frontier is empty. */
static int64_t bound_of(const uint64_t *qj, const uint64_t *or_img, const uint64_t *and_img, const int64_t *pmin,
                        const int64_t *pmax, int64_t nd) {
    const uint64_t *a = and_img ? and_img + nd * OR_WORDS : NULL;
    if (pmin) return or_node_bound_pop(qj, or_img + nd * OR_WORDS, a, pmin[nd], pmax[nd]);
    return or_node_bound(qj, or_img + nd * OR_WORDS, a);
}

static void tree_query(const uint64_t *db, const int32_t *child, const int64_t *begin, const int64_t *count,
                       const uint64_t *or_img, const uint64_t *and_img, const int64_t *pmin, const int64_t *pmax,
                       const uint32_t *perm, const uint64_t *qj, int k, const int64_t *score, or_cand *R,
                       int64_t *nr_out, int64_t stats[3]) {
    int64_t P = popcount_desc(qj);
    int64_t nr = 0;
    or_heap H = {0, 0, 0};
    int64_t visited = 0, bounds = 0, dists = 0;
    int64_t b0 = bound_of(qj, or_img, and_img, pmin, pmax, 0);
    bounds++;
    or_open root = {score ? score[0] : b0, 0, b0};
    heap_push(&H, root);
    while (H.n > 0) {
        or_open top = heap_pop(&H);
        int full = nr == k;
        if (full && top.bound > R[k - 1].key) {
            if (score) continue; /* cannot improve: skip */
            break;               /* plain order: nothing left can improve */
        }
        visited++;
        int64_t nd = top.node;
        if (child[2 * nd] < 0) {
            for (int64_t j = begin[nd]; j < begin[nd] + count[nd]; j++) {
                int64_t A, B;
                uint32_t row = perm[j];
                wh_counts(qj, db + (uint64_t)row * OR_WORDS, &A, &B);
                or_cand c = {or_wh_key(A, B, P), (int64_t)row, A, B};
                results_insert(R, &nr, k, c);
                dists++;
            }
        } else {
            for (int s = 0; s < 2; s++) {
                int64_t ch = child[2 * nd + s];
                int64_t kb = bound_of(qj, or_img, and_img, pmin, pmax, ch);
                bounds++;
                if (nr < k || kb <= R[k - 1].key) {
                    or_open o = {score ? score[ch] : kb, ch, kb};
                    heap_push(&H, o);
                }
            }
        }
    }
    free(H.h);
    *nr_out = nr;
    stats[0] = visited;
    stats[1] = bounds;
    stats[2] = dists;
}

/* k-NN for nq queries over a tree in the layout or_tree_build writes.
 * and_img may be NULL (sum-image bound only); pmin / pmax (both or neither)
 * give each node's row popcount range for the tightened bound.  stats (nullable) receives
 * per query: nodes visited (processed pops), bounds evaluated, distances
 * evaluated.  score (nullable) gives per query a node priority array
 * (score + j * n_nodes), replacing the bound as the pop order. */
int or_tree_knn(const uint64_t *db, const int32_t *child, const int64_t *begin, const int64_t *count,
                const uint64_t *or_img, const uint64_t *and_img, const int64_t *pmin, const int64_t *pmax,
                const uint32_t *perm, int64_t n_nodes,
                const uint64_t *q, int64_t nq, int k, const int64_t *score, uint32_t *idx, int32_t *missed,
                int32_t *extra, float *dist, int64_t *stats) {
    if (k <= 0 || n_nodes <= 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < nq; j++) {
        const uint64_t *qj = q + j * OR_WORDS;
        or_cand *R = (or_cand *)malloc((size_t)k * sizeof(or_cand));
        int64_t nr, st[3];
        tree_query(db, child, begin, count, or_img, and_img, pmin, pmax, perm, qj, k,
                   score ? score + j * n_nodes : NULL, R, &nr, st);
        emit(R, nr, popcount_desc(qj), k, idx + j * k, missed + j * k, extra + j * k, dist + j * k);
        if (stats) {
            stats[3 * j] = st[0];
            stats[3 * j + 1] = st[1];
            stats[3 * j + 2] = st[2];
        }
        free(R);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Voting (Section 3).  Query object g owns descriptors qoff[g] .. qoff[g+1]-1
 * in the order they are processed (the caller's random order).  Each of the
 * k neighbours of a descriptor casts one vote for the object that owns it;
 * the winner is the first object whose count reaches the threshold, counted
 * in processing order and, within a descriptor, in neighbour rank order.
 * used[g] = descriptors processed when the winner appeared (all of them if
 * none did; winner = -1).  votes[g][o] counts every descriptor's votes.
 * A neighbour whose row belongs to no object (id >= n_obj) casts no vote.
 * ------------------------------------------------------------------------- */
void or_votes(const uint32_t *nn_idx, int k, const uint16_t *obj_of, int64_t n_db, int64_t n_obj,
              const uint64_t *qoff, int64_t nqo, int64_t threshold, uint32_t *votes, int32_t *winner,
              uint32_t *used) {
    for (int64_t g = 0; g < nqo; g++) {
        uint32_t *v = votes + g * n_obj;
        for (int64_t o = 0; o < n_obj; o++) v[o] = 0;
        winner[g] = -1;
        used[g] = (uint32_t)(qoff[g + 1] - qoff[g]);
        for (uint64_t d = qoff[g]; d < qoff[g + 1]; d++)
            for (int r = 0; r < k; r++) {
                uint32_t row = nn_idx[d * (uint64_t)k + (uint64_t)r];
                if (row == 0xFFFFFFFFu || (int64_t)row >= n_db) continue;
                uint16_t o = obj_of[row];
                if ((int64_t)o >= n_obj) continue;
                v[o]++;
                if (winner[g] < 0 && (int64_t)v[o] >= threshold) {
                    winner[g] = (int32_t)o;
                    used[g] = (uint32_t)(d - qoff[g] + 1);
                }
            }
    }
}

/* ---------------------------------------------------------------------------
 * Object-level distance score (Section 6.4, the object matching experiment
 * behind Table 1 and the confusion matrices): the score of query object g
 * against database object o is the sum, over the query object's descriptors
 * in their given order, of the distance from the descriptor to its nearest
 * descriptor of object o.  The distance is Eq. 1 as the double quotient
 * K / (wA * wB) (not rounded to float); the sum is taken in double, one
 * descriptor after the other.  A query object with descriptors scores
 * +infinity against an object with no rows; an empty query object scores 0
 * against every object; rows whose object id is >= n_obj belong to no object.
 * scores: nqo x n_obj.
 * ------------------------------------------------------------------------- */
void or_object_scores(const uint64_t *db, int64_t n, const uint16_t *obj_of, int64_t n_obj, const uint64_t *q,
                      const uint64_t *qoff, int64_t nqo, double *scores) {
    enum { CHUNK = 64 }; /* descriptors whose minima are found together (in parallel) */
    int64_t *rows_of = (int64_t *)calloc((size_t)n_obj, sizeof(int64_t));
    int64_t *best = (int64_t *)malloc((size_t)CHUNK * (size_t)n_obj * sizeof(int64_t));
    for (int64_t t = 0; t < n; t++)
        if (obj_of[t] < n_obj) rows_of[obj_of[t]]++;
    for (int64_t g = 0; g < nqo; g++) {
        double *sg = scores + g * n_obj;
        for (int64_t o = 0; o < n_obj; o++) sg[o] = 0.0;
        for (uint64_t c0 = qoff[g]; c0 < qoff[g + 1]; c0 += CHUNK) {
            const int64_t m = (int64_t)(qoff[g + 1] - c0 < CHUNK ? qoff[g + 1] - c0 : CHUNK);
            /* nearest row of every object, for each descriptor of the chunk */
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t j = 0; j < m; j++) {
                const uint64_t *qq = q + (c0 + (uint64_t)j) * OR_WORDS;
                const int64_t P = popcount_desc(qq);
                int64_t *bj = best + j * n_obj;
                for (int64_t o = 0; o < n_obj; o++) bj[o] = INT64_MAX;
                for (int64_t t = 0; t < n; t++) {
                    const int64_t o = obj_of[t];
                    if (o >= n_obj) continue;
                    int64_t A, B;
                    wh_counts(qq, db + t * OR_WORDS, &A, &B);
                    const int64_t K = or_wh_key(A, B, P);
                    if (K < bj[o]) bj[o] = K;
                }
            }
            /* the terms, added in descriptor order; the minimum over no rows is +infinity */
            for (int64_t j = 0; j < m; j++) {
                const int64_t P = popcount_desc(q + (c0 + (uint64_t)j) * OR_WORDS);
                for (int64_t o = 0; o < n_obj; o++)
                    sg[o] += rows_of[o] ? (double)best[j * n_obj + o] / ((double)w_a(P) * (double)w_b(P))
                                        : __builtin_inf();
            }
        }
    }
    free(best);
    free(rows_of);
}

/* ---------------------------------------------------------------------------
 * Ranking and confusion-matrix rows (Section 6.4, Table 1 and the confusion
 * matrices).  For each query object g (one row of nqo x n_obj scores):
 * best[g] = the object of lowest score, ties to the lower id, -1 when no
 * score is finite (Table 1 counts the rows whose best object is the source).
 * With normalize set, the row is rescaled in place to [0, 1] as
 * (s - min) / (max - min) over its finite scores; a row whose finite scores
 * are all equal becomes 0 there; non-finite scores become 1.
 * ------------------------------------------------------------------------- */
void or_score_rows(double *scores, int64_t nqo, int64_t n_obj, int normalize, int32_t *best) {
    for (int64_t g = 0; g < nqo; g++) {
        double *s = scores + g * n_obj;
        int64_t arg = -1;
        double mn = __builtin_inf(), mx = -__builtin_inf();
        for (int64_t o = 0; o < n_obj; o++) {
            if (!__builtin_isfinite(s[o])) continue;
            if (s[o] < mn) {
                mn = s[o];
                arg = o;
            }
            if (s[o] > mx) mx = s[o];
        }
        best[g] = (int32_t)arg;
        if (!normalize) continue;
        for (int64_t o = 0; o < n_obj; o++) {
            if (!__builtin_isfinite(s[o]))
                s[o] = 1.0;
            else
                s[o] = mx > mn ? (s[o] - mn) / (mx - mn) : 0.0;
        }
    }
}

/* Threads of the parallel loops above (for timing the oracle on fewer cores). */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_max_threads(void) { return omp_get_max_threads(); }

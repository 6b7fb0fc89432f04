/*
 * qd — exact Weighted Hamming search over 64x64-bit QUICCI descriptors on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: van Blokland & Theoharis, "Partial 3D Object Retrieval using Local
 * Binary QUICCI Descriptors and Dissimilarity Tree Indexing" (2021).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Descriptor: 64 x uint64 = 4096 bits = 512 bytes.  Word r is image row r,
 *   bit c of that word is column c (bit index b = 64*r + c).  The image is
 *   N x N = 64 x 64 bits (Section 6).  Arrays of descriptors are row-major
 *   (descriptor i at word offset 64*i) and must be 16-byte aligned.
 * Distance (Eq. 1, Section 2.3), with |q| the query's popcount:
 *   A = #(query bit 1, target bit 0)   "missed" bits (type A errors)
 *   B = #(query bit 0, target bit 1)   "extra" bits  (type B errors)
 *   d = A / max(|q|,1) + B / max(4096 - |q|, 1)
 *   The second denominator is read as the number of query 0-bits, N*N - |q|.
 * Ranking: results are ordered by the exact integer key
 *   K = A * max(4096-|q|,1) + B * max(|q|,1)  (= d * wA * wB)
 *   and ties by ascending database index, so every result is unique and a
 *   pure function of the inputs.  The float distance is the double quotient
 *   K / (wA * wB) rounded to float; it is never used for ranking.
 * Results of a k-NN call: four caller-owned device arrays of nq*k elements,
 *   row j holding query j's neighbours in ascending (K, index):
 *   idx (uint32 database row), missed (int32 A), extra (int32 B),
 *   dist (float d).  When the database has fewer than k rows, the missing
 *   slots hold idx = QD_PAD_IDX, missed = extra = -1, dist = +inf.
 * Memory: every pointer named d_* is device memory owned by the caller; the
 *   library never frees it.  Inputs are only read.  Work runs asynchronously
 *   on `stream` (a hipStream_t passed as void*, NULL = the default stream)
 *   unless stated otherwise; outputs are valid once the stream reaches that
 *   point.  Scratch space is taken from the stream-ordered allocator.
 * Errors: every call returns QD_OK or a negative qd_status.  Argument errors
 *   are detected before any work is queued and leave outputs untouched.  A
 *   failed launch or allocation returns QD_ERR_DEVICE / QD_ERR_OOM.
 *   qd_last_error() gives a message for the calling thread's last failure.
 */
#ifndef QD_H
#define QD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QD_WORDS 64          /* uint64 words per descriptor */
#define QD_BITS 4096         /* bits per descriptor */
#define QD_MAX_K 64          /* largest k of any k-NN call */
#define QD_PAD_IDX 0xFFFFFFFFu
#define QD_MAX_ROWS 0xFFFFFFFEull /* database rows must fit a uint32 index */

typedef enum {
    QD_OK = 0,
    QD_ERR_INVALID = -1,     /* bad argument: null, misaligned, out of range */
    QD_ERR_OOM = -2,         /* device allocation failed */
    QD_ERR_DEVICE = -3,      /* HIP runtime or kernel launch failure */
    QD_ERR_UNSUPPORTED = -4, /* valid request the library does not serve */
    QD_ERR_ABORTED = -5,     /* stopped through an abort flag */
    QD_ERR_FORMAT = -6,      /* malformed serialized data */
    QD_ERR_IO = -7           /* a file could not be opened, read or written */
} qd_status;

/* Message for the calling thread's last non-OK status ("" if none). */
const char *qd_last_error(void);

/* Cancellation of long synchronous calls.  After qd_set_abort_flag(flag),
 * the calling thread's multi-step synchronous calls read *flag before each
 * step -- qd_tree_build before each level, qd_tree_load before its device
 * pass, qd_model_train before each step, qd_retrieve_objects_early before
 * each round, qd_autotune before each candidate -- and when it is non-zero
 * they wait for the work they queued, release their scratch and return
 * QD_ERR_ABORTED (their outputs are then undefined; a model keeps the steps
 * it took).  The flag may be written from another thread or a signal
 * handler; NULL removes it.  Asynchronous calls do not read it. */
int qd_set_abort_flag(const volatile int *flag);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int qd_version(void);

/* Kernel timing for measurement.  qd_profile_enable(1) clears the totals and
 * makes every following launch of a timed kernel record a HIP event pair on
 * its own stream; qd_profile_enable(0) stops.  qd_profile_read waits for the
 * recorded events and returns the summed duration (ms) and launch count of
 * the named kernel ("wh_scan_topk", "topk_merge", "tree_knn", ...; 0 and 0
 * if it never ran).  Process-wide; not meant for concurrent callers. */
int qd_profile_enable(int on);
int qd_profile_read(const char *kernel, double *total_ms, uint64_t *launches);
/* Named work counters kept while profiling is on (cleared with the totals):
 * "tree_block_tiles" = matrix-core tiles and "tree_block_short_pairs" =
 * (query, block) pairs evaluated on the vector ALUs by the blocked search.
 * *total = 0 for a counter that never counted. */
int qd_profile_counter(const char *name, uint64_t *total);

/* ---------------------------------------------------------------------------
 * Per-row popcount |t| (the sum over all bits of a descriptor, the column
 * sums of Eq. 1).  d_pop[i] = popcount(d_db[i]) for i < n, as uint16
 * (0..4096).  n may be 0.
 * ------------------------------------------------------------------------- */
int qd_popcount_rows(const uint64_t *d_db, uint64_t n, uint16_t *d_pop, void *stream);

/* ---------------------------------------------------------------------------
 * Exact k-NN by sequential search over the whole database: every row is
 * scored under Eq. 1 and the k best by (K, index) are returned (the
 * "sequential search" the tree is compared with in Section 6.2).
 *   d_db: n descriptors (1 <= n <= QD_MAX_ROWS), d_q: nq query descriptors.
 *   1 <= k <= QD_MAX_K.  nq = 0 is a no-op.  Outputs: see "Results" above.
 * ------------------------------------------------------------------------- */
int qd_knn_bruteforce(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                      uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream);

/* Same search with an explicit launch shape, for tuning and for tests that
 * check that results do not depend on it: query_tile = queries served per
 * pass over a row slice (1, 2, 4, 8 or 16 on the vector ALUs;
 * QD_QUERY_TILE_MATRIX: tiles of 16 queries whose overlap counts with 16 rows
 * at a time are one matrix-core product; 0 = automatic), row_parts = row
 * slices per query tile (1..4096, clipped to at least 256 rows per slice;
 * 0 = automatic).  Results are identical for every shape. */
#define QD_QUERY_TILE_MATRIX 256u
int qd_knn_bruteforce_shaped(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                             uint32_t query_tile, uint32_t row_parts, uint32_t *d_idx, int32_t *d_missed,
                             int32_t *d_extra, float *d_dist, void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as qd_knn_bruteforce, same arguments and results, on its row scan
 * (vector-ALU or matrix-core query tiles, chosen as there; never the
 * large-batch matrix-core path), with no device allocation and no allocating
 * library call.  Its scratch (each wave's top-k lists) is a fixed device array of
 * QD_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends; its address is looked up on the first call on each device.
 * Requests whose lists cannot fit (nq * k above QD_NOALLOC_SCRATCH_BYTES / 8)
 * return QD_ERR_INVALID; the row slices per query are reduced as needed
 * otherwise.  Calls on one GPU share that array: calls that overlap on one
 * device (other streams, other threads) race and must be serialised by the
 * caller.  Stream-ordered; nothing to free. */
#define QD_NOALLOC_SCRATCH_BYTES (32ull << 20)
int qd_knn_bruteforce_noalloc(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                              uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, void *stream);

/* ---------------------------------------------------------------------------
 * Bit-plane index for small query batches (the sequential search of Section
 * 6.2, reorganised).  qd_planes_build stores the n descriptors transposed:
 * plane b (one per bit position, 4096) holds bit b of every row, row i at bit
 * i % 64 of word i / 64, so a query reads only its |q| planes (and a
 * popcount per candidate row) instead of all 512-byte rows.  The index takes
 * about n x 512 bytes plus 2 bytes per row, keeps a pointer to d_db (which
 * must outlive it: the final step reads the result rows) and is built
 * synchronously on `stream`.  Free with qd_planes_free.
 * qd_knn_planes returns exactly qd_knn_bruteforce's results (same arguments
 * and outputs, see "Results" above).  Each wave counts, for one query and a
 * range of 64-row plane words, the overlaps of all 64 rows at once in
 * bit-sliced counters, and computes keys only for rows whose overlap can
 * still reach the wave's current k-th key.
 * ------------------------------------------------------------------------- */
typedef struct qd_planes_s *qd_planes_t;

int qd_planes_build(const uint64_t *d_db, uint64_t n, void *stream, qd_planes_t *out);
int qd_planes_free(qd_planes_t p);
int qd_knn_planes(qd_planes_t p, const uint64_t *d_q, uint32_t nq, uint32_t k, uint32_t *d_idx, int32_t *d_missed,
                  int32_t *d_extra, float *d_dist, void *stream);

/* ---------------------------------------------------------------------------
 * Dissimilarity Tree (Section 4).
 *
 * qd_tree_build indexes a fixed set of n descriptors (Section 4.1, Listing 1):
 * each node holding more than max_leaf descriptors is split in two; bit
 * positions are taken in ascending popularity over the node (ties: ascending
 * bit index) and every descriptor still in the "similar" set that has the
 * bit set moves to the "dissimilar" set, until the dissimilar set holds at
 * least half of the node; a move that would empty the similar set is not
 * applied, and a node that cannot be split stays a leaf.  Every node, leaves
 * included, stores the OR ("sum") image of its descriptors, the AND
 * ("product") image if store_and_image is set, and, unless plain_bound is
 * set, the smallest and largest popcount of its descriptors.
 * Numbering: nodes are numbered breadth first from the root (0), the similar
 * child before the dissimilar one.  Node i covers leaf-order positions
 * begin[i] .. begin[i]+count[i]-1; perm maps a leaf-order position to the
 * database row.  Within a leaf, rows keep ascending database order.
 * Ownership: the tree copies the rows into leaf order, so the caller may free
 * d_db after the call.  The call is synchronous (it returns once the tree is
 * complete) and uses `stream` for its device work.  Free with qd_tree_free.
 * ------------------------------------------------------------------------- */
typedef struct qd_tree_s *qd_tree_t;

typedef struct {
    uint32_t max_leaf;        /* leaf when a node holds <= max_leaf rows; 0 = 32 (Section 4.1) */
    uint32_t store_and_image; /* 0 = sum images only (the paper's choice for sparse QUICCI) */
    uint32_t plain_bound;     /* 1 = the paper's image bound only; 0 = also store each node's (and each
                                 256-row block's) row popcount range and tighten the bound with it */
} qd_build_params;

typedef struct {
    uint64_t n, n_nodes, n_leaves;
    uint32_t depth, max_leaf, has_and_image, has_pop_range;
} qd_tree_info_t;

int qd_tree_build(const uint64_t *d_db, uint64_t n, const qd_build_params *params, void *stream, qd_tree_t *out);
int qd_tree_free(qd_tree_t t);
int qd_tree_info(qd_tree_t t, qd_tree_info_t *info);

/* Save a tree to a file and load it back (Section 4.1: the index is built
 * once, offline, and queried afterwards).  The file holds the rows in leaf
 * order, the leaf-order permutation and the breadth-first structure (child
 * pairs, begin, count) behind a 64-byte versioned header with FNV-1a hashes
 * of the header and of the payload; the layout is documented in
 * csrc/tree_io.hip.  qd_tree_load reads the whole file and checks header,
 * hashes and structure on the host before any device work: a file that fails
 * returns QD_ERR_FORMAT (QD_ERR_IO if it cannot be opened or read) and
 * allocates nothing.  It then rebuilds every derived array (images,
 * popcounts, popcount ranges, block images) from the rows on the current
 * device, so the loaded tree answers every query exactly as the saved one.
 * Both calls are synchronous; qd_tree_load uses `stream` for its device
 * work.  The caller frees the loaded tree with qd_tree_free. */
int qd_tree_save(qd_tree_t t, const char *path);
int qd_tree_load(const char *path, void *stream, qd_tree_t *out);

/* Copy the tree's arrays to caller-owned HOST buffers (any may be NULL):
 * h_child n_nodes x 2 (similar, dissimilar; -1 for leaves), h_begin and
 * h_count n_nodes, h_or / h_and n_nodes x 64 words, h_perm n.  Synchronous. */
int qd_tree_export(qd_tree_t t, int32_t *h_child, uint32_t *h_begin, uint32_t *h_count, uint64_t *h_or,
                   uint64_t *h_and, uint32_t *h_perm);

/* ---------------------------------------------------------------------------
 * Exact k-NN through the tree (Section 4.2, Listing 2).
 *
 * A node's lower bound (minWHDist): every query 1-bit that is 0 in the
 * node's sum image is a type A error for all its rows, and every query 0-bit
 * that is 1 in its product image (when stored) a type B error, so all rows
 * under the node have key K >= Kb = A_lb*wB + B_lb*wA.  With popcount
 * ranges (qd_build_params.plain_bound = 0) a row t shares at most
 * min(ov, |t|) bits with q, ov = popcount(q AND sum image), so
 * A_lb = |q| - min(ov, pmax) and B_lb = max(product-image term, pmin - ov, 0)
 * for the node's popcount range [pmin, pmax]; the results do not change.  A child is queued
 * when fewer than k results exist or Kb <= the current k-th key; a popped
 * node with Kb above the k-th key is not expanded.  The result equals
 * qd_knn_bruteforce's exactly, whatever the order.
 * Orders:
 *   QD_ORDER_BEST_FIRST (default, the paper's priority queue): nodes leave
 *     the frontier in ascending floor(Kb / wB), which is the exact bound
 *     order for the sum-image bound alone; the search stops once that floor
 *     exceeds the k-th key (nodes above the key in a lower bucket are
 *     skipped).
 *   QD_ORDER_DEPTH_FIRST: a stack; each expansion visits the preferred child
 *     first: the higher score in d_scores when given (nq x n_scored floats,
 *     query-major, nodes 0..n_scored-1; e.g. a learned model's output), else
 *     the lower bound (ties: the similar child).  Runs until the stack is
 *     empty, skipping popped nodes that cannot improve the result.
 *   QD_ORDER_BLOCKED: the whole batch at once on the matrix cores.  The leaf
 *     order is cut into blocks of 256 rows, each with the sum image of its
 *     rows (and their popcount range); the same bound, rounded down to a
 *     multiple of wB (A_lb + floor(B_lb*wA/wB), at most 4096, times wB), is
 *     computed for every (query, block) pair, and
 *     each query evaluates its blocks in rounds of ascending bound (a first
 *     round of 16 blocks, then growing about 4x), keeping only blocks whose
 *     bound is <= its current k-th key, until no block is left that could
 *     hold a better key.  A query whose candidate buffer overflows repeats
 *     the round with a tighter key; one whose key cannot tighten (more rows
 *     tie at its k-th key than a buffer holds) is searched again depth-first.
 *     A direct call waits for the stream between rounds; plans run it
 *     without host waits (see qd_plan_create).  Takes no scores or traces.  Per-query stats mean: blocks
 *     evaluated, rounds taken part in, blocks bounded, distances evaluated.
 * d_query_stats (nullable): nq x 4 uint32 per query: nodes visited
 * (expanded pops, leaves and inner nodes), leaves visited, bounds evaluated,
 * distances evaluated.  h_stats (nullable): totals; filling it waits for the
 * stream.  waves_per_cu = 0 picks a default occupancy.  d_visited records
 * which of the first n_traced nodes each query expanded (traversal traces).
 * ------------------------------------------------------------------------- */
typedef enum { QD_ORDER_BEST_FIRST = 0, QD_ORDER_DEPTH_FIRST = 1, QD_ORDER_BLOCKED = 2 } qd_order;
typedef struct qd_model_s *qd_model_t; /* learned-order model, see below */

typedef struct {
    qd_order order;
    const float *d_scores; /* depth-first only; nullable */
    uint32_t n_scored;
    uint32_t waves_per_cu;
    uint32_t *d_visited;   /* nullable: trace bitmap, nq x ceil(n_traced/32) uint32; bit (node % 32) of word
                              node / 32 of query j's row is set when the search expands node (< n_traced).
                              The library clears it first. */
    uint32_t n_traced;
    /* QD_ORDER_BLOCKED round schedule (0 = default): blocks in round 1
       (default 16, at most 64), blocks covered after round 2 (default: enough
       for ~128 queries per block list on average), growth factor of the
       covered prefix per later round (default 4, 2..64). */
    uint32_t round1_blocks;
    uint32_t round2_blocks;
    uint32_t round_growth;
    /* Learned order (nullable; see "Learned frontier order" below).
       QD_ORDER_DEPTH_FIRST: the library scores nodes 0 .. n_scored-1 of the
       tree for every query (n_scored 0 = min(2047, nodes)) and visits the
       higher-scoring child first, as with d_scores (which must then be NULL).
       QD_ORDER_BLOCKED: round 1 starts where the model leads: from the root,
       the search enters at every inner node holding more than round1_blocks
       x 256 rows the child the model scores higher (ties: the similar child),
       and round 1 evaluates the round1_blocks consecutive blocks of the leaf
       order that begin with the reached node's first block; the other blocks
       follow in the bound-ordered rounds.  Results are identical with and
       without a model. */
    qd_model_t model;
    /* QD_ORDER_BLOCKED without a model: where round 1 starts.
       QD_START_LOWEST_BOUND (0): the round1_blocks blocks of lowest bound.
       QD_START_BOUND_DESCENT: the round1_blocks consecutive blocks that begin
       with the first block of the node reached from the root by entering, at
       every inner node above round1_blocks x 256 rows, the child of lower
       bound (ties: the similar child); the other blocks follow in the
       bound-ordered rounds, as with a model.  Results are identical. */
    uint32_t round1_start;
    /* QD_ORDER_BEST_FIRST / QD_ORDER_DEPTH_FIRST: concurrent searches per
       query (0 = default 16; 1 = one wave searches the whole tree; else a
       power of two up to 16).  With n > 1 the tree is cut log2(n) levels
       below the root, each subtree is searched in the same order by its own
       wave, the searches of a query prune with the least k-th key any of them
       has reached (shared through device memory), and their k-lists are
       merged.  Results are identical for every n; the statistics count the
       work of all of a query's searches, which depends on their timing.  A
       traced search (d_visited) runs unsplit.  A batch of nq queries runs
       nq x n searches, at most 2^31. */
    uint32_t query_split;
} qd_search_params;
enum { QD_START_LOWEST_BOUND = 0, QD_START_BOUND_DESCENT = 1 };

typedef struct {
    uint64_t nodes_visited, leaves_visited, bounds_evaluated, dists_evaluated;
} qd_stats;

int qd_knn_tree(qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k, const qd_search_params *params,
                uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, uint32_t *d_query_stats,
                qd_stats *h_stats, void *stream);

/* ---------------------------------------------------------------------------
 * Partial-object retrieval by voting (Section 3).
 *
 * nqo query objects; query object g owns the query descriptors
 * d_qoff[g] .. d_qoff[g+1]-1 of d_qdesc (d_qoff: nqo+1 uint64 on the device,
 * d_qoff[0] = 0, d_qoff[nqo] = n_qdesc), in the order they are processed (the
 * paper draws them at random; the caller supplies that order).  Every
 * descriptor's k nearest database descriptors are found exactly (through tree
 * t, or by sequential search over d_db when t is NULL), all in one batched
 * launch; each neighbour casts one vote for its object d_obj_of[row]
 * (uint16, n rows; object ids < n_obj <= 65536; a row whose id is >= n_obj
 * casts no vote).
 * Outputs: d_votes nqo x n_obj uint32 (all votes), d_winner[g] = the first
 * object whose count reaches vote_threshold (1..255; the paper uses 10),
 * counting votes in descriptor order and, within a descriptor, in neighbour
 * rank order, or -1 if none does; d_used[g] = descriptors processed when the
 * winner was decided (all of them if none).  d_nn_idx (nullable, n_qdesc x k
 * uint32) receives the neighbour rows.  params (nullable) picks the tree
 * frontier order and occupancy; d_scores must be NULL.
 * ------------------------------------------------------------------------- */
int qd_retrieve_objects(qd_tree_t t, const uint64_t *d_db, uint64_t n, const uint16_t *d_obj_of, uint32_t n_obj,
                        const uint64_t *d_qdesc, uint64_t n_qdesc, const uint64_t *d_qoff, uint32_t nqo, uint32_t k,
                        uint32_t vote_threshold, const qd_search_params *params, uint32_t *d_votes,
                        int32_t *d_winner, uint32_t *d_used, uint32_t *d_nn_idx, void *stream);

/* Retrieval that stops at the vote threshold (Section 3: descriptors are
 * processed in order until an object reaches the threshold).  Same arguments
 * and outputs as qd_retrieve_objects (vote_threshold 1..255), but each query
 * object's descriptors are searched in rounds, in their given order, and an
 * object stops as soon as its votes so far decide a winner: round r searches
 * the next 16 * 2^(r-1) descriptors of every undecided object, all objects'
 * in one batched k-NN call.  d_winner and d_used equal qd_retrieve_objects'
 * exactly; d_votes counts the votes of the first d_used[g] descriptors of
 * object g (all of them if it has no winner).  *h_searched (nullable)
 * receives the number of descriptors searched (at least the sum of d_used,
 * at most n_qdesc).  Synchronous (waits for the stream between rounds). */
int qd_retrieve_objects_early(qd_tree_t t, const uint64_t *d_db, uint64_t n, const uint16_t *d_obj_of, uint32_t n_obj,
                              const uint64_t *d_qdesc, uint64_t n_qdesc, const uint64_t *d_qoff, uint32_t nqo,
                              uint32_t k, uint32_t vote_threshold, const qd_search_params *params, uint32_t *d_votes,
                              int32_t *d_winner, uint32_t *d_used, uint64_t *h_searched, void *stream);

/* Object-level distance scores (Section 6.4: the object matching behind
 * Table 1 and the confusion matrices).  d_scores[g * n_obj + o] (float64,
 * device, nqo x n_obj, written whole) = the sum, over query object g's
 * descriptors d_qdesc[d_qoff[g] .. d_qoff[g+1]) in that order, of
 * K / (wA * wB) for the row of object o nearest to the descriptor (Eq. 1;
 * K, wA, wB as defined at the top of this file; the quotient and the running
 * sum in float64, one descriptor after the other).  An object with no rows adds
 * +inf per descriptor; an empty query object scores 0 against every object.
 *   d_db: n x 64 words (device, 16-byte aligned; may be null when n = 0),
 *   n < 2^32.  d_obj_of: n object ids (device uint16); rows with an id >=
 *   n_obj belong to no object.  1 <= n_obj <= 65536.  d_qoff: nqo + 1
 *   device offsets with d_qoff[0] = 0 <= ... <= d_qoff[nqo] = n_qdesc.
 *   nqo = 0 is a no-op.
 * Stream-ordered; allocates and frees its scratch on the stream (row order
 * by object, and at most 1 GiB of per-descriptor minima per batch of query
 * descriptors). */
int qd_object_scores(const uint64_t *d_db, uint64_t n, const uint16_t *d_obj_of, uint32_t n_obj,
                     const uint64_t *d_qdesc, uint64_t n_qdesc, const uint64_t *d_qoff, uint32_t nqo,
                     double *d_scores, void *stream);

/* Ranking and confusion-matrix rows (Section 6.4: Table 1 counts the query
 * objects whose best-ranked object is their source; the confusion matrices
 * show each row of scores rescaled to [0, 1]).  d_scores: nqo x n_obj
 * float64 (device, as written by qd_object_scores).  d_best[g] (device
 * int32, nqo) = the object of lowest score in row g, ties to the lower id,
 * -1 when no score of the row is finite.  With normalize != 0 each row is
 * rewritten in place as (s - min) / (max - min) over its finite scores (0
 * where they are all equal); non-finite scores become 1.  nqo = 0 is a
 * no-op; n_obj >= 1.  Stream-ordered; allocates nothing. */
int qd_score_rows(double *d_scores, uint32_t nqo, uint32_t n_obj, int normalize, int32_t *d_best, void *stream);

/* ---------------------------------------------------------------------------
 * Learned frontier order (an extension: the paper orders the frontier by the
 * bound only).  A multilayer perceptron scores (query, node) pairs; the
 * depth-first search visits the higher-scoring child first.  Pruning keeps
 * using the exact bounds, so the k-NN result is the same for any scores.
 *   x = [query bits (4096, 0/1), node features (32)]
 *   h1 = ReLU(x W1 + b1), h2 = ReLU(h1 W2 + b2), score = h2 . w3 + b3
 * Parameters (fp32, QD_MLP_NPARAMS floats, this order, matrices stored
 * [input][output] row-major): W1q 4096 x 256 (query-bit rows of W1),
 * W1f 32 x 256 (feature rows), b1 256, W2 256 x 256, b2 256, w3 256, b3 1.
 * Inference and training run BF16 weights with FP32 accumulation; the model
 * keeps FP32 masters and Adam moments.
 * Features of pair (q, node), |q| read as max(|q|,1), a_lb =
 * popcount(q AND NOT OR(node)), ov = popcount(q AND OR(node)), bands =
 * image rows 0-5, 6-11, ..., 54-59, 60-63:
 *   0 a_lb/|q|  1 ov/|q|  2 popcount(OR)/4096  3 the sibling's a_lb/|q| (0 for
 *   the root)  4 depth/32  5 log2(rows under the node)/24  6 is a leaf
 *   7 is the similar child  8 |q|/512  9 popcount(OR AND NOT q)/4096
 *   10..20 a_lb per band / |q|   21..31 ov per band / |q|
 * ------------------------------------------------------------------------- */
#define QD_MLP_HIDDEN 256
#define QD_MLP_FEATURES 32
#define QD_MLP_NPARAMS 1123073

/* New model from device fp32 parameters (copied); synchronous. */
int qd_model_create(const float *d_params, void *stream, qd_model_t *out);
int qd_model_free(qd_model_t m);
/* Copy the fp32 master parameters to d_params (QD_MLP_NPARAMS floats). */
int qd_model_params(qd_model_t m, float *d_params, void *stream);
/* Features (n_pairs x 32 fp32) of pairs (d_q[d_pair_q[p]], d_pair_node[p]). */
int qd_model_features(qd_tree_t t, const uint64_t *d_q, const uint32_t *d_pair_q, const uint32_t *d_pair_node,
                      uint64_t n_pairs, float *d_feat, void *stream);
/* Scores (logits) of pairs with given features; pair p uses query d_pair_q[p] < nq. */
int qd_model_forward(qd_model_t m, const uint64_t *d_q, uint32_t nq, const uint32_t *d_pair_q, const float *d_feat,
                     uint64_t n_pairs, float *d_scores, void *stream);
/* Gradient of the mean binary cross-entropy (labels 0/1 against the logit)
 * over the pairs, which must be grouped by query: query j owns pairs
 * d_qoff[j] .. d_qoff[j+1]-1 (device, nq+1).  d_grads: QD_MLP_NPARAMS floats
 * in the parameter layout; d_loss (nullable): the mean loss.  Reductions run
 * in a fixed order, so the gradient is reproducible. */
int qd_model_gradients(qd_model_t m, const uint64_t *d_q, uint32_t nq, const uint64_t *d_qoff,
                       const uint32_t *d_pair_q, const float *d_feat, const float *d_labels, uint64_t n_pairs,
                       float *d_grads, float *d_loss, void *stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with the given gradient. */
int qd_model_adam_step(qd_model_t m, const float *d_grads, float lr, void *stream);
/* Scores of nodes 0 .. n_scored-1 for every query: d_scores is nq x n_scored,
 * ready for qd_search_params.d_scores. */
int qd_model_score_tree(qd_model_t m, qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t n_scored,
                        float *d_scores, void *stream);
/* Training pairs from a traced search: for each query j and node 1 <=
 * node < n_traced whose parent the search expanded (d_visited, as written by
 * qd_knn_tree), a pair (j, node) with label 1 if one of the query's k result
 * rows (d_result_idx, nq x k) lies under the node, else 0.  Pairs come grouped
 * by query in ascending node order; d_qoff (nq+1 uint64) gets the groups.
 * Writes at most `capacity` pairs and returns the total in *h_n_pairs (if it
 * exceeds capacity nothing is written: call again with enough room).
 * Synchronous. */
int qd_trace_pairs(qd_tree_t t, uint32_t nq, uint32_t k, const uint32_t *d_result_idx, const uint32_t *d_visited,
                   uint32_t n_traced, uint32_t *d_pair_q, uint32_t *d_pair_node, float *d_labels, uint64_t capacity,
                   uint64_t *d_qoff, uint64_t *h_n_pairs, void *stream);

/* Train on traversal traces: trace the exact best-first search of the nq
 * training queries (k results, nodes < n_traced), form the labelled pairs as
 * qd_trace_pairs does, then run `epochs` passes of Adam (learning rate lr)
 * over batches of batch_queries consecutive queries, taken in the order
 * h_batch_order gives (host array of ceil(nq / batch_queries) batch indices;
 * NULL = ascending).  h_losses (nullable, host, epochs x batches floats):
 * mean loss of every step (NaN for a batch without pairs).  *h_n_pairs: the
 * number of training pairs.  Synchronous. */
int qd_model_train(qd_model_t m, qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k, uint32_t n_traced,
                   uint32_t epochs, uint32_t batch_queries, float lr, const uint32_t *h_batch_order,
                   float *h_losses, uint64_t *h_n_pairs, void *stream);

/* ---------------------------------------------------------------------------
 * Batched retrieval plans (an extension: the paper runs query objects one
 * descriptor at a time).  A plan fixes the search (tree t, or sequential
 * search over d_db when t is NULL), k, the vote threshold and the largest
 * batch (max_qdesc descriptors in max_qobj query objects).  params picks the
 * tree's order (best-first, depth-first or blocked, with occupancy or round
 * schedule; a model only with the blocked order, where it sets the start of
 * round 1, its descent running on the plan's memory; no scores or traces);
 * query_tile picks the sequential
 * scan: 0 = the matrix cores when max_qdesc >= 160 over >= 65,536 rows (as
 * qd_knn_bruteforce decides for a batch of max_qdesc), else the row scan with
 * that query tile (as in qd_knn_bruteforce_shaped; 0 = the one
 * qd_knn_bruteforce picks for max_qdesc queries).  It allocates all its device memory at
 * creation and records one batch -- the k-NN of every descriptor, then the
 * votes -- into a hipGraph whose kernels read the batch size from device
 * memory and never wait for the host: the blocked order runs a fixed number
 * of rounds per batch of up to 16,384 descriptors (queries still running
 * after them, and queries whose candidates overflow, are searched again one
 * by one, exactly), the matrix-core scan's overflow fallback takes its count
 * from the device.  qd_plan_run serves one batch exactly as
 * qd_retrieve_objects would (same arguments and outputs): it copies the
 * inputs into the plan, replays the graph on `stream` and copies the outputs
 * out; it allocates nothing and never waits for the device.  Runs of one
 * plan must not overlap (they share its buffers).  The plan keeps pointers to
 * t, d_db, d_obj_of and params->model, which must outlive it.
 * ------------------------------------------------------------------------- */
typedef struct qd_plan_s *qd_plan_t;

int qd_plan_create(qd_tree_t t, const uint64_t *d_db, uint64_t n, const uint16_t *d_obj_of, uint32_t n_obj,
                   uint64_t max_qdesc, uint32_t max_qobj, uint32_t k, uint32_t vote_threshold,
                   const qd_search_params *params, uint32_t query_tile, qd_plan_t *out);
int qd_plan_run(qd_plan_t p, const uint64_t *d_qdesc, uint64_t n_qdesc, const uint64_t *d_qoff, uint32_t nqo,
                uint32_t *d_votes, int32_t *d_winner, uint32_t *d_used, void *stream);
int qd_plan_free(qd_plan_t p);

/* ---------------------------------------------------------------------------
 * Autotuner: times every launch configuration of a k-NN batch (tree t:
 * best-first and depth-first x waves per CU, and the blocked order x round
 * schedules -- round-1 blocks 8, 16, 32, growth 2, 4, 8, round-2 coverage
 * half, default and double, round 1 at the lowest bounds or at the bound's
 * descent; sequential search: automatic path and query
 * tiles 4, 8, 16 and QD_QUERY_TILE_MATRIX) over `reps` runs after one warm-up on the caller's sample
 * batch, and returns the fastest in *best (every configuration returns the
 * same exact result).  With `all`, every candidate's timing is written too.
 * Results are cached per (device, rows, nodes, nq, k) for the process, and in
 * the file named by the environment variable QD_TUNE_CACHE when it is set (a
 * cached entry is returned without timing unless `all` is requested).
 * Synchronous.
 * ------------------------------------------------------------------------- */
typedef struct {
    int path;              /* 1 = tree search, 0 = sequential search */
    qd_order order;        /* tree: frontier order */
    uint32_t waves_per_cu; /* tree, per-query orders: occupancy (0 = default) */
    uint32_t query_tile;   /* sequential: query tile (0 = automatic; see qd_knn_bruteforce_shaped) */
    float ms;              /* mean time of one batch */
    uint32_t round1_blocks, round2_blocks, round_growth; /* blocked order: qd_search_params' schedule */
    uint32_t round1_start; /* blocked order: qd_search_params.round1_start */
} qd_tuning;

/* order_mask (tree only): the frontier orders to time, bit (1 << order) for
 * each qd_order; 0 = all.  The cache key includes it. */
int qd_autotune(qd_tree_t t, const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                uint32_t reps, uint32_t order_mask, qd_tuning *best, qd_tuning *all, uint32_t max_all,
                uint32_t *n_all, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QD_H */

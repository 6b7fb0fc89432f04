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
    QD_ERR_UNSUPPORTED = -4, /* valid request this build does not serve */
    QD_ERR_ABORTED = -5,     /* stopped through an abort flag */
    QD_ERR_FORMAT = -6       /* malformed serialized data */
} qd_status;

/* Message for the calling thread's last non-OK status ("" if none). */
const char *qd_last_error(void);

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
 * pass over a row slice (1, 2, 4, 8 or 16; 0 = automatic), row_parts = row
 * slices per query tile (1..4096, clipped to at least 256 rows per slice;
 * 0 = automatic).  Results are identical for every shape. */
int qd_knn_bruteforce_shaped(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq, uint32_t k,
                             uint32_t query_tile, uint32_t row_parts, uint32_t *d_idx, int32_t *d_missed,
                             int32_t *d_extra, float *d_dist, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QD_H */

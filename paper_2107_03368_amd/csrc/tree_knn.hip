// Dissimilarity Tree k-NN search (Section 4.2, Listing 2) as a persistent
// kernel: each wave takes queries from a global counter until none are left,
// and searches one query at a time.
//
// Node bound (minWHDist): a query 1-bit that is 0 in a node's sum image is a
// type A error for every row under the node, so with
//   A_lb = |q| - popcount(q AND OR)   (and, with product images,
//   B_lb = popcount(NOT q AND AND))
// every row under the node has key K >= Kb = A_lb*wB + B_lb*wA.  With the
// popcount range [pmin, pmax] of the node's rows, a row shares at most
// min(ov, pmax) bits with q (ov = popcount(q AND OR)): A_lb = |q| -
// min(ov, pmax), and B_lb is at least pmin - ov.  Children are
// bounded when their parent is expanded; a child is queued when fewer than k
// results exist or Kb <= the current k-th key; a popped node whose Kb exceeds
// the k-th key is not expanded.
//
// Frontier orders:
//  best-first (the paper's priority queue): a bucket queue on
//    floor(Kb / 2wB) (2 levels of A_lb per bucket for the sum-image bound
//    alone: the buckets' state then takes half the LDS, so 16 waves fit on a
//    CU instead of 8; registers hold 12); the search stops once the popped
//    bucket's lower end exceeds the k-th key, and a popped node above the key
//    is skipped, so the result stays exact.  Each bucket is a stack of
//    16-entry chunks in the wave's global workspace, its (chunk, fill) word in
//    LDS, and a 2048-bit occupancy map spread over the 64 lanes finds the
//    lowest non-empty bucket with one ballot.  Lane 0 writes the chunks; a
//    chunk is read back whole, one lane per entry.
//  depth-first: a stack in LDS; at every expansion the preferred child is
//    visited first (lower bound, or higher learned score where scores are
//    given); popped nodes are re-checked against the k-th key and skipped
//    when they cannot improve the result; the search ends with an empty stack.
// Both orders return exactly the sequential-search result.
//
// Intra-query split: one query's search can run as n concurrent tasks (n a
// power of two up to 16), each searching one subtree of the tree cut at
// depth log2(n) (a leaf above that depth is one task's whole subtree) in the
// same order.  The subtrees partition the rows, so the query's k nearest are
// the k smallest of the tasks' k-lists (merge_kernel).  Every task prunes
// with the least k-th key any task of its query has published: a device word
// per query, lowered with an atomic minimum after each leaf (the atomic also
// returns the word, taken in at the next leaf, by when it has long
// returned).  A task's k-th key is never below the query's final one, so the
// pruning stays exact.  With n tasks a query's search is spread over n waves,
// so a batch no longer waits for its last few long searches.
#include "qd_device.h"
#include "qd_internal.h"
#include "qd_launch.h"
#include "qd_tree.h"

namespace qd {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kBuckets = 2048;
constexpr uint32_t kBucketLevels = 2;  // bound levels (multiples of wB) per bucket
constexpr uint32_t kChunk = 16;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kMaxStack = 256;
// Best-first: entries of the bucket being popped live in a small LDS stack of
// the wave ("hot" bucket) while it has room; the other buckets' entries live
// in the wave's chunks in global memory.  A child's bound is never below its
// parent's, so pushes never go below the bucket being popped.  When a bucket
// becomes the hot one, its newest chunk moves to the LDS stack in one load,
// so every pop takes an entry from LDS and a chunk costs one wait for global
// memory instead of one per entry.
constexpr uint32_t kHot = 32;

struct TreeView {
    const uint4 *sorted;
    const uint32_t *perm;
    const uint4 *orimg;
    const uint4 *andimg;  // nullable
    const int32_t *child;
    const uint32_t *begin;
    const uint32_t *count;
    const uint16_t *pop;
    const uint16_t *pmin;  // nullable: per node, the smallest and largest row popcount
    const uint16_t *pmax;
};

struct Scores {
    const float *s;       // nq x n_scored (nullable): learned preference, higher = visit first
    uint32_t n_scored;    // nodes 0 .. n_scored-1 carry a score
};

constexpr uint32_t kMaxSplit = 16;
constexpr uint32_t kDefaultSplit = 16;
// The tasks' area, one allocation for nq_max queries of n tasks each:
// subtree roots (n int32, -1: an empty task) | per query, the least k-th key
// its tasks have published | per task, its k-list (k keys) | their payloads
// (A | B << 16) | its statistics (nodes visited, leaves, bounds, distances,
// |q|; 8 words).  Byte offsets from the area's start; the kernels take the
// start alone and compute the rest, so few pointers stay in registers.
struct SplitLayout {
    uint64_t kshared, key, pay, stat, bytes;
};
__host__ __device__ inline SplitLayout split_layout(uint64_t nq_max, uint32_t n, uint32_t k) {
    const uint64_t nt = nq_max * n;
    SplitLayout L;
    L.kshared = 256;
    L.key = L.kshared + (nq_max * 4 + 255) / 256 * 256;
    L.pay = L.key + nt * k * 8;
    L.stat = L.pay + (nt * k * 4 + 255) / 256 * 256;
    L.bytes = L.stat + nt * 32;
    return L;
}

__device__ __forceinline__ uint32_t sum32(uint32_t v) { return sum32_half(v); }

template <bool kBest>
__global__ __launch_bounds__(kBlock, kBest ? 3 : 4) void tree_knn_kernel(TreeView T, const uint4 *__restrict__ q, uint32_t nq,
                                                          uint32_t k, uint32_t *__restrict__ next_task,
                                                          u64 *__restrict__ pool, uint32_t *__restrict__ chunk_prev,
                                                          uint64_t pool_chunks, Scores S, uint32_t *trace,
                                                          uint32_t n_traced, const uint32_t *__restrict__ nq_dev,
                                                          char *__restrict__ sw, uint32_t nsplit) {
    __shared__ uint32_t bstate_all[kBest ? kWaves * kBuckets : 1];
    __shared__ u64 stack_all[kBest ? kWaves * kHot : kWaves * kMaxStack];  // best-first: the hot bucket's entries
    __shared__ u64 sinfo_all[kBest ? kWaves * kHot : kWaves * kMaxStack];  // the entries' node info
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 3, j = lane & 7;
    const uint64_t slot = (uint64_t)blockIdx.x * kWaves + wave;
    // this wave's chunks: each entry is one 16-byte record (the entry, then its node info)
    ulonglong2 *mypool = reinterpret_cast<ulonglong2 *>(pool) + slot * pool_chunks * kChunk;
    uint32_t *myprev = chunk_prev + slot * pool_chunks * 2;
    uint32_t *myfree = myprev + pool_chunks;
    uint32_t *bstate = bstate_all + (kBest ? wave * kBuckets : 0);
    u64 *stack = stack_all + wave * (kBest ? kHot : kMaxStack);
    u64 *sinfo = sinfo_all + wave * (kBest ? kHot : kMaxStack);
    const bool has_and = T.andimg != nullptr;
    const uint32_t nq_max = nq;  // the tasks' area is laid out for nq queries
    if (nq_dev) nq = readfirst(*nq_dev);  // size given on the device (captured graphs)
    const uint32_t tsh = (uint32_t)__builtin_ctz(nsplit);  // tasks per query = 1 << tsh
    const uint64_t ntasks = (uint64_t)nq << tsh;
    uint32_t *const kshared = reinterpret_cast<uint32_t *>(sw + 256);  // the layout's first offset

    for (;;) {
        // every lane takes part in the atomic (lane 0 adds 1, the others 0) so
        // that no lane-dependent branch guards the loop head; control values
        // below are passed through readfirstlane so the compiler keeps the
        // whole traversal wave-uniform.  A query's tasks are consecutive.
        const uint32_t task = readfirst(atomicAdd(next_task, lane == 0 ? 1u : 0u));
        if (task >= ntasks) break;
        const uint32_t qi = task >> tsh;
        const int32_t root =
            nsplit == 1 ? 0 : (int32_t)readfirst((uint32_t) reinterpret_cast<const int32_t *>(sw)[task & (nsplit - 1)]);
        // this task's list and statistics, for merge_kernel
        auto put = [&](u64 key, uint32_t pay, uint32_t visited, uint32_t leaves, uint32_t bounds, uint32_t dists,
                       uint32_t pq) {
            const SplitLayout SL = split_layout(nq_max, nsplit, k);
            if (lane < (int)k) {
                reinterpret_cast<u64 *>(sw + SL.key)[(uint64_t)task * k + lane] = key;
                reinterpret_cast<uint32_t *>(sw + SL.pay)[(uint64_t)task * k + lane] = pay;
            }
            if (lane == 0) {
                uint32_t *st = reinterpret_cast<uint32_t *>(sw + SL.stat) + (uint64_t)task * 8;
                st[0] = visited;
                st[1] = leaves;
                st[2] = bounds;
                st[3] = dists;
                st[4] = pq;
            }
        };
        if (root < 0) {  // no subtree at this position: an empty list
            put(KEY_NONE, 0, 0, 0, 0, 0, 0);
            continue;
        }

        // query in two layouts: row slices (chunks j, j+8, j+16, j+24) for the
        // leaf scan, and chunk (lane & 31) for bounding two children at once
        uint4 qv[4];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            qv[i] = q[(uint64_t)qi * 32 + j + 8 * i];
            s += popc4(qv[i]);
        }
        const uint32_t pq = readfirst(sum8(s));
        const uint4 qn = q[(uint64_t)qi * 32 + (lane & 31)];
        const uint4 nqn = make_uint4(~qn.x, ~qn.y, ~qn.z, ~qn.w);
        const uint32_t wa = pq > 1 ? pq : 1;
        const uint32_t wb = (QD_BITS - pq) > 1 ? QD_BITS - pq : 1;
        const float *qs = S.s ? S.s + (uint64_t)qi * S.n_scored : nullptr;

        u64 list = KEY_NONE;      // k best (K << 32 | row), lane r = r-th best
        uint32_t payload = 0;     // A | B << 16 of the entry in `list`
        uint32_t kworst = kNone;  // K of the k-th entry (kNone until k entries)
        // split: the least k-th key of the query's tasks known here, and the
        // value the last publishing atomic returned (lane 0; taken in at the
        // next leaf)
        uint32_t ucut = nsplit == 1 ? kNone : readfirst(lane == 0 ? atomicMin(&kshared[qi], kNone) : 0u);
        uint32_t uret = kNone;
        uint32_t visited = 0, leaves = 0, bounds = 0, dists = 0;

        // frontier
        u64 occ = 0;        // best-first: bucket occupancy bits 64*lane .. 64*lane+63
        u64 touched = 0;    // best-first: buckets whose state word is valid for this query
        uint32_t alloc = 0; // best-first: chunks handed out so far
        uint32_t nfree = 0; // best-first: chunks on the free list
        int sp = 0;         // depth-first: stack depth; best-first: entries of the hot bucket in LDS
        uint32_t hot_b = kNone;  // best-first: the bucket whose new entries go to LDS

        // bound of node c from its images (each half-wave holds one node's
        // 32 chunks) and, when stored, its rows' popcount range
        auto node_bound = [&](int32_t c) -> uint32_t {
            const uint4 o = T.orimg[(uint64_t)c * 32 + (lane & 31)];
            const uint32_t ov = sum32(popc_and4(qn, o));
            uint32_t bl = 0;
            if (has_and) bl = sum32(popc_and4(nqn, T.andimg[(uint64_t)c * 32 + (lane & 31)]));
            uint32_t al = pq - ov;
            if (T.pmin) {
                const uint32_t lo = T.pmin[c], hi = T.pmax[c];
                al = pq - (ov < hi ? ov : hi);
                bl = lo > ov && lo - ov > bl ? lo - ov : bl;
            }
            return al * wb + bl * wa;
        };
        // what a node's expansion needs, fetched when the node is bounded (in
        // parallel with its images) and kept with its queue entry, so popping
        // it waits for no load: a leaf's row range (bit 63 set) or its children
        auto info_of = [&](int32_t c) -> u64 {
            const int32_t a = T.child[2 * (uint64_t)c], b = T.child[2 * (uint64_t)c + 1];
            const uint32_t bg = T.begin[c], ct = T.count[c];
            return a < 0 ? ((1ull << 63) | ((u64)ct << 32) | bg) : (((u64)(uint32_t)b << 32) | (uint32_t)a);
        };
        auto bound_pair = [&](int32_t c0, int32_t c1, uint32_t &kb0, uint32_t &kb1, u64 &in0, u64 &in1) {
            const int32_t c = lane < 32 ? c0 : c1;
            const uint32_t kb = node_bound(c);
            const u64 in = info_of(c);
            kb0 = readlane(kb, 0);
            kb1 = readlane(kb, 32);
            in0 = readlane64(in, 0);
            in1 = readlane64(in, 32);
        };
        auto take_chunk = [&]() -> uint32_t {  // lane 0 only; capacity is sized so it never runs out
            const uint32_t c = nfree > 0 ? myfree[nfree - 1] : alloc;
            return c < pool_chunks ? c : (uint32_t)(pool_chunks - 1);
        };
        auto push = [&](uint32_t kb, uint32_t node, u64 info) {
            const u64 e = ((u64)kb << 32) | node;
            if (kBest) {
                uint32_t b = kb / (kBucketLevels * wb);
                b = b < kBuckets ? b : kBuckets - 1;
                // the hot bucket's entries go to the LDS stack while it has room
                const bool to_hot = b == hot_b && readfirst((uint32_t)sp) < kHot;
                const bool tb = (readlane64(touched, (int)(b >> 6)) >> (b & 63)) & 1ull;
                uint32_t took = 0;
                if (lane == 0) {
                    if (to_hot) {
                        stack[sp] = e;
                        sinfo[sp] = info;
                    } else if (!tb) {
                        const uint32_t c = take_chunk();
                        took = 1;
                        myprev[c] = kNone;
                        mypool[(uint64_t)c * kChunk] = make_ulonglong2(e, info);
                        bstate[b] = (c << 5) | 1u;
                    } else {
                        const uint32_t st = bstate[b];
                        const uint32_t c = st >> 5, f = st & 31u;
                        if (f == kChunk) {
                            const uint32_t c2 = take_chunk();
                            took = 1;
                            myprev[c2] = c;
                            mypool[(uint64_t)c2 * kChunk] = make_ulonglong2(e, info);
                            bstate[b] = (c2 << 5) | 1u;
                        } else {
                            mypool[(uint64_t)c * kChunk + f] = make_ulonglong2(e, info);
                            bstate[b] = (c << 5) | (f + 1);
                        }
                    }
                }
                sp = (int)readfirst((uint32_t)sp + (to_hot ? 1u : 0u));
                if (readfirst(took)) {
                    if (nfree > 0)
                        nfree--;
                    else
                        alloc++;
                }
                // the bucket is non-empty; its chunk state is valid once a chunk was written
                const u64 bit = lane == (int)(b >> 6) ? 1ull << (b & 63) : 0ull;
                occ |= bit;
                touched |= to_hot ? 0ull : bit;
            } else {
                if (readfirst((uint32_t)sp) < (uint32_t)kMaxStack) {
                    if (lane == 0) {
                        stack[sp] = e;
                        sinfo[sp] = info;
                    }
                    sp = (int)readfirst((uint32_t)sp + 1);
                }
            }
        };

        // the task's subtree root (the tree's root without a split)
        {
            const uint32_t kb = readlane(node_bound(root), 0);
            const u64 in = readlane64(info_of(root), 0);
            bounds++;
            if (kBest) hot_b = readfirst(kb / (kBucketLevels * wb) < (uint32_t)kBuckets ? kb / (kBucketLevels * wb)
                                                                                          : kBuckets - 1);
            push(kb, (uint32_t)root, in);
        }

        for (;;) {
            u64 e, ninfo;
            uint32_t floor_kb = 0;  // best-first: lower end of the popped bucket, a bound on every open node
            if (kBest) {
                const u64 nz = ballot(occ != 0);
                if (!nz) break;
                const int L = __builtin_ctzll(nz);
                const uint32_t b = 64u * (uint32_t)L + (uint32_t)__builtin_ctzll(readlane64(occ, L));
                floor_kb = b * kBucketLevels * wb;
                if (!(b == hot_b && readfirst((uint32_t)sp) > 0)) {
                    // the bucket's entries are in its chunks; it becomes the hot
                    // bucket (the LDS stack is empty: buckets below hot_b are
                    // empty), and its newest chunk moves to the LDS stack at
                    // once, one lane per entry: one wait for up to kChunk pops
                    hot_b = b;
                    const uint32_t st = readfirst(bstate[b]);
                    const uint32_t c = st >> 5, f = st & 31u;  // f >= 1: the bucket is not empty
                    const uint32_t pc = readfirst(myprev[c]);
                    if ((uint32_t)lane < f) {
                        const ulonglong2 ent = mypool[(uint64_t)c * kChunk + lane];
                        stack[lane] = ent.x;
                        sinfo[lane] = ent.y;
                    }
                    if (lane == 0) {
                        if (pc == kNone) {
                            bstate[b] = c << 5;  // keep the emptied chunk for this bucket
                        } else {
                            bstate[b] = (pc << 5) | kChunk;
                            myfree[nfree] = c;
                        }
                    }
                    if (pc != kNone) nfree++;
                    sp = (int)f;
                }
                // the hot bucket's newest entry, from LDS
                sp = (int)readfirst((uint32_t)sp - 1);
                e = readlane64(lane == 0 ? stack[sp] : 0ull, 0);
                ninfo = readlane64(lane == 0 ? sinfo[sp] : 0ull, 0);
                // once the stack is empty, the bucket is empty unless its chunks still hold entries
                const bool tb = (readlane64(touched, (int)(b >> 6)) >> (b & 63)) & 1ull;
                const uint32_t fill = readfirst(sp != 0 ? 1u : (tb && lane == 0 ? bstate[b] & 31u : 0u));
                occ &= fill == 0 && lane == L ? ~(1ull << (b & 63)) : ~0ull;
            } else {
                if (readfirst((uint32_t)sp) == 0) break;
                sp = (int)readfirst((uint32_t)sp - 1);
                e = readlane64(lane == 0 ? stack[sp] : 0ull, 0);
                ninfo = readlane64(lane == 0 ? sinfo[sp] : 0ull, 0);
            }
            const uint32_t kb = readfirst((uint32_t)(e >> 32)), node = readfirst((uint32_t)e);
            const uint32_t kcut = kworst < ucut ? kworst : ucut;  // kNone: no k-th key yet
            if (kcut != kNone && kb > kcut) {
                // best-first: once the bucket's lower end is past the k-th key,
                // every open node is; a node of a lower bucket is only skipped
                if (kBest && floor_kb > kcut) break;
                continue;  // this entry cannot improve the result
            }
            visited++;
            if (trace && node < n_traced && lane == 0)
                atomicOr(&trace[(uint64_t)qi * ((n_traced + 31) / 32) + node / 32], 1u << (node & 31));
            if (ninfo >> 63) {
                leaves++;
                const uint32_t b0 = readfirst((uint32_t)ninfo), m = readfirst((uint32_t)(ninfo >> 32) & 0x7FFFFFFFu);
                dists += m;
                for (uint32_t base0 = 0; base0 < m; base0 += 32) {
                    // up to 32 rows (4 groups of 8) loaded before any is reduced,
                    // so a whole leaf costs one round trip to memory
                    uint32_t cs[4], tps[4], rows[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const uint32_t r = base0 + 8 * u + (uint32_t)g;
                        const uint64_t pos = (uint64_t)b0 + (r < m ? r : 0);
                        uint4 tv[4];
#pragma unroll
                        for (int i = 0; i < 4; i++) tv[i] = T.sorted[pos * 32 + j + 8 * i];
                        cs[u] = popc_and4(tv[0], qv[0]) + popc_and4(tv[1], qv[1]) + popc_and4(tv[2], qv[2]) +
                                popc_and4(tv[3], qv[3]);
                        tps[u] = T.pop[pos];
                        rows[u] = T.perm[pos];
                    }
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                    const uint32_t base = base0 + 8 * u;
                    if (base >= m) break;
                    const uint32_t r = base + (uint32_t)g;
                    const bool valid = r < m;
                    const uint32_t c = sum8(cs[u]);
                    const uint32_t tp = tps[u];
                    const uint32_t A = pq - c, B = tp - c;
                    const uint32_t K = A * wb + B * wa;
                    const uint32_t row = rows[u];
                    const u64 key = valid ? ((u64)K << 32) | row : KEY_NONE;
                    const u64 thr = kworst == kNone ? KEY_NONE : readlane64(list, (int)k - 1);
                    u64 mk = ballot(j == 0 && key < thr);
                    while (mk) {
                        const int L = __builtin_ctzll(mk);
                        mk &= mk - 1;
                        const u64 cand = readlane64(key, L);
                        const uint32_t cpay = readlane(A | (B << 16), L);
                        const u64 t2 = readlane64(list, (int)k - 1);
                        if (cand < t2) {
                            const int pos2 = __popcll(ballot(list < cand));
                            const u64 up = shift_up64(list);
                            const uint32_t pup =
                                (uint32_t)__builtin_amdgcn_ds_bpermute((lane > 0 ? lane - 1 : 0) << 2, (int)payload);
                            const u64 nl = lane < pos2 ? list : (lane == pos2 ? cand : up);
                            const uint32_t np = lane < pos2 ? payload : (lane == pos2 ? cpay : pup);
                            list = lane < (int)k ? nl : KEY_NONE;
                            payload = lane < (int)k ? np : 0;
                        }
                    }
                    kworst = readfirst(readlane((uint32_t)(readlane64(list, (int)k - 1) >> 32), 0));
                    }
                }
                if (nsplit > 1) {
                    // take in what the previous leaf's atomic returned (the
                    // loads since then were waited for, so it has returned),
                    // then publish this task's k-th key and read the word again
                    ucut = min(ucut, readfirst(uret));
                    uret = lane == 0 ? atomicMin(&kshared[qi], kworst) : 0u;
                }
            } else {
                const int32_t c0 = (int32_t)readfirst((uint32_t)ninfo), c1 = (int32_t)readfirst((uint32_t)(ninfo >> 32));
                uint32_t kb0, kb1;
                u64 in0, in1;
                bound_pair(c0, c1, kb0, kb1, in0, in1);
                bounds += 2;
                const bool ok0 = kcut == kNone || kb0 <= kcut;
                const bool ok1 = kcut == kNone || kb1 <= kcut;
                if (kBest) {
                    if (ok0) push(kb0, (uint32_t)c0, in0);
                    if (ok1) push(kb1, (uint32_t)c1, in1);
                } else {
                    // preferred child last, so it is popped first
                    bool first1 = kb1 < kb0;  // lower bound first; ties: similar child
                    if (qs && (uint32_t)c0 < S.n_scored && (uint32_t)c1 < S.n_scored) first1 = qs[c1] > qs[c0];
                    if (first1) {
                        if (ok0) push(kb0, (uint32_t)c0, in0);
                        if (ok1) push(kb1, (uint32_t)c1, in1);
                    } else {
                        if (ok1) push(kb1, (uint32_t)c1, in1);
                        if (ok0) push(kb0, (uint32_t)c0, in0);
                    }
                }
            }
        }

        put(list, payload, visited, leaves, bounds, dists, pq);
        if (lane == 0) {
            // totals: after the task counter in the workspace head
            unsigned long long *gstats = reinterpret_cast<unsigned long long *>(next_task + 16);
            atomicAdd(&gstats[0], (unsigned long long)visited);
            atomicAdd(&gstats[1], (unsigned long long)leaves);
            atomicAdd(&gstats[2], (unsigned long long)bounds);
            atomicAdd(&gstats[3], (unsigned long long)dists);
        }
    }
}

// The n subtree roots of a split, from the tree's table (positions n - 1 ..
// 2n - 2), into the tasks' area.
__global__ void roots_kernel(const int32_t *__restrict__ table, uint32_t n, int32_t *__restrict__ roots) {
    if (threadIdx.x < n) roots[threadIdx.x] = table[n - 1 + threadIdx.x];
}

__global__ void fill_words_kernel(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__device__ __forceinline__ u64 shfl_xor64(u64 v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m), hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    return (u64)lo | ((u64)hi << 32);
}

// A query's n task lists -> its k nearest, and its statistics summed over
// the tasks (n = 1: a copy).  One wave per query: the lists go to LDS, then
// k steps each take the least head among the lists (the keys are distinct:
// the subtrees partition the rows).
constexpr int kMergeWaves = 4;
__global__ __launch_bounds__(64 * kMergeWaves) void merge_kernel(uint32_t nq, const uint32_t *__restrict__ nq_dev,
                                                                 uint32_t k, uint32_t n, const char *__restrict__ sw,
                                                                 uint32_t *idx, int32_t *missed, int32_t *extra,
                                                                 float *dist, uint32_t *qstats) {
    __shared__ u64 s_key[kMergeWaves][kMaxSplit * QD_MAX_K];
    __shared__ uint32_t s_pay[kMergeWaves][kMaxSplit * QD_MAX_K];
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const SplitLayout SL = split_layout(nq, n, k);  // laid out for nq queries
    const u64 *key = reinterpret_cast<const u64 *>(sw + SL.key);
    const uint32_t *pay = reinterpret_cast<const uint32_t *>(sw + SL.pay);
    const uint32_t *stat = reinterpret_cast<const uint32_t *>(sw + SL.stat);
    if (nq_dev) nq = min(nq, *nq_dev);
    const uint32_t qi = blockIdx.x * kMergeWaves + w;
    if (qi >= nq) return;  // the whole wave; nothing below waits for other waves
    const uint32_t nk = n * k;
    const uint64_t base = (uint64_t)qi * nk;
    u64 *sk = s_key[w];
    uint32_t *sp = s_pay[w];
    for (uint32_t e = (uint32_t)lane; e < nk; e += 64) {
        sk[e] = key[base + e];
        sp[e] = pay[base + e];
    }
    // statistics: lane t < n holds task t's
    uint32_t v0 = 0, v1 = 0, v2 = 0, v3 = 0, pq = 0;
    if ((uint32_t)lane < n) {
        const uint32_t *st = stat + ((uint64_t)qi * n + lane) * 8;
        v0 = st[0];
        v1 = st[1];
        v2 = st[2];
        v3 = st[3];
        pq = st[4];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        v0 += (uint32_t)__shfl_xor((int)v0, m);
        v1 += (uint32_t)__shfl_xor((int)v1, m);
        v2 += (uint32_t)__shfl_xor((int)v2, m);
        v3 += (uint32_t)__shfl_xor((int)v3, m);
        pq = max(pq, (uint32_t)__shfl_xor((int)pq, m));  // an empty task reports 0
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t h = 0;  // lane t < n: entries of list t taken
    u64 head = (uint32_t)lane < n ? sk[lane * k] : KEY_NONE;
    u64 mine = KEY_NONE;  // lane r < k: the r-th nearest
    uint32_t mpay = 0;
    for (uint32_t r = 0; r < k; r++) {
        u64 m = head;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            const u64 o = shfl_xor64(m, s);
            m = o < m ? o : m;
        }
        if (m == KEY_NONE) break;  // every list is exhausted
        const int L = __builtin_ctzll(ballot(head == m));
        const uint32_t hl = readlane(h, L);
        const uint32_t pl = sp[(uint32_t)L * k + hl];
        if ((uint32_t)lane == r) {
            mine = m;
            mpay = pl;
        }
        if (lane == L) {
            h++;
            head = h < k ? sk[lane * k + h] : KEY_NONE;
        }
    }
    if ((uint32_t)lane < k) {
        const uint64_t o = (uint64_t)qi * k + lane;
        if (mine == KEY_NONE) {
            idx[o] = QD_PAD_IDX;
            missed[o] = -1;
            extra[o] = -1;
            dist[o] = __builtin_inff();
        } else {
            const uint32_t wa = pq > 1 ? pq : 1;
            const uint32_t wb = (QD_BITS - pq) > 1 ? QD_BITS - pq : 1;
            idx[o] = (uint32_t)mine;
            missed[o] = (int32_t)(mpay & 0xFFFF);
            extra[o] = (int32_t)(mpay >> 16);
            dist[o] = (float)((double)(mine >> 32) / ((double)wa * (double)wb));
        }
    }
    if (qstats && lane == 0) {
        qstats[(uint64_t)qi * 4 + 0] = v0;
        qstats[(uint64_t)qi * 4 + 1] = v1;
        qstats[(uint64_t)qi * 4 + 2] = v2;
        qstats[(uint64_t)qi * 4 + 3] = v3;
    }
}

}  // namespace

__global__ void zero_words_kernel(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

bool depth_first_fits(qd_tree_t t) { return t->depth + 2 <= (uint32_t)kMaxStack; }

TreeLaunch tree_launch_shape(qd_tree_t t, uint32_t nq_max, uint32_t k, int order, uint32_t waves_per_cu,
                             uint32_t split) {
    TreeLaunch L;
    const int cus = device_cus();
    if (waves_per_cu == 0) waves_per_cu = order == QD_ORDER_BEST_FIRST ? 12 : 16;  // as many as registers hold
    if (split == 0) split = kDefaultSplit;
    L.split = split;
    uint64_t blocks = ((uint64_t)cus * waves_per_cu + kWaves - 1) / kWaves;
    const uint64_t need = ((uint64_t)(nq_max ? nq_max : 1) * split + kWaves - 1) / kWaves;
    if (blocks > need) blocks = need;
    L.blocks = blocks;
    L.slots = blocks * kWaves;
    // A search queues each node of its subtree at most once.  Live chunks: a
    // bucket holds at most one partly filled chunk (or one kept empty chunk)
    // besides full ones, and emptied chunks go to a free list, so (the
    // subtree's nodes)/kChunk + 2 per bucket chunks never run out.
    const uint64_t sub = t->split_nodes[__builtin_ctz(split)];
    L.pool_chunks = order == QD_ORDER_BEST_FIRST ? sub / kChunk + 2 * kBuckets + 2 : 1;
    L.head = 256;  // [counter | pad | stats x4 | pad]
    L.prev_bytes = (size_t)(L.slots * L.pool_chunks * 8 + 255) / 256 * 256;  // prev + free list
    L.pool_bytes = (size_t)L.slots * L.pool_chunks * kChunk * 16;  // 16-byte records: entry, node info
    L.split_bytes = split_layout(nq_max ? nq_max : 1, split, k).bytes;  // the tasks' lists, also unsplit
    return L;
}

bool split_ok(uint32_t split) { return split == 0 || (split <= kMaxSplit && (split & (split - 1)) == 0); }

int tree_launch(qd_tree_t t, const TreeLaunch &L, char *ws, const uint64_t *d_q, uint32_t nq,
                const uint32_t *nq_dev, uint32_t k, int order, const float *d_scores, uint32_t n_scored,
                uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist, uint32_t *d_qstats,
                uint32_t *d_trace, uint32_t n_traced, hipStream_t s) {
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(ws),
                       (uint32_t)(L.head / 4));
    uint32_t *counter = reinterpret_cast<uint32_t *>(ws);  // the kernel adds its totals at ws + 64
    uint32_t *chunk_prev = reinterpret_cast<uint32_t *>(ws + L.head);
    u64 *pool = reinterpret_cast<u64 *>(ws + L.head + L.prev_bytes);
    TreeView T{reinterpret_cast<const uint4 *>(t->d_sorted), t->d_perm, reinterpret_cast<const uint4 *>(t->d_or),
               reinterpret_cast<const uint4 *>(t->d_and), t->d_child, t->d_begin, t->d_count, t->d_pop,
               t->d_pmin, t->d_pmax};
    Scores S{d_scores, d_scores ? n_scored : 0};
    if (L.split > 1 && d_trace) return fail(QD_ERR_INVALID, "a traced search runs unsplit");
    char *sw = ws + L.head + L.prev_bytes + L.pool_bytes;  // the tasks' area
    if (L.split > 1) {
        hipLaunchKernelGGL(roots_kernel, dim3(1), dim3(64), 0, s, t->d_split_roots, L.split,
                           reinterpret_cast<int32_t *>(sw));
        const uint32_t fg = (nq + 255) / 256;
        hipLaunchKernelGGL(fill_words_kernel, dim3(fg < 1 ? 1 : fg < 1024 ? fg : 1024), dim3(256), 0, s,
                           reinterpret_cast<uint32_t *>(sw + split_layout(nq, L.split, k).kshared), (uint64_t)nq,
                           kNone);
    }
    {
        KernelTimer timer("tree_knn", s);
        if (order == QD_ORDER_BEST_FIRST)
            hipLaunchKernelGGL(tree_knn_kernel<true>, dim3((uint32_t)L.blocks), dim3(kBlock), 0, s, T,
                               reinterpret_cast<const uint4 *>(d_q), nq, k, counter, pool, chunk_prev, L.pool_chunks,
                               S, d_trace, n_traced, nq_dev, sw, L.split);
        else
            hipLaunchKernelGGL(tree_knn_kernel<false>, dim3((uint32_t)L.blocks), dim3(kBlock), 0, s, T,
                               reinterpret_cast<const uint4 *>(d_q), nq, k, counter, pool, chunk_prev, L.pool_chunks,
                               S, d_trace, n_traced, nq_dev, sw, L.split);
    }
    QD_HIP_CHECK(hipGetLastError());
    {
        KernelTimer timer("tree_merge", s);
        hipLaunchKernelGGL(merge_kernel, dim3((nq + kMergeWaves - 1) / kMergeWaves), dim3(64 * kMergeWaves), 0, s,
                           nq, nq_dev, k, L.split, sw, d_idx, d_missed, d_extra, d_dist, d_qstats);
    }
    QD_HIP_CHECK(hipGetLastError());
    return QD_OK;
}

int knn_tree_impl(qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k, int order, const float *d_scores,
                  uint32_t n_scored, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist,
                  uint32_t *d_qstats, qd_stats *h_stats, void *stream, uint32_t waves_per_cu, uint32_t *d_trace,
                  uint32_t n_traced, uint32_t split) {
    if (!t) return fail(QD_ERR_INVALID, "null tree");
    if (!split_ok(split)) return fail(QD_ERR_INVALID, "query_split %u: 0 or a power of two up to %u", split, kMaxSplit);
    if (k < 1 || k > QD_MAX_K) return fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
    if (order != QD_ORDER_BEST_FIRST && order != QD_ORDER_DEPTH_FIRST && order != QD_ORDER_BLOCKED)
        return fail(QD_ERR_INVALID, "unknown frontier order %d", order);
    if (h_stats) *h_stats = qd_stats{0, 0, 0, 0};
    if (nq == 0) return QD_OK;
    if (!d_q || !d_idx || !d_missed || !d_extra || !d_dist) return fail(QD_ERR_INVALID, "null pointer");
    if (!aligned16(d_q)) return fail(QD_ERR_INVALID, "queries must be 16-byte aligned");
    if (order == QD_ORDER_BLOCKED) {
        if (d_scores || d_trace) return fail(QD_ERR_INVALID, "the blocked order takes no scores or traces");
        return knn_tree_blocked(t, d_q, nq, k, nullptr, d_idx, d_missed, d_extra, d_dist, d_qstats, h_stats,
                                (hipStream_t)stream);
    }
    if (order == QD_ORDER_DEPTH_FIRST && !depth_first_fits(t))
        return fail(QD_ERR_UNSUPPORTED, "tree depth %u exceeds the depth-first stack (%d)", t->depth, kMaxStack);
    if (n_traced > t->n_nodes) return fail(QD_ERR_INVALID, "n_traced above the node count");
    if (d_trace && n_traced) split = 1;  // traces follow the one-wave traversal
    if ((uint64_t)nq * (split ? split : kDefaultSplit) > 0x7FFFFFFFull)
        return fail(QD_ERR_INVALID, "%u queries x %u subtree searches: too many tasks", nq, split ? split : kDefaultSplit);
    hipStream_t s = (hipStream_t)stream;
    const TreeLaunch L = tree_launch_shape(t, nq, k, order, waves_per_cu, split);
    char *ws = nullptr;
    QD_HIP_CHECK(hipMallocAsync((void **)&ws, L.total(), s));
    if (d_trace && n_traced)
        QD_HIP_CHECK(hipMemsetAsync(d_trace, 0, (size_t)nq * ((n_traced + 31) / 32) * 4, s));
    int rc = tree_launch(t, L, ws, d_q, nq, nullptr, k, order, d_scores, n_scored, d_idx, d_missed, d_extra, d_dist,
                         d_qstats, d_trace, n_traced, s);
    hipError_t e = hipSuccess;
    if (rc == QD_OK && h_stats) {
        unsigned long long hs[4];
        e = hipMemcpyAsync(hs, ws + 64, sizeof hs, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) *h_stats = qd_stats{hs[0], hs[1], hs[2], hs[3]};
    }
    hipError_t e2 = hipFreeAsync(ws, s);
    if (rc != QD_OK) return rc;
    if (e != hipSuccess) return fail(QD_ERR_DEVICE, "tree search: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(QD_ERR_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e2));
    return QD_OK;
}

}  // namespace qd

extern "C" int qd_knn_tree(qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k, const qd_search_params *p,
                           uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist,
                           uint32_t *d_query_stats, qd_stats *h_stats, void *stream) {
    const int order = p ? (int)p->order : QD_ORDER_BEST_FIRST;
    const float *sc = p ? p->d_scores : nullptr;
    uint32_t ns = p ? p->n_scored : 0;
    const uint32_t wpc = p ? p->waves_per_cu : 0;
    qd_model_t model = p ? p->model : nullptr;
    if (sc && order != QD_ORDER_DEPTH_FIRST)
        return qd::fail(QD_ERR_INVALID, "node scores order the depth-first frontier only");
    if (model && order == QD_ORDER_BEST_FIRST)
        return qd::fail(QD_ERR_INVALID, "a model orders the depth-first and blocked searches only");
    if (model && sc) return qd::fail(QD_ERR_INVALID, "give node scores or a model, not both");
    if (model && order == QD_ORDER_DEPTH_FIRST && t && nq > 0) {
        // score the top nodes for every query, then search in that order
        if (ns == 0) ns = (uint32_t)std::min<uint64_t>(2047, t->n_nodes);
        if (ns > t->n_nodes) return qd::fail(QD_ERR_INVALID, "n_scored %u above the node count", ns);
        if (k < 1 || k > QD_MAX_K) return qd::fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
        if (!d_q || !d_idx || !d_missed || !d_extra || !d_dist) return qd::fail(QD_ERR_INVALID, "null pointer");
        hipStream_t s = (hipStream_t)stream;
        float *scores = nullptr;
        QD_HIP_CHECK(hipMallocAsync((void **)&scores, (size_t)nq * ns * sizeof(float), s));
        int rc = qd_model_score_tree(model, t, d_q, nq, ns, scores, stream);
        if (rc == QD_OK)
            rc = qd::knn_tree_impl(t, d_q, nq, k, order, scores, ns, d_idx, d_missed, d_extra, d_dist, d_query_stats,
                                   h_stats, stream, wpc, p->d_visited, p->n_traced, p->query_split);
        (void)hipFreeAsync(scores, s);
        return rc;
    }
    if (order == QD_ORDER_BLOCKED && t && nq > 0) {
        if (k < 1 || k > QD_MAX_K) return qd::fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
        if (!d_q || !d_idx || !d_missed || !d_extra || !d_dist) return qd::fail(QD_ERR_INVALID, "null pointer");
        if (!qd::aligned16(d_q)) return qd::fail(QD_ERR_INVALID, "queries must be 16-byte aligned");
        if (p && p->d_visited) return qd::fail(QD_ERR_INVALID, "the blocked order takes no traces");
        return qd::knn_tree_blocked(t, d_q, nq, k, p, d_idx, d_missed, d_extra, d_dist, d_query_stats, h_stats,
                                    (hipStream_t)stream);
    }
    return qd::knn_tree_impl(t, d_q, nq, k, order, sc, ns, d_idx, d_missed, d_extra, d_dist, d_query_stats, h_stats,
                             stream, wpc, p ? p->d_visited : nullptr, p ? p->n_traced : 0, p ? p->query_split : 0);
}

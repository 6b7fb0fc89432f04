// Dissimilarity Tree construction on the GPU (Section 4.1, Listing 1).
//
// The paper's split of a node takes bit positions in ascending popularity
// (ties: ascending bit index) and moves every descriptor still in the similar
// set that has the bit set, stopping once the dissimilar set holds at least
// half of the node and never applying a move that would empty the similar
// set.  A descriptor therefore leaves with the first processed bit it has
// set: its least popular set bit, fr(t) = the set bit b minimising the key
// (popularity(b), b).  With the keys of all members known, the loop collapses
// to a cut on that key:
//   x* = the ceil(n/2)-th smallest member key (zero rows have no key and
//        sort last);
//   D  = {t : key(t) <= x*}, unless that is the whole node, then
//   D  = {t : key(t) <  x*};
//   if every member's key is absent or fewer than ceil(n/2) rows are nonzero,
//   D = the nonzero rows.
// The tree is built level by level.  Each node is a segment of a permutation
// of the rows; a split writes the similar rows, then the dissimilar rows, each
// in their previous order (a stable partition), so the layout matches a
// breadth-first numbering with the similar child first.  Nodes of at most
// kSmall rows are split by one block entirely in LDS; larger nodes use a
// multi-block path with global counters.  Sum (OR) and product (AND) images
// are then formed for every node, leaves from their rows and inner nodes from
// their children, deepest level first.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "qd_device.h"
#include "qd_internal.h"
#include "qd_tree.h"

namespace qd {
namespace {

constexpr int kBlock = 256;
constexpr uint32_t kSmall = 2048;  // rows a single block splits in LDS
constexpr uint32_t kChunk = 2048;  // rows per work item of a large node
constexpr uint16_t kNoBit = 0xFFFF;
constexpr u64 kCutAllNonzero = ~0ull - 1;

__device__ __forceinline__ uint32_t min8(uint32_t v) {
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false));
    return v;
}

// Per-lane slice of a row: lane j of an 8-lane group holds 16-byte chunks
// j, j+8, j+16, j+24.  Dword d of chunk c covers bits 32*(4c+d) .. +31.
struct RowSlice {
    uint4 v[4];
};

__device__ __forceinline__ RowSlice load_row(const uint4 *db, uint32_t row, int j) {
    RowSlice s;
#pragma unroll
    for (int i = 0; i < 4; i++) s.v[i] = db[(uint64_t)row * 32 + j + 8 * i];
    return s;
}

__device__ __forceinline__ uint32_t dword_of(const RowSlice &s, int i, int d) {
    return d == 0 ? s.v[i].x : d == 1 ? s.v[i].y : d == 2 ? s.v[i].z : s.v[i].w;
}

// Add the row's set bits to the 4096 counters in cnt.
__device__ __forceinline__ void count_bits(const RowSlice &s, int j, uint32_t *cnt) {
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int d = 0; d < 4; d++) {
            uint32_t w = dword_of(s, i, d);
            const uint32_t base = 32u * (4u * (uint32_t)(j + 8 * i) + (uint32_t)d);
            while (w) {
                const int b = __builtin_ctz(w);
                w &= w - 1;
                atomicAdd(&cnt[base + b], 1u);
            }
        }
}

// Least popular set bit of the row under the 4096 counters cnt; the result
// (key = cnt << 12 | bit, as 64 bits) is valid in every lane of the group.
__device__ __forceinline__ u64 first_ranked(const RowSlice &s, int j, const uint32_t *cnt) {
    u64 best = ~0ull;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int d = 0; d < 4; d++) {
            uint32_t w = dword_of(s, i, d);
            const uint32_t base = 32u * (4u * (uint32_t)(j + 8 * i) + (uint32_t)d);
            while (w) {
                const int b = __builtin_ctz(w);
                w &= w - 1;
                const u64 key = ((u64)cnt[base + b] << 12) | (base + b);
                best = key < best ? key : best;
            }
        }
    // min over the 8 lanes of the group, 64-bit: reduce high then low words
    uint32_t hi = min8((uint32_t)(best >> 32));
    uint32_t lo = (uint32_t)(best >> 32) == hi ? (uint32_t)best : 0xFFFFFFFFu;
    lo = min8(lo);
    return ((u64)hi << 32) | lo;
}

// Block-wide cut from the first-ranked-bit histogram.  keys[0..nb) are the
// sorted keys (cnt << 12 | bit) of the bits with hist > 0.  Writes the cut
// key and the size of the dissimilar side to *cut / *nd (thread 0's view is
// broadcast through LDS).
__device__ void find_cut(const u64 *keys, uint32_t nb, const uint32_t *hist, uint32_t m, u64 *cut, uint32_t *nd,
                         uint32_t *scan /* kBlock + 1 */) {
    const uint32_t t = threadIdx.x;
    const uint32_t per = (nb + kBlock - 1) / kBlock;
    const uint32_t lo = t * per, hi = lo + per < nb ? lo + per : nb;
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; i++) s += hist[keys[i] & 4095];
    scan[t + 1] = s;
    if (t == 0) scan[0] = 0;
    __syncthreads();
    if (t == 0) {
        for (uint32_t i = 1; i <= kBlock; i++) scan[i] += scan[i - 1];
    }
    __syncthreads();
    const uint32_t total = scan[kBlock];
    const uint32_t half = (m + 1) / 2;
    if (total < half) {
        if (t == 0) {
            *cut = kCutAllNonzero;
            *nd = total;
        }
    } else {
        uint32_t run = scan[t];
        for (uint32_t i = lo; i < hi; i++) {
            const uint32_t h = hist[keys[i] & 4095];
            if (run < half && run + h >= half) {
                if (run + h == m) {
                    *cut = keys[i] - 1;
                    *nd = run;
                } else {
                    *cut = keys[i];
                    *nd = run + h;
                }
            }
            run += h;
        }
    }
    __syncthreads();
}

// Collect the keys of bits with hist > 0 into keys[], sort them, return count.
__device__ uint32_t collect_sorted_keys(const uint32_t *hist, const uint32_t *cnt, u64 *keys, uint32_t *counter) {
    if (threadIdx.x == 0) *counter = 0;
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < 4096; b += kBlock)
        if (hist[b]) keys[atomicAdd(counter, 1u)] = ((u64)cnt[b] << 12) | b;
    __syncthreads();
    const uint32_t nb = *counter;
    const uint32_t np = next_pow2(nb < 2 ? 2 : nb);
    for (uint32_t i = nb + threadIdx.x; i < np; i += kBlock) keys[i] = ~0ull;
    __syncthreads();
    block_bitonic_sort(keys, np);
    return nb;
}

// Stable partition of one node segment given per-member dissimilar flags held
// as bits in flags[] (member r -> bit r).  Each thread owns a run of `per`
// consecutive members.
__device__ void stable_partition(const uint32_t *perm_in, uint32_t *perm_out, uint64_t begin, uint32_t m,
                                 uint32_t nd, const uint8_t *flag, uint32_t *scan) {
    const uint32_t t = threadIdx.x;
    const uint32_t per = (m + kBlock - 1) / kBlock;
    const uint32_t lo = t * per, hi = lo + per < m ? lo + per : m;
    uint32_t c = 0;
    for (uint32_t r = lo; r < hi; r++) c += flag[r];
    scan[t + 1] = c;
    if (t == 0) scan[0] = 0;
    __syncthreads();
    if (t == 0)
        for (uint32_t i = 1; i <= kBlock; i++) scan[i] += scan[i - 1];
    __syncthreads();
    uint32_t dpos = scan[t];
    uint32_t spos = lo - dpos;
    const uint32_t ns = m - nd;
    for (uint32_t r = lo; r < hi; r++) {
        const uint32_t v = perm_in[begin + r];
        if (flag[r])
            perm_out[begin + ns + dpos++] = v;
        else
            perm_out[begin + spos++] = v;
    }
    __syncthreads();
}

// One block splits one node of m <= kSmall rows entirely in LDS.
__global__ __launch_bounds__(kBlock) void split_small_kernel(const uint4 *__restrict__ db,
                                                             const uint32_t *__restrict__ perm_in,
                                                             uint32_t *__restrict__ perm_out,
                                                             const uint64_t *__restrict__ nbegin,
                                                             const uint32_t *__restrict__ ncount,
                                                             uint32_t *__restrict__ nd_out) {
    __shared__ uint32_t cnt[4096];
    __shared__ uint32_t hist[4096];
    __shared__ u64 keys[4096];
    __shared__ uint16_t fr[kSmall];
    __shared__ uint8_t flag[kSmall];
    __shared__ uint32_t scan[kBlock + 1];
    __shared__ uint32_t counter;
    __shared__ u64 cut;
    __shared__ uint32_t nd;
    const uint64_t begin = nbegin[blockIdx.x];
    const uint32_t m = ncount[blockIdx.x];
    const int lane = threadIdx.x & 63, j = lane & 7;
    const uint32_t group = threadIdx.x >> 3;  // 32 groups of 8 lanes
    for (uint32_t i = threadIdx.x; i < 4096; i += kBlock) {
        cnt[i] = 0;
        hist[i] = 0;
    }
    __syncthreads();
    for (uint32_t r = group; r < m; r += kBlock / 8) count_bits(load_row(db, perm_in[begin + r], j), j, cnt);
    __syncthreads();
    for (uint32_t r = group; r < m; r += kBlock / 8) {
        const u64 key = first_ranked(load_row(db, perm_in[begin + r], j), j, cnt);
        if (j == 0) {
            const uint16_t b = key == ~0ull ? kNoBit : (uint16_t)(key & 4095);
            fr[r] = b;
            if (b != kNoBit) atomicAdd(&hist[b], 1u);
        }
    }
    __syncthreads();
    const uint32_t nb = collect_sorted_keys(hist, cnt, keys, &counter);
    if (threadIdx.x == 0) {
        cut = 0;
        nd = 0;
    }
    __syncthreads();
    find_cut(keys, nb, hist, m, &cut, &nd, scan);
    const u64 c = cut;
    for (uint32_t r = threadIdx.x; r < m; r += kBlock)
        flag[r] = fr[r] != kNoBit && ((((u64)cnt[fr[r]]) << 12) | fr[r]) <= c;
    __syncthreads();
    stable_partition(perm_in, perm_out, begin, m, nd, flag, scan);
    if (threadIdx.x == 0) nd_out[blockIdx.x] = nd;
}

// ---- large nodes: work items are (node slot, row range) chunks ----

struct Item {
    uint32_t slot;  // index among the level's large nodes
    uint32_t first; // first member (relative to node begin)
    uint32_t count; // members in this chunk
    uint32_t pad;
};

__global__ __launch_bounds__(kBlock) void big_count_kernel(const uint4 *__restrict__ db,
                                                           const uint32_t *__restrict__ perm_in,
                                                           const uint64_t *__restrict__ nbegin,
                                                           const Item *__restrict__ items,
                                                           uint32_t *__restrict__ gcnt) {
    __shared__ uint32_t cnt[4096];
    const Item it = items[blockIdx.x];
    const uint64_t begin = nbegin[it.slot] + it.first;
    const int j = threadIdx.x & 7;
    const uint32_t group = threadIdx.x >> 3;
    for (uint32_t i = threadIdx.x; i < 4096; i += kBlock) cnt[i] = 0;
    __syncthreads();
    for (uint32_t r = group; r < it.count; r += kBlock / 8) count_bits(load_row(db, perm_in[begin + r], j), j, cnt);
    __syncthreads();
    uint32_t *g = gcnt + (uint64_t)it.slot * 4096;
    for (uint32_t i = threadIdx.x; i < 4096; i += kBlock)
        if (cnt[i]) atomicAdd(&g[i], cnt[i]);
}

__global__ __launch_bounds__(kBlock) void big_first_kernel(const uint4 *__restrict__ db,
                                                           const uint32_t *__restrict__ perm_in,
                                                           const uint64_t *__restrict__ nbegin,
                                                           const Item *__restrict__ items,
                                                           const uint32_t *__restrict__ gcnt,
                                                           uint16_t *__restrict__ fr_pos,
                                                           uint32_t *__restrict__ ghist) {
    __shared__ uint32_t cnt[4096];
    __shared__ uint32_t hist[4096];
    const Item it = items[blockIdx.x];
    const uint64_t begin = nbegin[it.slot] + it.first;
    const int j = threadIdx.x & 7;
    const uint32_t group = threadIdx.x >> 3;
    const uint32_t *gc = gcnt + (uint64_t)it.slot * 4096;
    for (uint32_t i = threadIdx.x; i < 4096; i += kBlock) {
        cnt[i] = gc[i];
        hist[i] = 0;
    }
    __syncthreads();
    for (uint32_t r = group; r < it.count; r += kBlock / 8) {
        const u64 key = first_ranked(load_row(db, perm_in[begin + r], j), j, cnt);
        if (j == 0) {
            const uint16_t b = key == ~0ull ? kNoBit : (uint16_t)(key & 4095);
            fr_pos[begin + r] = b;
            if (b != kNoBit) atomicAdd(&hist[b], 1u);
        }
    }
    __syncthreads();
    uint32_t *g = ghist + (uint64_t)it.slot * 4096;
    for (uint32_t i = threadIdx.x; i < 4096; i += kBlock)
        if (hist[i]) atomicAdd(&g[i], hist[i]);
}

__global__ __launch_bounds__(kBlock) void big_cut_kernel(const uint32_t *__restrict__ gcnt,
                                                         const uint32_t *__restrict__ ghist,
                                                         const uint32_t *__restrict__ ncount, u64 *__restrict__ cut_out,
                                                         uint32_t *__restrict__ nd_out) {
    __shared__ uint32_t cnt[4096];
    __shared__ uint32_t hist[4096];
    __shared__ u64 keys[4096];
    __shared__ uint32_t scan[kBlock + 1];
    __shared__ uint32_t counter;
    __shared__ u64 cut;
    __shared__ uint32_t nd;
    const uint32_t slot = blockIdx.x;
    for (uint32_t i = threadIdx.x; i < 4096; i += kBlock) {
        cnt[i] = gcnt[(uint64_t)slot * 4096 + i];
        hist[i] = ghist[(uint64_t)slot * 4096 + i];
    }
    if (threadIdx.x == 0) {
        cut = 0;
        nd = 0;
    }
    __syncthreads();
    const uint32_t nb = collect_sorted_keys(hist, cnt, keys, &counter);
    find_cut(keys, nb, hist, ncount[slot], &cut, &nd, scan);
    if (threadIdx.x == 0) {
        cut_out[slot] = cut;
        nd_out[slot] = nd;
    }
}

__device__ __forceinline__ bool big_is_d(uint16_t b, const uint32_t *gc, u64 cut) {
    return b != kNoBit && ((((u64)gc[b]) << 12) | b) <= cut;
}

__global__ __launch_bounds__(kBlock) void big_dcount_kernel(const uint64_t *__restrict__ nbegin,
                                                            const Item *__restrict__ items,
                                                            const uint32_t *__restrict__ gcnt,
                                                            const u64 *__restrict__ cuts,
                                                            const uint16_t *__restrict__ fr_pos,
                                                            uint32_t *__restrict__ dcount) {
    __shared__ uint32_t total;
    const Item it = items[blockIdx.x];
    const uint64_t begin = nbegin[it.slot] + it.first;
    const uint32_t *gc = gcnt + (uint64_t)it.slot * 4096;
    const u64 cut = cuts[it.slot];
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    uint32_t c = 0;
    for (uint32_t r = threadIdx.x; r < it.count; r += kBlock) c += big_is_d(fr_pos[begin + r], gc, cut);
    atomicAdd(&total, c);
    __syncthreads();
    if (threadIdx.x == 0) dcount[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void big_scatter_kernel(const uint32_t *__restrict__ perm_in,
                                                             uint32_t *__restrict__ perm_out,
                                                             const uint64_t *__restrict__ nbegin,
                                                             const uint32_t *__restrict__ ncount,
                                                             const Item *__restrict__ items,
                                                             const uint32_t *__restrict__ gcnt,
                                                             const u64 *__restrict__ cuts,
                                                             const uint32_t *__restrict__ nds,
                                                             const uint16_t *__restrict__ fr_pos,
                                                             const uint32_t *__restrict__ doff) {
    __shared__ uint32_t scan[kBlock + 1];
    const Item it = items[blockIdx.x];
    const uint64_t nb0 = nbegin[it.slot];
    const uint64_t begin = nb0 + it.first;
    const uint32_t *gc = gcnt + (uint64_t)it.slot * 4096;
    const u64 cut = cuts[it.slot];
    const uint32_t t = threadIdx.x;
    const uint32_t per = (it.count + kBlock - 1) / kBlock;
    const uint32_t lo = t * per, hi = lo + per < it.count ? lo + per : it.count;
    uint32_t c = 0;
    for (uint32_t r = lo; r < hi; r++) c += big_is_d(fr_pos[begin + r], gc, cut);
    scan[t + 1] = c;
    if (t == 0) scan[0] = 0;
    __syncthreads();
    if (t == 0)
        for (uint32_t i = 1; i <= kBlock; i++) scan[i] += scan[i - 1];
    __syncthreads();
    const uint32_t ns = ncount[it.slot] - nds[it.slot];
    const uint32_t d_before = doff[blockIdx.x];
    uint32_t dpos = d_before + scan[t];
    uint32_t spos = it.first + lo - dpos;
    for (uint32_t r = lo; r < hi; r++) {
        const uint32_t v = perm_in[begin + r];
        if (big_is_d(fr_pos[begin + r], gc, cut))
            perm_out[nb0 + ns + dpos++] = v;
        else
            perm_out[nb0 + spos++] = v;
    }
}

// ---- images and the leaf-ordered copy ----

// sorted[i] = db[perm[i]]
__global__ __launch_bounds__(kBlock) void gather_rows_kernel(const uint4 *__restrict__ db,
                                                             const uint32_t *__restrict__ perm, uint64_t n,
                                                             uint4 *__restrict__ sorted) {
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t e = tid; e < n * 32; e += stride) sorted[e] = db[(uint64_t)perm[e >> 5] * 32 + (e & 31)];
}

// Smallest and largest of a wave's 64 values (every lane gets them).
__device__ __forceinline__ void wave_min_max(uint32_t &mn, uint32_t &mx) {
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) {
        const uint32_t a = (uint32_t)__shfl_xor((int)mn, sh), b = (uint32_t)__shfl_xor((int)mx, sh);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
}

// One wave per leaf: OR / AND over its rows of the leaf-ordered copy, and
// the popcount range of the rows (when pmin is given).
__global__ __launch_bounds__(kBlock) void leaf_images_kernel(const uint4 *__restrict__ sorted,
                                                             const uint32_t *__restrict__ leaf_ids, uint32_t n_leaves,
                                                             const uint32_t *__restrict__ begin,
                                                             const uint32_t *__restrict__ count,
                                                             uint4 *__restrict__ or_img, uint4 *__restrict__ and_img,
                                                             const uint16_t *__restrict__ pop,
                                                             uint16_t *__restrict__ pmin, uint16_t *__restrict__ pmax) {
    const uint32_t w = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (w >= n_leaves) return;
    const uint32_t node = leaf_ids[w];
    const int lane = threadIdx.x & 63;
    const uint32_t c = lane & 31, half = lane >> 5;
    const uint64_t b = begin[node];
    const uint32_t m = count[node];
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint32_t r = half; r < m; r += 2) {
        const uint4 v = sorted[(b + r) * 32 + c];
        o.x |= v.x; o.y |= v.y; o.z |= v.z; o.w |= v.w;
        a.x &= v.x; a.y &= v.y; a.z &= v.z; a.w &= v.w;
    }
    // combine the two half-waves (lane l with lane l^32)
    uint4 o2, a2;
    o2.x = __shfl_xor(o.x, 32); o2.y = __shfl_xor(o.y, 32); o2.z = __shfl_xor(o.z, 32); o2.w = __shfl_xor(o.w, 32);
    a2.x = __shfl_xor(a.x, 32); a2.y = __shfl_xor(a.y, 32); a2.z = __shfl_xor(a.z, 32); a2.w = __shfl_xor(a.w, 32);
    if (half == 0) {
        or_img[(uint64_t)node * 32 + c] = make_uint4(o.x | o2.x, o.y | o2.y, o.z | o2.z, o.w | o2.w);
        if (and_img) and_img[(uint64_t)node * 32 + c] = make_uint4(a.x & a2.x, a.y & a2.y, a.z & a2.z, a.w & a2.w);
    }
    if (pmin) {
        uint32_t mn = 0xFFFFu, mx = 0;
        for (uint32_t r = lane; r < m; r += 64) {
            const uint32_t v = pop[b + r];
            mn = v < mn ? v : mn;
            mx = v > mx ? v : mx;
        }
        wave_min_max(mn, mx);
        if (lane == 0) {
            pmin[node] = (uint16_t)mn;
            pmax[node] = (uint16_t)mx;
        }
    }
}

// Inner nodes of one level: images and popcount range combine the two
// children's.
__global__ __launch_bounds__(kBlock) void inner_images_kernel(const uint32_t *__restrict__ ids, uint32_t n_ids,
                                                              const int32_t *__restrict__ child,
                                                              uint4 *__restrict__ or_img, uint4 *__restrict__ and_img,
                                                              uint16_t *__restrict__ pmin, uint16_t *__restrict__ pmax) {
    const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= (uint64_t)n_ids * 32) return;
    const uint32_t node = ids[e >> 5], c = e & 31;
    const int32_t s = child[2 * node], d = child[2 * node + 1];
    const uint4 x = or_img[(uint64_t)s * 32 + c], y = or_img[(uint64_t)d * 32 + c];
    or_img[(uint64_t)node * 32 + c] = make_uint4(x.x | y.x, x.y | y.y, x.z | y.z, x.w | y.w);
    if (and_img) {
        const uint4 p = and_img[(uint64_t)s * 32 + c], r = and_img[(uint64_t)d * 32 + c];
        and_img[(uint64_t)node * 32 + c] = make_uint4(p.x & r.x, p.y & r.y, p.z & r.z, p.w & r.w);
    }
    if (pmin && c == 0) {
        pmin[node] = pmin[s] < pmin[d] ? pmin[s] : pmin[d];
        pmax[node] = pmax[s] > pmax[d] ? pmax[s] : pmax[d];
    }
}

__global__ __launch_bounds__(kBlock) void invert_perm_kernel(const uint32_t *__restrict__ perm, uint64_t n,
                                                             uint32_t *__restrict__ iperm) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock)
        iperm[perm[i]] = (uint32_t)i;
}

template <class T>
struct DevBuf {
    T *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n) { return hipMalloc((void **)&p, std::max<size_t>(n, 1) * sizeof(T)); }
};

}  // namespace

void tree_release(qd_tree_s *t) {
    if (!t) return;
    void *ptrs[] = {t->d_sorted, t->d_perm,  t->d_or,     t->d_and,   t->d_child, t->d_begin, t->d_count,
                    t->d_pop,    t->d_parent, t->d_depth, t->d_iperm, t->d_blk,   t->d_pmin,  t->d_pmax,
                    t->d_bpop,   t->d_split_roots};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete t;
}

int tree_build_impl(const uint64_t *d_db, uint64_t n, const qd_build_params *params, void *stream, qd_tree_t *out) {
    if (!out) return fail(QD_ERR_INVALID, "null output handle");
    *out = nullptr;
    if (!d_db) return fail(QD_ERR_INVALID, "null database");
    if (n < 1 || n > QD_MAX_ROWS) return fail(QD_ERR_INVALID, "n=%llu outside 1..%llu", (u64)n, (u64)QD_MAX_ROWS);
    if (!aligned16(d_db)) return fail(QD_ERR_INVALID, "database must be 16-byte aligned");
    const uint32_t max_leaf = params && params->max_leaf ? params->max_leaf : 32;
    const bool want_and = params && params->store_and_image;
    const bool want_pop = !(params && params->plain_bound);
    if (max_leaf > kSmall) return fail(QD_ERR_INVALID, "max_leaf %u above %u", max_leaf, kSmall);
    if (abort_requested()) return fail(QD_ERR_ABORTED, "tree build aborted");
    hipStream_t s = (hipStream_t)stream;
    const uint4 *db4 = reinterpret_cast<const uint4 *>(d_db);

    DevBuf<uint32_t> perm_a, perm_b, gcnt, ghist, dcount, doff, nd_dev, ids_dev;
    DevBuf<uint16_t> fr_pos;
    DevBuf<uint64_t> nbegin_dev;
    DevBuf<uint32_t> ncount_dev;
    DevBuf<u64> cuts;
    DevBuf<Item> items_dev;
    QD_HIP_CHECK(perm_a.alloc(n));
    QD_HIP_CHECK(perm_b.alloc(n));
    QD_HIP_CHECK(fr_pos.alloc(n));

    // identity permutation
    {
        std::vector<uint32_t> id(n);
        for (uint64_t i = 0; i < n; i++) id[i] = (uint32_t)i;
        QD_HIP_CHECK(hipMemcpyAsync(perm_a.p, id.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        QD_HIP_CHECK(hipStreamSynchronize(s));
    }

    std::vector<uint64_t> begin{0};
    std::vector<uint32_t> count{(uint32_t)n};
    std::vector<int32_t> child{-1, -1};
    std::vector<uint32_t> level_first{0};
    uint32_t *pin = perm_a.p, *pout = perm_b.p;
    uint64_t lv0 = 0, lv1 = 1;
    while (lv0 < lv1) {
        if (abort_requested()) {  // between levels: nothing of this level is queued yet
            (void)hipStreamSynchronize(s);
            return fail(QD_ERR_ABORTED, "tree build aborted");
        }
        std::vector<uint32_t> small, big;
        for (uint64_t i = lv0; i < lv1; i++) {
            if (count[i] <= max_leaf) continue;
            (count[i] <= kSmall ? small : big).push_back((uint32_t)i);
        }
        if (small.empty() && big.empty()) break;
        QD_HIP_CHECK(hipMemcpyAsync(pout, pin, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        const size_t nsplit = small.size() + big.size();
        std::vector<uint64_t> hb(nsplit);
        std::vector<uint32_t> hc(nsplit);
        for (size_t i = 0; i < small.size(); i++) {
            hb[i] = begin[small[i]];
            hc[i] = count[small[i]];
        }
        for (size_t i = 0; i < big.size(); i++) {
            hb[small.size() + i] = begin[big[i]];
            hc[small.size() + i] = count[big[i]];
        }
        DevBuf<uint64_t> db_begin;
        DevBuf<uint32_t> db_count, db_nd;
        QD_HIP_CHECK(db_begin.alloc(nsplit));
        QD_HIP_CHECK(db_count.alloc(nsplit));
        QD_HIP_CHECK(db_nd.alloc(nsplit));
        QD_HIP_CHECK(hipMemcpyAsync(db_begin.p, hb.data(), nsplit * 8, hipMemcpyHostToDevice, s));
        QD_HIP_CHECK(hipMemcpyAsync(db_count.p, hc.data(), nsplit * 4, hipMemcpyHostToDevice, s));
        if (!small.empty()) {
            hipLaunchKernelGGL(split_small_kernel, dim3((uint32_t)small.size()), dim3(kBlock), 0, s, db4, pin, pout,
                               db_begin.p, db_count.p, db_nd.p);
            QD_HIP_CHECK(hipGetLastError());
        }
        if (!big.empty()) {
            const size_t nbig = big.size();
            std::vector<Item> items;
            std::vector<uint32_t> item_node;
            for (size_t i = 0; i < nbig; i++) {
                const uint32_t m = count[big[i]];
                for (uint32_t f = 0; f < m; f += kChunk) items.push_back({(uint32_t)i, f, std::min(kChunk, m - f), 0});
            }
            const size_t ni = items.size();
            DevBuf<Item> it_dev;
            DevBuf<uint32_t> gc, gh, dc, dof, bnd;
            DevBuf<u64> cu;
            QD_HIP_CHECK(it_dev.alloc(ni));
            QD_HIP_CHECK(gc.alloc(nbig * 4096));
            QD_HIP_CHECK(gh.alloc(nbig * 4096));
            QD_HIP_CHECK(dc.alloc(ni));
            QD_HIP_CHECK(dof.alloc(ni));
            QD_HIP_CHECK(cu.alloc(nbig));
            QD_HIP_CHECK(hipMemcpyAsync(it_dev.p, items.data(), ni * sizeof(Item), hipMemcpyHostToDevice, s));
            QD_HIP_CHECK(hipMemsetAsync(gc.p, 0, nbig * 4096 * 4, s));
            QD_HIP_CHECK(hipMemsetAsync(gh.p, 0, nbig * 4096 * 4, s));
            const uint64_t *bbeg = db_begin.p + small.size();
            const uint32_t *bcnt = db_count.p + small.size();
            uint32_t *bnd_out = db_nd.p + small.size();
            hipLaunchKernelGGL(big_count_kernel, dim3((uint32_t)ni), dim3(kBlock), 0, s, db4, pin, bbeg, it_dev.p, gc.p);
            hipLaunchKernelGGL(big_first_kernel, dim3((uint32_t)ni), dim3(kBlock), 0, s, db4, pin, bbeg, it_dev.p, gc.p,
                               fr_pos.p, gh.p);
            hipLaunchKernelGGL(big_cut_kernel, dim3((uint32_t)nbig), dim3(kBlock), 0, s, gc.p, gh.p, bcnt, cu.p,
                               bnd_out);
            hipLaunchKernelGGL(big_dcount_kernel, dim3((uint32_t)ni), dim3(kBlock), 0, s, bbeg, it_dev.p, gc.p, cu.p,
                               fr_pos.p, dc.p);
            QD_HIP_CHECK(hipGetLastError());
            std::vector<uint32_t> hdc(ni), hdoff(ni);
            QD_HIP_CHECK(hipMemcpyAsync(hdc.data(), dc.p, ni * 4, hipMemcpyDeviceToHost, s));
            QD_HIP_CHECK(hipStreamSynchronize(s));
            uint32_t run = 0;
            for (size_t i = 0; i < ni; i++) {
                if (i == 0 || items[i].slot != items[i - 1].slot) run = 0;
                hdoff[i] = run;
                run += hdc[i];
            }
            QD_HIP_CHECK(hipMemcpyAsync(dof.p, hdoff.data(), ni * 4, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(big_scatter_kernel, dim3((uint32_t)ni), dim3(kBlock), 0, s, pin, pout, bbeg, bcnt,
                               it_dev.p, gc.p, cu.p, bnd_out, fr_pos.p, dof.p);
            QD_HIP_CHECK(hipGetLastError());
            QD_HIP_CHECK(hipStreamSynchronize(s));
        }
        std::vector<uint32_t> hnd(nsplit);
        QD_HIP_CHECK(hipMemcpyAsync(hnd.data(), db_nd.p, nsplit * 4, hipMemcpyDeviceToHost, s));
        QD_HIP_CHECK(hipStreamSynchronize(s));
        // children in breadth-first order: parents in id order, similar first
        std::vector<std::pair<uint32_t, uint32_t>> split_nd;  // (node, nd)
        split_nd.reserve(nsplit);
        for (size_t i = 0; i < small.size(); i++) split_nd.push_back({small[i], hnd[i]});
        for (size_t i = 0; i < big.size(); i++) split_nd.push_back({big[i], hnd[small.size() + i]});
        std::sort(split_nd.begin(), split_nd.end());
        const uint64_t next0 = begin.size();
        for (auto &pn : split_nd) {
            const uint32_t node = pn.first, nd = pn.second, m = count[node];
            if (nd == 0 || nd >= m) continue;  // no split possible: the node stays a leaf
            const int32_t sid = (int32_t)begin.size();
            begin.push_back(begin[node]);
            count.push_back(m - nd);
            begin.push_back(begin[node] + (m - nd));
            count.push_back(nd);
            child[2 * node] = sid;
            child[2 * node + 1] = sid + 1;
            child.push_back(-1);
            child.push_back(-1);
            child.push_back(-1);
            child.push_back(-1);
        }
        std::swap(pin, pout);
        lv0 = next0;
        lv1 = begin.size();
        if (lv1 > lv0) level_first.push_back((uint32_t)lv0);
    }
    level_first.push_back((uint32_t)begin.size());

    // The final permutation is in `pin`.
    const uint64_t nn = begin.size();
    qd_tree_s *t = new qd_tree_s();
    t->n = n;
    t->n_nodes = nn;
    t->max_leaf = max_leaf;
    t->has_and = want_and;
    if (hipMalloc((void **)&t->d_sorted, n * 512) != hipSuccess || hipMalloc((void **)&t->d_perm, n * 4) != hipSuccess) {
        tree_release(t);
        return fail(QD_ERR_OOM, "tree allocation failed");
    }
    if (hipMemcpyAsync(t->d_perm, pin, n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        tree_release(t);
        return fail(QD_ERR_DEVICE, "tree upload failed");
    }
    {
        uint64_t blocks = std::min<uint64_t>((n * 32 + kBlock - 1) / kBlock, (uint64_t)device_cus() * 64);
        hipLaunchKernelGGL(gather_rows_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, s, db4, t->d_perm, n,
                           reinterpret_cast<uint4 *>(t->d_sorted));
    }
    std::vector<uint32_t> hb32(nn);
    for (uint64_t i = 0; i < nn; i++) hb32[i] = (uint32_t)begin[i];
    const int rc = tree_finish(t, child, hb32, count, want_pop, s);
    if (rc != QD_OK) return rc;  // tree_finish released t
    *out = t;
    return QD_OK;
}

int tree_finish(qd_tree_s *t, const std::vector<int32_t> &child, const std::vector<uint32_t> &begin,
                const std::vector<uint32_t> &count, bool want_pop, hipStream_t s) {
    const uint64_t n = t->n, nn = t->n_nodes;
    const bool want_and = t->has_and;
    auto cleanup = [&](int code) {
        tree_release(t);
        return code;
    };
    if (hipMalloc((void **)&t->d_or, nn * 512) != hipSuccess || hipMalloc((void **)&t->d_child, nn * 8) != hipSuccess ||
        hipMalloc((void **)&t->d_begin, nn * 4) != hipSuccess || hipMalloc((void **)&t->d_count, nn * 4) != hipSuccess ||
        hipMalloc((void **)&t->d_pop, n * 2) != hipSuccess || hipMalloc((void **)&t->d_parent, nn * 4) != hipSuccess ||
        hipMalloc((void **)&t->d_depth, nn) != hipSuccess || hipMalloc((void **)&t->d_iperm, n * 4) != hipSuccess ||
        (want_and && hipMalloc((void **)&t->d_and, nn * 512) != hipSuccess) ||
        (want_pop && (hipMalloc((void **)&t->d_pmin, nn * 2) != hipSuccess ||
                      hipMalloc((void **)&t->d_pmax, nn * 2) != hipSuccess)))
        return cleanup(fail(QD_ERR_OOM, "tree allocation failed"));
    std::vector<uint32_t> leaf_ids;
    for (uint64_t i = 0; i < nn; i++)
        if (child[2 * i] < 0) leaf_ids.push_back((uint32_t)i);
    const uint32_t n_leaves = (uint32_t)leaf_ids.size();
    t->n_leaves = n_leaves;
    // breadth-first numbering: a level's nodes are consecutive, children after parents
    std::vector<int32_t> parent(nn, -1);
    std::vector<uint32_t> level(nn, 0);
    std::vector<uint8_t> depth(nn, 0);
    for (uint64_t i = 0; i < nn; i++)
        if (child[2 * i] >= 0) {
            parent[child[2 * i]] = parent[child[2 * i + 1]] = (int32_t)i;
            level[child[2 * i]] = level[child[2 * i + 1]] = level[i] + 1;
        }
    std::vector<uint32_t> level_first{0};
    for (uint64_t i = 1; i < nn; i++)
        if (level[i] != level[i - 1]) level_first.push_back((uint32_t)i);
    level_first.push_back((uint32_t)nn);
    t->depth = (uint32_t)level_first.size() - 1;
    t->level_max.assign(t->depth, 0);
    for (uint64_t i = 0; i < nn; i++) {
        depth[i] = (uint8_t)std::min<uint32_t>(255, level[i]);
        t->level_max[level[i]] = std::max(t->level_max[level[i]], count[i]);
    }
    // The per-query search split into n subtree searches: position p (its
    // log2(n) bits from the most significant, 0 = the similar child) is the
    // node reached from the root along p's bits; a leaf met on the way is the
    // subtree of the first position below it, the other positions below it
    // are empty.  With the nodes under each node (children come after their
    // parents), the most nodes of any subtree bounds one search's queue.
    std::vector<int32_t> split_roots(31, -1);
    {
        std::vector<uint32_t> under(nn, 1);
        for (uint64_t i = nn; i-- > 0;)
            if (child[2 * i] >= 0) under[i] = 1 + under[child[2 * i]] + under[child[2 * i + 1]];
        for (uint32_t e = 0; e < 5; e++) {
            const uint32_t ns = 1u << e;
            uint64_t most = 0;
            for (uint32_t p = 0; p < ns; p++) {
                int32_t c = 0;
                for (uint32_t l = 0; l < e; l++) {
                    const int32_t a = child[2 * (uint64_t)c], b = child[2 * (uint64_t)c + 1];
                    if (a < 0) {
                        if ((p & ((1u << (e - l)) - 1u)) != 0) c = -1;
                        break;
                    }
                    c = (p >> (e - 1 - l)) & 1u ? b : a;
                }
                split_roots[ns - 1 + p] = c;
                if (c >= 0) most = std::max<uint64_t>(most, under[c]);
            }
            t->split_nodes[e] = most;
        }
    }
    if (hipMalloc((void **)&t->d_split_roots, 31 * 4) != hipSuccess)
        return cleanup(fail(QD_ERR_OOM, "tree allocation failed"));
    if (hipMemcpyAsync(t->d_split_roots, split_roots.data(), 31 * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_parent, parent.data(), nn * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_depth, depth.data(), nn, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_child, child.data(), nn * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_begin, begin.data(), nn * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(t->d_count, count.data(), nn * 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return cleanup(fail(QD_ERR_DEVICE, "tree upload failed"));
    DevBuf<uint32_t> lid;
    if (lid.alloc(std::max<uint64_t>(n_leaves, nn)) != hipSuccess) return cleanup(fail(QD_ERR_OOM, "alloc"));
    if (hipMemcpyAsync(lid.p, leaf_ids.data(), n_leaves * 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return cleanup(fail(QD_ERR_DEVICE, "upload"));
    {
        const int rc = qd_popcount_rows(t->d_sorted, n, t->d_pop, s);  // leaf-order rows
        if (rc != QD_OK) return cleanup(rc);
    }
    hipLaunchKernelGGL(leaf_images_kernel, dim3((n_leaves + 3) / 4), dim3(kBlock), 0, s,
                       reinterpret_cast<const uint4 *>(t->d_sorted), lid.p, n_leaves, t->d_begin, t->d_count,
                       reinterpret_cast<uint4 *>(t->d_or), reinterpret_cast<uint4 *>(t->d_and), t->d_pop, t->d_pmin,
                       t->d_pmax);
    if (hipStreamSynchronize(s) != hipSuccess) return cleanup(fail(QD_ERR_DEVICE, "leaf images"));
    // inner nodes, deepest level first
    for (int L = (int)level_first.size() - 2; L >= 0; L--) {
        std::vector<uint32_t> inner;
        for (uint32_t i = level_first[L]; i < level_first[L + 1]; i++)
            if (child[2 * i] >= 0) inner.push_back(i);
        if (inner.empty()) continue;
        if (hipMemcpyAsync(lid.p, inner.data(), inner.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
            return cleanup(fail(QD_ERR_DEVICE, "upload"));
        const uint64_t work = (uint64_t)inner.size() * 32;
        hipLaunchKernelGGL(inner_images_kernel, dim3((uint32_t)((work + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           lid.p, (uint32_t)inner.size(), t->d_child, reinterpret_cast<uint4 *>(t->d_or),
                           reinterpret_cast<uint4 *>(t->d_and), t->d_pmin, t->d_pmax);
        if (hipStreamSynchronize(s) != hipSuccess) return cleanup(fail(QD_ERR_DEVICE, "inner images"));
    }
    hipLaunchKernelGGL(invert_perm_kernel, dim3((uint32_t)std::min<uint64_t>((n + kBlock - 1) / kBlock, 65535)),
                       dim3(kBlock), 0, s, t->d_perm, n, t->d_iperm);
    int rc = tree_block_images(t, s);
    if (rc != QD_OK) return cleanup(rc);
    if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
        return cleanup(fail(QD_ERR_DEVICE, "tree build kernels failed"));
    (void)hipGetDevice(&t->device);
    return QD_OK;
}

}  // namespace qd

extern "C" int qd_tree_build(const uint64_t *d_db, uint64_t n, const qd_build_params *p, void *stream,
                             qd_tree_t *out) {
    return qd::tree_build_impl(d_db, n, p, stream, out);
}

extern "C" int qd_tree_free(qd_tree_t t) {
    qd::tree_release(t);
    return QD_OK;
}

extern "C" int qd_tree_info(qd_tree_t t, qd_tree_info_t *info) {
    if (!t || !info) return qd::fail(QD_ERR_INVALID, "null argument");
    info->n = t->n;
    info->n_nodes = t->n_nodes;
    info->n_leaves = t->n_leaves;
    info->depth = t->depth;
    info->max_leaf = t->max_leaf;
    info->has_and_image = t->has_and ? 1 : 0;
    info->has_pop_range = t->d_pmin ? 1 : 0;
    return QD_OK;
}

extern "C" int qd_tree_export(qd_tree_t t, int32_t *h_child, uint32_t *h_begin, uint32_t *h_count, uint64_t *h_or,
                              uint64_t *h_and, uint32_t *h_perm) {
    if (!t) return qd::fail(QD_ERR_INVALID, "null tree");
    if (h_and && !t->has_and) return qd::fail(QD_ERR_INVALID, "tree stores no product images");
    (void)hipSetDevice(t->device);
    struct {
        void *dst;
        const void *src;
        size_t bytes;
    } cp[] = {{h_child, t->d_child, t->n_nodes * 8}, {h_begin, t->d_begin, t->n_nodes * 4},
              {h_count, t->d_count, t->n_nodes * 4}, {h_or, t->d_or, t->n_nodes * 512},
              {h_and, t->d_and, t->n_nodes * 512},   {h_perm, t->d_perm, t->n * 4}};
    for (auto &c : cp)
        if (c.dst) QD_HIP_CHECK(hipMemcpy(c.dst, c.src, c.bytes, hipMemcpyDeviceToHost));
    return QD_OK;
}

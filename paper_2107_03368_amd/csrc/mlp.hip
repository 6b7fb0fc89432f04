// Learned frontier order: a small MLP that scores (query, tree node) pairs,
// with hand-written BF16 kernels (FP32 accumulation) for inference and
// training.  The score only decides which child the depth-first search visits
// first; pruning uses the exact bounds, so results never depend on it.
//
// Network: x = [query bits (4096, 0/1); node features f (32)]
//   h1 = ReLU(x W1 + b1)      W1 = [W1q (4096 x 256); W1f (32 x 256)]
//   h2 = ReLU(h1 W2 + b2)     W2: 256 x 256
//   s  = h2 . w3 + b3
// All weight matrices are stored [input][output].  Because the query part of
// x is binary and shared by every node scored for that query, u_q = b1 +
// sum over the query's set bits of the W1q rows is formed once per query (a
// gather-add); a pair then costs u_q + f W1f (32 x 256), the 256 x 256 layer
// as a BF16 MFMA GEMM over a batch of pairs, and the 256-wide head.  The
// layer-1 activations enter that GEMM as two BF16 terms (hi + lo, with lo the
// rounding residual), i.e. one GEMM of depth 512 against W2 stacked twice, so
// only the weights are rounded to BF16.
// Training (binary cross-entropy on the logit, mean over pairs) runs the same
// kernels backwards; every reduction has a fixed order, so gradients are
// reproducible bit for bit.  Parameters are FP32 masters with Adam moments;
// each update refreshes their BF16 copies.
#include <math.h>

#include <algorithm>
#include <vector>

#include "qd_device.h"
#include "qd_internal.h"
#include "qd_tree.h"

struct qd_model_s {
    int device = 0;
    float *p = nullptr;      // QD_MLP_NPARAMS fp32 master parameters
    float *m = nullptr;      // Adam first moments
    float *v = nullptr;      // Adam second moments
    uint16_t *w = nullptr;   // bf16 copy of p (same layout)
    uint16_t *w2x2 = nullptr;  // bf16 W2 stacked twice (512 x 256): the layer-2 operand for hi/lo activations
    uint64_t step = 0;
};

namespace qd {
namespace {

constexpr int kBlock = 256;
constexpr int H = QD_MLP_HIDDEN;
constexpr int NF = QD_MLP_FEATURES;
constexpr size_t OFF_W1Q = 0;
constexpr size_t OFF_W1F = OFF_W1Q + (size_t)QD_BITS * H;
constexpr size_t OFF_B1 = OFF_W1F + (size_t)NF * H;
constexpr size_t OFF_W2 = OFF_B1 + H;
constexpr size_t OFF_B2 = OFF_W2 + (size_t)H * H;
constexpr size_t OFF_W3 = OFF_B2 + H;
constexpr size_t OFF_B3 = OFF_W3 + H;
static_assert(OFF_B3 + 1 == QD_MLP_NPARAMS, "parameter layout");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
// float -> bf16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ---------------------------------------------------------------------------
// BF16 GEMM on MFMA: C[M][N] = sum_k A(m,k) B(k,n), fp32 accumulate.
//   A(m,k) = TA ? A[k*lda + m] : A[m*lda + k];  B(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n]
// M, N multiples of 64, K a multiple of 32.  A block of 4 waves owns a 64x64
// tile, each wave a 32x32 quarter as 2x2 tiles of v_mfma_f32_16x16x32_bf16:
// lane l supplies A rows (l % 16) at k = 8*(l/16) .. +7 and B columns (l % 16)
// at the same k; it receives C rows 4*(l/16) .. +3 of column (l % 16).
// ---------------------------------------------------------------------------
template <bool TA, bool TB>
__global__ __launch_bounds__(kBlock) void gemm_bf16_kernel(const uint16_t *__restrict__ A,
                                                           const uint16_t *__restrict__ B, float *__restrict__ C,
                                                           int K, int lda, int ldb, int ldc, int accumulate) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 64 + (w >> 1) * 32, n0 = blockIdx.x * 64 + (w & 1) * 32;
    const int li = lane & 15, lk = (lane >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int t = 0; t < 2; t++) {
            const int m = m0 + 16 * t + li;
            uint16_t e[8];
            if (!TA) {
                const uint4 v = *reinterpret_cast<const uint4 *>(A + (size_t)m * lda + k0 + lk);
                __builtin_memcpy(e, &v, 16);
            } else {
#pragma unroll
                for (int i = 0; i < 8; i++) e[i] = A[(size_t)(k0 + lk + i) * lda + m];
            }
            __builtin_memcpy(&af[t], e, 16);
            const int n = n0 + 16 * t + li;
            if (TB) {
                const uint4 v = *reinterpret_cast<const uint4 *>(B + (size_t)n * ldb + k0 + lk);
                __builtin_memcpy(e, &v, 16);
            } else {
#pragma unroll
                for (int i = 0; i < 8; i++) e[i] = B[(size_t)(k0 + lk + i) * ldb + n];
            }
            __builtin_memcpy(&bfr[t], e, 16);
        }
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int r = 0; r < 4; r++)
            {
                float *c = C + (size_t)(m0 + 16 * a + 4 * (lane >> 4) + r) * ldc + n0 + 16 * b + li;
                *c = accumulate ? *c + acc[a][b][r] : acc[a][b][r];
            }
}

// ---------------------------------------------------------------------------
// Node features for (query, node) pairs.  Pair p is (pair_q[p], pair_node[p]),
// or, with null pair arrays, (q0 + p / n_nodes_per_q, p % n_nodes_per_q).
// Features (|q| read as max(|q|,1); a_lb = popcount(q AND NOT OR),
// ov = popcount(q AND OR); bands = image rows 0-5, 6-11, ..., 54-59, 60-63):
//   0 a_lb/|q|  1 ov/|q|  2 popcount(OR)/4096  3 sibling's a_lb/|q| (0 at the
//   root)  4 depth/32  5 log2(rows under the node)/24  6 is leaf
//   7 is the similar child  8 |q|/512  9 popcount(OR AND NOT q)/4096
//   10..20 band a_lb/|q|  21..31 band ov/|q|
// Two pairs per wave, one per 32-lane half; lane c of a half holds the
// 16-byte chunk c (image rows 2c, 2c+1).
// ---------------------------------------------------------------------------
struct PairIdx {
    const uint32_t *pq, *pn;
    uint32_t q0, per_q;
    __device__ __forceinline__ uint32_t q(uint64_t p) const { return pq ? pq[p] : q0 + (uint32_t)(p / per_q); }
    __device__ __forceinline__ uint32_t node(uint64_t p) const { return pn ? pn[p] : (uint32_t)(p % per_q); }
};

__global__ __launch_bounds__(kBlock) void features_kernel(const uint4 *__restrict__ q, const uint4 *__restrict__ orimg,
                                                          const int32_t *__restrict__ child,
                                                          const int32_t *__restrict__ parent,
                                                          const uint8_t *__restrict__ depth,
                                                          const uint32_t *__restrict__ count, PairIdx P,
                                                          uint64_t n_pairs, float *__restrict__ feat) {
    __shared__ uint32_t band_a[kBlock / 32][32], band_o[kBlock / 32][32];
    const int half = threadIdx.x >> 5, c = threadIdx.x & 31;
    const uint64_t p = (uint64_t)blockIdx.x * (kBlock / 32) + half;
    const bool live = p < n_pairs;
    const uint64_t pp = live ? p : 0;
    const uint32_t qi = P.q(pp), node = P.node(pp);
    const int32_t par = parent[node];
    const int32_t sib = par < 0 ? -1 : (child[2 * par] == (int32_t)node ? child[2 * par + 1] : child[2 * par]);
    const uint4 qv = q[(uint64_t)qi * 32 + c];
    const uint4 ov = orimg[(uint64_t)node * 32 + c];
    const uint4 sv = sib >= 0 ? orimg[(uint64_t)sib * 32 + c] : make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
    // rows 2c (x, y) and 2c+1 (z, w)
    const uint32_t a0 = __popc(qv.x & ~ov.x) + __popc(qv.y & ~ov.y), a1 = __popc(qv.z & ~ov.z) + __popc(qv.w & ~ov.w);
    const uint32_t o0 = __popc(qv.x & ov.x) + __popc(qv.y & ov.y), o1 = __popc(qv.z & ov.z) + __popc(qv.w & ov.w);
    band_a[half][c] = a0 + a1;
    band_o[half][c] = o0 + o1;
    const uint32_t pq = sum32_half(popc4(qv));
    const uint32_t a_lb = sum32_half(a0 + a1);
    const uint32_t ovl = sum32_half(o0 + o1);
    const uint32_t orp = sum32_half(popc4(ov));
    const uint32_t extra = sum32_half(__popc(ov.x & ~qv.x) + __popc(ov.y & ~qv.y) + __popc(ov.z & ~qv.z) +
                                      __popc(ov.w & ~qv.w));
    const uint32_t sib_a = sum32_half(__popc(qv.x & ~sv.x) + __popc(qv.y & ~sv.y) + __popc(qv.z & ~sv.z) +
                                      __popc(qv.w & ~sv.w));
    __syncthreads();
    if (!live) return;
    const float inv = 1.0f / (float)(pq > 1 ? pq : 1);
    float *f = feat + p * NF;
    if (c == 0) {
        f[0] = (float)a_lb * inv;
        f[1] = (float)ovl * inv;
        f[2] = (float)orp * (1.0f / 4096.0f);
        f[3] = sib >= 0 ? (float)sib_a * inv : 0.0f;
        f[4] = (float)depth[node] * (1.0f / 32.0f);
        f[5] = log2f((float)count[node]) * (1.0f / 24.0f);
        f[6] = child[2 * node] < 0 ? 1.0f : 0.0f;
        f[7] = (par >= 0 && child[2 * par] == (int32_t)node) ? 1.0f : 0.0f;
        f[8] = (float)pq * (1.0f / 512.0f);
        f[9] = (float)extra * (1.0f / 4096.0f);
    }
    if (c < 11) {
        // band c covers chunks 3c .. 3c+2 (the last band chunks 30, 31)
        const int c0 = 3 * c, c1 = c == 10 ? 32 : 3 * c + 3;
        uint32_t sa = 0, so = 0;
        for (int i = c0; i < c1; i++) {
            sa += band_a[half][i];
            so += band_o[half][i];
        }
        f[10 + c] = (float)sa * inv;
        f[21 + c] = (float)so * inv;
    }
}

// u[qi][j] = b1[j] + sum over set bits b of query q0+qi of W1q[b][j] (bf16
// weights; bits summed in ascending order).  One block per query.
__global__ __launch_bounds__(kBlock) void uq_kernel(const uint64_t *__restrict__ q, uint32_t q0,
                                                    const uint16_t *__restrict__ w, float *__restrict__ u) {
    __shared__ uint16_t bits[QD_BITS];
    __shared__ uint32_t offs[65];
    const uint64_t *qq = q + (uint64_t)(q0 + blockIdx.x) * QD_WORDS;
    const int t = threadIdx.x;
    if (t < 64) offs[t + 1] = __popcll(qq[t]);
    if (t == 0) offs[0] = 0;
    __syncthreads();
    if (t == 0)
        for (int i = 1; i <= 64; i++) offs[i] += offs[i - 1];
    __syncthreads();
    if (t < 64) {
        uint64_t x = qq[t];
        uint32_t o = offs[t];
        while (x) {
            bits[o++] = (uint16_t)(64 * t + __builtin_ctzll(x));
            x &= x - 1;
        }
    }
    __syncthreads();
    float acc = bf2f(w[OFF_B1 + t]);
    const uint32_t nb = offs[64];
    for (uint32_t i = 0; i < nb; i++) acc += bf2f(w[OFF_W1Q + (size_t)bits[i] * H + t]);
    u[(size_t)blockIdx.x * H + t] = acc;
}

// h = ReLU(u[q(p) - q0][j] + sum_f feat[p][f] W1f[f][j]) stored as two bf16
// terms: h1[p][j] = bf16(h), h1[p][256 + j] = bf16(h - bf16(h)).  Rows
// p >= n_pairs (padding up to the GEMM tile) are zero.
__global__ __launch_bounds__(kBlock) void layer1_kernel(const float *__restrict__ u, PairIdx P, uint32_t q0,
                                                        const float *__restrict__ feat, uint64_t n_pairs,
                                                        const uint16_t *__restrict__ w, uint16_t *__restrict__ h1) {
    const uint64_t p = blockIdx.x;
    const int j = threadIdx.x;
    if (p >= n_pairs) {
        h1[p * 2 * H + j] = 0;
        h1[p * 2 * H + H + j] = 0;
        return;
    }
    const float *f = feat + p * NF;
    float z = u[(size_t)(P.q(p) - q0) * H + j];
#pragma unroll 8
    for (int i = 0; i < NF; i++) z += f[i] * bf2f(w[OFF_W1F + (size_t)i * H + j]);
    const float h = z > 0.f ? z : 0.f;
    const uint16_t hi = f2bf(h);
    h1[p * 2 * H + j] = hi;
    h1[p * 2 * H + H + j] = f2bf(h - bf2f(hi));
}

// s[p] = b3 + sum_j w3[j] ReLU(z2[p][j] + b2[j]); one wave per pair.  With
// labels: h2 (fp32) is kept, ds[p] = (sigmoid(s) - y) / n_pairs, loss[p] =
// softplus(s) - y s, and d2[p][j] = bf16(ds * w3[j] * [z2 + b2 > 0]).
__global__ __launch_bounds__(kBlock) void head_kernel(const float *__restrict__ z2, uint64_t n_pairs,
                                                      const uint16_t *__restrict__ w, const float *__restrict__ y,
                                                      float *__restrict__ s_out, float *__restrict__ h2_out,
                                                      float *__restrict__ ds_out, float *__restrict__ loss_out,
                                                      uint16_t *__restrict__ d2, uint64_t n_padded) {
    const uint64_t p = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= n_padded) return;
    if (p >= n_pairs) {
        if (d2)
            for (int i = 0; i < 4; i++) d2[p * H + lane + 64 * i] = 0;
        return;
    }
    float h[4], acc = 0.f;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int j = lane + 64 * i;
        const float zz = z2[p * H + j] + bf2f(w[OFF_B2 + j]);
        h[i] = zz > 0.f ? zz : 0.f;
        acc += h[i] * bf2f(w[OFF_W3 + j]);
    }
    // wave sum in a fixed order
    acc = wave_sum_f(acc);
    const float s = acc + bf2f(w[OFF_B3]);
    if (lane == 0 && s_out) s_out[p] = s;
    if (y) {
        const float yy = y[p];
        const float sig = 1.f / (1.f + expf(-s));
        const float ds = (sig - yy) / (float)n_pairs;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int j = lane + 64 * i;
            h2_out[p * H + j] = h[i];
            d2[p * H + j] = f2bf(h[i] > 0.f ? ds * bf2f(w[OFF_W3 + j]) : 0.f);
        }
        if (lane == 0) {
            ds_out[p] = ds;
            loss_out[p] = (s > 0.f ? s + log1pf(expf(-s)) : log1pf(expf(s))) - yy * s;
        }
    }
}

// Column reductions for the head and layer-2 biases, in two deterministic
// stages (fixed chunks of pairs, then a fixed-order sum over the chunks):
//   g[W3+j] = sum_p ds[p] h2[p][j]   g[B2+j] = w3[j] sum_p ds[p] [h2[p][j] > 0]
//   g[B3] = sum_p ds[p]              loss = mean_p loss[p]
constexpr uint32_t kHeadParts = 128;
constexpr uint32_t kHeadPartLen = 2 * H + 2;  // a[H], b[H], sum ds, sum loss

__global__ __launch_bounds__(kBlock) void head_partial_kernel(const float *__restrict__ h2,
                                                              const float *__restrict__ ds,
                                                              const float *__restrict__ lossv, uint64_t n_pairs,
                                                              float *__restrict__ part) {
    const uint32_t g = blockIdx.x;
    const uint64_t chunk = (n_pairs + kHeadParts - 1) / kHeadParts;
    const uint64_t p0 = g * chunk, p1 = p0 + chunk < n_pairs ? p0 + chunk : n_pairs;
    const int j = threadIdx.x;
    float a = 0.f, b = 0.f;
    for (uint64_t p = p0; p < p1; p++) {
        const float h = h2[p * H + j];
        a += ds[p] * h;
        b += h > 0.f ? ds[p] : 0.f;
    }
    float *o = part + (size_t)g * kHeadPartLen;
    o[j] = a;
    o[H + j] = b;
    if (j == 0) {
        float sd = 0.f, sl = 0.f;
        for (uint64_t p = p0; p < p1; p++) {
            sd += ds[p];
            sl += lossv[p];
        }
        o[2 * H] = sd;
        o[2 * H + 1] = sl;
    }
}

__global__ __launch_bounds__(kBlock) void head_final_kernel(const float *__restrict__ part, uint64_t n_pairs,
                                                            const uint16_t *__restrict__ w, float *__restrict__ g,
                                                            float *__restrict__ loss) {
    const int j = threadIdx.x;
    float a = 0.f, b = 0.f;
    for (uint32_t k = 0; k < kHeadParts; k++) {
        a += part[(size_t)k * kHeadPartLen + j];
        b += part[(size_t)k * kHeadPartLen + H + j];
    }
    g[OFF_W3 + j] = a;
    g[OFF_B2 + j] = b * bf2f(w[OFF_W3 + j]);
    if (j == 0) {
        float sd = 0.f, sl = 0.f;
        for (uint32_t k = 0; k < kHeadParts; k++) {
            sd += part[(size_t)k * kHeadPartLen + 2 * H];
            sl += part[(size_t)k * kHeadPartLen + 2 * H + 1];
        }
        g[OFF_B3] = sd;
        if (loss) *loss = sl / (float)n_pairs;
    }
}

// dz1[p][j] = dh1[p][j] * [h1[p][j] > 0]; then
//   g[B1+j] = sum_p dz1   g[W1F + f*H + j] = sum_p feat[p][f] dz1[p][j]
//   du[q][j] = sum over the pairs of query q of dz1 (pairs grouped by query)
// Stage 1: block (q, c) sums chunk c of query q's pairs; stage 2 sums the
// chunks in a fixed order.
constexpr uint32_t kL1Chunks = 8;
constexpr uint32_t kL1PartLen = (NF + 1) * H;  // gf[NF][H], su[H]

__global__ __launch_bounds__(kBlock) void layer1_partial_kernel(const float *__restrict__ dh1,
                                                                const uint16_t *__restrict__ h1,
                                                                const float *__restrict__ feat,
                                                                const uint64_t *__restrict__ qoff,
                                                                uint64_t qoff_base, float *__restrict__ part) {
    const uint32_t qi = blockIdx.x / kL1Chunks, c = blockIdx.x % kL1Chunks;
    const int j = threadIdx.x;
    const uint64_t b0 = qoff[qi] - qoff_base, b1 = qoff[qi + 1] - qoff_base;
    const uint64_t chunk = (b1 - b0 + kL1Chunks - 1) / kL1Chunks;
    const uint64_t p0 = b0 + c * chunk < b1 ? b0 + c * chunk : b1;
    const uint64_t p1 = p0 + chunk < b1 ? p0 + chunk : b1;
    float su = 0.f, gf[NF];
#pragma unroll
    for (int i = 0; i < NF; i++) gf[i] = 0.f;
    for (uint64_t p = p0; p < p1; p++) {
        const float dz = bf2f(h1[p * 2 * H + j]) > 0.f ? dh1[p * H + j] : 0.f;
        su += dz;
#pragma unroll
        for (int i = 0; i < NF; i++) gf[i] += feat[p * NF + i] * dz;
    }
    float *o = part + (size_t)blockIdx.x * kL1PartLen;
#pragma unroll
    for (int i = 0; i < NF; i++) o[(size_t)i * H + j] = gf[i];
    o[(size_t)NF * H + j] = su;
}

// Block i < NF: g[W1F + i*H + j]; block NF: du and g[B1].
__global__ __launch_bounds__(kBlock) void layer1_final_kernel(const float *__restrict__ part, uint32_t nq,
                                                              float *__restrict__ g, float *__restrict__ du) {
    const uint32_t i = blockIdx.x;
    const int j = threadIdx.x;
    if (i < NF) {
        float a = 0.f;
        for (uint32_t k = 0; k < nq * kL1Chunks; k++) a += part[(size_t)k * kL1PartLen + (size_t)i * H + j];
        g[OFF_W1F + (size_t)i * H + j] = a;
    } else {
        float gb = 0.f;
        for (uint32_t qi = 0; qi < nq; qi++) {
            float su = 0.f;
            for (uint32_t c = 0; c < kL1Chunks; c++)
                su += part[(size_t)(qi * kL1Chunks + c) * kL1PartLen + (size_t)NF * H + j];
            du[(size_t)qi * H + j] = su;
            gb += su;
        }
        g[OFF_B1 + j] = gb;
    }
}

// g[W1Q + b*H + j] = sum_q bit(q, b) du[q][j]
__global__ __launch_bounds__(kBlock) void w1q_grad_kernel(const uint64_t *__restrict__ q, uint32_t nq,
                                                          const float *__restrict__ du, float *__restrict__ g) {
    const uint32_t b = blockIdx.x;
    const int j = threadIdx.x;
    float a = 0.f;
    for (uint32_t qi = 0; qi < nq; qi++)
        if ((q[(uint64_t)qi * QD_WORDS + (b >> 6)] >> (b & 63)) & 1ull) a += du[(size_t)qi * H + j];
    g[OFF_W1Q + (size_t)b * H + j] = a;
}

__global__ __launch_bounds__(kBlock) void copy_grad_w2_kernel(const float *__restrict__ dw2, float *__restrict__ g) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < (size_t)H * H) g[OFF_W2 + i] = dw2[i];
}

__global__ __launch_bounds__(kBlock) void to_bf16_kernel(const float *__restrict__ p, uint16_t *__restrict__ w,
                                                         size_t n) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        w[i] = f2bf(p[i]);
}

__global__ __launch_bounds__(kBlock) void adam_kernel(float *__restrict__ p, float *__restrict__ m,
                                                      float *__restrict__ v, uint16_t *__restrict__ w,
                                                      const float *__restrict__ g, size_t n, float lr, float b1,
                                                      float b2, float eps, float c1, float c2) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        w[i] = f2bf(pi);
    }
}

// scores of a chunk of pairs into out[p] (implicit pairs: out is nq x per_q)
__global__ __launch_bounds__(kBlock) void scatter_scores_kernel(const float *__restrict__ s, uint64_t n,
                                                                float *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = s[i];
}

inline uint64_t pad64(uint64_t x) { return (x + 63) / 64 * 64; }

void gemm(hipStream_t s, bool ta, bool tb, const uint16_t *A, const uint16_t *B, float *C, int M, int N, int K,
          int lda, int ldb, int ldc, int accumulate = 0) {
    dim3 grid(N / 64, M / 64);
    if (!ta && !tb)
        hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(kBlock), 0, s, A, B, C, K, lda, ldb, ldc, accumulate);
    if (!ta && tb)
        hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(kBlock), 0, s, A, B, C, K, lda, ldb, ldc, accumulate);
    if (ta && !tb)
        hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(kBlock), 0, s, A, B, C, K, lda, ldb, ldc, accumulate);
    if (ta && tb)
        hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(kBlock), 0, s, A, B, C, K, lda, ldb, ldc, accumulate);
}

// w2x2 = [W2; W2] in bf16
__global__ __launch_bounds__(kBlock) void stack_w2_kernel(const uint16_t *__restrict__ w, uint16_t *__restrict__ w2x2) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < (size_t)H * H) {
        w2x2[i] = w[OFF_W2 + i];
        w2x2[(size_t)H * H + i] = w[OFF_W2 + i];
    }
}

// Forward of one chunk of pairs (and, with labels, the gradients).
// Scratch layout per chunk of P (padded to 64) pairs is allocated by the caller.
struct Scratch {
    float *u = nullptr;     // nq_chunk x H
    uint16_t *h1 = nullptr; // P x 2H (hi, lo)
    float *z2 = nullptr;    // P x H   (also dh1 in the backward pass)
    float *s = nullptr;     // P
    float *h2 = nullptr;    // P x H   (training)
    float *ds = nullptr;    // P
    float *lossv = nullptr; // P
    uint16_t *d2 = nullptr; // P x H   (training)
    float *dw2 = nullptr;   // H x H
    float *du = nullptr;    // nq x H
    float *hpart = nullptr; // kHeadParts x kHeadPartLen
    float *lpart = nullptr; // nq x kL1Chunks x kL1PartLen
};

}  // namespace

// ---- entry points -------------------------------------------------------

static int check_model(qd_model_t m) { return m && m->p ? QD_OK : fail(QD_ERR_INVALID, "null model"); }

}  // namespace qd

extern "C" int qd_model_create(const float *d_params, void *stream, qd_model_t *out) {
    using namespace qd;
    if (!out || !d_params) return fail(QD_ERR_INVALID, "null pointer");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    qd_model_s *m = new qd_model_s();
    const size_t n = QD_MLP_NPARAMS;
    if (hipMalloc((void **)&m->p, n * 4) != hipSuccess || hipMalloc((void **)&m->m, n * 4) != hipSuccess ||
        hipMalloc((void **)&m->v, n * 4) != hipSuccess || hipMalloc((void **)&m->w, n * 2) != hipSuccess ||
        hipMalloc((void **)&m->w2x2, (size_t)2 * H * H * 2) != hipSuccess) {
        qd_model_free(m);
        return fail(QD_ERR_OOM, "model allocation failed");
    }
    (void)hipGetDevice(&m->device);
    QD_HIP_CHECK(hipMemcpyAsync(m->p, d_params, n * 4, hipMemcpyDeviceToDevice, s));
    QD_HIP_CHECK(hipMemsetAsync(m->m, 0, n * 4, s));
    QD_HIP_CHECK(hipMemsetAsync(m->v, 0, n * 4, s));
    hipLaunchKernelGGL(to_bf16_kernel, dim3(1024), dim3(kBlock), 0, s, m->p, m->w, n);
    hipLaunchKernelGGL(stack_w2_kernel, dim3(H * H / kBlock), dim3(kBlock), 0, s, m->w, m->w2x2);
    QD_HIP_CHECK(hipGetLastError());
    QD_HIP_CHECK(hipStreamSynchronize(s));
    *out = m;
    return QD_OK;
}

extern "C" int qd_model_free(qd_model_t m) {
    if (!m) return QD_OK;
    void *ptrs[] = {m->p, m->m, m->v, m->w, m->w2x2};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
    return QD_OK;
}

extern "C" int qd_model_params(qd_model_t m, float *d_params, void *stream) {
    using namespace qd;
    if (check_model(m) != QD_OK || !d_params) return fail(QD_ERR_INVALID, "null pointer");
    QD_HIP_CHECK(hipMemcpyAsync(d_params, m->p, QD_MLP_NPARAMS * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return QD_OK;
}

static int features_launch(qd_tree_t t, const uint64_t *d_q, qd::PairIdx P, uint64_t n_pairs, float *d_feat,
                           hipStream_t s) {
    using namespace qd;
    if (n_pairs == 0) return QD_OK;
    const uint64_t blocks = (n_pairs + (kBlock / 32) - 1) / (kBlock / 32);
    hipLaunchKernelGGL(features_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, s,
                       reinterpret_cast<const uint4 *>(d_q), reinterpret_cast<const uint4 *>(t->d_or), t->d_child,
                       t->d_parent, t->d_depth, t->d_count, P, n_pairs, d_feat);
    QD_HIP_CHECK(hipGetLastError());
    return QD_OK;
}

extern "C" int qd_model_features(qd_tree_t t, const uint64_t *d_q, const uint32_t *d_pair_q,
                                 const uint32_t *d_pair_node, uint64_t n_pairs, float *d_feat, void *stream) {
    using namespace qd;
    if (!t) return fail(QD_ERR_INVALID, "null tree");
    if (n_pairs && (!d_q || !d_pair_q || !d_pair_node || !d_feat)) return fail(QD_ERR_INVALID, "null pointer");
    return features_launch(t, d_q, PairIdx{d_pair_q, d_pair_node, 0, 1}, n_pairs, d_feat, (hipStream_t)stream);
}

// Forward (and optionally backward) over pairs grouped by query: queries
// q0 .. q0+nq-1 of d_q, pair p belongs to query P.q(p).  With labels y the
// full gradient goes to d_grads (QD_MLP_NPARAMS) and the mean loss to d_loss;
// this path needs the pairs as explicit arrays grouped by query (d_qoff).
// u_pre (nullable): the per-query layer-1 sums u (nq x H), already formed.
// ws_given (nullable): scratch of mlp_infer_bytes(n_pairs) for an inference
// with u_pre (no allocation then).
static size_t mlp_infer_bytes(uint64_t n_pairs) {
    const uint64_t np = qd::pad64(n_pairs ? n_pairs : 1);
    return np * qd::H * 4 + np * qd::H * 4 + np * 4 + 64 * 16;
}
static int mlp_run(qd_model_t m, const uint64_t *d_q, uint32_t q0, uint32_t nq, qd::PairIdx P,
                   const uint64_t *d_qoff, uint64_t qoff_base, const float *d_feat, uint64_t n_pairs, const float *y,
                   float *d_scores, float *d_grads, float *d_loss, hipStream_t s, float *u_pre = nullptr,
                   char *ws_given = nullptr) {
    using namespace qd;
    const uint64_t np = pad64(n_pairs ? n_pairs : 1);
    const bool train = y != nullptr;
    if (ws_given && (train || !u_pre)) return fail(QD_ERR_INVALID, "a given scratch serves inference with u only");
    size_t bytes = (u_pre ? 0 : (size_t)nq * H * 4) + np * H * 4 + np * H * 4 + np * 4;
    if (train)
        bytes += np * H * 4 + np * 4 + np * 4 + np * H * 2 + (size_t)H * H * 4 + (size_t)nq * H * 4 +
                 (size_t)kHeadParts * kHeadPartLen * 4 + (size_t)nq * kL1Chunks * kL1PartLen * 4;
    char *ws = ws_given;
    if (!ws) QD_HIP_CHECK(hipMallocAsync((void **)&ws, bytes + 64 * 16, s));
    char *c = ws;
    auto take = [&](size_t b) {
        char *r = c;
        c += (b + 63) / 64 * 64;
        return r;
    };
    Scratch S;
    S.u = u_pre ? u_pre : (float *)take((size_t)nq * H * 4);
    S.h1 = (uint16_t *)take(np * H * 4);
    S.z2 = (float *)take(np * H * 4);
    S.s = (float *)take(np * 4);
    if (train) {
        S.h2 = (float *)take(np * H * 4);
        S.ds = (float *)take(np * 4);
        S.lossv = (float *)take(np * 4);
        S.d2 = (uint16_t *)take(np * H * 2);
        S.dw2 = (float *)take((size_t)H * H * 4);
        S.du = (float *)take((size_t)nq * H * 4);
        S.hpart = (float *)take((size_t)kHeadParts * kHeadPartLen * 4);
        S.lpart = (float *)take((size_t)nq * kL1Chunks * kL1PartLen * 4);
    }
    {
        KernelTimer timer("mlp_forward", s);
        if (!u_pre) hipLaunchKernelGGL(uq_kernel, dim3(nq), dim3(kBlock), 0, s, d_q, q0, m->w, S.u);
        hipLaunchKernelGGL(layer1_kernel, dim3((uint32_t)np), dim3(kBlock), 0, s, S.u, P, q0, d_feat, n_pairs, m->w,
                           S.h1);
        gemm(s, false, false, S.h1, m->w2x2, S.z2, (int)np, H, 2 * H, 2 * H, H, H);
        hipLaunchKernelGGL(head_kernel, dim3((uint32_t)(np / 4)), dim3(kBlock), 0, s, S.z2, n_pairs, m->w, y,
                           d_scores ? d_scores : S.s, S.h2, S.ds, S.lossv, S.d2, np);
    }
    hipError_t e = hipGetLastError();
    if (train && e == hipSuccess) {
        KernelTimer timer("mlp_backward", s);
        hipLaunchKernelGGL(head_partial_kernel, dim3(kHeadParts), dim3(kBlock), 0, s, S.h2, S.ds, S.lossv, n_pairs,
                           S.hpart);
        hipLaunchKernelGGL(head_final_kernel, dim3(1), dim3(kBlock), 0, s, S.hpart, n_pairs, m->w, d_grads, d_loss);
        // dW2 = (h1_hi + h1_lo)^T d2 ; dh1 = d2 W2^T (into z2's buffer)
        gemm(s, true, false, S.h1, S.d2, S.dw2, H, H, (int)np, 2 * H, H, H);
        gemm(s, true, false, S.h1 + H, S.d2, S.dw2, H, H, (int)np, 2 * H, H, H, 1);
        gemm(s, false, true, S.d2, m->w + OFF_W2, S.z2, (int)np, H, H, H, H, H);
        hipLaunchKernelGGL(copy_grad_w2_kernel, dim3(H * H / kBlock), dim3(kBlock), 0, s, S.dw2, d_grads);
        hipLaunchKernelGGL(layer1_partial_kernel, dim3(nq * kL1Chunks), dim3(kBlock), 0, s, S.z2, S.h1, d_feat, d_qoff,
                           qoff_base, S.lpart);
        hipLaunchKernelGGL(layer1_final_kernel, dim3(NF + 1), dim3(kBlock), 0, s, S.lpart, nq, d_grads, S.du);
        hipLaunchKernelGGL(w1q_grad_kernel, dim3(QD_BITS), dim3(kBlock), 0, s, d_q + (uint64_t)q0 * QD_WORDS, nq,
                           S.du, d_grads);
        e = hipGetLastError();
    }
    if (!ws_given) (void)hipFreeAsync(ws, s);
    if (e != hipSuccess) return fail(QD_ERR_DEVICE, "mlp kernels: %s", hipGetErrorString(e));
    return QD_OK;
}

extern "C" int qd_model_forward(qd_model_t m, const uint64_t *d_q, uint32_t nq, const uint32_t *d_pair_q,
                                const float *d_feat, uint64_t n_pairs, float *d_scores, void *stream) {
    using namespace qd;
    if (check_model(m) != QD_OK) return QD_ERR_INVALID;
    if (n_pairs == 0) return QD_OK;
    if (!d_q || !d_pair_q || !d_feat || !d_scores || nq == 0) return fail(QD_ERR_INVALID, "null pointer");
    return mlp_run(m, d_q, 0, nq, PairIdx{d_pair_q, nullptr, 0, 1}, nullptr, 0, d_feat, n_pairs, nullptr, d_scores,
                   nullptr, nullptr, (hipStream_t)stream);
}

extern "C" int qd_model_gradients(qd_model_t m, const uint64_t *d_q, uint32_t nq, const uint64_t *d_qoff,
                                  const uint32_t *d_pair_q, const float *d_feat, const float *d_labels,
                                  uint64_t n_pairs, float *d_grads, float *d_loss, void *stream) {
    using namespace qd;
    if (check_model(m) != QD_OK) return QD_ERR_INVALID;
    if (!d_q || !d_qoff || !d_pair_q || !d_feat || !d_labels || !d_grads || nq == 0 || n_pairs == 0)
        return fail(QD_ERR_INVALID, "null pointer or empty batch");
    return mlp_run(m, d_q, 0, nq, PairIdx{d_pair_q, nullptr, 0, 1}, d_qoff, 0, d_feat, n_pairs, d_labels, nullptr,
                   d_grads, d_loss, (hipStream_t)stream);
}

extern "C" int qd_model_adam_step(qd_model_t m, const float *d_grads, float lr, void *stream) {
    using namespace qd;
    if (check_model(m) != QD_OK || !d_grads) return fail(QD_ERR_INVALID, "null pointer");
    m->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)m->step), c2 = 1.f - powf(b2, (float)m->step);
    hipLaunchKernelGGL(adam_kernel, dim3(1024), dim3(kBlock), 0, (hipStream_t)stream, m->p, m->m, m->v, m->w,
                       d_grads, (size_t)QD_MLP_NPARAMS, lr, b1, b2, 1e-8f, c1, c2);
    hipLaunchKernelGGL(stack_w2_kernel, dim3(H * H / kBlock), dim3(kBlock), 0, (hipStream_t)stream, m->w, m->w2x2);
    QD_HIP_CHECK(hipGetLastError());
    return QD_OK;
}

// Scores of nodes 0 .. n_scored-1 for every query: d_scores is nq x n_scored.
extern "C" int qd_model_score_tree(qd_model_t m, qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t n_scored,
                                   float *d_scores, void *stream) {
    using namespace qd;
    if (check_model(m) != QD_OK || !t) return fail(QD_ERR_INVALID, "null model or tree");
    if (nq == 0 || n_scored == 0) return QD_OK;
    if (!d_q || !d_scores) return fail(QD_ERR_INVALID, "null pointer");
    if (n_scored > t->n_nodes) return fail(QD_ERR_INVALID, "n_scored %u above the node count", n_scored);
    hipStream_t s = (hipStream_t)stream;
    // chunks of whole queries, about 1M pairs each
    const uint32_t per = std::max<uint32_t>(1, (uint32_t)((1u << 20) / n_scored));
    float *feat = nullptr;
    const uint64_t maxp = (uint64_t)per * n_scored;
    QD_HIP_CHECK(hipMallocAsync((void **)&feat, maxp * NF * 4, s));
    int rc = QD_OK;
    for (uint32_t q0 = 0; q0 < nq && rc == QD_OK; q0 += per) {
        const uint32_t cq = std::min(per, nq - q0);
        const uint64_t npair = (uint64_t)cq * n_scored;
        PairIdx P{nullptr, nullptr, q0, n_scored};
        {
            KernelTimer timer("mlp_features", s);
            rc = features_launch(t, d_q, P, npair, feat, s);
        }
        if (rc == QD_OK)
            rc = mlp_run(m, d_q, q0, cq, P, nullptr, 0, feat, npair, nullptr, d_scores + (uint64_t)q0 * n_scored,
                         nullptr, nullptr, s);
    }
    (void)hipFreeAsync(feat, s);
    return rc;
}

// ---- learned start of the blocked search --------------------------------

namespace qd {
namespace {

// The pair of children of every query's current node: pairs 2i and 2i + 1
// score the similar and the dissimilar child of cur[i] when that node is an
// inner node above max_rows rows; otherwise both name cur[i] (scored, unused).
__global__ void descend_pairs_kernel(const uint32_t *__restrict__ cur, uint32_t nq, const int32_t *__restrict__ child,
                                     const uint32_t *__restrict__ count, uint32_t max_rows,
                                     uint32_t *__restrict__ pq, uint32_t *__restrict__ pn) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const uint32_t node = cur[i];
    const int32_t a = child[2 * node];
    const bool go = a >= 0 && count[node] > max_rows;
    pq[2 * i] = pq[2 * i + 1] = i;
    pn[2 * i] = go ? (uint32_t)a : node;
    pn[2 * i + 1] = go ? (uint32_t)child[2 * node + 1] : node;
}

// Enter the higher-scoring child (ties: the similar child).
__global__ void descend_pick_kernel(uint32_t *__restrict__ cur, uint32_t nq, const int32_t *__restrict__ child,
                                    const uint32_t *__restrict__ count, uint32_t max_rows,
                                    const float *__restrict__ sc) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const uint32_t node = cur[i];
    const int32_t a = child[2 * node];
    if (a < 0 || count[node] <= max_rows) return;
    cur[i] = sc[2 * i + 1] > sc[2 * i] ? (uint32_t)child[2 * node + 1] : (uint32_t)a;
}

__global__ void fill_u32_kernel(uint32_t *__restrict__ p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

// Scratch of one descent: the per-query layer-1 sums, the level's (query,
// node) pairs, their features and scores, then the MLP's own scratch.
static size_t descend_own_bytes(uint32_t nq) {
    const uint64_t np = 2ull * nq;
    return (size_t)nq * H * 4 + np * 8 + np * NF * 4 + np * 4 + 5 * 256;
}

size_t model_descend_bytes(uint32_t nq) { return descend_own_bytes(nq) + mlp_infer_bytes(2ull * nq) + 256; }

int model_descend(qd_model_t m, qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t max_rows, uint32_t *d_node,
                  char *ws_given, hipStream_t s) {
    if (check_model(m) != QD_OK || !t) return fail(QD_ERR_INVALID, "null model or tree");
    if (nq == 0) return QD_OK;
    const uint64_t np = 2ull * nq;
    char *ws = ws_given;
    if (!ws) QD_HIP_CHECK(hipMallocAsync((void **)&ws, model_descend_bytes(nq), s));
    char *c = ws;
    auto take = [&](size_t b) {
        char *r = c;
        c += (b + 255) / 256 * 256;
        return r;
    };
    float *u = (float *)take((size_t)nq * H * 4);
    uint32_t *pq = (uint32_t *)take(np * 4), *pn = (uint32_t *)take(np * 4);
    float *feat = (float *)take(np * NF * 4), *sc = (float *)take(np * 4);
    const dim3 g((nq + 255) / 256);
    int rc = QD_OK;
    {
        KernelTimer timer("mlp_forward", s);
        hipLaunchKernelGGL(fill_u32_kernel, g, dim3(256), 0, s, d_node, nq, 0u);  // every query starts at the root
        hipLaunchKernelGGL(uq_kernel, dim3(nq), dim3(kBlock), 0, s, d_q, 0u, m->w, u);  // shared by every level
    }
    for (size_t L = 0; L < t->level_max.size() && t->level_max[L] > max_rows && rc == QD_OK; L++) {
        hipLaunchKernelGGL(descend_pairs_kernel, g, dim3(256), 0, s, d_node, nq, t->d_child, t->d_count, max_rows, pq,
                           pn);
        {
            KernelTimer timer("mlp_features", s);
            rc = features_launch(t, d_q, PairIdx{pq, pn, 0, 1}, np, feat, s);
        }
        if (rc == QD_OK)
            rc = mlp_run(m, d_q, 0, nq, PairIdx{pq, pn, 0, 1}, nullptr, 0, feat, np, nullptr, sc, nullptr, nullptr, s,
                         u, ws + (descend_own_bytes(nq) + 255) / 256 * 256);
        hipLaunchKernelGGL(descend_pick_kernel, g, dim3(256), 0, s, d_node, nq, t->d_child, t->d_count, max_rows, sc);
    }
    if (rc == QD_OK && hipGetLastError() != hipSuccess) rc = fail(QD_ERR_DEVICE, "model descent: launch failed");
    if (!ws_given) (void)hipFreeAsync(ws, s);
    return rc;
}

}  // namespace qd

// ---- training pairs from traversal traces ------------------------------

namespace qd {
namespace {

// One block per query.  Pass 1 (pair_q == nullptr) counts valid pairs into
// counts[j]; pass 2 writes them at qoff[j] in ascending node order.
__global__ __launch_bounds__(kBlock) void trace_pairs_kernel(const int32_t *__restrict__ parent,
                                                             const uint32_t *__restrict__ begin,
                                                             const uint32_t *__restrict__ count,
                                                             const uint32_t *__restrict__ iperm, uint64_t n_rows,
                                                             const uint32_t *__restrict__ result, uint32_t k,
                                                             const uint32_t *__restrict__ vis, uint32_t n_traced,
                                                             uint32_t *__restrict__ counts,
                                                             const uint64_t *__restrict__ qoff,
                                                             uint32_t *__restrict__ pair_q,
                                                             uint32_t *__restrict__ pair_node,
                                                             float *__restrict__ labels) {
    __shared__ uint32_t pos[QD_MAX_K];
    __shared__ uint32_t wave_cnt[kBlock / 64];
    const uint32_t j = blockIdx.x;
    const uint32_t words = (n_traced + 31) / 32;
    const uint32_t *v = vis + (uint64_t)j * words;
    if (threadIdx.x < k) {
        const uint32_t r = result[(uint64_t)j * k + threadIdx.x];
        pos[threadIdx.x] = r < n_rows ? iperm[r] : 0xFFFFFFFFu;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t out = pair_q ? qoff[j] : 0;
    uint32_t total = 0;
    for (uint32_t base = 1; base < n_traced; base += kBlock) {
        const uint32_t node = base + threadIdx.x;
        bool valid = false;
        float lab = 0.f;
        if (node < n_traced) {
            const int32_t par = parent[node];
            valid = par >= 0 && ((v[par >> 5] >> (par & 31)) & 1u);
            if (valid)
                for (uint32_t r = 0; r < k; r++) {
                    const uint32_t ps = pos[r];
                    if (ps != 0xFFFFFFFFu && ps >= begin[node] && ps - begin[node] < count[node]) lab = 1.f;
                }
        }
        const uint64_t b = ballot(valid);
        if (lane == 0) wave_cnt[w] = (uint32_t)__popcll(b);
        __syncthreads();
        uint32_t before = 0, chunk = 0;
        for (int i = 0; i < kBlock / 64; i++) {
            if (i < w) before += wave_cnt[i];
            chunk += wave_cnt[i];
        }
        if (valid && pair_q) {
            const uint64_t o = out + before + (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
            pair_q[o] = j;
            pair_node[o] = node;
            labels[o] = lab;
        }
        out += chunk;
        total += chunk;
        __syncthreads();
    }
    if (!pair_q && threadIdx.x == 0) counts[j] = total;
}

}  // namespace
}  // namespace qd

extern "C" int qd_trace_pairs(qd_tree_t t, uint32_t nq, uint32_t k, const uint32_t *d_result_idx,
                              const uint32_t *d_visited, uint32_t n_traced, uint32_t *d_pair_q,
                              uint32_t *d_pair_node, float *d_labels, uint64_t capacity, uint64_t *d_qoff,
                              uint64_t *h_n_pairs, void *stream) {
    using namespace qd;
    if (!t || !h_n_pairs) return fail(QD_ERR_INVALID, "null argument");
    if (k < 1 || k > QD_MAX_K) return fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
    if (n_traced > t->n_nodes) return fail(QD_ERR_INVALID, "n_traced above the node count");
    *h_n_pairs = 0;
    if (nq == 0) return QD_OK;
    if (!d_result_idx || !d_visited || !d_qoff) return fail(QD_ERR_INVALID, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    uint32_t *cnt = nullptr;
    QD_HIP_CHECK(hipMallocAsync((void **)&cnt, (size_t)nq * 4, s));
    hipLaunchKernelGGL(trace_pairs_kernel, dim3(nq), dim3(kBlock), 0, s, t->d_parent, t->d_begin, t->d_count,
                       t->d_iperm, t->n, d_result_idx, k, d_visited, n_traced, cnt, nullptr, nullptr, nullptr,
                       nullptr);
    std::vector<uint32_t> hc(nq);
    std::vector<uint64_t> off(nq + 1, 0);
    hipError_t e = hipMemcpyAsync(hc.data(), cnt, (size_t)nq * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFreeAsync(cnt, s);
        return fail(QD_ERR_DEVICE, "trace count: %s", hipGetErrorString(e));
    }
    for (uint32_t j = 0; j < nq; j++) off[j + 1] = off[j] + hc[j];
    *h_n_pairs = off[nq];
    if (off[nq] <= capacity && off[nq] > 0) {
        if (!d_pair_q || !d_pair_node || !d_labels) {
            (void)hipFreeAsync(cnt, s);
            return fail(QD_ERR_INVALID, "null pair arrays");
        }
        e = hipMemcpyAsync(d_qoff, off.data(), (nq + 1) * 8, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(trace_pairs_kernel, dim3(nq), dim3(kBlock), 0, s, t->d_parent, t->d_begin,
                               t->d_count, t->d_iperm, t->n, d_result_idx, k, d_visited, n_traced, cnt, d_qoff,
                               d_pair_q, d_pair_node, d_labels);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    } else if (off[nq] <= capacity) {
        e = hipMemcpyAsync(d_qoff, off.data(), (nq + 1) * 8, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    (void)hipFreeAsync(cnt, s);
    if (e != hipSuccess) return fail(QD_ERR_DEVICE, "trace pairs: %s", hipGetErrorString(e));
    return QD_OK;
}

// ---- training loop ------------------------------------------------------

namespace qd {
int knn_tree_impl(qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k, int order, const float *d_scores,
                  uint32_t n_scored, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra, float *d_dist,
                  uint32_t *d_qstats, qd_stats *h_stats, void *stream, uint32_t waves_per_cu, uint32_t *d_trace,
                  uint32_t n_traced, uint32_t split);
}

// Traces the exact best-first search of the training queries, forms the
// (query, node, useful) pairs, and runs `epochs` passes of Adam over batches
// of batch_queries queries, in the order h_batch_order gives (a permutation of
// the batch indices; NULL = ascending).  h_losses (nullable) receives the mean
// loss of every step.  Synchronous.
extern "C" int qd_model_train(qd_model_t m, qd_tree_t t, const uint64_t *d_q, uint32_t nq, uint32_t k,
                              uint32_t n_traced, uint32_t epochs, uint32_t batch_queries, float lr,
                              const uint32_t *h_batch_order, float *h_losses, uint64_t *h_n_pairs, void *stream) {
    using namespace qd;
    if (check_model(m) != QD_OK || !t || !d_q) return fail(QD_ERR_INVALID, "null argument");
    if (nq == 0 || batch_queries == 0 || n_traced < 2 || n_traced > t->n_nodes)
        return fail(QD_ERR_INVALID, "bad training shape");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t words = (n_traced + 31) / 32;
    struct Bufs {
        void *p[12] = {};
        ~Bufs() {
            for (void *x : p)
                if (x) (void)hipFree(x);
        }
    } B;
    uint32_t *idx, *vis;
    int32_t *mi, *ex;
    float *di;
    QD_HIP_CHECK(hipMalloc(&B.p[0], (size_t)nq * k * 4));
    QD_HIP_CHECK(hipMalloc(&B.p[1], (size_t)nq * k * 4));
    QD_HIP_CHECK(hipMalloc(&B.p[2], (size_t)nq * k * 4));
    QD_HIP_CHECK(hipMalloc(&B.p[3], (size_t)nq * k * 4));
    QD_HIP_CHECK(hipMalloc(&B.p[4], (size_t)nq * words * 4));
    idx = (uint32_t *)B.p[0];
    mi = (int32_t *)B.p[1];
    ex = (int32_t *)B.p[2];
    di = (float *)B.p[3];
    vis = (uint32_t *)B.p[4];
    int rc = knn_tree_impl(t, d_q, nq, k, QD_ORDER_BEST_FIRST, nullptr, 0, idx, mi, ex, di, nullptr, nullptr, stream, 0,
                           vis, n_traced, 1);
    if (rc != QD_OK) return rc;
    uint64_t np = 0;
    QD_HIP_CHECK(hipMalloc(&B.p[5], (size_t)(nq + 1) * 8));
    uint64_t *qoff = (uint64_t *)B.p[5];
    rc = qd_trace_pairs(t, nq, k, idx, vis, n_traced, nullptr, nullptr, nullptr, 0, qoff, &np, stream);
    if (rc != QD_OK) return rc;
    if (h_n_pairs) *h_n_pairs = np;
    if (np == 0) return fail(QD_ERR_INVALID, "the traced search produced no training pairs");
    QD_HIP_CHECK(hipMalloc(&B.p[6], np * 4));
    QD_HIP_CHECK(hipMalloc(&B.p[7], np * 4));
    QD_HIP_CHECK(hipMalloc(&B.p[8], np * 4));
    QD_HIP_CHECK(hipMalloc(&B.p[9], np * NF * 4));
    QD_HIP_CHECK(hipMalloc(&B.p[10], (size_t)QD_MLP_NPARAMS * 4));
    QD_HIP_CHECK(hipMalloc(&B.p[11], 4));
    uint32_t *pq = (uint32_t *)B.p[6], *pn = (uint32_t *)B.p[7];
    float *lab = (float *)B.p[8], *feat = (float *)B.p[9], *grads = (float *)B.p[10], *loss = (float *)B.p[11];
    rc = qd_trace_pairs(t, nq, k, idx, vis, n_traced, pq, pn, lab, np, qoff, &np, stream);
    if (rc != QD_OK) return rc;
    rc = features_launch(t, d_q, PairIdx{pq, pn, 0, 1}, np, feat, s);
    if (rc != QD_OK) return rc;
    std::vector<uint64_t> hoff(nq + 1);
    QD_HIP_CHECK(hipMemcpy(hoff.data(), qoff, (nq + 1) * 8, hipMemcpyDeviceToHost));
    const uint32_t nb = (nq + batch_queries - 1) / batch_queries;
    uint64_t step = 0;
    for (uint32_t e = 0; e < epochs; e++)
        for (uint32_t bi = 0; bi < nb; bi++) {
            if (abort_requested()) {  // between steps: the queued ones finish first
                (void)hipStreamSynchronize(s);
                return fail(QD_ERR_ABORTED, "training aborted after %llu steps", (unsigned long long)step);
            }
            const uint32_t b = h_batch_order ? h_batch_order[bi] % nb : bi;
            const uint32_t qa = b * batch_queries, qb = std::min(nq, qa + batch_queries);
            const uint64_t p0 = hoff[qa], p1 = hoff[qb];
            float lv = NAN;
            if (p1 > p0) {
                rc = mlp_run(m, d_q, qa, qb - qa, PairIdx{pq + p0, nullptr, 0, 1}, qoff + qa, p0, feat + p0 * NF,
                             p1 - p0, lab + p0, nullptr, grads, loss, s);
                if (rc != QD_OK) return rc;
                rc = qd_model_adam_step(m, grads, lr, stream);
                if (rc != QD_OK) return rc;
                if (h_losses) {
                    QD_HIP_CHECK(hipMemcpyAsync(&lv, loss, 4, hipMemcpyDeviceToHost, s));
                    QD_HIP_CHECK(hipStreamSynchronize(s));
                }
            }
            if (h_losses) h_losses[step] = lv;
            step++;
        }
    QD_HIP_CHECK(hipStreamSynchronize(s));
    return QD_OK;
}

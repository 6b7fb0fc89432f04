/*
 * Seeded synthetic inputs shaped like 64x64-bit QUICCI descriptors.
 *
 * This file only draws inputs.  It holds no part of the search method: no
 * distance, no tree, no selection, no vote.  Both the CPU oracle and the GPU
 * library consume what it writes, so nothing here may depend on either.
 *
 * Format: a descriptor is uint64[64]; word r is image row r and bit c of that
 * word is column c (bit index b = 64*r + c).  QUICCI images are 64x64 bits in
 * all of the paper's experiments (Section 6), and their set bits trace the
 * outlines where circle/surface intersection counts change (Section 2.2), so
 * the stand-in draws thin circular arcs centred on the image centre.
 *
 * Random numbers: splitmix64 (Steele, Lea, Flood 2014), one independent
 * stream per output item keyed as seed ^ (golden_gamma * (i + 1)), doubles
 * from the top 53 bits.  Every item depends only on (seed, its index), so the
 * output is identical for any thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SY_WORDS 64
#define SY_BITS 4096
#define SY_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sy_next(uint64_t *s) {
    uint64_t z = (*s += SY_GAMMA);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline double sy_unif(uint64_t *s) { return (double)(sy_next(s) >> 11) * 0x1.0p-53; }
/* uniform integer in [0, m) */
static inline uint64_t sy_below(uint64_t *s, uint64_t m) {
    uint64_t v = (uint64_t)(sy_unif(s) * (double)m);
    return v >= m ? m - 1 : v;
}
static inline uint64_t sy_key(uint64_t seed, uint64_t i) { return seed ^ (SY_GAMMA * (i + 1)); }

static int sy_popcount(const uint64_t *d) {
    int c = 0;
    for (int r = 0; r < SY_WORDS; r++) c += __builtin_popcountll(d[r]);
    return c;
}

/* Ring arc of radius rad around (31.5, 31.5), angles phi .. phi+len, one pixel
 * wide.  The angle advances by 1/(2*rad) per step (half a pixel of arc), the
 * rotation done by a fixed complex multiplier. */
static void sy_arc(uint64_t *img, double rad, double phi, double len) {
    double step = 1.0 / (2.0 * rad);
    long n = (long)floor(len / step) + 1;
    double c = cos(phi), s = sin(phi), cd = cos(step), sd = sin(step);
    for (long j = 0; j < n; j++) {
        int row = (int)floor(31.5 + rad * s);
        int col = (int)floor(31.5 + rad * c);
        if (row < 0) row = 0;
        if (row > 63) row = 63;
        if (col < 0) col = 0;
        if (col > 63) col = 63;
        img[row] |= 1ULL << col;
        double c2 = c * cd - s * sd;
        s = s * cd + c * sd;
        c = c2;
    }
}

/* One database descriptor: m ~ U{3..12} arcs with radius ~ U[2,31], start
 * angle ~ U[0,2pi), arc length ~ U[pi/4, 2pi]; an arc that would lift the
 * popcount above max_bits is skipped; after m draws, arcs keep coming (same
 * rule) until the popcount reaches min_bits.  Draws are capped so the loop
 * always ends. */
static void sy_one(uint64_t st, int min_bits, int max_bits, uint64_t *out) {
    uint64_t img[SY_WORDS], tmp[SY_WORDS];
    memset(img, 0, sizeof img);
    int m = 3 + (int)sy_below(&st, 10);
    int pop = 0;
    for (int draw = 0; draw < 4096 && (draw < m || pop < min_bits); draw++) {
        double rad = 2.0 + 29.0 * sy_unif(&st);
        double phi = 2.0 * M_PI * sy_unif(&st);
        double len = M_PI / 4.0 + (2.0 * M_PI - M_PI / 4.0) * sy_unif(&st);
        memcpy(tmp, img, sizeof img);
        sy_arc(tmp, rad, phi, len);
        int p = sy_popcount(tmp);
        if (p <= max_bits) {
            memcpy(img, tmp, sizeof img);
            pop = p;
        }
    }
    memcpy(out, img, sizeof img);
}

/* Rows first .. first+n-1 of the database for `seed`. */
void sy_gen_db(uint64_t *out, uint64_t first, uint64_t n, uint64_t seed, int min_bits, int max_bits) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < (int64_t)n; i++)
        sy_one(sy_key(seed, first + (uint64_t)i), min_bits, max_bits, out + (uint64_t)i * SY_WORDS);
}

/* Partial, noisy copy of src: clear round(p*|src|) distinct set bits chosen
 * uniformly, then flip nflip distinct uniformly chosen positions. */
static void sy_partial(const uint64_t *src, double p, int nflip, uint64_t *st, uint64_t *out) {
    uint16_t pos[SY_BITS];
    int cnt = 0;
    memcpy(out, src, SY_WORDS * sizeof(uint64_t));
    for (int b = 0; b < SY_BITS; b++)
        if ((src[b >> 6] >> (b & 63)) & 1) pos[cnt++] = (uint16_t)b;
    int nclear = (int)llround(p * cnt);
    if (nclear > cnt) nclear = cnt;
    for (int a = 0; a < nclear; a++) {
        int j = a + (int)sy_below(st, (uint64_t)(cnt - a));
        uint16_t t = pos[a];
        pos[a] = pos[j];
        pos[j] = t;
        out[pos[a] >> 6] &= ~(1ULL << (pos[a] & 63));
    }
    /* distinct flip positions by partial Fisher-Yates over all 4096 bits */
    uint16_t all[SY_BITS];
    for (int b = 0; b < SY_BITS; b++) all[b] = (uint16_t)b;
    for (int a = 0; a < nflip && a < SY_BITS; a++) {
        int j = a + (int)sy_below(st, (uint64_t)(SY_BITS - a));
        uint16_t t = all[a];
        all[a] = all[j];
        all[j] = t;
        out[all[a] >> 6] ^= 1ULL << (all[a] & 63);
    }
}

/* nq queries.  Query j draws its source row uniformly from [0, n) unless
 * src_in is given, its partiality p ~ U[pmin, pmax], then the partial copy.
 * The source row is written to src_out (ground truth for recall only). */
void sy_gen_queries(const uint64_t *db, uint64_t n, uint64_t nq, uint64_t seed, double pmin, double pmax,
                    int nflip, const uint32_t *src_in, uint64_t *out, uint32_t *src_out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < (int64_t)nq; j++) {
        uint64_t st = sy_key(seed, (uint64_t)j);
        uint64_t s = src_in ? src_in[j] : sy_below(&st, n);
        double p = pmin + (pmax - pmin) * sy_unif(&st);
        sy_partial(db + s * SY_WORDS, p, nflip, &st, out + (uint64_t)j * SY_WORDS);
        if (src_out) src_out[j] = (uint32_t)s;
    }
}

/* Query objects over a database of n_obj objects with per_obj rows each
 * (object o owns rows o*per_obj .. o*per_obj+per_obj-1).  Query object g
 * picks an object o_g ~ U{0..n_obj-1} and a size m_g ~ U{mmin..mmax}
 * (m_g <= per_obj), then m_g distinct rows of o_g in a uniformly random
 * order.  Pass 1 (rows == NULL) only writes sizes into off[g+1]; pass 2
 * writes the source rows (CSR by the prefix sums in off) and obj[g]. */
void sy_gen_query_objects(uint64_t n_obj, uint64_t per_obj, uint64_t nqo, uint64_t seed, uint64_t mmin,
                          uint64_t mmax, uint64_t *off, uint32_t *rows, int32_t *obj) {
    for (uint64_t g = 0; g < nqo; g++) {
        uint64_t st = sy_key(seed, g);
        uint64_t o = sy_below(&st, n_obj);
        uint64_t m = mmin + sy_below(&st, mmax - mmin + 1);
        if (m > per_obj) m = per_obj;
        if (!rows) {
            off[g + 1] = m;
            continue;
        }
        obj[g] = (int32_t)o;
        uint32_t *perm = (uint32_t *)malloc(per_obj * sizeof(uint32_t));
        for (uint64_t a = 0; a < per_obj; a++) perm[a] = (uint32_t)a;
        for (uint64_t a = 0; a < m; a++) {
            uint64_t j = a + sy_below(&st, per_obj - a);
            uint32_t t = perm[a];
            perm[a] = perm[j];
            perm[j] = t;
            rows[off[g] + a] = (uint32_t)(o * per_obj + perm[a]);
        }
        free(perm);
    }
}

/* Poisson-process arrival times (exponential gaps of mean 1/rate) for n
 * events, starting at 0; used to replay a stream of query objects. */
void sy_poisson_arrivals(uint64_t n, double rate, uint64_t seed, double *t_out) {
    uint64_t st = sy_key(seed, 0);
    double t = 0.0;
    for (uint64_t i = 0; i < n; i++) {
        double u = sy_unif(&st);
        t += -log1p(-u) / rate;
        t_out[i] = t;
    }
}

/* n floats uniform in [lo, hi): initial weights for the frontier-order model. */
void sy_uniform_f32(float *out, uint64_t n, uint64_t seed, float lo, float hi) {
    for (uint64_t i = 0; i < n; i++) {
        uint64_t st = sy_key(seed, i);
        out[i] = lo + (hi - lo) * (float)sy_unif(&st);
    }
}

/* A uniformly random permutation of 0..n-1 (Fisher-Yates on one stream). */
void sy_permutation(uint32_t *out, uint64_t n, uint64_t seed) {
    uint64_t st = sy_key(seed, 0);
    for (uint64_t i = 0; i < n; i++) out[i] = (uint32_t)i;
    for (uint64_t i = 0; i + 1 < n; i++) {
        uint64_t j = i + sy_below(&st, n - i);
        uint32_t t = out[i];
        out[i] = out[j];
        out[j] = t;
    }
}

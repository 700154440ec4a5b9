/*
 * Seeded synthetic column generator.
 *
 * Produces the encoded inputs that both the CPU oracle and the GPU library
 * consume: RLE columns (values + exclusive run ends), index-encoded sparse
 * columns (sorted unique int32 positions + values) and bit-packed columns
 * (dictionary codes or frame-of-reference offsets in an LSB-first stream of
 * little-endian uint32 words).  It holds no query arithmetic: no predicate,
 * alignment, grouping or aggregation happens here.
 *
 * Randomness is counter based, so every output element is a pure function of
 * (seed, stream, index) and the result does not depend on the thread count:
 *   key     = mix(seed ^ mix(stream + 1))
 *   draw(i) = mix(key + (i + 1) * 0x9E3779B97F4A7C15)
 * where mix is the SplitMix64 output function (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC dg.c -o libccq_datagen.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t dg_key(uint64_t seed, uint64_t stream) { return mix64(seed ^ mix64(stream + 1)); }

uint64_t dg_draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GOLDEN); }

/* uniform double in (0, 1]: 53 random bits, never 0 so log() is finite */
static inline double unit_open0(uint64_t u) { return ((double)(u >> 11) + 1.0) * (1.0 / 9007199254740992.0); }

/* uniform integer in [lo, hi) by multiply-high (Lemire); bias < 2^-64 * range */
static inline int64_t uniform_range(uint64_t u, int64_t lo, int64_t hi) {
    uint64_t span = (uint64_t)(hi - lo);
    return lo + (int64_t)(((unsigned __int128)u * span) >> 64);
}

/* ------------------------------------------------------------------ */
/* run lengths                                                         */
/* dist 0: geometric on {1,2,...} with mean m  (p = 1/m)               */
/* dist 1: max(1, round(X)), X ~ LogNormal(ln m - s^2/2, s)            */
/* ------------------------------------------------------------------ */
static inline int64_t run_len(uint64_t key, uint64_t i, int dist, double mean, double sigma) {
    if (dist == 0) {
        if (mean <= 1.0) return 1;
        double p = 1.0 / mean;
        double u = unit_open0(dg_draw(key, i));
        return 1 + (int64_t)floor(log(u) / log1p(-p));
    } else {
        double u1 = unit_open0(dg_draw(key, 2 * i));
        double u2 = unit_open0(dg_draw(key, 2 * i + 1));
        double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        double mu = log(mean) - 0.5 * sigma * sigma;
        double x = exp(mu + sigma * z);
        int64_t l = (int64_t)llround(x);
        return l < 1 ? 1 : l;
    }
}

#define RUN_BLOCK 65536

/* Number of runs needed to cover n_rows rows (the last run is clipped). */
int64_t dg_rle_count(uint64_t seed, uint64_t stream, int dist, double mean, double sigma, int64_t n_rows) {
    if (n_rows <= 0) return 0;
    uint64_t key = dg_key(seed, stream);
    int64_t est_blocks = (int64_t)((double)n_rows / mean * 1.25 / RUN_BLOCK) + 2;
    int64_t base_block = 0;
    int64_t covered = 0;
    for (;;) {
        int64_t nb = est_blocks;
        int64_t* sums = (int64_t*)malloc(sizeof(int64_t) * nb);
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = 0; b < nb; b++) {
            int64_t s = 0;
            uint64_t i0 = (uint64_t)(base_block + b) * RUN_BLOCK;
            for (int j = 0; j < RUN_BLOCK; j++) s += run_len(key, i0 + j, dist, mean, sigma);
            sums[b] = s;
        }
        for (int64_t b = 0; b < nb; b++) {
            if (covered + sums[b] >= n_rows) {
                uint64_t i0 = (uint64_t)(base_block + b) * RUN_BLOCK;
                int64_t c = covered;
                for (int j = 0; j < RUN_BLOCK; j++) {
                    c += run_len(key, i0 + j, dist, mean, sigma);
                    if (c >= n_rows) { free(sums); return (base_block + b) * RUN_BLOCK + j + 1; }
                }
            }
            covered += sums[b];
        }
        free(sums);
        base_block += nb;
        est_blocks = est_blocks / 4 + 2;
    }
}

/* Fill run_ends[0..n_runs) (exclusive ends, strictly increasing, last == n_rows). */
void dg_rle_fill(uint64_t seed, uint64_t stream, int dist, double mean, double sigma, int64_t n_rows,
                 int64_t* run_ends, int64_t n_runs) {
    if (n_runs <= 0) return;
    uint64_t key = dg_key(seed, stream);
    int64_t nb = (n_runs + RUN_BLOCK - 1) / RUN_BLOCK;
    int64_t* offs = (int64_t*)malloc(sizeof(int64_t) * (nb + 1));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; b++) {
        int64_t s = 0;
        int64_t j1 = (b + 1) * RUN_BLOCK < n_runs ? (b + 1) * RUN_BLOCK : n_runs;
        for (int64_t i = b * RUN_BLOCK; i < j1; i++) {
            s += run_len(key, (uint64_t)i, dist, mean, sigma);
            run_ends[i] = s;
        }
        offs[b + 1] = s;
    }
    offs[0] = 0;
    for (int64_t b = 0; b < nb; b++) offs[b + 1] += offs[b];
#pragma omp parallel for schedule(static)
    for (int64_t b = 1; b < nb; b++) {
        int64_t j1 = (b + 1) * RUN_BLOCK < n_runs ? (b + 1) * RUN_BLOCK : n_runs;
        for (int64_t i = b * RUN_BLOCK; i < j1; i++) run_ends[i] += offs[b];
    }
    run_ends[n_runs - 1] = n_rows;
    free(offs);
}

/* i.i.d. uniform integers in [lo, hi) */
void dg_uniform_i32(uint64_t seed, uint64_t stream, int64_t lo, int64_t hi, int32_t* out, int64_t n) {
    uint64_t key = dg_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) out[i] = (int32_t)uniform_range(dg_draw(key, (uint64_t)i), lo, hi);
}

void dg_uniform_i64(uint64_t seed, uint64_t stream, int64_t lo, int64_t hi, int64_t* out, int64_t n) {
    uint64_t key = dg_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) out[i] = uniform_range(dg_draw(key, (uint64_t)i), lo, hi);
}

/* ------------------------------------------------------------------ */
/* sparse positions: every row is listed independently with prob p     */
/* (geometric gaps), restarted at each 2^20-row block so blocks are    */
/* independent and can be generated in parallel.                       */
/* ------------------------------------------------------------------ */
#define SP_BLOCK (1 << 20)

/* out32 / out64: where to write the block's positions (at most one set) */
static int64_t sparse_block(uint64_t key, int64_t b, double p, int64_t n_rows, int32_t* out32, int64_t* out64) {
    int64_t r0 = b * (int64_t)SP_BLOCK;
    int64_t r1 = r0 + SP_BLOCK < n_rows ? r0 + SP_BLOCK : n_rows;
    uint64_t ctr = (uint64_t)b << 32;
    int64_t cnt = 0;
    double lq = log1p(-p);
    int64_t r = r0 - 1;
    for (;;) {
        double u = unit_open0(dg_draw(key, ctr++));
        int64_t gap = 1 + (int64_t)floor(log(u) / lq);
        r += gap;
        if (r >= r1) break;
        if (out32) out32[cnt] = (int32_t)r;
        if (out64) out64[cnt] = r;
        cnt++;
    }
    return cnt;
}

int64_t dg_sparse_count(uint64_t seed, uint64_t stream, double p, int64_t n_rows) {
    if (n_rows <= 0 || p <= 0) return 0;
    uint64_t key = dg_key(seed, stream);
    int64_t nb = (n_rows + SP_BLOCK - 1) / SP_BLOCK;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : total)
    for (int64_t b = 0; b < nb; b++) total += sparse_block(key, b, p, n_rows, NULL, NULL);
    return total;
}

static void sparse_fill(uint64_t seed, uint64_t stream, double p, int64_t n_rows, int32_t* p32, int64_t* p64,
                        int64_t n) {
    if (n <= 0) return;
    uint64_t key = dg_key(seed, stream);
    int64_t nb = (n_rows + SP_BLOCK - 1) / SP_BLOCK;
    int64_t* offs = (int64_t*)malloc(sizeof(int64_t) * (nb + 1));
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t b = 0; b < nb; b++) offs[b + 1] = sparse_block(key, b, p, n_rows, NULL, NULL);
    offs[0] = 0;
    for (int64_t b = 0; b < nb; b++) offs[b + 1] += offs[b];
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t b = 0; b < nb; b++)
        sparse_block(key, b, p, n_rows, p32 ? p32 + offs[b] : NULL, p64 ? p64 + offs[b] : NULL);
    free(offs);
}

/* int32 positions (tables below 2^31 rows) */
void dg_sparse_fill(uint64_t seed, uint64_t stream, double p, int64_t n_rows, int32_t* positions, int64_t n) {
    sparse_fill(seed, stream, p, n_rows, positions, NULL, n);
}

/* int64 positions (the same rows as dg_sparse_fill) */
void dg_sparse_fill64(uint64_t seed, uint64_t stream, double p, int64_t n_rows, int64_t* positions, int64_t n) {
    sparse_fill(seed, stream, p, n_rows, NULL, positions, n);
}

/* ------------------------------------------------------------------ */
/* codes and packing                                                   */
/* ------------------------------------------------------------------ */

/* Zipf over ranks k = 1..n_codes with P(k) ~ k^-s; the code is k - 1. */
static double* zipf_cdf(double s, int64_t n_codes) {
    double* cdf = (double*)malloc(sizeof(double) * n_codes);
    double acc = 0;
    for (int64_t k = 0; k < n_codes; k++) { acc += pow((double)(k + 1), -s); cdf[k] = acc; }
    for (int64_t k = 0; k < n_codes; k++) cdf[k] /= acc;
    cdf[n_codes - 1] = 1.0;
    return cdf;
}

static inline uint32_t zipf_code(const double* cdf, int64_t n_codes, uint64_t u) {
    double x = ((double)(u >> 11)) * (1.0 / 9007199254740992.0); /* [0,1) */
    int64_t lo = 0, hi = n_codes - 1;                          /* first k with cdf[k] > x */
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > x) hi = mid; else lo = mid + 1;
    }
    return (uint32_t)lo;
}

void dg_zipf_codes(uint64_t seed, uint64_t stream, double s, int64_t n_codes, uint32_t* out, int64_t n) {
    uint64_t key = dg_key(seed, stream);
    double* cdf = zipf_cdf(s, n_codes);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) out[i] = zipf_code(cdf, n_codes, dg_draw(key, (uint64_t)i));
    free(cdf);
}

void dg_zipf_pmf(double s, int64_t n_codes, double* out) {
    double* cdf = zipf_cdf(s, n_codes);
    double prev = 0;
    for (int64_t k = 0; k < n_codes; k++) { out[k] = cdf[k] - prev; prev = cdf[k]; }
    free(cdf);
}

/* Words needed for n codes of w bits, plus two pad words. */
int64_t dg_packed_words(int64_t n, int w) { return (n * (int64_t)w + 31) / 32 + 2; }

/* Pack cnt <= 32 consecutive codes into words[0 .. ceil(cnt*w/32)); a full
 * group of 32 codes fills exactly w words. */
static inline void pack32(const uint32_t* codes, int64_t cnt, int w, uint32_t* words) {
    uint64_t mask = w == 32 ? 0xFFFFFFFFULL : ((1ULL << w) - 1);
    int64_t nw = (cnt * (int64_t)w + 31) / 32;
    for (int64_t j = 0; j < nw; j++) words[j] = 0;
    for (int64_t j = 0; j < cnt; j++) {
        uint64_t bit = (uint64_t)j * (uint64_t)w;
        uint64_t c = (uint64_t)codes[j] & mask;
        uint64_t wi = bit >> 5, sh = bit & 31;
        uint64_t v = c << sh;
        words[wi] |= (uint32_t)v;
        if (sh + (uint64_t)w > 32) words[wi + 1] |= (uint32_t)(v >> 32);
    }
}

/* Pack arbitrary codes (low w bits each) into an LSB-first stream. */
void dg_pack(const uint32_t* codes, int64_t n, int w, uint32_t* packed, int64_t n_words) {
    memset(packed, 0, sizeof(uint32_t) * (size_t)n_words);
    int64_t ng = (n + 31) / 32;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < ng; g++) {
        int64_t cnt = n - g * 32 < 32 ? n - g * 32 : 32;
        pack32(codes + g * 32, cnt, w, packed + g * (int64_t)w);
    }
}

/* Generate and pack in one pass (no full code array in memory).
 * kind 0: Zipf(s) over n_codes; kind 1: uniform over [0, n_codes). */
void dg_codes_packed(uint64_t seed, uint64_t stream, int kind, double s, int64_t n_codes, int64_t n, int w,
                     uint32_t* packed, int64_t n_words) {
    uint64_t key = dg_key(seed, stream);
    double* cdf = kind == 0 ? zipf_cdf(s, n_codes) : NULL;
    int64_t ng = (n + 31) / 32;
    int64_t used = (n * (int64_t)w + 31) / 32;
    if (used < n_words) memset(packed + used, 0, sizeof(uint32_t) * (size_t)(n_words - used));
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < ng; g++) {
        uint32_t codes[32];
        int64_t cnt = n - g * 32 < 32 ? n - g * 32 : 32;
        for (int64_t j = 0; j < cnt; j++) {
            uint64_t u = dg_draw(key, (uint64_t)(g * 32 + j));
            codes[j] = kind == 0 ? zipf_code(cdf, n_codes, u) : (uint32_t)uniform_range(u, 0, n_codes);
        }
        pack32(codes, cnt, w, packed + g * (int64_t)w);
    }
    free(cdf);
}

int dg_max_threads(void) { return omp_get_max_threads(); }

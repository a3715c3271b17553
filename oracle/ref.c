/*
 * FP64 CPU oracle for preconditioned data sparsification
 * (Pourkamali-Anaraki & Becker, arXiv 1511.00152).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the
 * GPU library: every routine below is written out from the paper's
 * definitions (and, for the random choices the paper leaves open, from the
 * published definitions of the generators named at each routine).
 *
 * Conventions.  The paper stores samples as the columns of X (p x n).  Here
 * one sample is one contiguous row of a row-major n x p array; indices are
 * 0-based.  All arithmetic is IEEE double.  Parallel loops (OpenMP) split the
 * samples into contiguous ranges; sums over samples are formed per range and
 * then added range by range, which only changes the rounding order (the Gram
 * of the covariance estimator instead sums every entry in sample order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 block function (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11).  Each round multiplies counter words 0
 * and 2 by the two Philox multipliers, and recombines the 128-bit products with
 * counter words 1 and 3 and the round key; the key is bumped by the two Weyl
 * constants between rounds.                                                  */
/* ------------------------------------------------------------------------- */
#define ORC_PHILOX_MUL0 0xD2E7470EE14C6C93ULL
#define ORC_PHILOX_MUL1 0xCA5A826395121157ULL
#define ORC_PHILOX_WEYL0 0x9E3779B97F4A7C15ULL
#define ORC_PHILOX_WEYL1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += ORC_PHILOX_WEYL0;
            k1 += ORC_PHILOX_WEYL1;
        }
        unsigned __int128 prod0 = (unsigned __int128)ORC_PHILOX_MUL0 * c0;
        unsigned __int128 prod1 = (unsigned __int128)ORC_PHILOX_MUL1 * c2;
        uint64_t hi0 = (uint64_t)(prod0 >> 64), lo0 = (uint64_t)prod0;
        uint64_t hi1 = (uint64_t)(prod1 >> 64), lo1 = (uint64_t)prod1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A stream of 32-bit words: blocks b = 0, 1, 2, ... of Philox4x64-10 under key
 * (seed, 0) and counter (b, c1, c2, 0); within a block the four 64-bit words
 * are used in order, each low half first, then high half.                    */
typedef struct {
    uint64_t key[2];
    uint64_t ctr[4];
    uint64_t buf[4];
    int pos; /* next 32-bit word inside buf, 0..8; 8 = buffer empty */
} orc_stream;

static void stream_init(orc_stream* s, uint64_t seed, uint64_t c1, uint64_t c2)
{
    s->key[0] = seed;
    s->key[1] = 0;
    s->ctr[0] = 0;
    s->ctr[1] = c1;
    s->ctr[2] = c2;
    s->ctr[3] = 0;
    s->pos = 8;
}

static uint32_t stream_next32(orc_stream* s)
{
    if (s->pos == 8) {
        orc_philox4x64_10(s->ctr, s->key, s->buf);
        s->ctr[0] += 1;
        s->pos = 0;
    }
    uint64_t w = s->buf[s->pos >> 1];
    uint32_t r = (s->pos & 1) ? (uint32_t)(w >> 32) : (uint32_t)(w & 0xffffffffu);
    s->pos += 1;
    return r;
}

/* ------------------------------------------------------------------------- */
/* Uniform integer in [0, range) by Lemire's multiply-and-reject method
 * (Lemire, "Fast random integer generation in an interval", ACM TOMACS 2019),
 * written for a word width of `bits` (1..32) so that a test can enumerate it
 * exhaustively at small widths.  `next` supplies the words; returns the value. */
/* ------------------------------------------------------------------------- */
typedef uint32_t (*orc_word_fn)(void* ctx);

static uint32_t lemire_bits(uint32_t range, int bits, orc_word_fn next, void* ctx)
{
    const uint64_t mask = (bits == 32) ? 0xffffffffULL : ((1ULL << bits) - 1ULL);
    uint64_t product = (uint64_t)(next(ctx) & mask) * range;
    uint64_t low = product & mask;
    if (low < range) {
        /* 2^bits mod range: the number of low parts that must be rejected */
        uint64_t threshold = ((mask + 1ULL) - range) % range;
        while (low < threshold) {
            product = (uint64_t)(next(ctx) & mask) * range;
            low = product & mask;
        }
    }
    return (uint32_t)(product >> bits);
}

typedef struct {
    const uint32_t* words;
    int n;
    int used;
} orc_word_array;

static uint32_t word_array_next(void* ctx)
{
    orc_word_array* a = (orc_word_array*)ctx;
    uint32_t w = (a->used < a->n) ? a->words[a->used] : 0u;
    a->used += 1;
    return w;
}

/* Test hook: Lemire's method over an explicit word list; *consumed receives the
 * number of words read (may exceed nwords, which means the list ran short).   */
uint32_t orc_lemire_from_words(uint32_t range, int bits, const uint32_t* words, int nwords, int* consumed)
{
    orc_word_array a = {words, nwords, 0};
    uint32_t r = lemire_bits(range, bits, word_array_next, &a);
    *consumed = a.used;
    return r;
}

static uint32_t stream_word_fn(void* ctx) { return stream_next32((orc_stream*)ctx); }

/* ------------------------------------------------------------------------- */
/* Sampling m of p coordinates uniformly without replacement (Sec. I, setup
 * paragraph; Appendix B, Thm. "Properties of the sampling matrix").  The paper
 * does not say how the subset is drawn; Floyd's algorithm (Bentley & Floyd,
 * CACM 1987) gives every m-subset probability 1/C(p,m) from m uniform draws:
 * for t = p-m, ..., p-1 draw r uniform on {0..t}; keep r unless it is already
 * kept, in which case keep t.                                               */
/* ------------------------------------------------------------------------- */

/* Test hook: Floyd's set logic on an explicit list of draws (draw k must lie in
 * [0, p-m+k]).  Writes the kept set ascending into idx (m entries).          */
int orc_floyd_from_draws(int64_t p, int64_t m, const uint32_t* draws, uint16_t* idx)
{
    unsigned char* kept = (unsigned char*)calloc((size_t)p, 1);
    if (!kept) return -1;
    for (int64_t k = 0; k < m; ++k) {
        int64_t t = p - m + k;
        uint32_t r = draws[k];
        if (kept[r]) kept[t] = 1;
        else kept[r] = 1;
    }
    int64_t c = 0;
    for (int64_t j = 0; j < p; ++j)
        if (kept[j]) idx[c++] = (uint16_t)j;
    free(kept);
    return (c == m) ? 0 : -2;
}

/* The kept coordinates of sample i (global index): the draws are Lemire on the
 * 32-bit word stream of key (seed, 0), counter (b, i, 0, 0).                 */
void orc_sample_indices(uint64_t seed, uint64_t i, int64_t p, int64_t m, uint16_t* idx)
{
    orc_stream s;
    stream_init(&s, seed, i, 0);
    uint32_t* draws = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m);
    for (int64_t k = 0; k < m; ++k) {
        int64_t t = p - m + k;
        draws[k] = lemire_bits((uint32_t)(t + 1), 32, stream_word_fn, &s);
    }
    orc_floyd_from_draws(p, m, draws, idx);
    free(draws);
}

/* Number of 32-bit words sample i's draws consume (m when no draw was
 * rejected by Lemire's method).                                             */
int64_t orc_sample_words_used(uint64_t seed, uint64_t i, int64_t p, int64_t m)
{
    orc_stream s;
    stream_init(&s, seed, i, 0);
    for (int64_t k = 0; k < m; ++k) {
        int64_t t = p - m + k;
        (void)lemire_bits((uint32_t)(t + 1), 32, stream_word_fn, &s);
    }
    return (int64_t)(s.ctr[0] - 1) * 8 + s.pos;
}

/* ------------------------------------------------------------------------- */
/* The random sign diagonal D of the ROS (Sec. III, eq. ROS): one sign per
 * coordinate, shared by every sample (Alg. 1 applies one HD to all of X).
 * D_j = +1 if bit (j mod 64) of 64-bit word ((j div 64) mod 4) of the block
 * with key (seed, 0), counter (j div 256, 0, 1, 0) is 0, else -1.            */
/* ------------------------------------------------------------------------- */
void orc_signs(uint64_t seed, int64_t p, int8_t* D)
{
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    for (int64_t j = 0; j < p; ++j) {
        uint64_t ctr[4] = {(uint64_t)(j / 256), 0, 1, 0};
        orc_philox4x64_10(ctr, key, out);
        uint64_t word = out[(j / 64) % 4];
        D[j] = ((word >> (j % 64)) & 1ULL) ? (int8_t)-1 : (int8_t)1;
    }
}

/* ------------------------------------------------------------------------- */
/* Normalized Walsh-Hadamard transform, Sylvester (natural) order:
 * H[j][k] = (-1)^popcount(j & k) / sqrt(p).  Sec. III: H orthonormal, entries
 * +-1/sqrt(p), applied in O(p log p).  Butterflies h = 1, 2, 4, ..., then one
 * multiplication by 1/sqrt(p).                                              */
/* ------------------------------------------------------------------------- */
void orc_fwht_normalized(double* v, int64_t p)
{
    for (int64_t h = 1; h < p; h <<= 1)
        for (int64_t i = 0; i < p; i += 2 * h)
            for (int64_t j = i; j < i + h; ++j) {
                double a = v[j], b = v[j + h];
                v[j] = a + b;
                v[j + h] = a - b;
            }
    double s = 1.0 / sqrt((double)p);
    for (int64_t j = 0; j < p; ++j) v[j] *= s;
}

/* One entry of y = H D x straight from the definition (row j of H dotted with
 * D x), for spot checks of single outputs at sizes where whole rows would be
 * too slow to recompute.  x has p entries (float or double, see below).     */
static double y_entry_from(const int8_t* D, int64_t p, int64_t j, const double* xd, const float* xf)
{
    double acc = 0.0;
    for (int64_t k = 0; k < p; ++k) {
        double xk = xd ? xd[k] : (double)xf[k];
        int neg = __builtin_popcountll((unsigned long long)(j & k)) & 1;
        double h = neg ? -1.0 : 1.0;
        acc += h * (double)D[k] * xk;
    }
    return acc / sqrt((double)p);
}

double orc_y_entry_f64(const int8_t* D, int64_t p, int64_t j, const double* x)
{
    return y_entry_from(D, p, j, x, NULL);
}

double orc_y_entry_f32(const int8_t* D, int64_t p, int64_t j, const float* x)
{
    return y_entry_from(D, p, j, NULL, x);
}

/* ------------------------------------------------------------------------- */
/* One-pass compression (Alg. 1, first loop): y_i = H D x_i, then keep the m
 * sampled entries w_i = R_i R_i^T y_i, stored as (vals, idx) with idx
 * ascending.  Row r of X is sample i0 + r.  X is double (xd) or float (xf,
 * widened exactly to double).                                                */
/* ------------------------------------------------------------------------- */
static void compress_impl(uint64_t seed, int64_t p, int64_t m, const double* xd, const float* xf,
                          int64_t n, int64_t ldx, uint64_t i0, double* vals, uint16_t* idx, int nthreads)
{
    int8_t* D = (int8_t*)malloc((size_t)p);
    orc_signs(seed, p, D);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double* y = (double*)malloc(sizeof(double) * (size_t)p);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            for (int64_t j = 0; j < p; ++j) {
                double xj = xd ? xd[r * ldx + j] : (double)xf[r * ldx + j];
                y[j] = (double)D[j] * xj;
            }
            orc_fwht_normalized(y, p);
            uint16_t* row_idx = idx + r * m;
            orc_sample_indices(seed, i0 + (uint64_t)r, p, m, row_idx);
            for (int64_t k = 0; k < m; ++k) vals[r * m + k] = y[row_idx[k]];
        }
        free(y);
    }
    free(D);
}

void orc_compress_f64(uint64_t seed, int64_t p, int64_t m, const double* X, int64_t n, int64_t ldx,
                      uint64_t i0, double* vals, uint16_t* idx, int nthreads)
{
    compress_impl(seed, p, m, X, NULL, n, ldx, i0, vals, idx, nthreads);
}

void orc_compress_f32(uint64_t seed, int64_t p, int64_t m, const float* X, int64_t n, int64_t ldx,
                      uint64_t i0, double* vals, uint16_t* idx, int nthreads)
{
    compress_impl(seed, p, m, NULL, X, n, ldx, i0, vals, idx, nthreads);
}

/* ------------------------------------------------------------------------- */
/* Covariance estimator (Sec. V).  G = sum_i w_i w_i^T over the compressed
 * samples.  Every entry G[j][k] is summed over the samples in sample order
 * (i = 0, 1, ..., n-1), so the result does not depend on the thread count:
 * for each sample that keeps coordinate j, row j receives v_j * v_k for all
 * kept k of that sample, and a row is updated by one thread at a time.
 *
 * orc_gram_rows: rows[0..nrows-1] of G (distinct coordinates), added into the
 * nrows x p row-major array out.  orc_gram_accumulate: all p rows, added into
 * the p x p row-major G.                                                    */
/* ------------------------------------------------------------------------- */
void orc_gram_rows(int64_t p, int64_t m, const double* vals, const uint16_t* idx, int64_t n,
                   const int64_t* rows, int64_t nrows, double* out, int nthreads)
{
    /* Samples are taken in blocks of NB.  Within a block, the (sample, entry)
     * pairs of each wanted coordinate are listed in sample order (a stable
     * counting sort by coordinate), and each row of the output then walks its
     * own list: every entry of G still receives its terms in sample order, and
     * the row being updated stays in cache while it does.                   */
    const int64_t NB = 8192;
    int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)p);
    for (int64_t j = 0; j < p; ++j) slot[j] = -1;
    for (int64_t r = 0; r < nrows; ++r) slot[rows[r]] = r;
    int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nrows + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nrows + 1));
    int64_t* list = (int64_t*)malloc(sizeof(int64_t) * (size_t)(NB * m));  /* i * m + a */
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (int64_t i0 = 0; i0 < n; i0 += NB) {
        const int64_t i1 = (i0 + NB < n) ? i0 + NB : n;
        for (int64_t r = 0; r <= nrows; ++r) start[r] = 0;
        for (int64_t e = i0 * m; e < i1 * m; ++e) {
            const int64_t r = slot[idx[e]];
            if (r >= 0) ++start[r + 1];
        }
        for (int64_t r = 0; r < nrows; ++r) start[r + 1] += start[r];
        for (int64_t r = 0; r <= nrows; ++r) fill[r] = start[r];
        for (int64_t e = i0 * m; e < i1 * m; ++e) {
            const int64_t r = slot[idx[e]];
            if (r >= 0) list[fill[r]++] = e - i0 * m;
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; ++r) {
            double* orow = out + r * p;
            for (int64_t q = start[r]; q < start[r + 1]; ++q) {
                const int64_t e = i0 * m + list[q];
                const int64_t i = e / m;
                const double va = vals[e];
                const double* v = vals + i * m;
                const uint16_t* ix = idx + i * m;
                for (int64_t b = 0; b < m; ++b) orow[ix[b]] += va * v[b];
            }
        }
    }
    free(list);
    free(fill);
    free(start);
    free(slot);
}

void orc_gram_accumulate(int64_t p, int64_t m, const double* vals, const uint16_t* idx, int64_t n,
                         double* G, int nthreads)
{
    int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)p);
    for (int64_t j = 0; j < p; ++j) rows[j] = j;
    orc_gram_rows(p, m, vals, idx, n, rows, p, G, nthreads);
    free(rows);
}

/* C_emp_hat = p(p-1)/(m(m-1)) * G / n and
 * C_n = C_emp_hat - (p-m)/(p-1) * diag(C_emp_hat)   (Sec. V, the two displayed
 * definitions before Thm. "covariance").  Requires m >= 2.                  */
void orc_cov_finalize(int64_t p, int64_t m, int64_t n, const double* G, double* C)
{
    double rescale = ((double)p * (double)(p - 1)) / ((double)m * (double)(m - 1));
    for (int64_t e = 0; e < p * p; ++e) C[e] = rescale * (G[e] / (double)n);
    double shrink = (double)(p - m) / (double)(p - 1);
    for (int64_t j = 0; j < p; ++j) C[j * p + j] = C[j * p + j] - shrink * C[j * p + j];
}

/* ------------------------------------------------------------------------- */
/* Sparsified K-means (Sec. VI).  Distances use each sample's own m kept
 * coordinates only (eq. assignments); centers are the coordinate-wise means
 * of the kept entries over each cluster (eq. mu_update_two).  Where a count
 * n_k^(j) is zero the coordinate cannot be estimated; it keeps its previous
 * value.  Ties in the argmin go to the lowest cluster index.  Distances are
 * summed in ascending coordinate order with fused multiply-adds.            */
/* ------------------------------------------------------------------------- */
static double sparse_dist(int64_t p, int64_t m, const double* v, const uint16_t* ix, const double* mu)
{
    (void)p;
    double d = 0.0;
    for (int64_t a = 0; a < m; ++a) {
        double diff = v[a] - mu[ix[a]];
        d = fma(diff, diff, d);
    }
    return d;
}

/* margin[i] (optional) receives (second smallest - smallest distance) for
 * sample i, +inf when K == 1.                                               */
void orc_kmeans_step(int64_t p, int64_t m, const double* vals, const uint16_t* idx, int64_t n, int K,
                     const double* centers_in, double* centers_out, int32_t* assign, double* objective,
                     double* margin, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    double obj = 0.0;
    /* Step 1: assignments */
#pragma omp parallel for schedule(static) reduction(+ : obj)
    for (int64_t i = 0; i < n; ++i) {
        const double* v = vals + i * m;
        const uint16_t* ix = idx + i * m;
        int best = 0;
        double dbest = sparse_dist(p, m, v, ix, centers_in);
        double dsecond = INFINITY;
        for (int k = 1; k < K; ++k) {
            double d = sparse_dist(p, m, v, ix, centers_in + (int64_t)k * p);
            if (d < dbest) {
                dsecond = dbest;
                dbest = d;
                best = k;
            } else if (d < dsecond) {
                dsecond = d;
            }
        }
        assign[i] = best;
        if (margin) margin[i] = dsecond - dbest;
        obj += dbest;
    }
    *objective = obj;
    /* Step 2: coordinate-wise means over kept entries */
    double* sums = (double*)calloc((size_t)K * (size_t)p, sizeof(double));
    int64_t* counts = (int64_t*)calloc((size_t)K * (size_t)p, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        int k = assign[i];
        for (int64_t a = 0; a < m; ++a) {
            sums[(int64_t)k * p + idx[i * m + a]] += vals[i * m + a];
            counts[(int64_t)k * p + idx[i * m + a]] += 1;
        }
    }
    for (int64_t e = 0; e < (int64_t)K * p; ++e)
        centers_out[e] = (counts[e] > 0) ? sums[e] / (double)counts[e] : centers_in[e];
    free(sums);
    free(counts);
}

/* Two-pass sparsified K-means (Alg. "Sparsified K-means, 2-pass"): one pass
 * over the original rows X (n x p) after the one-pass run, given its
 * assignments c_hat and its centers mu_hat in the original domain.  Each row
 * is added to the center of its one-pass cluster (the pseudocode's garbled
 * increment is read as x_i), and is re-assigned to the nearest one-pass
 * center in the original domain (FP64, ascending coordinate order, fma; ties
 * to the lowest k).  A cluster with no rows keeps its one-pass center.
 * margin[i] (optional): second smallest - smallest distance, +inf if K == 1. */
void orc_kmeans_2pass(int64_t p, const double* X, int64_t n, int K, const int32_t* c_hat, const double* mu_hat,
                      double* mu_out, int32_t* c_out, double* margin, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* re-assignment to the nearest one-pass center */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double* x = X + i * p;
        int best = 0;
        double dbest = INFINITY, dsecond = INFINITY;
        for (int k = 0; k < K; ++k) {
            const double* mu = mu_hat + (int64_t)k * p;
            double d = 0.0;
            for (int64_t j = 0; j < p; ++j) {
                const double diff = x[j] - mu[j];
                d = fma(diff, diff, d);
            }
            if (d < dbest) {
                dsecond = dbest;
                dbest = d;
                best = k;
            } else if (d < dsecond) {
                dsecond = d;
            }
        }
        c_out[i] = best;
        if (margin) margin[i] = dsecond - dbest;
    }
    /* centers: mean of the rows of each one-pass cluster */
    double* sums = (double*)calloc((size_t)K * (size_t)p, sizeof(double));
    int64_t* counts = (int64_t*)calloc((size_t)K, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        const int k = c_hat[i];
        counts[k] += 1;
        for (int64_t j = 0; j < p; ++j) sums[(int64_t)k * p + j] += X[i * p + j];
    }
    for (int k = 0; k < K; ++k)
        for (int64_t j = 0; j < p; ++j)
            mu_out[(int64_t)k * p + j] =
                counts[k] > 0 ? sums[(int64_t)k * p + j] / (double)counts[k] : mu_hat[(int64_t)k * p + j];
    free(sums);
    free(counts);
}

/* Unmixing (eq. mu-mu'): mu = (HD)^T mu' = D H mu' since H is symmetric. */
void orc_unmix(uint64_t seed, int64_t p, const double* centers_pre, int K, double* centers_out)
{
    int8_t* D = (int8_t*)malloc((size_t)p);
    orc_signs(seed, p, D);
    double* t = (double*)malloc(sizeof(double) * (size_t)p);
    for (int k = 0; k < K; ++k) {
        memcpy(t, centers_pre + (int64_t)k * p, sizeof(double) * (size_t)p);
        orc_fwht_normalized(t, p);
        for (int64_t j = 0; j < p; ++j) centers_out[(int64_t)k * p + j] = (double)D[j] * t[j];
    }
    free(t);
    free(D);
}

/* K-means++ seeding (Arthur & Vassilvitskii, SODA 2007) on the compressed
 * samples (Alg. 1, "find initial cluster centers via K-means++").  The paper
 * does not say how the seeding sees sparse samples; here a chosen sample's
 * center is its zero-filled w_c and D^2 is the sparse distance above.  Uniform
 * doubles are 53-bit fractions of the 64-bit words of key (seed, 0), counter
 * (b, 0, 2, 0).  The first center is sample floor(u * n); each next one is the
 * first sample whose running D^2 sum exceeds u * (total D^2).                */
void orc_kmeanspp(uint64_t seed, int64_t p, int64_t m, const double* vals, const uint16_t* idx, int64_t n,
                  int K, uint64_t replicate, double* centers, int64_t* chosen)
{
    uint64_t key[2] = {seed, 0};
    uint64_t ctr[4] = {0, replicate, 2, 0};
    uint64_t buf[4];
    int pos = 4;
    double* d2 = (double*)malloc(sizeof(double) * (size_t)n);
    memset(centers, 0, sizeof(double) * (size_t)K * (size_t)p);
    for (int k = 0; k < K; ++k) {
        if (pos == 4) {
            orc_philox4x64_10(ctr, key, buf);
            ctr[0] += 1;
            pos = 0;
        }
        double u = (double)(buf[pos++] >> 11) * (1.0 / 9007199254740992.0);
        int64_t c;
        if (k == 0) {
            c = (int64_t)(u * (double)n);
            if (c >= n) c = n - 1;
        } else {
            double total = 0.0;
            for (int64_t i = 0; i < n; ++i) total += d2[i];
            double target = u * total;
            double run = 0.0;
            c = n - 1;
            for (int64_t i = 0; i < n; ++i) {
                run += d2[i];
                if (run > target) {
                    c = i;
                    break;
                }
            }
        }
        if (chosen) chosen[k] = c;
        double* mu = centers + (int64_t)k * p;
        for (int64_t a = 0; a < m; ++a) mu[idx[c * m + a]] = vals[c * m + a];
        for (int64_t i = 0; i < n; ++i) {
            double d = sparse_dist(p, m, vals + i * m, idx + i * m, mu);
            if (k == 0 || d < d2[i]) d2[i] = d;
        }
    }
    free(d2);
}

/* Sample-mean estimator (Thm. "sampleMean"): xbar_hat = (p/m)(1/n) sum_i w_i. */
void orc_mean_estimate(int64_t p, int64_t m, const double* vals, const uint16_t* idx, int64_t n, double* mean)
{
    memset(mean, 0, sizeof(double) * (size_t)p);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t a = 0; a < m; ++a) mean[idx[i * m + a]] += vals[i * m + a];
    double s = (double)p / ((double)m * (double)n);
    for (int64_t j = 0; j < p; ++j) mean[j] *= s;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Kept coordinates of samples i0 .. i0+n-1 (row r of idx is sample i0 + r). */
void orc_sample_batch(uint64_t seed, uint64_t i0, int64_t n, int64_t p, int64_t m, uint16_t* idx, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) orc_sample_indices(seed, i0 + (uint64_t)r, p, m, idx + r * m);
}

/* Principal submatrix G[J][J] of G = sum_i w_i w_i^T straight from the
 * definitions, for spot checks at sizes where the whole Gram is out of reach:
 * for every sample, its kept set (the sampler above) and, for each coordinate
 * of J that it keeps, y_ij = row j of H times D x_i (no fast transform).
 * X is float, row-major n x p (ld ldx); sample i0 + r is row r.
 * Gsub is nJ x nJ, added into.                                             */
void orc_gram_submatrix_f32(uint64_t seed, int64_t p, int64_t m, const float* X, int64_t n, int64_t ldx, uint64_t i0,
                            const int64_t* J, int64_t nJ, double* Gsub, int nthreads)
{
    int8_t* D = (int8_t*)malloc((size_t)p);
    orc_signs(seed, p, D);
    int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)p);
    for (int64_t j = 0; j < p; ++j) slot[j] = -1;
    for (int64_t a = 0; a < nJ; ++a) slot[J[a]] = a;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int T = omp_get_max_threads();
#else
    (void)nthreads;
    int T = 1;
#endif
    double* part = (double*)calloc((size_t)T * (size_t)(nJ * nJ), sizeof(double));
#pragma omp parallel num_threads(T)
    {
#ifdef _OPENMP
        int t = omp_get_thread_num();
#else
        int t = 0;
#endif
        double* Gt = part + (size_t)t * (size_t)(nJ * nJ);
        uint16_t* ix = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)m);
        int64_t* hit = (int64_t*)malloc(sizeof(int64_t) * (size_t)nJ);
        double* yv = (double*)malloc(sizeof(double) * (size_t)nJ);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            orc_sample_indices(seed, i0 + (uint64_t)r, p, m, ix);
            int64_t h = 0;
            for (int64_t k = 0; k < m; ++k)
                if (slot[ix[k]] >= 0) {
                    hit[h] = slot[ix[k]];
                    yv[h] = y_entry_from(D, p, ix[k], NULL, X + r * ldx);
                    ++h;
                }
            for (int64_t a = 0; a < h; ++a)
                for (int64_t b = 0; b < h; ++b) Gt[hit[a] * nJ + hit[b]] += yv[a] * yv[b];
        }
        free(ix);
        free(hit);
        free(yv);
    }
    for (int t = 0; t < T; ++t)
        for (int64_t e = 0; e < nJ * nJ; ++e) Gsub[e] += part[(size_t)t * (size_t)(nJ * nJ) + e];
    free(part);
    free(slot);
    free(D);
}

/*
 * discord_ref.c -- plain, slow, obviously correct FP64 reference for time-series
 * discord search.  TEST INFRASTRUCTURE ONLY: it is called by the tests, by the
 * smoke check and by the CPU-baseline leg of the benchmark, never by the
 * product library, and it shares no code with it.
 *
 * Definitions followed (the paper's section 2.1, "formal definitions"):
 *   - series T = (t_0 .. t_{m-1}); subsequence T_{i,n} = (t_i .. t_{i+n-1}),
 *     N = m - n + 1 subsequences (indices are 0-based here, 1-based in the paper);
 *   - T_{i,n} and T_{j,n} are non-self matches iff |i - j| >= n;
 *   - Euclidean distance, eq. (1); comparisons are made on its square, as the
 *     PotentialDiscord/RefineDiscord algorithms do, and the square root is taken
 *     once at the end;
 *   - the discord is the subsequence whose nearest non-self match is farthest.
 *   - z-normalisation, eq. (2): one mean and one standard deviation for the whole
 *     series.  It is an affine map, so every squared distance on the normalised
 *     series equals the raw one divided by sigma^2; the search is done on raw
 *     values and the reported distance is divided by sigma.
 *
 * Readings where the paper is silent:
 *   - ties: the lowest index among maximal nearest-neighbour distances wins, and
 *     the nearest neighbour reported is the lowest j among minimisers;
 *   - rows that have no non-self match at all (possible only when 2n <= m <= 3n-2)
 *     take no part in the argmax;
 *   - sigma^2 is computed two-pass (same real number as eq. (2)'s one-pass form).
 *
 * Arithmetic: every float32 input is promoted to double exactly; each squared
 * distance is the sequential sum over k = 0..n-1 of (a_k - b_k)^2 with separately
 * rounded multiply and add (built with -ffp-contract=off).
 *
 * Second reading (the *_z functions): Algorithm 2 applies Znormalize to the
 * subsequence matrix S, which read row by row normalises every window on its
 * own: x_{i,k} = (t_{i+k} - mu_i) / sigma_i with mu_i and sigma_i the mean and
 * standard deviation of eq. (2) taken over T_{i,n} alone (two-pass, sequential
 * sums), and the distance of eq. (1) is taken between the normalised windows.
 * A flat window (sigma_i == 0) normalises to the zero vector.  The answer then
 * differs from the global reading, so it is a mode of its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ECONST -2

/* Sum over k of (t[i+k] - t[j+k])^2, eq. (1) squared. */
double orc_pair_d2(const float *T, int64_t m, int32_t n, int64_t i, int64_t j)
{
    (void)m;
    double s = 0.0;
    for (int32_t k = 0; k < n; ++k) {
        double d = (double)T[i + k] - (double)T[j + k];
        s = s + d * d;
    }
    return s;
}

/* Mean and standard deviation of the whole series, eq. (2), two-pass. */
int orc_stats(const float *T, int64_t m, double *mu, double *sigma)
{
    if (!T || m < 1) return ORC_EINVAL;
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        if (!isfinite(T[i])) return ORC_EINVAL;
        s += (double)T[i];
    }
    double mean = s / (double)m;
    double v = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double d = (double)T[i] - mean;
        v += d * d;
    }
    *mu = mean;
    *sigma = sqrt(v / (double)m);
    return *sigma > 0.0 ? ORC_OK : ORC_ECONST;
}

/* Mean and standard deviation of every window T_{i,n} (eq. (2) over the window
 * alone), two-pass: mu_i = (sum_k t_{i+k}) / n, sigma_i = sqrt(sum_k (t_{i+k} -
 * mu_i)^2 / n), both sums sequential in k.  mu and sigma hold N = m - n + 1. */
int orc_row_zstats(const float *T, int64_t m, int32_t n, double *mu, double *sigma)
{
    if (!T || !mu || !sigma || n < 1 || m < n) return ORC_EINVAL;
    int64_t N = m - n + 1;
    for (int64_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int32_t k = 0; k < n; ++k) s = s + (double)T[i + k];
        double mean = s / (double)n;
        double q = 0.0;
        for (int32_t k = 0; k < n; ++k) {
            double d = (double)T[i + k] - mean;
            q = q + d * d;
        }
        mu[i] = mean;
        sigma[i] = sqrt(q / (double)n);
    }
    return ORC_OK;
}

/* Element k of the normalised window i: (t_{i+k} - mu_i) / sigma_i, 0 if flat. */
static double zval(const float *T, int64_t i, int32_t k, const double *mu, const double *sg)
{
    return sg[i] > 0.0 ? ((double)T[i + k] - mu[i]) / sg[i] : 0.0;
}

/* Sum over k of (x_{i,k} - x_{j,k})^2: eq. (1) squared between the windows
 * normalised one by one.  mu and sigma come from orc_row_zstats. */
double orc_pair_d2_z(const float *T, int64_t m, int32_t n, int64_t i, int64_t j,
                     const double *mu, const double *sigma)
{
    (void)m;
    double s = 0.0;
    for (int32_t k = 0; k < n; ++k) {
        double d = zval(T, i, k, mu, sigma) - zval(T, j, k, mu, sigma);
        s = s + d * d;
    }
    return s;
}

/* One pair's squared distance under either reading (zmu == NULL: raw values). */
static double pair_any(const float *T, int64_t m, int32_t n, int64_t i, int64_t j,
                       const double *zmu, const double *zsg)
{
    return zmu ? orc_pair_d2_z(T, m, n, i, j, zmu, zsg) : orc_pair_d2(T, m, n, i, j);
}

/* Nearest non-self match of one row: min over j with |i-j| >= n.  Returns 0 and
 * sets *jout = -1 when the row has no non-self match. */
static int row_nn(const float *T, int64_t m, int32_t n, int64_t i, double *dout, int64_t *jout,
                  const double *zmu, const double *zsg)
{
    int64_t N = m - n + 1;
    double best = INFINITY;
    int64_t bj = -1;
    for (int64_t j = 0; j < N; ++j) {
        if (llabs(i - j) < n) continue;
        double d = pair_any(T, m, n, i, j, zmu, zsg);
        if (d < best) { best = d; bj = j; }
    }
    *dout = best;
    *jout = bj;
    return bj >= 0;
}

/* The same minimum for one row with its columns shared among threads: each
 * thread scans a contiguous ascending range of j and keeps its first minimum;
 * merging takes the smallest distance and, among equal ones, the lowest j, so
 * the result is the sequential loop's.  Used where a single row of a long
 * series is asked for. */
static int row_nn_cols(const float *T, int64_t m, int32_t n, int64_t i, double *dout,
                       int64_t *jout, const double *zmu, const double *zsg, int threads)
{
    int64_t N = m - n + 1;
    double best = INFINITY;
    int64_t bj = -1;
    if (threads < 1) threads = 1;
#pragma omp parallel num_threads(threads)
    {
        double lb = INFINITY;
        int64_t lj = -1;
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            if (llabs(i - j) < n) continue;
            double d = pair_any(T, m, n, i, j, zmu, zsg);
            if (d < lb) { lb = d; lj = j; }
        }
#pragma omp critical
        if (lj >= 0 && (bj < 0 || lb < best || (lb == best && lj < bj))) { best = lb; bj = lj; }
    }
    *dout = best;
    *jout = bj;
    return bj >= 0;
}

/* Window statistics for the *_z entry points (NULL on allocation failure). */
static int zstats_alloc(const float *T, int64_t m, int32_t n, double **mu, double **sg)
{
    int64_t N = m - n + 1;
    *mu = (double *)malloc(sizeof(double) * N);
    *sg = (double *)malloc(sizeof(double) * N);
    if (!*mu || !*sg) { free(*mu); free(*sg); *mu = *sg = NULL; return ORC_EINVAL; }
    return orc_row_zstats(T, m, n, *mu, *sg);
}

/* Exact nearest non-self match for a list of rows. */
static int rows_nn_any(const float *T, int64_t m, int32_t n, const int64_t *rows, int64_t count,
                       double *nn_d2, int64_t *nn_j, int threads, const double *zmu,
                       const double *zsg)
{
    if (threads < 1) threads = 1;
    if (count < threads) {   /* few rows: share each row's columns instead */
        for (int64_t r = 0; r < count; ++r)
            row_nn_cols(T, m, n, rows[r], &nn_d2[r], &nn_j[r], zmu, zsg, threads);
        return ORC_OK;
    }
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
    for (int64_t r = 0; r < count; ++r)
        row_nn(T, m, n, rows[r], &nn_d2[r], &nn_j[r], zmu, zsg);
    return ORC_OK;
}

int orc_rows_nn(const float *T, int64_t m, int32_t n, const int64_t *rows, int64_t count,
                double *nn_d2, int64_t *nn_j, int threads)
{
    if (!T || n < 1 || m < n) return ORC_EINVAL;
    return rows_nn_any(T, m, n, rows, count, nn_d2, nn_j, threads, NULL, NULL);
}

int orc_rows_nn_z(const float *T, int64_t m, int32_t n, const int64_t *rows, int64_t count,
                  double *nn_d2, int64_t *nn_j, int threads)
{
    if (!T || n < 1 || m < n) return ORC_EINVAL;
    double *zmu, *zsg;
    int st = zstats_alloc(T, m, n, &zmu, &zsg);
    if (st == ORC_OK) st = rows_nn_any(T, m, n, rows, count, nn_d2, nn_j, threads, zmu, zsg);
    free(zmu);
    free(zsg);
    return st;
}

/* Brute-force discord: NN profile of every row, then the argmax (lowest index on
 * ties).  profile / profile_j may be NULL. */
static int discord_any(const float *T, int64_t m, int32_t n, int threads, int64_t *idx,
                       int64_t *nn_idx, double *d2, double *profile, int64_t *profile_j,
                       const double *zmu, const double *zsg)
{
    int64_t N = m - n + 1;
    double *prof = profile ? profile : (double *)malloc(sizeof(double) * N);
    int64_t *pj = profile_j ? profile_j : (int64_t *)malloc(sizeof(int64_t) * N);
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads)
    for (int64_t i = 0; i < N; ++i)
        row_nn(T, m, n, i, &prof[i], &pj[i], zmu, zsg);
    int64_t bi = -1;
    for (int64_t i = 0; i < N; ++i) {
        if (pj[i] < 0) continue;
        if (bi < 0 || prof[i] > prof[bi]) bi = i;
    }
    *idx = bi;
    *nn_idx = pj[bi];
    *d2 = prof[bi];
    if (!profile) free(prof);
    if (!profile_j) free(pj);
    return ORC_OK;
}

int orc_discord(const float *T, int64_t m, int32_t n, int threads,
                int64_t *idx, int64_t *nn_idx, double *d2, double *mu, double *sigma,
                double *profile, int64_t *profile_j)
{
    if (!T || n < 1 || m < 2 * (int64_t)n) return ORC_EINVAL;
    int st = orc_stats(T, m, mu, sigma);
    if (st != ORC_OK) return st;
    return discord_any(T, m, n, threads, idx, nn_idx, d2, profile, profile_j, NULL, NULL);
}

/* The discord under per-window normalisation.  A constant series is refused
 * (ECONST) as in the global reading: every window is flat and every distance 0. */
int orc_discord_z(const float *T, int64_t m, int32_t n, int threads,
                  int64_t *idx, int64_t *nn_idx, double *d2, double *mu, double *sigma,
                  double *profile, int64_t *profile_j)
{
    if (!T || n < 1 || m < 2 * (int64_t)n) return ORC_EINVAL;
    int st = orc_stats(T, m, mu, sigma);
    if (st != ORC_OK) return st;
    double *zmu, *zsg;
    st = zstats_alloc(T, m, n, &zmu, &zsg);
    if (st == ORC_OK)
        st = discord_any(T, m, n, threads, idx, nn_idx, d2, profile, profile_j, zmu, zsg);
    free(zmu);
    free(zsg);
    return st;
}

/* Witness certificate for a claimed discord (idx, d2):
 *  (i)  the exact NN of idx equals d2;
 *  (ii) every other row i that has a non-self match carries a witness j_i with
 *       |i - j_i| >= n and d(i, j_i) < d2, or d(i, j_i) <= d2 when i > idx.
 * Then no row can beat idx under the lowest-index rule.  Returns the number of
 * rows that fail (ii) and the first of them in *first_bad (-1 if none), or a
 * negative status.  *nn_of_idx receives the exact NN of idx, which is also the
 * threshold used for (ii); the caller checks (i) against it. */
static int64_t witness_any(const float *T, int64_t m, int32_t n, int64_t idx, const int64_t *wit,
                           int threads, int64_t *first_bad, double *nn_of_idx,
                           const double *zmu, const double *zsg)
{
    int64_t N = m - n + 1;
    if (idx < 0 || idx >= N) return ORC_EINVAL;
    double dd; int64_t jj;
    if (!row_nn_cols(T, m, n, idx, &dd, &jj, zmu, zsg, threads)) return ORC_EINVAL;
    *nn_of_idx = dd;
    /* part (ii) is checked against the exact NN of idx; the caller compares its
       claimed distance with *nn_of_idx */
    const double d2 = dd;
    int64_t bad = 0, first = -1;
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(static) num_threads(threads) reduction(+:bad)
    for (int64_t i = 0; i < N; ++i) {
        if (i == idx) continue;
        /* rows with no non-self match at all need no witness */
        int has = (i - n >= 0) || (i + n <= N - 1);
        if (!has) continue;
        int64_t j = wit[i];
        int ok = 0;
        if (j >= 0 && j < N && llabs(i - j) >= n) {
            double e = pair_any(T, m, n, i, j, zmu, zsg);
            ok = (e < d2) || (e == d2 && i > idx);
        }
        if (!ok) {
            bad += 1;
#pragma omp critical
            if (first < 0 || i < first) first = i;
        }
    }
    *first_bad = first;
    return bad;
}

int64_t orc_witness_check(const float *T, int64_t m, int32_t n, int64_t idx, double d2,
                          const int64_t *wit, int threads, int64_t *first_bad, double *nn_of_idx)
{
    (void)d2;
    if (!T || n < 1 || m < 2 * (int64_t)n) return ORC_EINVAL;
    return witness_any(T, m, n, idx, wit, threads, first_bad, nn_of_idx, NULL, NULL);
}

int64_t orc_witness_check_z(const float *T, int64_t m, int32_t n, int64_t idx, double d2,
                            const int64_t *wit, int threads, int64_t *first_bad,
                            double *nn_of_idx)
{
    (void)d2;
    if (!T || n < 1 || m < 2 * (int64_t)n) return ORC_EINVAL;
    double *zmu, *zsg;
    int64_t st = zstats_alloc(T, m, n, &zmu, &zsg);
    if (st == ORC_OK)
        st = witness_any(T, m, n, idx, wit, threads, first_bad, nn_of_idx, zmu, zsg);
    free(zmu);
    free(zsg);
    return st;
}

/* PAA, eq. (3), then SAX, eq. (4), then the word hash, eq. (9), of every row,
 * on the z-normalised series of eq. (2).
 *   - segment s of a row covers offsets [floor(s*n/w), floor((s+1)*n/w)); for
 *     n divisible by w these are the paper's equal blocks of n/w points;
 *   - the PAA value is the mean of the normalised points of the segment;
 *   - the symbol is the k (0-based) with beta_{k} <= value < beta_{k+1}, where
 *     beta_0 = -inf, beta_alpha = +inf and bp[0..alpha-2] are the inner points;
 *   - the word id is sum_s sym_s * alpha^(w-1-s): lexicographic rank of the word,
 *     first segment most significant. */
int orc_sax_words(const float *T, int64_t m, int32_t n, int32_t w, int32_t alpha,
                  const double *bp, double mu, double sigma, int32_t *words, int threads)
{
    if (!T || n < 1 || w < 1 || w > n || alpha < 2 || m < n) return ORC_EINVAL;
    int64_t N = m - n + 1;
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(static) num_threads(threads)
    for (int64_t i = 0; i < N; ++i) {
        int32_t code = 0;
        for (int32_t s = 0; s < w; ++s) {
            int64_t a = ((int64_t)s * n) / w, b = ((int64_t)(s + 1) * n) / w;
            double acc = 0.0;
            for (int64_t k = a; k < b; ++k)
                acc += ((double)T[i + k] - mu) / sigma;
            double paa = acc / (double)(b - a);
            int32_t sym = 0;
            while (sym < alpha - 1 && paa >= bp[sym]) ++sym;
            code = code * alpha + sym;
        }
        words[i] = code;
    }
    return ORC_OK;
}

/* The same words with every window normalised on its own (the *_z reading):
 * the PAA value of segment s is the mean over the segment of the normalised
 * points (t_{i+k} - mu_i) / sigma_i (0 for a flat window); mu and sigma come
 * from orc_row_zstats. */
int orc_sax_words_z(const float *T, int64_t m, int32_t n, int32_t w, int32_t alpha,
                    const double *bp, const double *mu, const double *sigma, int32_t *words,
                    int threads)
{
    if (!T || !mu || !sigma || n < 1 || w < 1 || w > n || alpha < 2 || m < n) return ORC_EINVAL;
    int64_t N = m - n + 1;
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(static) num_threads(threads)
    for (int64_t i = 0; i < N; ++i) {
        int32_t code = 0;
        for (int32_t s = 0; s < w; ++s) {
            int64_t a = ((int64_t)s * n) / w, b = ((int64_t)(s + 1) * n) / w;
            double acc = 0.0;
            for (int64_t k = a; k < b; ++k)
                acc += zval(T, i, (int32_t)k, mu, sigma);
            double paa = acc / (double)(b - a);
            int32_t sym = 0;
            while (sym < alpha - 1 && paa >= bp[sym]) ++sym;
            code = code * alpha + sym;
        }
        words[i] = code;
    }
    return ORC_OK;
}

/*
 * Plain CPU oracle for the discrete Frechet distance.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU library against an
 * independent, obviously correct implementation.  It shares no code, header
 * or constant with the GPU library.
 *
 * Definitions followed (Meinert, "Walking Your Frog Fast in 4 LoC",
 * arXiv 2404.05708):
 *   - Sec. 2: the discrete Frechet distance of Eiter and Mannila between
 *     p in R^{P x D} and q in R^{Q x D} under a ground distance f.
 *   - Algorithm 1 ("vanilla"): memoised top-down recursion over the table M.
 *   - Eq. (1): M_ij = max{ min{M_{i-1,j}, M_{i-1,j-1}, M_{i,j-1}}, d_ij },
 *     delta_dF = M_PQ, with the boundary branches of Algorithms 1 and 3.
 *   - Algorithm 3: the same recurrence bottom-up over the full table.
 *   - Sec. 3 (proof of Theorem 1): only two adjacent rows of M are live, so
 *     the rolling two-row form keeps rows i-1 and i only.
 *
 * Arithmetic: FP64 for float inputs (each float32 coordinate widened
 * exactly); the EUCLIDEAN ground distance is sqrt(sum (p_k - q_k)^2) per
 * cell, SQEUCLIDEAN the plain sum of squares, MANHATTAN sum |p_k - q_k|,
 * CHEBYSHEV max_k |p_k - q_k| (Sec. 3: the method assumes nothing about the
 * ground distance).  Integer inputs use exact int64 distances (squared,
 * Manhattan or Chebyshev) and int64 min/max.  Built without fast-math and
 * without FP contraction so that every operation is the one written here.
 *
 * HAVERSINE is the great-circle distance on the unit sphere between points
 * given as (latitude, longitude) in radians (dim 2): the central angle
 *   theta = 2 asin( sqrt( sin^2(dlat / 2) + cos lat_1 cos lat_2 sin^2(dlon / 2) ) ),
 * the haversine formula, evaluated per cell in FP64 (float inputs only).
 *
 * A separate "float replica" (ffdo_f32_replica) evaluates the distance with
 * the fixed float32 expression documented below and runs the recurrence in
 * float32; it exists only for a bit-exactness check of the GPU's FP32 path.
 *
 * Dynamic time warping (Appendix B, Algorithm B.1): the same table
 * with the outer max replaced by a sum,
 *   M_ij = min{M_{i-1,j}, M_{i-1,j-1}, M_{i,j-1}} + d_ij,  DTW = M_PQ,
 * whose first row is the running sum of d_1j (the +-scan of the DTW
 * algorithm) and whose first column is the running sum of d_i1.  Here the
 * ground distance enters the sum per cell, so EUCLIDEAN takes a square root
 * in every cell (ffdo_dtw_*).
 *
 * Levenshtein distance (Appendix B, Algorithm B.2) of two symbol sequences
 * (int32 points, equal when every coordinate is equal): the table
 *   M_ij = min{M_{i-1,j} + 1, M_{i,j-1} + 1, M_{i-1,j-1} + [p_i != q_j]}
 * with the boundary M_{-1,j} = j + 1, M_{i,-1} = i + 1, M_{-1,-1} = 0
 * (0-based; the algorithm's index vectors read as 0-based), result M_PQ
 * (ffdo_lev_*).
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define FFDO_OK 0
#define FFDO_EINVAL (-1)
#define FFDO_ENOMEM (-3)

#define FFDO_EUCLIDEAN 0
#define FFDO_SQEUCLIDEAN 1
#define FFDO_MANHATTAN 2
#define FFDO_CHEBYSHEV 3
#define FFDO_HAVERSINE 4

/* ---------------------------------------------------------------- ground distance */

/* Central angle between two (latitude, longitude) points in radians, by
 * the haversine formula; the haversine is clamped at 1 against rounding. */
static double haversine_f64(const float *a, const float *b)
{
    double lat1 = a[0], lon1 = a[1], lat2 = b[0], lon2 = b[1];
    double sa = sin(0.5 * (lat2 - lat1));
    double sb = sin(0.5 * (lon2 - lon1));
    double h = sa * sa + cos(lat1) * cos(lat2) * (sb * sb);
    if (h > 1.0) h = 1.0;
    return 2.0 * asin(sqrt(h));
}

/* d(p_i, q_j) in FP64 from float32 coordinates (Sec. 2, f(p_i, q_j)). */
static double cell_f64(const float *pi, const float *qj, int dim, int metric)
{
    if (metric == FFDO_HAVERSINE) return haversine_f64(pi, qj);
    double s = 0.0;
    for (int k = 0; k < dim; ++k) {
        double t = (double)pi[k] - (double)qj[k];
        if (metric == FFDO_MANHATTAN) s += fabs(t);
        else if (metric == FFDO_CHEBYSHEV) s = fabs(t) > s ? fabs(t) : s;
        else s += t * t;
    }
    return metric == FFDO_EUCLIDEAN ? sqrt(s) : s;
}

/* Exact distance of integer points: squared Euclidean, Manhattan or
 * Chebyshev. */
static int64_t cell_i64(const int32_t *pi, const int32_t *qj, int dim, int metric)
{
    int64_t s = 0;
    for (int k = 0; k < dim; ++k) {
        int64_t t = (int64_t)pi[k] - (int64_t)qj[k];
        int64_t a = t < 0 ? -t : t;
        if (metric == FFDO_MANHATTAN) s += a;
        else if (metric == FFDO_CHEBYSHEV) s = a > s ? a : s;
        else s += t * t;
    }
    return s;
}

static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }
static int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

static int check_args(const void *p, int64_t n, const void *q, int64_t m, int dim,
                      int metric, const void *out)
{
    if (!p || !q || !out) return FFDO_EINVAL;
    if (n < 1 || m < 1 || dim < 1) return FFDO_EINVAL;
    if (metric < FFDO_EUCLIDEAN || metric > FFDO_HAVERSINE) return FFDO_EINVAL;
    if (metric == FFDO_HAVERSINE && dim != 2) return FFDO_EINVAL;
    return FFDO_OK;
}

/* ------------------------------------------- Algorithm 1: memoised recursion */

/* The paper marks "not yet computed" with M_ij = -1, which silently assumes
 * f >= 0; a separate visited flag per cell is used instead. */
struct memo {
    const float *p, *q;
    int64_t n, m;
    int dim, metric;
    double *M;
    unsigned char *seen;
};

static double memo_eval(struct memo *s, int64_t i, int64_t j) /* 1-based i, j */
{
    int64_t idx = (i - 1) * s->m + (j - 1);
    if (s->seen[idx]) return s->M[idx];
    double d = cell_f64(s->p + (i - 1) * s->dim, s->q + (j - 1) * s->dim, s->dim, s->metric);
    double v;
    if (i == 1 && j == 1)
        v = d;
    else if (i > 1 && j == 1)
        v = dmax(memo_eval(s, i - 1, 1), d);
    else if (i == 1 && j > 1)
        v = dmax(memo_eval(s, 1, j - 1), d);
    else
        v = dmax(dmin(dmin(memo_eval(s, i - 1, j), memo_eval(s, i - 1, j - 1)),
                      memo_eval(s, i, j - 1)),
                 d);
    s->M[idx] = v;
    s->seen[idx] = 1;
    return v;
}

struct memo_job { struct memo *s; double result; };

static void *memo_thread(void *arg)
{
    struct memo_job *job = (struct memo_job *)arg;
    job->result = memo_eval(job->s, job->s->n, job->s->m);
    return NULL;
}

/* Recursion depth is at most n + m; it runs on a thread with a stack sized
 * for that depth so that the recursion itself is what the paper describes. */
int ffdo_recursive(const float *p, int64_t n, const float *q, int64_t m, int dim,
                   int metric, double *out)
{
    int rc = check_args(p, n, q, m, dim, metric, out);
    if (rc) return rc;
    if (n * m > (int64_t)1 << 28) return FFDO_ENOMEM;
    struct memo s = {p, q, n, m, dim, metric, NULL, NULL};
    s.M = (double *)malloc((size_t)(n * m) * sizeof(double));
    s.seen = (unsigned char *)calloc((size_t)(n * m), 1);
    if (!s.M || !s.seen) { free(s.M); free(s.seen); return FFDO_ENOMEM; }
    struct memo_job job = {&s, 0.0};
    pthread_attr_t attr;
    pthread_attr_init(&attr);
    size_t stack = (size_t)(n + m + 64) * 256u + ((size_t)1 << 20);
    pthread_attr_setstacksize(&attr, stack);
    pthread_t th;
    if (pthread_create(&th, &attr, memo_thread, &job) != 0) {
        pthread_attr_destroy(&attr);
        free(s.M); free(s.seen);
        return FFDO_ENOMEM;
    }
    pthread_join(th, NULL);
    pthread_attr_destroy(&attr);
    free(s.M); free(s.seen);
    *out = job.result;
    return FFDO_OK;
}

/* ------------------------------------------- Algorithm 3: full-table iteration */

int ffdo_table(const float *p, int64_t n, const float *q, int64_t m, int dim, int metric,
               double *out)
{
    int rc = check_args(p, n, q, m, dim, metric, out);
    if (rc) return rc;
    if (n * m > (int64_t)1 << 28) return FFDO_ENOMEM;
    double *M = (double *)malloc((size_t)(n * m) * sizeof(double));
    if (!M) return FFDO_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double d = cell_f64(p + i * dim, q + j * dim, dim, metric);
            double v;
            if (i == 0 && j == 0)
                v = d;
            else if (i > 0 && j == 0)
                v = dmax(M[(i - 1) * m], d);
            else if (i == 0 && j > 0)
                v = dmax(M[j - 1], d);
            else
                v = dmax(dmin(dmin(M[(i - 1) * m + j], M[(i - 1) * m + j - 1]), M[i * m + j - 1]), d);
            M[i * m + j] = v;
        }
    }
    *out = M[n * m - 1];
    free(M);
    return FFDO_OK;
}

/* Full table written out, for tests that inspect M itself (row-major n x m). */
int ffdo_table_full(const float *p, int64_t n, const float *q, int64_t m, int dim,
                    int metric, double *M)
{
    int rc = check_args(p, n, q, m, dim, metric, M);
    if (rc) return rc;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j) {
            double d = cell_f64(p + i * dim, q + j * dim, dim, metric);
            double v;
            if (i == 0 && j == 0) v = d;
            else if (i > 0 && j == 0) v = dmax(M[(i - 1) * m], d);
            else if (i == 0 && j > 0) v = dmax(M[j - 1], d);
            else v = dmax(dmin(dmin(M[(i - 1) * m + j], M[(i - 1) * m + j - 1]), M[i * m + j - 1]), d);
            M[i * m + j] = v;
        }
    return FFDO_OK;
}

/* -------------------------------- Algorithm 3 keeping rows i-1 and i only */

static int rolling_f64(const float *p, int64_t n, const float *q, int64_t m, int dim,
                       int metric, double *out, double *prev, double *cur)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double d = cell_f64(p + i * dim, q + j * dim, dim, metric);
            double v;
            if (i == 0 && j == 0) v = d;
            else if (i > 0 && j == 0) v = dmax(prev[0], d);
            else if (i == 0 && j > 0) v = dmax(cur[j - 1], d);
            else v = dmax(dmin(dmin(prev[j], prev[j - 1]), cur[j - 1]), d);
            cur[j] = v;
        }
        double *t = prev; prev = cur; cur = t;
    }
    *out = prev[m - 1];
    return FFDO_OK;
}

int ffdo_rolling(const float *p, int64_t n, const float *q, int64_t m, int dim, int metric,
                 double *out)
{
    int rc = check_args(p, n, q, m, dim, metric, out);
    if (rc) return rc;
    double *buf = (double *)malloc((size_t)(2 * m) * sizeof(double));
    if (!buf) return FFDO_ENOMEM;
    rc = rolling_f64(p, n, q, m, dim, metric, out, buf, buf + m);
    free(buf);
    return rc;
}

/* Rolling form run for the first `rows` rows only, returning the live row:
 * the whole DP state after row `rows` (Theorem 1's O(Q) memory claim). */
int ffdo_rolling_state(const float *p, int64_t rows, const float *q, int64_t m, int dim,
                       int metric, double *row_out)
{
    int rc = check_args(p, rows, q, m, dim, metric, row_out);
    if (rc) return rc;
    double *buf = (double *)malloc((size_t)(2 * m) * sizeof(double));
    if (!buf) return FFDO_ENOMEM;
    double *prev = buf, *cur = buf + m;
    for (int64_t i = 0; i < rows; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double d = cell_f64(p + i * dim, q + j * dim, dim, metric);
            double v;
            if (i == 0 && j == 0) v = d;
            else if (i > 0 && j == 0) v = dmax(prev[0], d);
            else if (i == 0 && j > 0) v = dmax(cur[j - 1], d);
            else v = dmax(dmin(dmin(prev[j], prev[j - 1]), cur[j - 1]), d);
            cur[j] = v;
        }
        double *t = prev; prev = cur; cur = t;
    }
    memcpy(row_out, prev, (size_t)m * sizeof(double));
    free(buf);
    return FFDO_OK;
}

/* Resume the rolling form from a saved row: rows [row0, n) of p given the
 * state after row row0 (row0 >= 1). */
int ffdo_rolling_resume(const float *p, int64_t row0, int64_t n, const float *q, int64_t m,
                        int dim, int metric, const double *row_in, double *out)
{
    int rc = check_args(p, n, q, m, dim, metric, out);
    if (rc) return rc;
    if (row0 < 1 || row0 > n || !row_in) return FFDO_EINVAL;
    double *buf = (double *)malloc((size_t)(2 * m) * sizeof(double));
    if (!buf) return FFDO_ENOMEM;
    double *prev = buf, *cur = buf + m;
    memcpy(prev, row_in, (size_t)m * sizeof(double));
    for (int64_t i = row0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double d = cell_f64(p + i * dim, q + j * dim, dim, metric);
            double v = (j == 0) ? dmax(prev[0], d)
                                : dmax(dmin(dmin(prev[j], prev[j - 1]), cur[j - 1]), d);
            cur[j] = v;
        }
        double *t = prev; prev = cur; cur = t;
    }
    *out = prev[m - 1];
    free(buf);
    return FFDO_OK;
}

/* ------------------------------------------------------ exact integer version */

static int rolling_i64(const int32_t *p, int64_t n, const int32_t *q, int64_t m, int dim,
                       int metric, int64_t *out, int64_t *prev, int64_t *cur)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            int64_t d = cell_i64(p + i * dim, q + j * dim, dim, metric);
            int64_t v;
            if (i == 0 && j == 0) v = d;
            else if (i > 0 && j == 0) v = imax(prev[0], d);
            else if (i == 0 && j > 0) v = imax(cur[j - 1], d);
            else v = imax(imin(imin(prev[j], prev[j - 1]), cur[j - 1]), d);
            cur[j] = v;
        }
        int64_t *t = prev; prev = cur; cur = t;
    }
    *out = prev[m - 1];
    return FFDO_OK;
}

/* Discrete Frechet distance of int32 curves, exact int64; metric is
 * SQEUCLIDEAN, MANHATTAN or CHEBYSHEV. */
int ffdo_i32(const int32_t *p, int64_t n, const int32_t *q, int64_t m, int dim, int metric, int64_t *out)
{
    int rc = check_args(p, n, q, m, dim, metric, out);
    if (rc) return rc;
    if (metric == FFDO_EUCLIDEAN || metric == FFDO_HAVERSINE) return FFDO_EINVAL;
    int64_t *buf = (int64_t *)malloc((size_t)(2 * m) * sizeof(int64_t));
    if (!buf) return FFDO_ENOMEM;
    rc = rolling_i64(p, n, q, m, dim, metric, out, buf, buf + m);
    free(buf);
    return rc;
}

/* ------------------------------------------- dynamic time warping (App. B) */

/* Rows i-1 and i of the DTW table: the DFD recurrence with max{., d}
 * replaced by . + d. */
static int dtw_rolling_f64(const float *p, int64_t n, const float *q, int64_t m, int dim,
                           int metric, double *out, double *prev, double *cur)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double d = cell_f64(p + i * dim, q + j * dim, dim, metric);
            double v;
            if (i == 0 && j == 0) v = d;
            else if (i > 0 && j == 0) v = prev[0] + d;
            else if (i == 0 && j > 0) v = cur[j - 1] + d;
            else v = dmin(dmin(prev[j], prev[j - 1]), cur[j - 1]) + d;
            cur[j] = v;
        }
        double *t = prev; prev = cur; cur = t;
    }
    *out = prev[m - 1];
    return FFDO_OK;
}

static int dtw_rolling_i64(const int32_t *p, int64_t n, const int32_t *q, int64_t m, int dim,
                           int metric, int64_t *out, int64_t *prev, int64_t *cur)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            int64_t d = cell_i64(p + i * dim, q + j * dim, dim, metric);
            int64_t v;
            if (i == 0 && j == 0) v = d;
            else if (i > 0 && j == 0) v = prev[0] + d;
            else if (i == 0 && j > 0) v = cur[j - 1] + d;
            else v = imin(imin(prev[j], prev[j - 1]), cur[j - 1]) + d;
            cur[j] = v;
        }
        int64_t *t = prev; prev = cur; cur = t;
    }
    *out = prev[m - 1];
    return FFDO_OK;
}

/* DTW of two float32 curves in FP64. */
int ffdo_dtw(const float *p, int64_t n, const float *q, int64_t m, int dim, int metric,
             double *out)
{
    int rc = check_args(p, n, q, m, dim, metric, out);
    if (rc) return rc;
    double *buf = (double *)malloc((size_t)(2 * m) * sizeof(double));
    if (!buf) return FFDO_ENOMEM;
    rc = dtw_rolling_f64(p, n, q, m, dim, metric, out, buf, buf + m);
    free(buf);
    return rc;
}

/* DTW of int32 curves, exact int64 (the caller keeps the sums below
 * 2^63); metric is SQEUCLIDEAN, MANHATTAN or CHEBYSHEV. */
int ffdo_dtw_i32(const int32_t *p, int64_t n, const int32_t *q, int64_t m, int dim, int metric, int64_t *out)
{
    int rc = check_args(p, n, q, m, dim, metric, out);
    if (rc) return rc;
    if (metric == FFDO_EUCLIDEAN || metric == FFDO_HAVERSINE) return FFDO_EINVAL;
    int64_t *buf = (int64_t *)malloc((size_t)(2 * m) * sizeof(int64_t));
    if (!buf) return FFDO_ENOMEM;
    rc = dtw_rolling_i64(p, n, q, m, dim, metric, out, buf, buf + m);
    free(buf);
    return rc;
}

/* ---------------------------------------- Levenshtein distance (App. B) */

static int sym_ne(const int32_t *pi, const int32_t *qj, int dim)
{
    for (int k = 0; k < dim; ++k)
        if (pi[k] != qj[k]) return 1;
    return 0;
}

/* Rows i-1 and i of the Levenshtein table. */
static int lev_rolling(const int32_t *p, int64_t n, const int32_t *q, int64_t m, int dim,
                       int64_t *out, int64_t *prev, int64_t *cur)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            int64_t d = sym_ne(p + i * dim, q + j * dim, dim);
            int64_t up = i > 0 ? prev[j] : j + 1;         /* M_{i-1,j}   */
            int64_t left = j > 0 ? cur[j - 1] : i + 1;    /* M_{i,j-1}   */
            int64_t diag = i > 0 ? (j > 0 ? prev[j - 1] : i) : j; /* M_{i-1,j-1} */
            cur[j] = imin(imin(up + 1, left + 1), diag + d);
        }
        int64_t *t = prev; prev = cur; cur = t;
    }
    *out = prev[m - 1];
    return FFDO_OK;
}

/* Levenshtein distance of two int32 symbol sequences (dim coordinates per
 * symbol). */
int ffdo_lev(const int32_t *p, int64_t n, const int32_t *q, int64_t m, int dim, int64_t *out)
{
    int rc = check_args(p, n, q, m, dim, FFDO_SQEUCLIDEAN, out);
    if (rc) return rc;
    int64_t *buf = (int64_t *)malloc((size_t)(2 * m) * sizeof(int64_t));
    if (!buf) return FFDO_ENOMEM;
    rc = lev_rolling(p, n, q, m, dim, out, buf, buf + m);
    free(buf);
    return rc;
}

/* ----------------------------------------------------------- float replica */

/* Float32 replica of one fixed evaluation order: d2 = dx*dx, then
 * d2 = fmaf(dk, dk, d2) for k = 1..D-1, recurrence in float32, and for
 * EUCLIDEAN one correctly rounded square root of the selected d2 at the end
 * (min and max commute with the monotone square root).  Used only to check
 * that a float32 implementation of that order selects the same cell. */
static float cell_f32_replica(const float *pi, const float *qj, int dim, int metric)
{
    float dx = pi[0] - qj[0];
    if (metric == FFDO_MANHATTAN || metric == FFDO_CHEBYSHEV) {
        /* s = |dx|, then s = s + |dk| (Manhattan) or max(s, |dk|) */
        float a = fabsf(dx);
        for (int k = 1; k < dim; ++k) {
            float t = fabsf(pi[k] - qj[k]);
            a = metric == FFDO_MANHATTAN ? a + t : fmaxf(a, t);
        }
        return a;
    }
    float s = dx * dx;
    for (int k = 1; k < dim; ++k) {
        float t = pi[k] - qj[k];
        s = fmaf(t, t, s);
    }
    return s;
}

int ffdo_f32_replica(const float *p, int64_t n, const float *q, int64_t m, int dim,
                     int metric, float *out)
{
    int rc = check_args(p, n, q, m, dim, metric, out);
    if (rc) return rc;
    if (metric == FFDO_HAVERSINE) return FFDO_EINVAL;
    float *buf = (float *)malloc((size_t)(2 * m) * sizeof(float));
    if (!buf) return FFDO_ENOMEM;
    float *prev = buf, *cur = buf + m;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            float d = cell_f32_replica(p + i * dim, q + j * dim, dim, metric);
            float v;
            if (i == 0 && j == 0) v = d;
            else if (i > 0 && j == 0) v = fmaxf(prev[0], d);
            else if (i == 0 && j > 0) v = fmaxf(cur[j - 1], d);
            else v = fmaxf(fminf(fminf(prev[j], prev[j - 1]), cur[j - 1]), d);
            cur[j] = v;
        }
        float *t = prev; prev = cur; cur = t;
    }
    float r = prev[m - 1];
    *out = metric == FFDO_EUCLIDEAN ? (float)sqrt((double)r) : r;
    free(buf);
    return FFDO_OK;
}

/* Float32 replica of DTW in one fixed order: the cell distance as above,
 * then (EUCLIDEAN) its correctly rounded float32 square root, then
 * v = fminf(fminf(...)) + d in float32.  Minima are exact, so only the
 * order of the additions along the selected path matters, and that order is
 * fixed by the recurrence. */
int ffdo_dtw_f32_replica(const float *p, int64_t n, const float *q, int64_t m, int dim,
                         int metric, float *out)
{
    int rc = check_args(p, n, q, m, dim, metric, out);
    if (rc) return rc;
    if (metric == FFDO_HAVERSINE) return FFDO_EINVAL;
    float *buf = (float *)malloc((size_t)(2 * m) * sizeof(float));
    if (!buf) return FFDO_ENOMEM;
    float *prev = buf, *cur = buf + m;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            float d = cell_f32_replica(p + i * dim, q + j * dim, dim, metric);
            if (metric == FFDO_EUCLIDEAN) d = sqrtf(d);
            float v;
            if (i == 0 && j == 0) v = d;
            else if (i > 0 && j == 0) v = prev[0] + d;
            else if (i == 0 && j > 0) v = cur[j - 1] + d;
            else v = fminf(fminf(prev[j], prev[j - 1]), cur[j - 1]) + d;
            cur[j] = v;
        }
        float *t = prev; prev = cur; cur = t;
    }
    *out = prev[m - 1];
    free(buf);
    return FFDO_OK;
}

/* ------------------------------------------------ many pairs on a thread pool */

/* Pair k is P[p_start[k] .. p_start[k]+p_len[k]) against
 * Q[q_start[k] .. q_start[k]+q_len[k]) (starts and lengths in points).  Each
 * pair runs the rolling form; pairs are handed to `nthreads` workers in the
 * order of `order` (NULL = natural order), so that a longest-first order can
 * be used.  out[k] receives pair k's distance. */
struct pool_ctx {
    const void *P, *Q;
    const int64_t *p_start, *p_len, *q_start, *q_len;
    const int64_t *order;
    int64_t npairs;
    int dim, metric, is_int;
    int dtw;               /* 0: discrete Frechet distance, 1: DTW, 2: Levenshtein (int) */
    void *out;
    int64_t next;
    pthread_mutex_t mu;
    int error;
};

static void *pool_worker(void *arg)
{
    struct pool_ctx *c = (struct pool_ctx *)arg;
    size_t cap = 0;
    void *buf = NULL;
    for (;;) {
        pthread_mutex_lock(&c->mu);
        int64_t t = c->next++;
        pthread_mutex_unlock(&c->mu);
        if (t >= c->npairs) break;
        int64_t k = c->order ? c->order[t] : t;
        int64_t n = c->p_len[k];
        int64_t m = c->q_len[k];
        if (n < 1 || m < 1) { c->error = FFDO_EINVAL; continue; }
        size_t need = (size_t)(2 * m) * 8u;
        if (need > cap) {
            free(buf);
            buf = malloc(need);
            cap = need;
            if (!buf) { c->error = FFDO_ENOMEM; cap = 0; continue; }
        }
        if (c->is_int) {
            const int32_t *P = (const int32_t *)c->P, *Q = (const int32_t *)c->Q;
            int64_t *b = (int64_t *)buf;
            if (c->dtw == 2)
                lev_rolling(P + c->p_start[k] * c->dim, n, Q + c->q_start[k] * c->dim, m, c->dim,
                            (int64_t *)c->out + k, b, b + m);
            else
                (c->dtw ? dtw_rolling_i64 : rolling_i64)(P + c->p_start[k] * c->dim, n,
                                                         Q + c->q_start[k] * c->dim, m, c->dim,
                                                         c->metric, (int64_t *)c->out + k, b, b + m);
        } else {
            const float *P = (const float *)c->P, *Q = (const float *)c->Q;
            double *b = (double *)buf;
            (c->dtw ? dtw_rolling_f64 : rolling_f64)(P + c->p_start[k] * c->dim, n,
                                                     Q + c->q_start[k] * c->dim, m, c->dim,
                                                     c->metric, (double *)c->out + k, b, b + m);
        }
    }
    free(buf);
    return NULL;
}

static int run_pool(struct pool_ctx *c, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    pthread_mutex_init(&c->mu, NULL);
    c->next = 0;
    c->error = FFDO_OK;
    int started = 0;
    for (int i = 0; i < nthreads; ++i)
        if (pthread_create(&th[i], NULL, pool_worker, c) == 0) ++started;
    if (started == 0) pool_worker(c);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&c->mu);
    return c->error;
}

static int pool_args(const void *P, const void *Q, const int64_t *ps, const int64_t *pl,
                     const int64_t *qs, const int64_t *ql, int64_t npairs, int dim,
                     const void *out)
{
    if (!P || !Q || !ps || !pl || !qs || !ql || !out || npairs < 0 || dim < 1)
        return FFDO_EINVAL;
    return FFDO_OK;
}

static int pairs_f32(const float *P, const int64_t *p_start, const int64_t *p_len, const float *Q,
                     const int64_t *q_start, const int64_t *q_len, int64_t npairs, int dim,
                     int metric, const int64_t *order, int nthreads, double *out, int dtw)
{
    int rc = pool_args(P, Q, p_start, p_len, q_start, q_len, npairs, dim, out);
    if (rc) return rc;
    if (metric < FFDO_EUCLIDEAN || metric > FFDO_HAVERSINE) return FFDO_EINVAL;
    if (metric == FFDO_HAVERSINE && dim != 2) return FFDO_EINVAL;
    struct pool_ctx c;
    memset(&c, 0, sizeof c);
    c.P = P; c.Q = Q; c.p_start = p_start; c.p_len = p_len; c.q_start = q_start;
    c.q_len = q_len; c.order = order; c.npairs = npairs; c.dim = dim; c.metric = metric;
    c.is_int = 0; c.dtw = dtw; c.out = out;
    return run_pool(&c, nthreads);
}

static int pairs_i32(const int32_t *P, const int64_t *p_start, const int64_t *p_len,
                     const int32_t *Q, const int64_t *q_start, const int64_t *q_len,
                     int64_t npairs, int dim, int metric, const int64_t *order, int nthreads,
                     int64_t *out, int dtw)
{
    int rc = pool_args(P, Q, p_start, p_len, q_start, q_len, npairs, dim, out);
    if (rc) return rc;
    if (metric < FFDO_SQEUCLIDEAN || metric > FFDO_CHEBYSHEV) return FFDO_EINVAL;
    struct pool_ctx c;
    memset(&c, 0, sizeof c);
    c.P = P; c.Q = Q; c.p_start = p_start; c.p_len = p_len; c.q_start = q_start;
    c.q_len = q_len; c.order = order; c.npairs = npairs; c.dim = dim;
    c.metric = metric; c.is_int = 1; c.dtw = dtw; c.out = out;
    return run_pool(&c, nthreads);
}

int ffdo_pairs(const float *P, const int64_t *p_start, const int64_t *p_len, const float *Q,
               const int64_t *q_start, const int64_t *q_len, int64_t npairs, int dim,
               int metric, const int64_t *order, int nthreads, double *out)
{
    return pairs_f32(P, p_start, p_len, Q, q_start, q_len, npairs, dim, metric, order, nthreads,
                     out, 0);
}

int ffdo_pairs_i32(const int32_t *P, const int64_t *p_start, const int64_t *p_len,
                   const int32_t *Q, const int64_t *q_start, const int64_t *q_len,
                   int64_t npairs, int dim, int metric, const int64_t *order, int nthreads,
                   int64_t *out)
{
    return pairs_i32(P, p_start, p_len, Q, q_start, q_len, npairs, dim, metric, order, nthreads, out, 0);
}

int ffdo_dtw_pairs(const float *P, const int64_t *p_start, const int64_t *p_len, const float *Q,
                   const int64_t *q_start, const int64_t *q_len, int64_t npairs, int dim,
                   int metric, const int64_t *order, int nthreads, double *out)
{
    return pairs_f32(P, p_start, p_len, Q, q_start, q_len, npairs, dim, metric, order, nthreads,
                     out, 1);
}

int ffdo_lev_pairs(const int32_t *P, const int64_t *p_start, const int64_t *p_len,
                   const int32_t *Q, const int64_t *q_start, const int64_t *q_len,
                   int64_t npairs, int dim, const int64_t *order, int nthreads, int64_t *out)
{
    return pairs_i32(P, p_start, p_len, Q, q_start, q_len, npairs, dim, FFDO_SQEUCLIDEAN, order, nthreads,
                     out, 2);
}

int ffdo_dtw_pairs_i32(const int32_t *P, const int64_t *p_start, const int64_t *p_len,
                       const int32_t *Q, const int64_t *q_start, const int64_t *q_len,
                       int64_t npairs, int dim, int metric, const int64_t *order, int nthreads,
                       int64_t *out)
{
    return pairs_i32(P, p_start, p_len, Q, q_start, q_len, npairs, dim, metric, order, nthreads, out, 1);
}

/* Seconds on the monotonic clock, for the CPU-baseline timer. */
double ffdo_now(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

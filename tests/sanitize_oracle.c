/* The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built and run by tests/test_sanitizers.py): every oracle form on seeded
 * random walks and integer sequences of ragged sizes (one-point curves,
 * D = 1 ... 4), the pair pool on several threads, and the checkpoint of the
 * live row; the forms must agree with each other (the table, rolling and
 * memoised recursive forms exactly), and the sanitizers must report
 * nothing. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int ffdo_recursive(const float *p, int64_t n, const float *q, int64_t m, int dim, int metric, double *out);
int ffdo_table(const float *p, int64_t n, const float *q, int64_t m, int dim, int metric, double *out);
int ffdo_rolling(const float *p, int64_t n, const float *q, int64_t m, int dim, int metric, double *out);
int ffdo_rolling_state(const float *p, int64_t rows, const float *q, int64_t m, int dim, int metric,
                       double *row_out);
int ffdo_rolling_resume(const float *p, int64_t row0, int64_t n, const float *q, int64_t m, int dim, int metric,
                        const double *row_in, double *out);
int ffdo_f32_replica(const float *p, int64_t n, const float *q, int64_t m, int dim, int metric, float *out);
int ffdo_dtw(const float *p, int64_t n, const float *q, int64_t m, int dim, int metric, double *out);
int ffdo_dtw_f32_replica(const float *p, int64_t n, const float *q, int64_t m, int dim, int metric, float *out);
int ffdo_i32(const int32_t *p, int64_t n, const int32_t *q, int64_t m, int dim, int metric, int64_t *out);
int ffdo_dtw_i32(const int32_t *p, int64_t n, const int32_t *q, int64_t m, int dim, int metric, int64_t *out);
int ffdo_lev(const int32_t *p, int64_t n, const int32_t *q, int64_t m, int dim, int64_t *out);
int ffdo_pairs(const float *P, const int64_t *p_start, const int64_t *p_len, const float *Q,
               const int64_t *q_start, const int64_t *q_len, int64_t npairs, int dim, int metric,
               const int64_t *order, int nthreads, double *out);

static uint64_t rng = 88172645463325252ull;
static double unif(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (double)(rng >> 11) / 9007199254740992.0;
}

static float *walk(int64_t n, int dim) {
  float *x = (float *)malloc((size_t)(n * dim) * sizeof(float));
  for (int k = 0; k < dim; ++k) x[k] = (float)(unif() * 4 - 2);
  for (int64_t i = 1; i < n; ++i)
    for (int k = 0; k < dim; ++k) x[i * dim + k] = x[(i - 1) * dim + k] + (float)(unif() * 2 - 1);
  return x;
}

static int fails = 0;
#define CHECK(c, ...)                     \
  do {                                    \
    if (!(c)) {                           \
      fprintf(stderr, __VA_ARGS__);       \
      fprintf(stderr, "\n");              \
      ++fails;                            \
    }                                     \
  } while (0)

int main(void) {
  const int64_t lens[] = {1, 2, 3, 17, 64, 65, 130, 257};
  const int nl = (int)(sizeof lens / sizeof lens[0]);
  int cases = 0;
  for (int dim = 1; dim <= 4; ++dim)
    for (int a = 0; a < nl; ++a)
      for (int b = 0; b < nl; b += 2) {
        const int64_t n = lens[a], m = lens[(a + b) % nl];
        float *p = walk(n, dim), *q = walk(m, dim);
        for (int metric = 0; metric <= 3; ++metric) {
          double t = 0, r = 0, rec = 0, dt = 0;
          CHECK(ffdo_table(p, n, q, m, dim, metric, &t) == 0, "table %lld %lld", (long long)n, (long long)m);
          CHECK(ffdo_rolling(p, n, q, m, dim, metric, &r) == 0, "rolling");
          CHECK(t == r, "table %.17g != rolling %.17g (n %lld m %lld D %d metric %d)", t, r, (long long)n,
                (long long)m, dim, metric);
          if (n * m <= 4096) {
            CHECK(ffdo_recursive(p, n, q, m, dim, metric, &rec) == 0, "recursive");
            CHECK(rec == t, "recursive %.17g != table %.17g", rec, t);
          }
          CHECK(ffdo_dtw(p, n, q, m, dim, metric, &dt) == 0, "dtw");
          CHECK(dt >= t - 1e-12 * fabs(t), "dtw %.17g below the Frechet distance %.17g", dt, t);
          if (metric <= 1) {
            float f = 0, fd = 0;
            CHECK(ffdo_f32_replica(p, n, q, m, dim, metric, &f) == 0, "replica");
            CHECK(fabs((double)f - t) <= 1e-5 * fabs(t) + 1e-6, "replica %.9g vs table %.17g", f, t);
            CHECK(ffdo_dtw_f32_replica(p, n, q, m, dim, metric, &fd) == 0, "dtw replica");
          }
          if (n > 2) {
            // checkpoint after row n / 2, then resume: the same value
            double *row = (double *)malloc((size_t)m * sizeof(double)), res = 0;
            CHECK(ffdo_rolling_state(p, n / 2, q, m, dim, metric, row) == 0, "state");
            CHECK(ffdo_rolling_resume(p, n / 2, n, q, m, dim, metric, row, &res) == 0, "resume");
            CHECK(res == t, "resume %.17g != %.17g", res, t);
            free(row);
          }
          ++cases;
        }
        // integer forms on the rounded coordinates
        int32_t *pi = (int32_t *)malloc((size_t)(n * dim) * sizeof(int32_t));
        int32_t *qi = (int32_t *)malloc((size_t)(m * dim) * sizeof(int32_t));
        for (int64_t i = 0; i < n * dim; ++i) pi[i] = (int32_t)lrintf(p[i] * 8);
        for (int64_t i = 0; i < m * dim; ++i) qi[i] = (int32_t)lrintf(q[i] * 8) % 4;
        int64_t fi = 0, di = 0, lv = 0;
        CHECK(ffdo_i32(pi, n, qi, m, dim, 1, &fi) == 0, "i32");
        CHECK(ffdo_dtw_i32(pi, n, qi, m, dim, 1, &di) == 0, "dtw i32");
        CHECK(di >= fi, "int dtw below Frechet");
        CHECK(ffdo_lev(pi, n, qi, m, dim, &lv) == 0, "lev");
        CHECK(lv >= (n > m ? n - m : m - n) && lv <= (n > m ? n : m), "levenshtein %lld out of its bounds",
              (long long)lv);
        free(pi);
        free(qi);
        free(p);
        free(q);
      }
  // the pair pool on three threads against single calls
  enum { NP = 40 };
  int64_t ps[NP], pl[NP], qs[NP], ql[NP], tot_p = 0, tot_q = 0;
  for (int k = 0; k < NP; ++k) {
    pl[k] = 1 + (int64_t)(unif() * 200);
    ql[k] = 1 + (int64_t)(unif() * 200);
    ps[k] = tot_p;
    qs[k] = tot_q;
    tot_p += pl[k];
    tot_q += ql[k];
  }
  float *P = walk(tot_p, 2), *Q = walk(tot_q, 2);
  double out[NP];
  CHECK(ffdo_pairs(P, ps, pl, Q, qs, ql, NP, 2, 0, NULL, 3, out) == 0, "pairs");
  for (int k = 0; k < NP; ++k) {
    double t = 0;
    ffdo_table(P + ps[k] * 2, pl[k], Q + qs[k] * 2, ql[k], 2, 0, &t);
    CHECK(t == out[k], "pair %d: pool %.17g != single %.17g", k, out[k], t);
  }
  free(P);
  free(Q);
  // refused arguments
  double x = 0;
  float one[4] = {0, 0, 0, 0};
  CHECK(ffdo_table(one, 0, one, 1, 1, 0, &x) != 0, "n = 0 accepted");
  CHECK(ffdo_table(NULL, 1, one, 1, 1, 0, &x) != 0, "NULL accepted");
  CHECK(ffdo_table(one, 1, one, 1, 1, 9, &x) != 0, "unknown metric accepted");
  if (fails) {
    printf("FAILED %d checks\n", fails);
    return 1;
  }
  printf("ok %d cases\n", cases);
  return 0;
}

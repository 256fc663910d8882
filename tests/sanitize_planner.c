/* The library's host planner under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by tests/test_sanitizers.py):
 * a planning-only context plans batches of seeded ragged lengths with
 * every tuning knob, forced band splitting, cross requests, single pairs
 * (pipelined and not), the other measures, workspace and scratch sizes,
 * and reads an autotune cache file; each plan's job table is read back in
 * full.  Exits 0 when every call returns the expected status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ffd.h"

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static int64_t lenu(int64_t lo, int64_t hi) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return lo + (int64_t)(rng % (uint64_t)(hi - lo + 1));
}

static int fails = 0;
#define EXPECT(c, what)                               \
  do {                                                \
    if (!(c)) {                                       \
      fprintf(stderr, "failed: %s\n", what);          \
      ++fails;                                        \
    }                                                 \
  } while (0)

static void offsets(int64_t *off, int64_t n, int64_t lo, int64_t hi) {
  off[0] = 0;
  for (int64_t k = 0; k < n; ++k) off[k + 1] = off[k] + lenu(lo, hi);
}

/* plan, then read the whole job table back */
static int describe(ffd_ctx *c, int op, const int64_t *a, int64_t na, const int64_t *b, int64_t nb, int dim,
                    int exact, int measure, int metric) {
  ffd_plan_summary sm;
  int rc = ffd_plan_describe(c, op, a, na, b, nb, dim, exact, measure, metric, &sm, NULL, 0, NULL, 0);
  if (rc != FFD_OK && rc != FFD_E_NOMEM) return rc;
  ffd_plan_job *jobs = (ffd_plan_job *)malloc(sizeof(ffd_plan_job) * (size_t)(sm.jobs + 1));
  int32_t *wj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(sm.waves + 1));
  rc = ffd_plan_describe(c, op, a, na, b, nb, dim, exact, measure, metric, &sm, jobs, sm.jobs, wj, sm.waves + 1);
  if (rc == FFD_OK && !sm.pipelined) {
    for (int32_t w = 0; w < sm.waves; ++w)
      if (wj[w] > wj[w + 1] || wj[w + 1] > sm.jobs) rc = -100;
  }
  free(jobs);
  free(wj);
  return rc;
}

int main(void) {
  ffd_ctx *c = NULL;
  EXPECT(ffd_create_planner(256, 160 * 1024, &c) == FFD_OK, "planner");
  enum { NP = 700 };
  int64_t *p = (int64_t *)malloc(sizeof(int64_t) * (NP + 1)), *q = (int64_t *)malloc(sizeof(int64_t) * (NP + 1));
  offsets(p, NP, 1, 2600);
  offsets(q, NP, 1, 2600);
  const int Rs[] = {0, 1, 2, 4, 8};
  const int Ws[] = {0, 1, 2, 3};
  const float splits[] = {0.f, 1e-9f, -1.f, 1.5f};
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 4; ++j)
      for (int s = 0; s < 4; ++s) {
        EXPECT(ffd_set_tuning(c, Rs[i], Ws[j]) == FFD_OK, "tuning");
        EXPECT(ffd_set_split(c, splits[s]) == FFD_OK, "split");
        for (int dim = 1; dim <= 4; dim += 3)
          EXPECT(describe(c, FFD_OP_BATCH, p, NP, q, NP, dim, 0, 0, 0) == FFD_OK, "batch plan");
      }
  ffd_set_tuning(c, 0, 0);
  ffd_set_split(c, 0.f);
  /* curves of 5 to 16 coordinates: the wide kernels' one rows-per-lane each */
  for (int dim = 5; dim <= 16; dim += 11) {
    EXPECT(describe(c, FFD_OP_BATCH, p, NP, q, NP, dim, 0, 0, 0) == FFD_OK, "wide batch plan");
    EXPECT(describe(c, FFD_OP_BATCH, p, NP, q, NP, dim, 1, 0, 1) == FFD_OK, "wide exact batch plan");
    EXPECT(describe(c, FFD_OP_CROSS, p, 30, q, 400, dim, 0, 1, 0) == FFD_OK, "wide dtw cross plan");
  }
  ffd_set_tuning(c, 4, 0);
  EXPECT(describe(c, FFD_OP_BATCH, p, NP, q, NP, 6, 0, 0, 0) == FFD_E_UNSUPPORTED, "wide shape other than its R");
  ffd_set_tuning(c, 0, 0);
  /* cross: 30 queries x 400 curves, float and exact */
  EXPECT(describe(c, FFD_OP_CROSS, p, 30, q, 400, 2, 0, 0, 0) == FFD_OK, "cross plan");
  EXPECT(describe(c, FFD_OP_CROSS, p, 30, q, 400, 2, 1, 0, 1) == FFD_OK, "exact cross plan");
  /* single pairs: long ones on the pipelined kernel, forced and not */
  const int64_t shapes[][2] = {{131072, 131072}, {5000, 3}, {300, 20000}, {100, 90}, {1, 1}, {1, 7000}};
  for (int k = 0; k < 6; ++k) {
    int64_t a[2] = {0, shapes[k][0]}, b[2] = {0, shapes[k][1]};
    for (int w = -1; w <= 0; ++w) {
      ffd_set_tuning(c, 0, w);
      EXPECT(describe(c, FFD_OP_PAIR, a, 1, b, 1, 3, 0, 0, 0) == FFD_OK, "pair plan");
      EXPECT(describe(c, FFD_OP_PAIR, a, 1, b, 1, 2, 1, 0, 1) == FFD_OK, "exact pair plan");
      EXPECT(describe(c, FFD_OP_PAIR, a, 1, b, 1, 11, 0, 0, 0) == FFD_OK, "wide pair plan");
    }
  }
  ffd_set_tuning(c, 0, 0);
  /* other measures: DTW on both cells, Manhattan, Chebyshev, Levenshtein */
  EXPECT(describe(c, FFD_OP_BATCH, p, 200, q, 200, 2, 0, 1, 0) == FFD_OK, "dtw plan");
  EXPECT(describe(c, FFD_OP_BATCH, p, 200, q, 200, 2, 0, 1, 1) == FFD_OK, "dtw squared plan");
  EXPECT(describe(c, FFD_OP_BATCH, p, 200, q, 200, 2, 0, 0, FFD_MANHATTAN) == FFD_OK, "manhattan plan");
  EXPECT(describe(c, FFD_OP_BATCH, p, 200, q, 200, 2, 0, 0, FFD_CHEBYSHEV) == FFD_OK, "chebyshev plan");
  EXPECT(describe(c, FFD_OP_BATCH, p, 200, q, 200, 1, 1, 2, 0) == FFD_OK, "levenshtein plan");
  EXPECT(describe(c, FFD_OP_BATCH, p, 200, q, 200, 2, 0, 0, FFD_HAVERSINE) == FFD_OK, "great-circle plan");
  /* refused requests */
  EXPECT(describe(c, FFD_OP_BATCH, p, 0, q, 0, 2, 0, 0, 0) == FFD_E_INVALID, "empty batch refused");
  EXPECT(describe(c, 99, p, 2, q, 2, 2, 0, 0, 0) == FFD_E_INVALID, "unknown op refused");
  EXPECT(describe(c, FFD_OP_BATCH, p, 2, q, 2, 17, 0, 0, 0) == FFD_E_UNSUPPORTED, "dim 17 refused");
  /* sizes of every op */
  size_t bytes = 0;
  const int ops[] = {FFD_OP_BATCH, FFD_OP_CROSS, FFD_OP_DECIDE, FFD_OP_KNN};
  for (int k = 0; k < 4; ++k) {
    int64_t na = ops[k] == FFD_OP_CROSS || ops[k] == FFD_OP_KNN ? 5 : NP;
    EXPECT(ffd_workspace_size(c, ops[k], p, na, q, NP, 2, &bytes) == FFD_OK && bytes > 0, "size");
  }
  int64_t a1[2] = {0, 90000}, b1[2] = {0, 70000};
  EXPECT(ffd_workspace_size(c, FFD_OP_PAIR, a1, 1, b1, 1, 2, &bytes) == FFD_OK && bytes > 0, "pair scratch");
  /* an autotune cache file with a good line, a broken one and junk */
  const char *path = "sanitize_tune.json";
  FILE *f = fopen(path, "w");
  if (f) {
    fprintf(f, "{\n\"gfx950/cu256/op1/k0/f32/D2/L10/M10/N9/Q9\": {\"rows_per_lane\": 4, \"waves_per_simd\": 1, "
               "\"split\": 0},\n\"broken\n\"x\": {\"rows_per_lane\": 99}\n}\n");
    fclose(f);
  }
  EXPECT(ffd_set_tune_cache(c, path) == FFD_OK, "tune cache");
  EXPECT(describe(c, FFD_OP_BATCH, p, NP, q, NP, 2, 0, 0, 0) == FFD_OK, "batch plan with a cache");
  EXPECT(ffd_set_tune_cache(c, NULL) == FFD_OK, "no cache");
  remove(path);
  ffd_destroy(c);
  free(p);
  free(q);
  if (fails) {
    printf("FAILED %d checks\n", fails);
    return 1;
  }
  printf("ok\n");
  return 0;
}

// Decider and k-nearest-neighbour search on the early-abandoning sweep
// (ffd_bounded.hip): host-side checks, scratch management and the two-stage
// search.
//
// k nearest neighbours of a query q in a database of curves:
//   1. a lower bound per database curve, the larger of the squared
//      first-point and last-point distances (every coupling contains both
//      corner cells), computed on the GPU;
//   2. exact squared distances of 128 curves (at least k) with the smallest
//      bounds, among curves of moderate length: the k-th smallest is the
//      threshold tau;
//   3. every other curve whose bound is at most tau runs through the sweep
//      with threshold tau, which drops a pair as soon as a crossing set of
//      its table exceeds tau;
//   4. the k smallest (distance, index) pairs of stages 2 and 3.
// Every curve at distance <= tau is evaluated exactly in stage 2 or 3 (its
// bound is at most its distance), and at least k curves are within tau, so
// the result is the exact k nearest, ties broken by the smaller index.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <vector>

#include "ffd.h"
#include "ffd_bounded.h"
#include "ffd_internal.h"

using namespace ffdi;

namespace {

constexpr int64_t kStageOne = 128;  // exact evaluations before the threshold is set (at least k)

// Largest float x whose square root, taken in FP64 and rounded once to
// float (the stored form of a Euclidean result), is at most eps: then
// delta <= eps exactly when delta^2 <= x.
float eps2_of(float eps, int32_t metric) {
  if (metric == FFD_SQEUCLIDEAN || std::isinf(eps)) return eps;
  if (eps < 0.f) return -1.f;
  auto root = [](float x) { return (float)std::sqrt((double)x); };
  float x = (float)((double)eps * (double)eps);
  while (x > 0.f && root(x) > eps) x = std::nextafter(x, 0.f);
  for (;;) {
    float y = std::nextafter(x, std::numeric_limits<float>::infinity());
    if (std::isinf(y) || root(y) > eps) break;
    x = y;
  }
  return x;
}

// Rows per lane: the smallest R whose band holds a typical row curve
// (curves of more than four coordinates: the wide kernels' R).
int rows_per_lane(int64_t n, int32_t dim) {
  if (dim > 4) return ffd::wide_rows(dim);
  if (n <= 64) return 1;
  if (n <= 128) return 2;
  if (n <= 256) return 4;
  return 8;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_search(ffd_ctx *ctx, int32_t dim, int32_t metric) {
  if (!ctx) return FFD_E_INVALID;
  if (dim < 1) return fail(ctx, FFD_E_INVALID, "dim must be >= 1");
  if (dim > FFD_MAX_DIM) return fail(ctx, FFD_E_UNSUPPORTED, "dim exceeds FFD_MAX_DIM");
  if (metric < FFD_EUCLIDEAN || metric > FFD_HAVERSINE) return fail(ctx, FFD_E_INVALID, "unknown metric");
  if (metric != FFD_EUCLIDEAN && metric != FFD_SQEUCLIDEAN)
    return fail(ctx, FFD_E_UNSUPPORTED, "the search calls take the Euclidean and squared Euclidean metrics");
  return FFD_OK;
}

// The scratch the caller registered (ffd_set_scratch), at least `bytes`
// long; work of an earlier call that used it on another stream is waited
// for on the device.
int search_scratch(ffd_ctx *ctx, size_t bytes, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return fail(ctx, FFD_E_UNSUPPORTED, "the search calls cannot be recorded into a graph");
  if (ctx->scratch_bytes < bytes)
    return fail(ctx, FFD_E_NOMEM,
                "the search calls need device scratch: register at least ffd_workspace_size(FFD_OP_DECIDE or "
                "FFD_OP_KNN) bytes with ffd_set_scratch");
  return use_begin(ctx, ctx->scratch_use, ctx->scratch, st, false);
}

// Pinned host staging of the k-nearest search, grown on demand (copies
// from and to pageable memory go through the runtime's own staging and
// cost more per query).  Every search call ends with a stream
// synchronisation, so no copy from an earlier call is pending when it is
// reused or replaced.
int search_host(ffd_ctx *ctx, size_t bytes) {
  if (ctx->search_host_bytes >= bytes) return FFD_OK;
  if (ctx->search_host) {
    hipHostFree(ctx->search_host);
    ctx->search_host = nullptr;
    ctx->search_host_bytes = 0;
  }
  hipError_t e = hipHostMalloc(&ctx->search_host, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipHostMalloc (search staging)");
  ctx->search_host_bytes = bytes;
  return FFD_OK;
}

// Waves of a launch, in whole workgroups of four: at most one per pair,
// and between one and two per SIMD -- as many as keep the average wave's
// steps (total / waves) above the longest pair's, since one wave sweeps a
// whole pair and the longest one would otherwise set the launch time.
int search_waves(ffd_ctx *ctx, int64_t npairs, double total_steps = 0, double longest = 0) {
  int64_t lo = (int64_t)ctx->cus * 4, hi = (int64_t)ctx->cus * 8;
  int64_t w = hi;
  if (longest > 0) w = std::max<int64_t>(lo, std::min<int64_t>(hi, (int64_t)(total_steps / longest)));
  w = std::min<int64_t>(w, npairs);
  return (int)std::max<int64_t>(4, (w + 3) / 4 * 4);
}

// Steps of one pair on a wave: its bands, each a ramp of 64 steps and the
// column curve, in groups of 16.
double pair_steps(int64_t n, int64_t m, int R) {
  int64_t nb = (n + 64 * R - 1) / (64 * R);
  return (double)nb * (double)((m + 63 + 15) / 16 * 16);
}

struct Layout {
  size_t off0, off1, order, out, counter, lb, eps, rows, total;
};

Layout layout(int64_t n0, int64_t n1, int64_t npairs, int64_t nout, int64_t nlb, int nwaves, int64_t row_cap,
              int64_t neps = 0) {
  Layout L{};
  size_t o = 0;
  L.off0 = o; o = al256(o + (size_t)(n0 + 1) * 8);
  L.off1 = o; o = al256(o + (size_t)(n1 + 1) * 8);
  L.order = o; o = al256(o + (size_t)std::max<int64_t>(npairs, 1) * 4);
  L.out = o; o = al256(o + (size_t)std::max<int64_t>(nout, 1) * 4);
  L.counter = o; o = al256(o + 8);
  L.lb = o; o = al256(o + (size_t)std::max<int64_t>(nlb, 1) * 4);
  L.eps = o; o = al256(o + (size_t)std::max<int64_t>(neps, 1) * 4);
  L.rows = o; o = al256(o + (size_t)nwaves * 3 * (size_t)row_cap * 4);
  L.total = o;
  return L;
}

int launch(ffd_ctx *ctx, ffd::BoundedArgs &a, int R, int D, int nwaves, hipStream_t st) {
  hipError_t e = ffd::clear_words(reinterpret_cast<uint64_t *>(a.counter), 1, st);
  if (e == hipSuccess) e = ffd::launch_bounded(R, D, a, nwaves, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "search launch");
  return use_end(ctx, ctx->scratch_use, ctx->scratch, st, false);
}

// Launch shape and scratch layout of a decider call.
struct DecideShape {
  int R, nwaves;
  int64_t row_cap;
  Layout L;
};

// Each pair is swept with the curve whose bands waste the fewest rows (and
// ramp steps) as the row curve: swap[k] when Q_k takes that role.
DecideShape decide_shape(ffd_ctx *ctx, const int64_t *p_off, const int64_t *q_off, int64_t npairs, int32_t dim,
                         std::vector<uint8_t> *swap = nullptr) {
  int64_t nsum = 0;
  for (int64_t k = 0; k < npairs; ++k) nsum += p_off[k + 1] - p_off[k];
  DecideShape d;
  d.R = rows_per_lane(nsum / npairs, dim);
  if (swap) swap->assign(npairs, 0);
  int64_t cmax = 0;
  bool banded = false;
  double total = 0, longest = 0;
  for (int64_t k = 0; k < npairs; ++k) {
    const int64_t n = p_off[k + 1] - p_off[k], m = q_off[k + 1] - q_off[k];
    const double a = pair_steps(n, m, d.R), b = pair_steps(m, n, d.R);
    const bool sw = b < a;
    if (swap) (*swap)[k] = sw ? 1 : 0;
    const int64_t rows = sw ? m : n, cols = sw ? n : m;
    banded = banded || rows > 64 * d.R;
    cmax = std::max(cmax, cols);
    const double st = sw ? b : a;
    total += st;
    longest = std::max(longest, st);
  }
  d.row_cap = banded ? cmax + 1 : 0;
  d.nwaves = search_waves(ctx, npairs, total, longest);
  d.L = layout(npairs, npairs, npairs, 0, 0, d.nwaves, d.row_cap);
  return d;
}

// Launch shape and scratch layout of a k-nearest search of nq queries (the
// largest stage; the others launch fewer waves): rows per lane for the
// median query length, the bound, value and order arrays for every
// (query, curve) pair, one threshold per query.
DecideShape knn_shape(ffd_ctx *ctx, const int64_t *q_off, int64_t nq, const int64_t *db_off, int64_t ndb,
                      int32_t dim) {
  int64_t mmax = 0, nmax = 0;
  for (int64_t c = 0; c < ndb; ++c) mmax = std::max(mmax, db_off[c + 1] - db_off[c]);
  std::vector<int64_t> lens(nq);
  for (int64_t i = 0; i < nq; ++i) {
    lens[i] = q_off[i + 1] - q_off[i];
    nmax = std::max(nmax, lens[i]);
  }
  std::nth_element(lens.begin(), lens.begin() + nq / 2, lens.end());
  DecideShape d;
  d.R = rows_per_lane(lens[nq / 2], dim);
  d.row_cap = nmax > 64 * d.R ? mmax + 1 : 0;
  d.nwaves = search_waves(ctx, nq * ndb);
  d.L = layout(nq, ndb, nq * ndb, nq * ndb, nq * ndb, d.nwaves, d.row_cap, nq);
  return d;
}

}  // namespace

namespace ffdi {

int search_scratch_size(ffd_ctx *ctx, int32_t op, const int64_t *a_off, int64_t na, const int64_t *b_off,
                        int64_t nb, int32_t dim, size_t *bytes) {
  if (op == FFD_OP_DECIDE) {
    if (na != nb) return fail(ctx, FFD_E_INVALID, "the decider needs na == nb");
    // eps = +inf runs ffd_batch in the same scratch
    size_t batch = 0;
    int rc = ffd_workspace_size(ctx, FFD_OP_BATCH, a_off, na, b_off, nb, dim, &batch);
    if (rc) return rc;
    *bytes = std::max(decide_shape(ctx, a_off, b_off, na, dim).L.total, batch);
    return FFD_OK;
  }
  if (na < 1) return fail(ctx, FFD_E_INVALID, "a k-nearest search takes at least one query");
  *bytes = knn_shape(ctx, a_off, na, b_off, nb, dim).L.total;
  return FFD_OK;
}

}  // namespace ffdi

extern "C" {

int ffd_decide_batch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
                     int64_t npairs, int32_t dim, int32_t metric, float eps, float *out, void *stream) {
  int rc = check_search(ctx, dim, metric);
  if (rc) return rc;
  if (std::isnan(eps)) return fail(ctx, FFD_E_INVALID, "eps is NaN");
  if (npairs < 0) return fail(ctx, FFD_E_INVALID, "npairs < 0");
  if (npairs == 0) return FFD_OK;
  if (npairs > INT32_MAX / 2) return fail(ctx, FFD_E_UNSUPPORTED, "too many pairs");
  if (!P || !Q || !out) return fail(ctx, FFD_E_INVALID, "NULL pointer");
  if ((rc = check_offsets(ctx, p_off, npairs, "p_off is NULL"))) return rc;
  if ((rc = check_offsets(ctx, q_off, npairs, "q_off is NULL"))) return rc;
  int64_t mmax = 0;
  for (int64_t k = 0; k < npairs; ++k) mmax = std::max(mmax, q_off[k + 1] - q_off[k]);
  if (mmax * dim >= ((int64_t)1 << 31)) return fail(ctx, FFD_E_UNSUPPORTED, "column curve too long");
  if (ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot launch");
  hipStream_t st = (hipStream_t)stream;
  if (std::isinf(eps) && eps > 0) {
    // no pair can be dropped: the decider is a batch, and the streaming
    // kernel computes it faster than the early-abandoning sweep (the
    // batch's own check reports a scratch too small for its plan)
    if ((rc = search_scratch(ctx, 0, st))) return rc;
    return batch_in_scratch(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, st);
  }
  std::vector<uint8_t> swap;
  const DecideShape sh = decide_shape(ctx, p_off, q_off, npairs, dim, &swap);
  const int R = sh.R, nwaves = sh.nwaves;
  const int64_t row_cap = sh.row_cap;
  const Layout &L = sh.L;
  if ((rc = search_scratch(ctx, L.total, st))) return rc;
  // larger pairs first, so that the work counter ends with small ones; the
  // top bit marks a swapped pair
  std::vector<int32_t> order(npairs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return (p_off[x + 1] - p_off[x]) * (q_off[x + 1] - q_off[x]) >
           (p_off[y + 1] - p_off[y]) * (q_off[y + 1] - q_off[y]);
  });
  for (int32_t &o : order)
    if (swap[o]) o = (int32_t)((uint32_t)o | 0x80000000u);
  char *base = static_cast<char *>(ctx->scratch);
  hipError_t e = hipMemcpyAsync(base + L.off0, p_off, (size_t)(npairs + 1) * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + L.off1, q_off, (size_t)(npairs + 1) * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + L.order, order.data(), (size_t)npairs * 4, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "search upload");
  ffd::BoundedArgs a{};
  a.X0 = P;
  a.X1 = Q;
  a.off0 = reinterpret_cast<const int64_t *>(base + L.off0);
  a.off1 = reinterpret_cast<const int64_t *>(base + L.off1);
  a.order = reinterpret_cast<const int32_t *>(base + L.order);
  a.fixed_row = -1;
  a.metric = metric;
  a.npairs = npairs;
  a.eps2 = eps2_of(eps, metric);
  a.out = out;
  a.rows = reinterpret_cast<float *>(base + L.rows);
  a.row_cap = row_cap;
  a.counter = reinterpret_cast<uint32_t *>(base + L.counter);
  a.dim = dim;
  return launch(ctx, a, R, dim, nwaves, st);
}

int ffd_knn_batch(ffd_ctx *ctx, const float *Q, const int64_t *q_off, int64_t nq, const float *DB,
                  const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, int32_t k, int64_t *out_idx,
                  float *out_dist, void *stream) {
  int rc = check_search(ctx, dim, metric);
  if (rc) return rc;
  if (k < 1) return fail(ctx, FFD_E_INVALID, "k must be >= 1");
  if (nq < 1) return fail(ctx, FFD_E_INVALID, "nq must be >= 1");
  if (ndb < 1) return fail(ctx, FFD_E_INVALID, "the database must hold at least one curve");
  if (nq * ndb > INT32_MAX / 2) return fail(ctx, FFD_E_UNSUPPORTED, "too many (query, curve) pairs");
  if (!Q || !DB || !out_idx || !out_dist) return fail(ctx, FFD_E_INVALID, "NULL pointer");
  if ((rc = check_offsets(ctx, q_off, nq, "q_off is NULL"))) return rc;
  if ((rc = check_offsets(ctx, db_off, ndb, "db_off is NULL"))) return rc;
  for (int64_t i = 0; i < nq; ++i)
    if (q_off[i + 1] - q_off[i] < 1) return fail(ctx, FFD_E_INVALID, "every query must have at least one point");
  int64_t mmax = 0;
  for (int64_t c = 0; c < ndb; ++c) mmax = std::max(mmax, db_off[c + 1] - db_off[c]);
  if (mmax * dim >= ((int64_t)1 << 31)) return fail(ctx, FFD_E_UNSUPPORTED, "database curve too long");
  if (ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot launch");
  hipStream_t st = (hipStream_t)stream;
  const int64_t kk = std::min<int64_t>(k, ndb);
  const int64_t np = nq * ndb;
  const DecideShape sh = knn_shape(ctx, q_off, nq, db_off, ndb, dim);
  const int R = sh.R;
  const Layout &L = sh.L;
  if ((rc = search_scratch(ctx, L.total, st))) return rc;
  char *base = static_cast<char *>(ctx->scratch);
  // pinned staging: both offset arrays, the bounds, the values, the order,
  // the thresholds
  const size_t h_off = 0, h_lb = al256((size_t)(nq + ndb + 2) * 8), h_vals = h_lb + al256((size_t)np * 4),
               h_order = h_vals + al256((size_t)np * 4), h_eps = h_order + al256((size_t)np * 4),
               h_total = h_eps + al256((size_t)nq * 4);
  if ((rc = search_host(ctx, h_total))) return rc;
  char *hb = static_cast<char *>(ctx->search_host);
  int64_t *hoff = reinterpret_cast<int64_t *>(hb + h_off);
  float *lb = reinterpret_cast<float *>(hb + h_lb);
  float *vals = reinterpret_cast<float *>(hb + h_vals);
  int32_t *horder = reinterpret_cast<int32_t *>(hb + h_order);
  float *heps = reinterpret_cast<float *>(hb + h_eps);
  memcpy(hoff, q_off, (size_t)(nq + 1) * 8);
  memcpy(hoff + nq + 1, db_off, (size_t)(ndb + 1) * 8);
  hipError_t e = hipMemcpyAsync(base + L.off0, hoff, (size_t)(nq + 1) * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + L.off1, hoff + nq + 1, (size_t)(ndb + 1) * 8, hipMemcpyHostToDevice, st);
  float *lb_dev = reinterpret_cast<float *>(base + L.lb);
  if (e == hipSuccess)
    e = ffd::launch_endpoint_bound_batch(dim, Q, reinterpret_cast<const int64_t *>(base + L.off0), nq, DB,
                                         reinterpret_cast<const int64_t *>(base + L.off1), ndb, lb_dev, st);
  if (e == hipSuccess) e = hipMemcpyAsync(lb, lb_dev, (size_t)np * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(ctx, e, "search bounds");

  ffd::BoundedArgs a{};
  a.X0 = Q;
  a.X1 = DB;
  a.off0 = reinterpret_cast<const int64_t *>(base + L.off0);
  a.off1 = reinterpret_cast<const int64_t *>(base + L.off1);
  a.order = reinterpret_cast<const int32_t *>(base + L.order);
  a.fixed_row = -1;
  a.col_count = ndb;
  a.metric = FFD_SQEUCLIDEAN;
  a.out = reinterpret_cast<float *>(base + L.out);
  a.rows = reinterpret_cast<float *>(base + L.rows);
  a.row_cap = sh.row_cap;
  a.counter = reinterpret_cast<uint32_t *>(base + L.counter);
  a.dim = dim;
  // one stage: exact squared distances of the npairs (query, curve) pairs in
  // horder, each at its query's threshold (heps) or at +inf
  auto stage = [&](int64_t npairs, bool thresholds) -> int {
    if (npairs == 0) return FFD_OK;
    a.npairs = npairs;
    a.eps2 = std::numeric_limits<float>::infinity();
    a.row_eps2 = thresholds ? reinterpret_cast<const float *>(base + L.eps) : nullptr;
    hipError_t err = hipMemcpyAsync(base + L.order, horder, (size_t)npairs * 4, hipMemcpyHostToDevice, st);
    if (err == hipSuccess && thresholds)
      err = hipMemcpyAsync(base + L.eps, heps, (size_t)nq * 4, hipMemcpyHostToDevice, st);
    if (err != hipSuccess) return hip_fail(ctx, err, "search upload");
    int r = launch(ctx, a, R, dim, search_waves(ctx, npairs), st);
    if (r) return r;
    err = hipMemcpyAsync(vals, a.out, (size_t)np * 4, hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) return hip_fail(ctx, err, "search results");
    return FFD_OK;
  };

  // per query: the curves with the smallest bounds first (ties by index);
  // the rest is only split by the threshold later, so no full sort is needed
  std::vector<int64_t> lens(ndb);
  for (int64_t c = 0; c < ndb; ++c) lens[c] = db_off[c + 1] - db_off[c];
  int64_t cap = 0;
  {
    std::vector<int64_t> tmp(lens);
    std::nth_element(tmp.begin(), tmp.begin() + ndb / 2, tmp.end());
    cap = 4 * tmp[ndb / 2];
  }
  const int64_t s1 = std::min<int64_t>(ndb, std::max<int64_t>(kk, kStageOne));
  std::vector<std::vector<int32_t>> idx(nq);
  int64_t n1 = 0;
  for (int64_t i = 0; i < nq; ++i) {
    const float *lbi = lb + i * ndb;
    std::vector<int32_t> &ix = idx[i];
    ix.resize(ndb);
    std::iota(ix.begin(), ix.end(), 0);
    if (s1 < ndb) {
      // one wave sweeps one curve, so the longest curve of the first stage
      // sets its time: take its curves from those no longer than four times
      // the median length when enough of them exist (any k curves give a
      // valid threshold; shorter ones give it sooner)
      auto by_bound = [&](int32_t x, int32_t y) { return lbi[x] < lbi[y] || (lbi[x] == lbi[y] && x < y); };
      auto mid = std::partition(ix.begin(), ix.end(), [&](int32_t c) { return lens[c] <= cap; });
      if (mid - ix.begin() >= s1) std::nth_element(ix.begin(), ix.begin() + s1, mid, by_bound);
      else std::nth_element(ix.begin(), ix.begin() + s1, ix.end(), by_bound);
    }
    for (int64_t j = 0; j < s1; ++j) horder[n1++] = (int32_t)(i * ndb + ix[j]);
  }
  if ((rc = stage(n1, false))) return rc;
  std::vector<std::vector<std::pair<float, int32_t>>> pool(nq);
  std::vector<int64_t> s2(nq);
  int64_t n2 = 0;
  for (int64_t i = 0; i < nq; ++i) {
    const float *lbi = lb + i * ndb, *vi = vals + i * ndb;
    std::vector<int32_t> &ix = idx[i];
    auto &pl = pool[i];
    for (int64_t j = 0; j < s1; ++j) pl.emplace_back(vi[ix[j]], ix[j]);
    std::nth_element(pl.begin(), pl.begin() + (kk - 1), pl.end());
    const float tau2 = pl[kk - 1].first;
    heps[i] = tau2;
    s2[i] = std::partition(ix.begin() + s1, ix.end(), [&](int32_t c) { return lbi[c] <= tau2; }) - ix.begin();
    for (int64_t j = s1; j < s2[i]; ++j) horder[n2++] = (int32_t)(i * ndb + ix[j]);
  }
  if ((rc = stage(n2, true))) return rc;
  ctx->last_search = ffd_search_info{s1 * nq, n2, 0};
  std::vector<int64_t> ri((size_t)nq * k, -1);
  std::vector<float> rd((size_t)nq * k, std::numeric_limits<float>::infinity());
  for (int64_t i = 0; i < nq; ++i) {
    const float *vi = vals + i * ndb;
    std::vector<int32_t> &ix = idx[i];
    auto &pl = pool[i];
    for (int64_t j = s1; j < s2[i]; ++j) {
      if (vi[ix[j]] <= heps[i]) pl.emplace_back(vi[ix[j]], ix[j]);
      else ctx->last_search.rejected += 1;
    }
    std::partial_sort(pl.begin(), pl.begin() + kk, pl.end());
    for (int64_t j = 0; j < kk; ++j) {
      ri[i * k + j] = pl[j].second;
      rd[i * k + j] = metric == FFD_EUCLIDEAN ? (float)std::sqrt((double)pl[j].first) : pl[j].first;
    }
  }
  e = hipMemcpyAsync(out_idx, ri.data(), (size_t)nq * k * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(out_dist, rd.data(), (size_t)nq * k * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(ctx, e, "search output");
  return FFD_OK;
}

int ffd_knn(ffd_ctx *ctx, const float *q, int64_t n, const float *DB, const int64_t *db_off, int64_t ndb,
            int32_t dim, int32_t metric, int32_t k, int64_t *out_idx, float *out_dist, void *stream) {
  if (ctx && n < 1) return fail(ctx, FFD_E_INVALID, "the query must have at least one point");
  const int64_t q_off[2] = {0, n};
  return ffd_knn_batch(ctx, q, q_off, 1, DB, db_off, ndb, dim, metric, k, out_idx, out_dist, stream);
}

int ffd_last_search(const ffd_ctx *ctx, ffd_search_info *info) {
  if (!ctx || !info) return FFD_E_INVALID;
  *info = ctx->last_search;
  return FFD_OK;
}

}  // extern "C"

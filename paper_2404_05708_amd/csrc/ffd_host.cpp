// Host side of the library: argument checks, planning, plan upload, launch.
//
// Planning follows Sec. 4 of the paper (batches of curves, sorting by length
// before batching) in the form that suits one wavefront per stream:
//  * every pair is oriented so that the cheaper curve becomes the row curve
//    (the distance is symmetric and the float evaluation is exactly
//    symmetric, so both orientations give the same bits);
//  * jobs are assigned to waves longest-first onto the least loaded wave
//    (LPT), which is the "sort by length" rule applied to a fixed number of
//    workers;
//  * the plan (jobs, per-wave job ranges, curve offsets) is copied into the
//    caller's workspace and reused while the offsets do not change.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "ffd.h"
#include "ffd_plan.h"

namespace ffd {
hipError_t launch_stream(bool exact, int R, int D, const KernelArgs &a, int wpb, hipStream_t st);
}

using ffd::Job;
using ffd::KernelArgs;

struct PlanCacheBase;

struct ffd_ctx {
  int device = 0;
  int cus = 0;
  size_t lds_block_max = 0;
  int tune_R = 0;
  int tune_W = 0;
  std::string last_error;
  // plan most recently written to a workspace (skip the upload if unchanged)
  void *plan_ws = nullptr;
  uint64_t plan_ws_key = 0;
  void *pinned = nullptr;  // staging buffer for plan uploads
  size_t pinned_bytes = 0;
  hipEvent_t upload_done = nullptr;
  PlanCacheBase *plans_ptr = nullptr;
};

namespace {

const char *kVersion = "ffd 0.1.0 (gfx950)";

int fail(ffd_ctx *ctx, int code, const char *msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

int hip_fail(ffd_ctx *ctx, hipError_t e, const char *what) {
  if (ctx) ctx->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return FFD_E_DEVICE;
}

// Modelled VALU instructions per lane for one step with R rows per lane:
// (2D + 2) per cell (D subtractions, one multiply, D-1 FMAs, min, min, max
// with min3 fused as two) plus a few per step (lane shift, addressing).
double step_cost(int R, int D) { return (double)R * (2 * D + 2) + 3.0; }

struct Orient {
  bool swap;        // true: row curve is the second curve
  int64_t steps;    // stream steps of the job
  int64_t hcap;     // hand-off entries needed (0 if a single band)
};

Orient orient_pair(int64_t n, int64_t m, int R, bool allow_swap) {
  auto steps = [&](int64_t rows, int64_t cols, int64_t *hc) {
    int64_t nb = ffd::bands_for(rows, R);
    int64_t L = ffd::task_len(cols, nb > 1);
    *hc = nb > 1 ? L : 0;
    return nb * L;
  };
  Orient o{false, 0, 0};
  int64_t h1, h2;
  int64_t s1 = steps(n, m, &h1);
  o.steps = s1;
  o.hcap = h1;
  if (allow_swap) {
    int64_t s2 = steps(m, n, &h2);
    if (s2 < s1 || (s2 == s1 && h2 < h1)) {
      o.swap = true;
      o.steps = s2;
      o.hcap = h2;
    }
  }
  return o;
}

uint64_t fnv(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = (const unsigned char *)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

int check_offsets(ffd_ctx *ctx, const int64_t *off, int64_t count, const char *name) {
  if (!off) return fail(ctx, FFD_E_INVALID, name);
  if (off[0] != 0) return fail(ctx, FFD_E_INVALID, "offsets must start at 0");
  for (int64_t k = 0; k < count; ++k)
    if (off[k + 1] <= off[k]) return fail(ctx, FFD_E_INVALID, "offsets must be strictly increasing (empty curve)");
  return FFD_OK;
}

int check_common(ffd_ctx *ctx, int32_t dim, int32_t metric, bool exact) {
  if (!ctx) return FFD_E_INVALID;
  if (dim < 1) return fail(ctx, FFD_E_INVALID, "dim must be >= 1");
  if (metric != FFD_EUCLIDEAN && metric != FFD_SQEUCLIDEAN) return fail(ctx, FFD_E_INVALID, "unknown metric");
  if (dim > FFD_MAX_DIM) return fail(ctx, FFD_E_UNSUPPORTED, "dim exceeds FFD_MAX_DIM");
  if (exact && metric != FFD_SQEUCLIDEAN)
    return fail(ctx, FFD_E_UNSUPPORTED, "int32 coordinates support the squared Euclidean metric only");
  return FFD_OK;
}

int lds_bytes(int R, int D, bool exact, int64_t hcap) {
  return ffd::lds_layout(R, D, exact ? 8 : 4, (int)hcap).total;
}

const int kRs[4] = {1, 2, 4, 8};

// A planned launch over jobs.
struct Plan {
  int R = 4;
  int nwaves = 0;
  int wpb = 1;
  int64_t hcap = 0;
  int64_t max_steps = 0;         // largest stream of any wave
  std::vector<Job> jobs;         // grouped by wave
  std::vector<int32_t> wave_jobs;
};

// Assign jobs (with modelled costs) to nwaves waves, longest first onto the
// least loaded wave, and lay them out grouped by wave.
void lpt(std::vector<Job> &jobs, const std::vector<double> &cost, int nwaves, Plan &pl) {
  std::vector<int64_t> order(jobs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
  using Item = std::pair<double, int>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int w = 0; w < nwaves; ++w) heap.push({0.0, w});
  std::vector<int> owner(jobs.size());
  std::vector<int32_t> count(nwaves, 0);
  std::vector<double> load(nwaves, 0.0);
  for (int64_t i : order) {
    Item it = heap.top();
    heap.pop();
    owner[i] = it.second;
    count[it.second]++;
    load[it.second] += cost[i];
    heap.push({it.first + cost[i], it.second});
  }
  double mx = 0;
  for (double x : load) mx = std::max(mx, x);
  pl.max_steps = (int64_t)mx;
  pl.wave_jobs.assign(nwaves + 1, 0);
  for (int w = 0; w < nwaves; ++w) pl.wave_jobs[w + 1] = pl.wave_jobs[w] + count[w];
  std::vector<int32_t> fillp(pl.wave_jobs.begin(), pl.wave_jobs.end() - 1);
  pl.jobs.resize(jobs.size());
  for (int64_t i : order) pl.jobs[fillp[owner[i]]++] = jobs[i];
}

int waves_for(ffd_ctx *ctx, int W, size_t njobs) {
  int nw = ctx->cus * 4 * W;
  if ((size_t)nw > njobs) nw = (int)njobs;
  return nw < 1 ? 1 : nw;
}

int choose_wpb(ffd_ctx *ctx, int lds_wave) {
  int wpb = 4;
  while (wpb > 1 && (size_t)lds_wave * wpb > ctx->lds_block_max) wpb /= 2;
  return wpb;
}

// Plan a batch of independent pairs.
int plan_batch(ffd_ctx *ctx, const int64_t *p_off, const int64_t *q_off, int64_t npairs, int D,
               bool exact, Plan &pl) {
  int W = ctx->tune_W > 0 ? ctx->tune_W : 2;
  double best = -1;
  int bestR = 4;
  for (int R : kRs) {
    if (ctx->tune_R && R != ctx->tune_R) continue;
    double tot = 0;
    int64_t hc = 0;
    for (int64_t k = 0; k < npairs; ++k) {
      Orient o = orient_pair(p_off[k + 1] - p_off[k], q_off[k + 1] - q_off[k], R, true);
      tot += (double)o.steps * step_cost(R, D);
      hc = std::max(hc, o.hcap);
    }
    if ((size_t)lds_bytes(R, D, exact, hc) > ctx->lds_block_max) continue;
    if (best < 0 || tot < best) {
      best = tot;
      bestR = R;
    }
  }
  if (best < 0) return fail(ctx, FFD_E_UNSUPPORTED, "curves too long for the LDS hand-off row");
  pl.R = bestR;
  std::vector<Job> jobs(npairs);
  std::vector<double> cost(npairs);
  pl.hcap = 0;
  for (int64_t k = 0; k < npairs; ++k) {
    Orient o = orient_pair(p_off[k + 1] - p_off[k], q_off[k + 1] - q_off[k], pl.R, true);
    Job &jb = jobs[k];
    jb.out_base = k;
    jb.row_sel = o.swap ? 1 : 0;
    jb.row_idx = (int32_t)k;
    jb.col_sel = o.swap ? 0 : 1;
    jb.col_first = (int32_t)k;
    jb.col_count = 1;
    jb.out_stride = 1;
    cost[k] = (double)o.steps;  // exact stream length of the job
    pl.hcap = std::max(pl.hcap, o.hcap);
  }
  pl.nwaves = waves_for(ctx, W, jobs.size());
  pl.wpb = choose_wpb(ctx, lds_bytes(pl.R, D, exact, pl.hcap));
  lpt(jobs, cost, pl.nwaves, pl);
  return FFD_OK;
}

// Plan queries x database: job = one query against a run of database curves.
int plan_cross(ffd_ctx *ctx, const int64_t *q_off, int64_t nq, const int64_t *db_off, int64_t ndb,
               int D, bool exact, Plan &pl) {
  int W = ctx->tune_W > 0 ? ctx->tune_W : 2;
  int64_t dbmax = 0;
  for (int64_t k = 0; k < ndb; ++k) dbmax = std::max(dbmax, db_off[k + 1] - db_off[k]);
  double best = -1;
  int bestR = 4;
  for (int R : kRs) {
    if (ctx->tune_R && R != ctx->tune_R) continue;
    double tot = 0;
    bool chained = false;
    for (int64_t i = 0; i < nq; ++i) {
      int64_t nb = ffd::bands_for(q_off[i + 1] - q_off[i], R);
      chained |= nb > 1;
      tot += (double)nb;
    }
    double cols = 0;
    for (int64_t k = 0; k < ndb; ++k) cols += (double)ffd::task_len(db_off[k + 1] - db_off[k], chained);
    tot *= cols * step_cost(R, D);
    int64_t hc = chained ? ffd::task_len(dbmax, true) : 0;
    if ((size_t)lds_bytes(R, D, exact, hc) > ctx->lds_block_max) continue;
    if (best < 0 || tot < best) {
      best = tot;
      bestR = R;
    }
  }
  if (best < 0) return fail(ctx, FFD_E_UNSUPPORTED, "database curves too long for the LDS hand-off row");
  pl.R = bestR;
  bool any_chained = false;
  for (int64_t i = 0; i < nq; ++i) any_chained |= ffd::bands_for(q_off[i + 1] - q_off[i], pl.R) > 1;
  pl.hcap = any_chained ? ffd::task_len(dbmax, true) : 0;
  // total modelled steps -> chunk target so that each wave gets several jobs
  int nw_full = ctx->cus * 4 * W;
  std::vector<double> colcost(ndb);
  for (int64_t k = 0; k < ndb; ++k) {
    bool chained_any = any_chained;
    colcost[k] = (double)ffd::task_len(db_off[k + 1] - db_off[k], chained_any);
  }
  double total = 0;
  std::vector<double> qb(nq);
  for (int64_t i = 0; i < nq; ++i) {
    qb[i] = (double)ffd::bands_for(q_off[i + 1] - q_off[i], pl.R);
    total += qb[i];
  }
  double colsum = 0;
  for (double x : colcost) colsum += x;
  total *= colsum;
  double target = total / ((double)nw_full * 8.0);
  std::vector<Job> jobs;
  std::vector<double> cost;
  for (int64_t i = 0; i < nq; ++i) {
    int64_t k = 0;
    while (k < ndb) {
      int64_t k0 = k;
      double c = 0;
      while (k < ndb && (c == 0 || c + qb[i] * colcost[k] <= target)) {
        c += qb[i] * colcost[k];
        ++k;
      }
      Job jb;
      jb.out_base = i * ndb + k0;
      jb.row_sel = 0;
      jb.row_idx = (int32_t)i;
      jb.col_sel = 1;
      jb.col_first = (int32_t)k0;
      jb.col_count = (int32_t)(k - k0);
      jb.out_stride = 1;
      jobs.push_back(jb);
      cost.push_back(c);
    }
  }
  pl.nwaves = waves_for(ctx, W, jobs.size());
  pl.wpb = choose_wpb(ctx, lds_bytes(pl.R, D, exact, pl.hcap));
  lpt(jobs, cost, pl.nwaves, pl);
  return FFD_OK;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
  size_t jobs, wj, off0, off1, total;
};

WsLayout ws_layout(size_t njobs, int nwaves, int64_t n0, int64_t n1) {
  WsLayout w;
  size_t o = 0;
  w.jobs = o; o = al256(o + njobs * sizeof(Job));
  w.wj = o;   o = al256(o + (size_t)(nwaves + 1) * sizeof(int32_t));
  w.off0 = o; o = al256(o + (size_t)(n0 + 1) * sizeof(int64_t));
  w.off1 = o; o = al256(o + (size_t)(n1 + 1) * sizeof(int64_t));
  w.total = o;
  return w;
}

int ensure_pinned(ffd_ctx *ctx, size_t bytes) {
  if (ctx->pinned_bytes >= bytes) {
    // previous upload must have finished reading the staging buffer
    if (ctx->upload_done) hipEventSynchronize(ctx->upload_done);
    return FFD_OK;
  }
  if (ctx->pinned) {
    if (ctx->upload_done) hipEventSynchronize(ctx->upload_done);
    hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
  }
  hipError_t e = hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipHostMalloc");
  ctx->pinned_bytes = bytes;
  return FFD_OK;
}

// Run a planned launch: upload the plan into the workspace unless the same
// plan is already there, then launch.
int run_plan(ffd_ctx *ctx, const Plan &pl, uint64_t key, const void *X0, const int64_t *off0,
             int64_t n0, const void *X1, const int64_t *off1, int64_t n1, int D, bool exact,
             int metric, void *out, void *ws, size_t ws_bytes, hipStream_t st) {
  WsLayout wl = ws_layout(pl.jobs.size(), pl.nwaves, n0, n1);
  if (!ws || ws_bytes < wl.total) return fail(ctx, FFD_E_NOMEM, "workspace too small (see ffd_workspace_size)");
  unsigned char *w = (unsigned char *)ws;
  if (!(ctx->plan_ws == ws && ctx->plan_ws_key == key)) {
    int rc = ensure_pinned(ctx, wl.total);
    if (rc) return rc;
    unsigned char *h = (unsigned char *)ctx->pinned;
    memcpy(h + wl.jobs, pl.jobs.data(), pl.jobs.size() * sizeof(Job));
    memcpy(h + wl.wj, pl.wave_jobs.data(), pl.wave_jobs.size() * sizeof(int32_t));
    memcpy(h + wl.off0, off0, (size_t)(n0 + 1) * sizeof(int64_t));
    memcpy(h + wl.off1, off1, (size_t)(n1 + 1) * sizeof(int64_t));
    hipError_t e = hipMemcpyAsync(w, h, wl.total, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync (plan)");
    if (!ctx->upload_done) {
      e = hipEventCreateWithFlags(&ctx->upload_done, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
    }
    hipEventRecord(ctx->upload_done, st);
    ctx->plan_ws = ws;
    ctx->plan_ws_key = key;
  }
  KernelArgs a;
  memset(&a, 0, sizeof a);
  a.X[0] = X0;
  a.X[1] = X1;
  a.off[0] = (const int64_t *)(w + wl.off0);
  a.off[1] = (const int64_t *)(w + wl.off1);
  a.jobs = (const Job *)(w + wl.jobs);
  a.wave_jobs = (const int32_t *)(w + wl.wj);
  a.out = out;
  a.nwaves = pl.nwaves;
  a.metric = metric;
  a.hcap = (int32_t)pl.hcap;
  a.lds_per_wave = lds_bytes(pl.R, D, exact, pl.hcap);
  if (pl.max_steps + 4 * ffd::kRing > INT32_MAX) return fail(ctx, FFD_E_UNSUPPORTED, "stream too long");
  a.max_steps = (int32_t)(pl.max_steps + 4 * ffd::kRing);
  hipError_t e = ffd::launch_stream(exact, pl.R, D, a, pl.wpb, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  return FFD_OK;
}

uint64_t key_of(int op, int D, bool exact, int R, int W, const int64_t *a, int64_t na, const int64_t *b,
                int64_t nb) {
  uint64_t h = 1469598103934665603ull;
  int hdr[6] = {op, D, exact ? 1 : 0, R, W, 0};
  h = fnv(h, hdr, sizeof hdr);
  h = fnv(h, &na, sizeof na);
  h = fnv(h, &nb, sizeof nb);
  h = fnv(h, a, (size_t)(na + 1) * sizeof(int64_t));
  h = fnv(h, b, (size_t)(nb + 1) * sizeof(int64_t));
  return h;
}

struct PlanCache {
  uint64_t key = 0;
  Plan plan;
  bool valid = false;
};

PlanCache &plans_of(ffd_ctx *ctx) {
  if (!ctx->plans_ptr) ctx->plans_ptr = reinterpret_cast<PlanCacheBase *>(new PlanCache());
  return *reinterpret_cast<PlanCache *>(ctx->plans_ptr);
}

int cached_plan(ffd_ctx *ctx, PlanCache &pc, int op, const int64_t *a_off, int64_t na,
                const int64_t *b_off, int64_t nb, int D, bool exact, const Plan **out, uint64_t &key) {
  key = key_of(op, D, exact, ctx->tune_R, ctx->tune_W, a_off, na, b_off, nb);
  if (pc.valid && pc.key == key) {
    *out = &pc.plan;
    return FFD_OK;
  }
  Plan pl;
  int rc = op == FFD_OP_BATCH ? plan_batch(ctx, a_off, b_off, na, D, exact, pl)
                              : plan_cross(ctx, a_off, na, b_off, nb, D, exact, pl);
  if (rc) return rc;
  pc.plan = std::move(pl);
  pc.key = key;
  pc.valid = true;
  *out = &pc.plan;
  return FFD_OK;
}

int pair_common(ffd_ctx *ctx, const void *p, int64_t n, const void *q, int64_t m, int32_t dim,
                int32_t metric, void *out, hipStream_t st, bool exact) {
  int rc = check_common(ctx, dim, metric, exact);
  if (rc) return rc;
  if (!p || !q || !out) return fail(ctx, FFD_E_INVALID, "NULL pointer");
  if (n < 1 || m < 1) return fail(ctx, FFD_E_INVALID, "curves must have at least one point");
  // choose R and orientation for one stream
  double best = -1;
  int bestR = 4;
  Orient bestO{false, 0, 0};
  for (int R : kRs) {
    if (ctx->tune_R && R != ctx->tune_R) continue;
    Orient o = orient_pair(n, m, R, true);
    if ((size_t)lds_bytes(R, dim, exact, o.hcap) > ctx->lds_block_max) {
      Orient o2 = orient_pair(n, m, R, false);
      Orient o3 = orient_pair(m, n, R, false);
      o3.swap = true;
      if ((size_t)lds_bytes(R, dim, exact, o2.hcap) <= ctx->lds_block_max) o = o2;
      else if ((size_t)lds_bytes(R, dim, exact, o3.hcap) <= ctx->lds_block_max) o = o3;
      else continue;
    }
    double c = (double)(o.steps + ffd::kWave) * step_cost(R, dim);
    if (best < 0 || c < best) {
      best = c;
      bestR = R;
      bestO = o;
    }
  }
  if (best < 0) return fail(ctx, FFD_E_UNSUPPORTED, "pair too long for the LDS hand-off row");
  KernelArgs a;
  memset(&a, 0, sizeof a);
  a.X[0] = p;
  a.X[1] = q;
  a.inl_off[0][0] = 0;
  a.inl_off[0][1] = n;
  a.inl_off[1][0] = 0;
  a.inl_off[1][1] = m;
  a.jobs = nullptr;
  a.inl_job.out_base = 0;
  a.inl_job.row_sel = bestO.swap ? 1 : 0;
  a.inl_job.row_idx = 0;
  a.inl_job.col_sel = bestO.swap ? 0 : 1;
  a.inl_job.col_first = 0;
  a.inl_job.col_count = 1;
  a.inl_job.out_stride = 1;
  a.out = out;
  a.nwaves = 1;
  a.metric = metric;
  a.hcap = (int32_t)bestO.hcap;
  a.lds_per_wave = lds_bytes(bestR, dim, exact, bestO.hcap);
  if (bestO.steps + 4 * ffd::kRing > INT32_MAX) return fail(ctx, FFD_E_UNSUPPORTED, "stream too long");
  a.max_steps = (int32_t)(bestO.steps + 4 * ffd::kRing);
  if (ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot launch");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  e = ffd::launch_stream(exact, bestR, dim, a, 1, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  return FFD_OK;
}

int batch_common(ffd_ctx *ctx, const void *P, const int64_t *p_off, const void *Q, const int64_t *q_off,
                 int64_t npairs, int32_t dim, int32_t metric, void *out, void *ws, size_t ws_bytes,
                 hipStream_t st, bool exact) {
  int rc = check_common(ctx, dim, metric, exact);
  if (rc) return rc;
  if (npairs < 0) return fail(ctx, FFD_E_INVALID, "npairs < 0");
  if (npairs == 0) return FFD_OK;
  if (npairs > INT32_MAX / 2) return fail(ctx, FFD_E_UNSUPPORTED, "too many pairs");
  if (!P || !Q || !out) return fail(ctx, FFD_E_INVALID, "NULL pointer");
  if ((rc = check_offsets(ctx, p_off, npairs, "p_off is NULL"))) return rc;
  if ((rc = check_offsets(ctx, q_off, npairs, "q_off is NULL"))) return rc;
  const Plan *pl;
  uint64_t key;
  rc = cached_plan(ctx, plans_of(ctx), FFD_OP_BATCH, p_off, npairs, q_off, npairs, dim, exact, &pl, key);
  if (rc) return rc;
  if (ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot launch");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  return run_plan(ctx, *pl, key, P, p_off, npairs, Q, q_off, npairs, dim, exact, metric, out, ws, ws_bytes, st);
}

int cross_common(ffd_ctx *ctx, const void *Qs, const int64_t *q_off, int64_t nq, const void *DB,
                 const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, void *out, void *ws,
                 size_t ws_bytes, hipStream_t st, bool exact) {
  int rc = check_common(ctx, dim, metric, exact);
  if (rc) return rc;
  if (nq < 0 || ndb < 0) return fail(ctx, FFD_E_INVALID, "negative count");
  if (nq == 0 || ndb == 0) return FFD_OK;
  if (nq > INT32_MAX / 2 || ndb > INT32_MAX / 2) return fail(ctx, FFD_E_UNSUPPORTED, "too many curves");
  if (!Qs || !DB || !out) return fail(ctx, FFD_E_INVALID, "NULL pointer");
  if ((rc = check_offsets(ctx, q_off, nq, "q_off is NULL"))) return rc;
  if ((rc = check_offsets(ctx, db_off, ndb, "db_off is NULL"))) return rc;
  const Plan *pl;
  uint64_t key;
  rc = cached_plan(ctx, plans_of(ctx), FFD_OP_CROSS, q_off, nq, db_off, ndb, dim, exact, &pl, key);
  if (rc) return rc;
  if (ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot launch");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  return run_plan(ctx, *pl, key, Qs, q_off, nq, DB, db_off, ndb, dim, exact, metric, out, ws, ws_bytes, st);
}

}  // namespace

extern "C" {

const char *ffd_version(void) { return kVersion; }

const char *ffd_strerror(int status) {
  switch (status) {
    case FFD_OK: return "ok";
    case FFD_E_INVALID: return "invalid argument";
    case FFD_E_UNSUPPORTED: return "unsupported request";
    case FFD_E_NOMEM: return "workspace or arena too small";
    case FFD_E_DEVICE: return "HIP device error";
    case FFD_E_BUSY: return "busy";
    case FFD_E_TIMEOUT: return "timed out";
  }
  return "unknown status";
}

const char *ffd_last_error(const ffd_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int ffd_create(int device, ffd_ctx **out) {
  if (!out) return FFD_E_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return FFD_E_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FFD_E_DEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FFD_E_DEVICE;
  ffd_ctx *c = new (std::nothrow) ffd_ctx();
  if (!c) return FFD_E_NOMEM;
  c->device = device;
  c->cus = prop.multiProcessorCount;
  c->lds_block_max = prop.sharedMemPerBlock < 65536 ? prop.sharedMemPerBlock : 65536;
  *out = c;
  return FFD_OK;
}

int ffd_create_planner(int32_t compute_units, int64_t lds_per_block, ffd_ctx **out) {
  if (!out) return FFD_E_INVALID;
  *out = nullptr;
  if (compute_units < 1 || lds_per_block < 16384) return FFD_E_INVALID;
  ffd_ctx *c = new (std::nothrow) ffd_ctx();
  if (!c) return FFD_E_NOMEM;
  c->device = -1;
  c->cus = compute_units;
  c->lds_block_max = (size_t)lds_per_block;
  *out = c;
  return FFD_OK;
}

void ffd_destroy(ffd_ctx *ctx) {
  if (!ctx) return;
  if (ctx->upload_done) {
    hipEventSynchronize(ctx->upload_done);
    hipEventDestroy(ctx->upload_done);
  }
  if (ctx->pinned) hipHostFree(ctx->pinned);

  delete ctx;
}

int ffd_set_tuning(ffd_ctx *ctx, int32_t rows_per_lane, int32_t waves_per_simd) {
  if (!ctx) return FFD_E_INVALID;
  if (rows_per_lane != 0 && rows_per_lane != 1 && rows_per_lane != 2 && rows_per_lane != 4 &&
      rows_per_lane != 8)
    return fail(ctx, FFD_E_INVALID, "rows_per_lane must be 0, 1, 2, 4 or 8");
  if (waves_per_simd < 0 || waves_per_simd > 8) return fail(ctx, FFD_E_INVALID, "waves_per_simd must be 0..8");
  ctx->tune_R = rows_per_lane;
  ctx->tune_W = waves_per_simd;
  return FFD_OK;
}

int ffd_distance(ffd_ctx *ctx, const float *p, int64_t n, const float *q, int64_t m, int32_t dim,
                 int32_t metric, float *out, void *stream) {
  return pair_common(ctx, p, n, q, m, dim, metric, out, (hipStream_t)stream, false);
}

int ffd_distance_i32(ffd_ctx *ctx, const int32_t *p, int64_t n, const int32_t *q, int64_t m, int32_t dim,
                     int32_t metric, int64_t *out, void *stream) {
  return pair_common(ctx, p, n, q, m, dim, metric, out, (hipStream_t)stream, true);
}

int ffd_batch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
              int64_t npairs, int32_t dim, int32_t metric, float *out, void *workspace, size_t ws_bytes,
              void *stream) {
  return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, workspace, ws_bytes,
                      (hipStream_t)stream, false);
}

int ffd_batch_i32(ffd_ctx *ctx, const int32_t *P, const int64_t *p_off, const int32_t *Q,
                  const int64_t *q_off, int64_t npairs, int32_t dim, int32_t metric, int64_t *out,
                  void *workspace, size_t ws_bytes, void *stream) {
  return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, workspace, ws_bytes,
                      (hipStream_t)stream, true);
}

int ffd_cross(ffd_ctx *ctx, const float *Qs, const int64_t *q_off, int64_t nq, const float *DB,
              const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, float *out, void *workspace,
              size_t ws_bytes, void *stream) {
  return cross_common(ctx, Qs, q_off, nq, DB, db_off, ndb, dim, metric, out, workspace, ws_bytes,
                      (hipStream_t)stream, false);
}

int ffd_cross_i32(ffd_ctx *ctx, const int32_t *Qs, const int64_t *q_off, int64_t nq, const int32_t *DB,
                  const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, int64_t *out,
                  void *workspace, size_t ws_bytes, void *stream) {
  return cross_common(ctx, Qs, q_off, nq, DB, db_off, ndb, dim, metric, out, workspace, ws_bytes,
                      (hipStream_t)stream, true);
}

int ffd_workspace_size(ffd_ctx *ctx, int32_t op, const int64_t *a_off, int64_t na, const int64_t *b_off,
                       int64_t nb, int32_t dim, size_t *bytes) {
  if (!ctx || !bytes) return FFD_E_INVALID;
  if (op != FFD_OP_BATCH && op != FFD_OP_CROSS) return fail(ctx, FFD_E_INVALID, "unknown op");
  if (dim < 1) return fail(ctx, FFD_E_INVALID, "dim must be >= 1");
  if (dim > FFD_MAX_DIM) return fail(ctx, FFD_E_UNSUPPORTED, "dim exceeds FFD_MAX_DIM");
  if (na < 0 || nb < 0) return fail(ctx, FFD_E_INVALID, "negative count");
  if (op == FFD_OP_BATCH && na != nb) return fail(ctx, FFD_E_INVALID, "batch needs na == nb");
  *bytes = 0;
  if (na == 0 || nb == 0) return FFD_OK;
  int rc;
  if ((rc = check_offsets(ctx, a_off, na, "offsets are NULL"))) return rc;
  if ((rc = check_offsets(ctx, b_off, nb, "offsets are NULL"))) return rc;
  size_t worst = 0;
  for (int ex = 0; ex < 2; ++ex) {
    const Plan *pl;
    uint64_t key;
    PlanCache tmp;
    rc = cached_plan(ctx, tmp, op, a_off, na, b_off, nb, dim, ex == 1, &pl, key);
    if (rc == FFD_E_UNSUPPORTED) continue;
    if (rc) return rc;
    worst = std::max(worst, ws_layout(pl->jobs.size(), pl->nwaves, na, nb).total);
  }
  if (worst == 0) return fail(ctx, FFD_E_UNSUPPORTED, "request not supported by any path");
  *bytes = worst;
  return FFD_OK;
}

}  // extern "C"

// Host side of the library: argument checks, planning, plan upload, launch.
//
// Planning follows Sec. 4 of the paper (batches of curves, sorting by length
// before batching) in the form that suits one wavefront per stream:
//  * a "unit" is one row curve against a run of column curves (a pair of a
//    batch, or a query against a chunk of the database); every pair is
//    oriented so that the cheaper curve becomes the row curve (the distance
//    is symmetric and the float evaluation is exactly symmetric, so both
//    orientations give the same bits);
//  * units much longer than a wave's fair share are split into their bands
//    of 64*R rows, which run on different waves and hand their boundary rows
//    on through global "links" (release/acquire progress flags); a unit
//    whose boundary row does not fit a wave's LDS keeps its bands on one
//    wave, in order, chained through links in the same way;
//  * tasks are placed by list scheduling: the highest-priority ready task
//    (longest remaining chain; longest first otherwise, the paper's sort by
//    length) goes to the wave that frees first.  A band that reads a link
//    starts, in its wave's stream, at least kLinkLag steps after the band
//    that writes it starts in its own (idle jobs pad the stream where
//    needed), so every wait is for a strictly earlier stream position: no
//    deadlock, whatever the actual timing;
//  * the plan (jobs, per-wave job ranges, curve offsets) is copied into the
//    caller's workspace and reused while the offsets do not change.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "ffd_internal.h"

using ffd::Job;
using ffd::KernelArgs;

namespace ffdi {

const char *kVersion = "ffd 0.2.0 (gfx950)";

int fail(ffd_ctx *ctx, int code, const char *msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

int hip_fail(ffd_ctx *ctx, hipError_t e, const char *what) {
  if (ctx) ctx->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return FFD_E_DEVICE;
}

// Modelled shader clocks of one stream step of a wave with R rows per lane.
// A step issues I VALU instructions per wave: (2D + 2) per cell (D
// subtractions, one multiply, D-1 FMAs, min3, max; FP64 needs two mins) and
// about 8 per step (lane shift, LDS stores, bookkeeping).  Fitted to
// measured lone waves (one per SIMD; 3-D single pairs at R = 2, 4, 8 and the
// 2-D batch at R = 8): about 104 + 3.9 I clocks.  Waves sharing a SIMD also
// share its wave64 issue slots (4 clocks each), which they keep about three
// quarters busy.  Other kernels (op = measure + 2 * cell): Euclidean cells
// add a square root per cell, a quarter-rate instruction (4 issue slots);
// Manhattan and Chebyshev cells take D subtractions and D - 1 additions or
// maxima with free absolute values, one instruction less; great-circle
// cells (ops 10, 11) are FP64 squared chords of unit vectors (D = 3), and
// DTW adds a float square root and arcsine per cell (about 20 instructions).
double step_clocks(int R, int D, bool exact, double waves_per_simd, int op) {
  D = ffd::kernel_dim(D);  // the wide kernels compute their zero coordinates too
  int cell = op >> 1;
  double per_cell = 2 * D + (exact ? 3 : 2) + (cell == 1 ? 4 : 0) - (cell == 2 || cell == 3 ? 1 : 0);
  if (op == 8) per_cell = 2 * D + 5;  // Levenshtein: a compare per coordinate, the flag, a select, 4 ops
  if (op == 11) per_cell += 20;
  double I = (double)R * per_cell + 8.0;
  double lone = 104.0 + 3.9 * I;
  double shared = 0.75 * std::max(1.0, waves_per_simd) * I * 4.0;
  return std::max(lone, shared);
}

// Stream steps a consumer band starts after its producer band.  At its
// refill at step t the consumer waits for the entries of its chunk
// [t + kFill, t + 2 kFill), i.e. up to t + 2 kFill - S_consumer; the
// producer publishes at its refill at step t' the count stored by its
// previous flush, t' - kFill - kWave - S_producer columns.  The wait
// therefore ends once the producer reaches t' = t + 3 kFill + kWave - lag:
// with lag = 5 kFill that is t - kFill, strictly before the waiting wave's
// own position.
constexpr double kLinkLag = 5.0 * ffd::kFill;

// Hash of 64-bit words (a multiply-xorshift mix per word): only used to
// tell requests apart quickly; equality is always decided on the words.
uint64_t mix_words(uint64_t h, const int64_t *w, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    h ^= (uint64_t)w[i] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h *= 0xFF51AFD7ED558CCDull;
    h ^= h >> 33;
  }
  return h;
}

int check_offsets(ffd_ctx *ctx, const int64_t *off, int64_t count, const char *name) {
  if (!off) return fail(ctx, FFD_E_INVALID, name);
  if (off[0] != 0) return fail(ctx, FFD_E_INVALID, "offsets must start at 0");
  bool bad = false;  // one pass without an early exit, which the compiler vectorises
  for (int64_t k = 0; k < count; ++k) bad |= off[k + 1] <= off[k];
  if (bad) return fail(ctx, FFD_E_INVALID, "offsets must be strictly increasing (empty curve)");
  return FFD_OK;
}

// kernel ops of the Frechet distance and of DTW on great-circle cells
constexpr int kOpGeo = 10;
constexpr int kOpGeoDtw = 11;

int check_common(ffd_ctx *ctx, int32_t dim, int32_t metric, bool exact) {
  if (!ctx) return FFD_E_INVALID;
  if (dim < 1) return fail(ctx, FFD_E_INVALID, "dim must be >= 1");
  if (metric < FFD_EUCLIDEAN || metric > FFD_HAVERSINE) return fail(ctx, FFD_E_INVALID, "unknown metric");
  if (dim > FFD_MAX_DIM) return fail(ctx, FFD_E_UNSUPPORTED, "dim exceeds FFD_MAX_DIM");
  // great-circle requests arrive here with the kernel's shape (geo_shape)
  if (metric == FFD_HAVERSINE && ctx->measure != kOpGeo && ctx->measure != kOpGeoDtw)
    return fail(ctx, FFD_E_UNSUPPORTED, "the great-circle distance is available for float32 curves");
  if (exact && metric == FFD_EUCLIDEAN)
    return fail(ctx, FFD_E_UNSUPPORTED, "int32 coordinates take the squared Euclidean, Manhattan or Chebyshev metric");
  return FFD_OK;
}

int lds_bytes(int R, int D, bool exact, int64_t hcap, bool rings, int measure) {
  D = ffd::kernel_dim(D);
  return ffd::lds_layout(R, D, exact ? 8 : 4, (int)hcap, rings, measure == 8 ? ffd::lev_dim(D) : 0).total;
}

const int kRs[4] = {1, 2, 4, 8};

// ---------------------------------------------------------------- units

// One row curve against a run of column curves, all bands of the row curve.
struct Unit {
  int32_t row_sel, row_idx, col_sel, col_first, col_count, out_stride;
  int64_t out_base;
  int64_t nrows;
  int32_t nb;      // bands
  int64_t sumL;    // stream steps of one band over all column curves
  int64_t maxL;    // longest task of the unit
  double steps() const { return (double)nb * (double)sumL; }
};

struct CurveSet {
  const int64_t *off;
  int64_t count;
  int64_t len(int64_t k) const { return off[k + 1] - off[k]; }
};

// Units of a batch: pair k, oriented to the cheaper number of steps.
void batch_units(const CurveSet &P, const CurveSet &Q, int R, std::vector<Unit> &units) {
  units.resize(P.count);
  for (int64_t k = 0; k < P.count; ++k) {
    int64_t n = P.len(k), m = Q.len(k);
    int64_t nb1 = ffd::bands_for(n, R), nb2 = ffd::bands_for(m, R);
    int64_t L1 = ffd::task_len(m, nb1 > 1), L2 = ffd::task_len(n, nb2 > 1);
    bool swap = nb2 * L2 < nb1 * L1;
    Unit &u = units[k];
    u.row_sel = swap ? 1 : 0;
    u.col_sel = swap ? 0 : 1;
    u.row_idx = u.col_first = (int32_t)k;
    u.col_count = 1;
    u.out_base = k;
    u.out_stride = 1;
    u.nrows = swap ? m : n;
    u.nb = (int32_t)(swap ? nb2 : nb1);
    u.sumL = u.maxL = swap ? L2 : L1;
  }
}

// Units of the pairs listed in idx only (the rest of a batch runs elsewhere).
void batch_units_of(const CurveSet &P, const CurveSet &Q, int R, const std::vector<int32_t> &idx,
                    std::vector<Unit> &units) {
  std::vector<Unit> all;
  units.clear();
  units.reserve(idx.size());
  for (int32_t k : idx) {
    int64_t off_p[2] = {0, P.len(k)}, off_q[2] = {0, Q.len(k)};
    CurveSet p1{off_p, 1}, q1{off_q, 1};
    batch_units(p1, q1, R, all);
    Unit u = all[0];
    u.row_idx = u.col_first = k;
    u.out_base = k;
    units.push_back(u);
  }
}

// Units of queries x database: query i against runs of consecutive database
// curves of about `target` steps each.
void cross_units(const CurveSet &Qs, const CurveSet &DB, int R, double target, std::vector<Unit> &units) {
  units.clear();
  for (int64_t i = 0; i < Qs.count; ++i) {
    int64_t nb = ffd::bands_for(Qs.len(i), R);
    int64_t k = 0;
    while (k < DB.count) {
      Unit u;
      u.row_sel = 0;
      u.row_idx = (int32_t)i;
      u.col_sel = 1;
      u.col_first = (int32_t)k;
      u.out_base = i * DB.count + k;
      u.out_stride = 1;
      u.nrows = Qs.len(i);
      u.nb = (int32_t)nb;
      u.sumL = 0;
      u.maxL = 0;
      while (k < DB.count) {
        int64_t L = ffd::task_len(DB.len(k), nb > 1);
        if (u.sumL > 0 && (double)nb * (double)(u.sumL + L) > target) break;
        u.sumL += L;
        u.maxL = std::max(u.maxL, L);
        ++k;
      }
      u.col_count = (int32_t)(k - u.col_first);
      units.push_back(u);
    }
  }
}

// ------------------------------------------------------------- scheduling

struct Task {
  int32_t unit;
  int32_t band_first, band_count;  // band_count 0: all bands
  int32_t pred;                    // task writing this task's incoming link, -1 none
  int32_t succ;                    // task reading this task's outgoing link, -1 none
  double dur;                      // stream steps
  double prio;                     // longest remaining chain (steps)
  int64_t chain_gap = 0;           // self-chained unit: idle steps between its bands, -1 not one
};

// Idle steps a band must wait after the previous band of its unit on the
// same wave when the boundary row goes through global memory.
int64_t self_gap(int64_t sumL) {
  if ((double)sumL >= kLinkLag) return 0;
  int64_t gap = std::max<int64_t>((int64_t)std::ceil(kLinkLag - (double)sumL), ffd::kMinTask);
  return (gap + ffd::kGroup - 1) / ffd::kGroup * ffd::kGroup;
}

// List scheduling with precedence (see the file comment).  Fills
// owner/order: the wave of every task and the tasks in placement order.
// Returns the modelled makespan in steps.
double list_schedule(const std::vector<Task> &tasks, int nwaves, std::vector<int> &owner,
                     std::vector<int32_t> &order, std::vector<double> &wave_steps) {
  const size_t nt = tasks.size();
  owner.assign(nt, -1);
  order.clear();
  order.reserve(nt);
  wave_steps.assign(nwaves, 0.0);
  using WaveItem = std::pair<double, int>;  // free time, wave
  std::priority_queue<WaveItem, std::vector<WaveItem>, std::greater<WaveItem>> waves;
  for (int w = 0; w < nwaves; ++w) waves.push({0.0, w});
  using Ready = std::pair<double, int32_t>;  // priority, task
  std::priority_queue<Ready> avail;          // ready now, highest priority first
  using Pending = std::pair<double, int32_t>;  // ready time, task
  std::priority_queue<Pending, std::vector<Pending>, std::greater<Pending>> pending;
  for (size_t i = 0; i < nt; ++i)
    if (tasks[i].pred < 0) avail.push({tasks[i].prio, (int32_t)i});
  double makespan = 0;
  std::vector<double> start(nt, 0.0);
  while (!avail.empty() || !pending.empty()) {
    WaveItem w = waves.top();
    waves.pop();
    double now = w.first;
    while (!pending.empty() && pending.top().first <= now) {
      avail.push({tasks[pending.top().second].prio, pending.top().second});
      pending.pop();
    }
    if (avail.empty()) {  // nothing ready yet: this wave idles until the next task is
      now = pending.top().first;
      avail.push({tasks[pending.top().second].prio, pending.top().second});
      pending.pop();
    }
    int32_t t = avail.top().second;
    avail.pop();
    double st = now;
    if (tasks[t].pred >= 0) st = std::max(st, start[tasks[t].pred] + kLinkLag);
    start[t] = st;
    owner[t] = w.second;
    order.push_back(t);
    wave_steps[w.second] += tasks[t].dur;
    double fin = st + tasks[t].dur;
    makespan = std::max(makespan, fin);
    waves.push({fin, w.second});
    if (tasks[t].succ >= 0) pending.push({st + kLinkLag, tasks[t].succ});
  }
  return makespan;
}


// Launch resources for R rows per lane and W waves per SIMD: every wave gets
// an equal share of the CU's LDS, which bounds the LDS hand-off row; all
// waves of the launch are resident at once (a wave waiting on a link may
// only wait on a running wave).
Resources resources(ffd_ctx *ctx, int R, int D, bool exact, int W) {
  Resources r;
  r.wpb = 4;
  while (r.wpb > 1 && (size_t)r.wpb * (ctx->lds_cu / (size_t)(4 * W)) > ctx->lds_block_max) r.wpb /= 2;
  // LDS is allocated to workgroups in granules; a block's share is rounded
  // down to 1 KiB so that 4W/wpb blocks surely fit one CU's LDS at once
  size_t blocks_per_cu = (size_t)std::max(1, 4 * W / r.wpb);
  size_t block_lds = ctx->lds_cu / blocks_per_cu / 1024 * 1024;
  size_t per_wave = block_lds / (size_t)r.wpb / 16 * 16;
  int vs = exact ? 8 : 4;
  int fixed = lds_bytes(R, D, exact, 0, false, ctx->measure);
  int64_t hand = ((int64_t)per_wave - fixed - 16) / vs;
  r.hand_max = hand > 0 ? hand : 0;
  r.nwaves_max = ctx->cus * 4 * W;
  size_t lds = (size_t)r.wpb * (size_t)lds_bytes(R, D, exact, r.hand_max, false, ctx->measure);
  if (ctx->device >= 0) {
    // registers may allow fewer resident waves than the LDS share assumes
    int blocks = 0;
    if (ffd::occupancy_stream(exact, R, D, r.wpb, lds, &blocks, false, ctx->measure) == hipSuccess && blocks > 0)
      r.nwaves_max = std::min(r.nwaves_max, ctx->cus * blocks * r.wpb);
  }
  // A launch whose waves wait on other waves needs every wave resident.
  // Count a workgroup's LDS in whole 4 KiB units (no coarser allocation
  // granule is assumed): a full CU at 3 workgroups of 53 KB did not hold
  // all of them at once in measurements, although the occupancy query said
  // it would.
  size_t rounded = (lds + 4095) / 4096 * 4096;
  int fit = (int)std::min<size_t>(blocks_per_cu, ctx->lds_cu / std::max<size_t>(rounded, 1));
  r.nwaves_coop = std::min(r.nwaves_max, ctx->cus * std::max(fit, 1) * r.wpb);
  return r;
}

// Turn units into tasks (splitting the long ones), schedule them on nwaves
// waves and lay the plan out.
void build_plan(const std::vector<Unit> &units, int R, int nwaves, double split_share, int64_t hand_max,
                Plan &pl) {
  double total = 0;
  for (const Unit &u : units) total += u.steps();
  double fair = total / std::max(1, nwaves);
  std::vector<Task> tasks;
  tasks.reserve(units.size());
  std::vector<char> split(units.size(), 0);  // 1: bands on several waves, 2: chained on one wave
  pl.coop = false;
  for (size_t i = 0; i < units.size(); ++i) {
    const Unit &u = units[i];
    bool need = u.nb > 1 && u.maxL > hand_max;
    bool want = u.nb > 1 && split_share >= 0 && u.steps() > split_share * fair;
    split[i] = want ? 1 : (need ? 2 : 0);
    if (split[i] == 0) {
      tasks.push_back({(int32_t)i, 0, 0, -1, -1, u.steps(), u.steps(), -1});
    } else if (split[i] == 2) {
      // the boundary row does not fit the LDS hand-off: the bands stay on
      // one wave in order and hand their rows on through global links
      int64_t gap = self_gap(u.sumL);
      double dur = u.steps() + (double)(u.nb - 1) * (double)gap;
      tasks.push_back({(int32_t)i, 0, 0, -1, -1, dur, dur, gap});
    } else {
      pl.coop = true;
      int32_t first = (int32_t)tasks.size();
      for (int32_t bnd = 0; bnd < u.nb; ++bnd) {
        double chain = (double)(u.nb - 1 - bnd) * kLinkLag + (double)u.sumL;
        tasks.push_back({(int32_t)i, bnd, 1, bnd > 0 ? first + bnd - 1 : -1,
                         bnd + 1 < u.nb ? first + bnd + 1 : -1, (double)u.sumL, chain, -1});
      }
    }
  }
  std::vector<int> owner;
  std::vector<int32_t> order;
  std::vector<double> wsteps;
  pl.makespan = list_schedule(tasks, nwaves, owner, order, wsteps);
  // links: one per band boundary of a split unit, sumL entries each
  std::vector<int64_t> link_of(tasks.size(), -1);  // outgoing link element start
  std::vector<int32_t> flag_of(tasks.size(), -1);
  pl.link_elems = 0;
  pl.nflags = 0;
  for (size_t t = 0; t < tasks.size(); ++t) {
    const Unit &u = units[tasks[t].unit];
    if (tasks[t].succ >= 0) {
      link_of[t] = pl.link_elems;
      flag_of[t] = pl.nflags++;
      pl.link_elems += u.sumL;
    } else if (tasks[t].chain_gap >= 0) {
      // one boundary row, rewritten in place by every band (a band reads
      // each entry, into LDS, well before it overwrites it), and one flag
      // per band boundary (each flag's count only grows)
      link_of[t] = pl.link_elems;
      flag_of[t] = pl.nflags;
      pl.nflags += u.nb - 1;
      pl.link_elems += u.sumL;
    }
  }
  pl.hcap = 0;
  for (size_t i = 0; i < units.size(); ++i)
    if (!split[i] && units[i].nb > 1) pl.hcap = std::max(pl.hcap, units[i].maxL);
  // Stream positions.  A wave runs its tasks back to back, so a task starts
  // at the sum of the stream lengths before it on its wave, whatever idle
  // time the model gave it.  Every consumer band must start at least
  // kLinkLag stream steps after its producer band: then each wait is for a
  // position strictly earlier than the waiting wave's own, so no set of
  // waves can wait on each other in a cycle.  Where the positions do not
  // give that, an idle job pads the consumer's stream.
  std::vector<double> spos(tasks.size(), 0.0), wpos(nwaves, 0.0);
  std::vector<int64_t> idle(tasks.size(), 0);
  for (int32_t t : order) {
    int w = owner[t];
    double s = wpos[w];
    if (tasks[t].pred >= 0 && s < spos[tasks[t].pred] + kLinkLag) {
      int64_t gap = (int64_t)std::ceil(spos[tasks[t].pred] + kLinkLag - s);
      gap = std::max<int64_t>(gap, ffd::kMinTask);
      gap = (gap + ffd::kGroup - 1) / ffd::kGroup * ffd::kGroup;
      idle[t] = gap;
      s += (double)gap;
    }
    spos[t] = s;
    wpos[w] = s + tasks[t].dur;
  }
  std::vector<int32_t> count(nwaves, 0);
  for (int32_t t : order) {
    const Task &tk = tasks[t];
    int32_t nbands = tk.chain_gap >= 0 ? units[tk.unit].nb : 1;
    count[owner[t]] += (idle[t] > 0 ? 1 : 0) + nbands + (tk.chain_gap > 0 ? nbands - 1 : 0);
  }
  pl.wave_jobs.assign(nwaves + 1, 0);
  for (int w = 0; w < nwaves; ++w) pl.wave_jobs[w + 1] = pl.wave_jobs[w] + count[w];
  std::vector<int32_t> fillp(pl.wave_jobs.begin(), pl.wave_jobs.end() - 1);
  pl.jobs.resize(pl.wave_jobs[nwaves]);
  for (int32_t t : order) {
    const Task &tk = tasks[t];
    const Unit &u = units[tk.unit];
    Job jb;
    if (idle[t] > 0) {
      memset(&jb, 0, sizeof jb);
      jb.row_sel = ffd::kRowIdle;
      jb.col_count = (int32_t)idle[t];
      jb.link_in = jb.link_out = -1;
      jb.flag_in = jb.flag_out = -1;
      pl.jobs[fillp[owner[t]]++] = jb;
    }
    jb.out_base = u.out_base;
    jb.row_sel = u.row_sel;
    jb.row_idx = u.row_idx;
    jb.col_sel = u.col_sel;
    jb.col_first = u.col_first;
    jb.col_count = u.col_count;
    jb.out_stride = u.out_stride;
    if (tk.chain_gap < 0) {
      jb.band_first = tk.band_first;
      jb.band_count = tk.band_count;
      jb.link_in = tk.pred >= 0 ? link_of[tk.pred] : -1;
      jb.flag_in = tk.pred >= 0 ? flag_of[tk.pred] : -1;
      jb.link_out = link_of[t];
      jb.flag_out = flag_of[t];
      pl.jobs[fillp[owner[t]]++] = jb;
      continue;
    }
    // self-chained unit: one job per band, each band after an idle job
    // where the bands are too short to keep kLinkLag apart
    for (int32_t b = 0; b < u.nb; ++b) {
      if (b > 0 && tk.chain_gap > 0) {
        Job idle_job;
        memset(&idle_job, 0, sizeof idle_job);
        idle_job.row_sel = ffd::kRowIdle;
        idle_job.col_count = (int32_t)tk.chain_gap;
        idle_job.link_in = idle_job.link_out = -1;
        idle_job.flag_in = idle_job.flag_out = -1;
        pl.jobs[fillp[owner[t]]++] = idle_job;
      }
      jb.band_first = b;
      jb.band_count = 1;
      jb.link_in = b > 0 ? link_of[t] : -1;
      jb.flag_in = b > 0 ? flag_of[t] + b - 1 : -1;
      jb.link_out = b + 1 < u.nb ? link_of[t] : -1;
      jb.flag_out = b + 1 < u.nb ? flag_of[t] + b : -1;
      pl.jobs[fillp[owner[t]]++] = jb;
    }
  }
  double mx = 0;
  for (double x : wpos) mx = std::max(mx, x);
  pl.max_steps = (int64_t)mx;
  pl.nwaves = nwaves;
  pl.R = R;
}

// Batched and cross launches split a unit into bands over several waves
// when it is longer than 1.25 times a wave's fair share of the launch: a
// unit that long would otherwise set the launch's makespan, while splitting
// shorter units costs more in link lag and waiting than the balance gains
// (measured on the 4096-pair workload: 1.07 ms at 1.25, 1.10 ms at 1.0,
// 1.16 ms at 1.5, 1.23 ms without splitting).
double split_share(ffd_ctx *ctx) {
  if (ctx->split == 0.f) return 1.25;
  if (ctx->split < 0.f) return -1.0;
  return ctx->split;
}

// Plan the units produced by `make(R, W, units)` for the R with the lowest
// modelled stream length times per-step clocks.
// A single long pair as a pipeline of its bands, band b on wave b: bands
// of one workgroup hand their bottom rows on through LDS rings and start
// kWave + kGroup stream steps after each other; bands of consecutive
// workgroups hand them on through global links and start kLinkLag steps
// after each other.  Every wave is resident at once (cooperative launch).
// Returns false when the pair has too many bands for that.
bool build_pipeline(ffd_ctx *ctx, const Unit &u, int R, int D, bool exact, Plan &pl) {
  const int wpb = 4;
  if (u.nb < 2) return false;
  int lds_wave = lds_bytes(R, D, exact, 0, true);
  size_t block = (size_t)wpb * (size_t)lds_wave;
  if (block > ctx->lds_block_max) return false;
  size_t rounded = (block + 4095) / 4096 * 4096;
  int fit = (int)std::min<size_t>(16 / wpb, ctx->lds_cu / rounded);
  if (ctx->device >= 0) {
    int blocks = 0;
    if (ffd::occupancy_stream(exact, R, D, wpb, block, &blocks, true) != hipSuccess || blocks < 1) return false;
    fit = std::min(fit, blocks);
  }
  if ((int64_t)u.nb > (int64_t)ctx->cus * fit * wpb) return false;
  const int32_t nb = u.nb;
  pl = Plan();
  pl.R = R;
  pl.nwaves = nb;
  pl.wpb = std::min(wpb, nb);
  pl.hcap = 0;
  pl.rings = true;
  pl.coop = nb > wpb;
  pl.wave_jobs.assign(nb + 1, 0);
  pl.jobs.clear();
  int64_t start = 0;
  int64_t gl_link = -1;
  int32_t gl_flag = -1;
  for (int32_t b = 0; b < nb; ++b) {
    bool ring_in = b > 0 && b % wpb != 0;
    if (b > 0) start += ring_in ? (int64_t)(ffd::kWave + ffd::kGroup) : (int64_t)kLinkLag;
    pl.wave_jobs[b] = (int32_t)pl.jobs.size();
    if (start > 0) {
      Job idle;
      memset(&idle, 0, sizeof idle);
      idle.row_sel = ffd::kRowIdle;
      idle.col_count = (int32_t)start;
      idle.link_in = idle.link_out = -1;
      idle.flag_in = idle.flag_out = -1;
      pl.jobs.push_back(idle);
    }
    Job jb;
    memset(&jb, 0, sizeof jb);
    jb.out_base = u.out_base;
    jb.row_sel = u.row_sel;
    jb.row_idx = u.row_idx;
    jb.col_sel = u.col_sel;
    jb.col_first = u.col_first;
    jb.col_count = u.col_count;
    jb.out_stride = u.out_stride;
    jb.band_first = b;
    jb.band_count = 1;
    jb.link_in = jb.link_out = -1;
    jb.flag_in = jb.flag_out = -1;
    if (ring_in) {
      jb.flag_in = -2 - ((b - 1) % wpb);
    } else if (b > 0) {
      jb.link_in = gl_link;
      jb.flag_in = gl_flag;
    }
    if (b + 1 < nb) {
      if ((b + 1) % wpb != 0) {
        jb.flag_out = -2;
      } else {
        gl_link = pl.link_elems;
        gl_flag = pl.nflags++;
        pl.link_elems += u.sumL;
        jb.link_out = gl_link;
        jb.flag_out = gl_flag;
      }
    }
    pl.jobs.push_back(jb);
  }
  pl.wave_jobs[nb] = (int32_t)pl.jobs.size();
  pl.max_steps = start + u.sumL;
  pl.makespan = (double)pl.max_steps;
  return true;
}

template <typename MakeUnits>
int plan_units(ffd_ctx *ctx, int D, bool exact, int W, double share, bool single, MakeUnits make, Plan &best,
               double *best_cost_out = nullptr) {
  double best_cost = -1;
  for (int R : kRs) {
    if (ctx->tune_R && R != ctx->tune_R) continue;
    if (D > 4 && R != ffd::wide_rows(D)) continue;  // the wide kernels' only shape
    // great-circle DTW inlines an arcsine per cell and row: at R = 8 the
    // kernel spills registers to scratch memory
    if (!ctx->tune_R && ctx->measure == kOpGeoDtw && R > 4) continue;
    Resources rs = resources(ctx, R, D, exact, W);
    std::vector<Unit> units;
    make(R, W, units);
    size_t ntasks = 0;
    for (const Unit &u : units) ntasks += (size_t)u.nb;  // tasks if every unit were split
    int nwaves = rs.nwaves_max;
    if ((size_t)nwaves > ntasks) nwaves = (int)std::max<size_t>(1, ntasks);
    Plan pl;
    build_plan(units, R, nwaves, share, rs.hand_max, pl);
    if (pl.coop && pl.nwaves > rs.nwaves_coop) {
      Plan fewer;
      build_plan(units, R, rs.nwaves_coop, share, rs.hand_max, fewer);
      pl = std::move(fewer);
    }
    if (single && pl.link_elems > 0) {
      // a single pair: compare with the whole pair on one wave
      Plan whole;
      build_plan(units, R, 1, -1.0, rs.hand_max, whole);
      if (whole.link_elems == 0 && whole.max_steps <= pl.max_steps) pl = std::move(whole);
    }
    pl.wpb = std::min(rs.wpb, pl.nwaves);
    double wps = std::ceil((double)pl.nwaves / (4.0 * ctx->cus));
    double cost = ((double)pl.max_steps + ffd::kWave) * step_clocks(R, D, exact, wps, ctx->measure);
    Plan pipe;
    if (single && share >= 0 && units.size() == 1 && ctx->measure == 0 &&
        build_pipeline(ctx, units[0], R, D, exact, pipe)) {
      double pw = std::ceil((double)pipe.nwaves / (4.0 * ctx->cus));
      double pc = ((double)pipe.max_steps + ffd::kWave) * step_clocks(R, D, exact, pw);
      if (pc < cost) {
        cost = pc;
        pl = std::move(pipe);
      }
    }
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = std::move(pl);
    }
  }
  if (best_cost < 0) return fail(ctx, FFD_E_UNSUPPORTED, "no feasible launch shape");
  if (best_cost_out) *best_cost_out = best_cost;
  return FFD_OK;
}

// ------------------------------------------------------ pipelined single pair
//
// A single long pair on the pipelined kernel (ffd_pipe.h): one band of 64 R
// rows per wave, four waves per workgroup in lockstep (kPipeLag groups of
// 16 steps apart), workgroups chained through link rows in global memory.
// Modelled stream steps: the last band starts about 88 steps per band
// after the first (5 groups inside a workgroup, about 7 between
// workgroups: the last wave stores a group's link values when it starts
// its fifth group after it, and the next workgroup needs them one group
// before their own group), or, with several passes, when its wave has
// swept its earlier bands; each band sweeps the columns plus the lanes'
// ramp and the link flush.
// Clocks per step: one instruction per 4 clocks (one wave per SIMD issues
// alone), R cells of 2 D + 2 instructions (FP64: 2 D + 3) and about 7 per
// step of lane shift, LDS traffic and bookkeeping.
constexpr double kPipeBandLag = (3 * ffd::kPipeLag * ffd::kPipeGroup + 7 * ffd::kPipeGroup) / 4.0;

double pipe_step_clocks(int R, int D, bool exact) {
  return 4.0 * (R * (2 * D + 2 + (exact ? 1 : 0)) + 7 + (exact ? 2 : 0));
}

// A pipelined plan for rows x cols with R rows per lane; false when the
// kernel cannot run it.
bool build_pipe(ffd_ctx *ctx, int64_t rows, int64_t cols, int R, int D, bool exact, Plan &pl, double &cost) {
  if (R != 2 && R != 4) return false;
  if (D > 4) return false;  // instantiated for up to four coordinates
  const int64_t nb = ffd::bands_for(rows, R);
  if (nb < 2 || nb > INT32_MAX / 2 || cols < 2) return false;
  size_t lds = ffd::pipe_lds(exact, D);
  if (lds > ctx->lds_block_hw) return false;
  // one workgroup (four waves, one per SIMD) per compute unit: request more
  // than half of a compute unit's LDS where a workgroup may, so that the
  // hardware cannot place two workgroups on one compute unit (two waves
  // sharing a SIMD would halve the pace of the whole chain)
  if (ctx->lds_cu / 2 + 4096 <= ctx->lds_block_hw) lds = std::max(lds, ctx->lds_cu / 2 + 4096);
  int64_t nwg = (nb + ffd::kPipeWaves - 1) / ffd::kPipeWaves;
  int64_t cap = ctx->cus;
  if (ctx->device >= 0) {
    int blocks = 0;
    if (ffd::occupancy_pipe(exact, R, D, lds, &blocks) != hipSuccess || blocks < 1) return false;
  }
  if (nwg > cap) nwg = cap;
  int32_t xcd = 0;
  if (nwg >= 8) {
    int64_t up = (nwg + 7) / 8 * 8;
    if (up > cap) up = cap / 8 * 8;
    if (up >= nwg || up >= 8) {
      nwg = up;
      xcd = (int32_t)(nwg / 8);
    }
  }
  const int64_t W = nwg * ffd::kPipeWaves;
  const int64_t passes = (nb + W - 1) / W;
  const double sweep = (double)(((cols - 1) / ffd::kPipeGroup + 6) * ffd::kPipeGroup);
  const double chain = (double)(nb - 1) * kPipeBandLag;
  const double wrap = (double)(passes - 1) * sweep + (double)((nb - 1) % W) * kPipeBandLag;
  const double steps = std::max(chain, wrap) + sweep;
  if (steps + 64 > (double)INT32_MAX) return false;
  pl = Plan();
  pl.R = R;
  pl.nwaves = (int)W;
  pl.wpb = ffd::kPipeWaves;
  pl.coop = true;
  pl.pipe = true;
  pl.pipe_nb = (int32_t)nb;
  pl.pipe_nwg = (int32_t)nwg;
  pl.pipe_xcd = xcd;
  pl.pipe_rows = rows;
  pl.pipe_cols = cols;
  pl.pipe_stride = (cols + 63) / 64 * 64;
  // one link row per band that hands its bottom row to another workgroup
  pl.pipe_nlinks = (nb - 1) / ffd::kPipeWaves;
  pl.pipe_lds = lds;
  pl.link_elems = pl.pipe_nlinks * pl.pipe_stride;
  pl.max_steps = (int64_t)steps;
  pl.makespan = steps;
  cost = steps * pipe_step_clocks(R, D, exact);
  return true;
}

// Scratch of a pipelined launch: the error word, then the link rows (none
// for a pair inside one workgroup, which then needs no scratch at all).
struct PipeLayout {
  size_t err, links, total;
};

PipeLayout pipe_layout(const Plan &pl, bool exact) {
  PipeLayout L{0, 0, 0};
  if (pl.pipe_nlinks == 0) return L;
  L.err = 0;
  L.links = 256;
  L.total = L.links + (size_t)pl.link_elems * (exact ? 8 : 4);
  L.total = (L.total + 255) & ~(size_t)255;
  return L;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
  size_t jobs, wj, off0, off1, lo0, lo1, order, flags, err, links, total;
};

WsLayout ws_layout(const Plan &pl, int64_t n0, int64_t n1, bool exact) {
  WsLayout w;
  size_t o = 0;
  w.jobs = o;  o = al256(o + pl.jobs.size() * sizeof(Job));
  w.wj = o;    o = al256(o + (size_t)(pl.nwaves + 1) * sizeof(int32_t));
  // 64-bit offsets for the streaming kernel, 32-bit ones for the lane kernel
  const bool stream = !pl.lanes || !pl.jobs.empty();
  w.off0 = o;  o = al256(o + (stream ? (size_t)(n0 + 1) * sizeof(int64_t) : 0));
  w.off1 = o;  o = al256(o + (stream ? (size_t)(n1 + 1) * sizeof(int64_t) : 0));
  w.lo0 = o;   o = al256(o + (pl.lanes ? (size_t)(n0 + 1) * sizeof(int32_t) : 0));
  w.lo1 = o;   o = al256(o + (pl.lanes ? (size_t)(n1 + 1) * sizeof(int32_t) : 0));
  w.order = o; o = al256(o + pl.lane_order.size() * sizeof(int32_t));
  w.flags = o; o = al256(o + (size_t)pl.nflags * sizeof(uint64_t));
  w.err = o;   o = al256(o + sizeof(uint64_t));
  w.links = o; o = al256(o + (size_t)pl.link_elems * (exact ? 8 : 4));
  w.total = o;
  return w;
}

// ------------------------------------------------------ short pairs per lane
//
// A batch whose pairs all have a curve of at most lane_cols_max points runs
// on the one-pair-per-lane kernel (ffd_lanes.hip) when the model says it is
// faster: each lane sweeps the longer curve's rows against the shorter
// curve held in registers, padded to a multiple of 8 columns (classes of
// column count, the widest first, in one launch), the pairs of a class in decreasing row
// count so that the lanes of a wavefront sweep about as many rows.
// Modelled clocks: per row of a lane, M cells of 2 D + 2 instructions
// (FP64: 2 D + 3) and about 8 of loop and load work; a wavefront takes its
// longest lane's rows; the wavefronts share the SIMDs at about one
// instruction per 4.5 clocks, and no wavefront can finish before its own
// rows at one per 5 clocks (alone on a SIMD).
// With `rest`, pairs whose curves are both longer than a lane holds are
// listed there instead of making the batch ineligible (false: no pair fits).
// With col_count > 0, the pairs are (query, database curve): p_off holds
// the npairs / col_count queries, q_off the col_count database curves, pair
// i * col_count + c.
// Cells a lane sweeps for rows x cols: the rows two at a time, the columns
// padded to the next multiple of kLaneColStep.
int64_t lane_padded(int64_t rows, int64_t cols) {
  return (rows + 1) / 2 * 2 * ((cols + ffd::kLaneColStep - 1) / ffd::kLaneColStep * ffd::kLaneColStep);
}

bool build_lanes(ffd_ctx *ctx, const int64_t *p_off, const int64_t *q_off, int64_t npairs, int D, bool exact,
                 Plan &pl, double &cost, std::vector<int32_t> *rest = nullptr, int64_t col_count = 0) {
  // the Frechet distance on squared Euclidean, Manhattan or Chebyshev cells,
  // DTW on those or on Euclidean cells (ops 0 ... 7), Levenshtein (op 8)
  const int op = ctx->measure;
  if (op < 0 || op > 8 || op == 2 || D > 4 || npairs < 1 || npairs > INT32_MAX) return false;
  // the kernel reads 32-bit offsets (half the upload of every call)
  const int64_t n0 = col_count > 0 ? npairs / col_count : npairs, n1 = col_count > 0 ? col_count : npairs;
  if (p_off[n0] > INT32_MAX || q_off[n1] > INT32_MAX) return false;
  const int cmax = ffd::lane_cols_max(exact, D);
  struct Item {
    int64_t rows;
    int32_t key;
  };
  std::vector<Item> cls[ffd::kLaneClasses];
  for (int64_t k = 0; k < npairs; ++k) {
    const int64_t i0 = col_count > 0 ? k / col_count : k, i1 = col_count > 0 ? k % col_count : k;
    const int64_t n = p_off[i0 + 1] - p_off[i0], m = q_off[i1 + 1] - q_off[i1];
    // the shorter curve holds the columns.  Levenshtein: when both fit, the
    // curve that leaves less padded work (rows go two at a time, columns to
    // a multiple of kLaneColStep); the table's values are the same either
    // way.  (Measured on 262,144 pairs of 8 ... 64: 3 % faster for
    // Levenshtein, 6 % slower for the Frechet distance of 2-D float curves,
    // whose longer column curve is a longer burst of loads before the sweep)
    bool swap = n < m;
    if (op == 8 && n <= cmax && m <= cmax) {
      const int64_t keep = lane_padded(n, m), turn = lane_padded(m, n);
      swap = turn < keep || (turn == keep && n < m);
    }
    const int64_t cols = swap ? n : m, rows = swap ? m : n;
    if (cols > cmax) {
      if (!rest) return false;
      rest->push_back((int32_t)k);
      continue;
    }
    const int c = (int)((cols - 1) / ffd::kLaneColStep);  // columns padded to (c + 1) * kLaneColStep
    cls[c].push_back({rows, (int32_t)((uint32_t)k | (swap ? 0x80000000u : 0u))});
  }
  if (rest && rest->size() == (size_t)npairs) return false;
  pl = Plan();
  pl.lanes = true;
  pl.lane_cross = col_count;
  pl.R = 0;
  pl.wpb = 4;
  double total = 0, longest = 0;
  for (int c = ffd::kLaneClasses - 1; c >= 0; --c) {
    if (cls[c].empty()) continue;
    std::stable_sort(cls[c].begin(), cls[c].end(), [](const Item &a, const Item &b) { return a.rows > b.rows; });
    const int i = pl.lane_classes++;
    pl.lane_cols[i] = (c + 1) * ffd::kLaneColStep;
    pl.lane_first[i] = (int64_t)pl.lane_order.size();
    const double per_cell =
        op == 8 ? 2 * D + 5 : 2 * D + (exact ? 3 : 2) + ((op >> 1) == 1 ? 4 : 0);  // Levenshtein: 2 D + 5
    const double per_row = (double)((c + 1) * ffd::kLaneColStep) * per_cell + 8.0;
    for (size_t w = 0; w < cls[c].size(); w += ffd::kWave) {
      const double v = (double)cls[c][w].rows * per_row;  // the wavefront's longest lane
      total += v;
      longest = std::max(longest, v);
      pl.max_steps = std::max<int64_t>(pl.max_steps, cls[c][w].rows);
    }
    for (const Item &it : cls[c]) pl.lane_order.push_back(it.key);
    pl.lane_first[i + 1] = (int64_t)pl.lane_order.size();
    pl.nwaves += (int)((cls[c].size() + ffd::kWave - 1) / ffd::kWave);
  }
  pl.makespan = (double)pl.max_steps;
  cost = std::max(total * 4.5 / (4.0 * ctx->cus), longest * 5.0);
  return true;
}

int plan_batch(ffd_ctx *ctx, const int64_t *p_off, const int64_t *q_off, int64_t npairs, int D, bool exact,
               Plan &pl) {
  CurveSet P{p_off, npairs}, Q{q_off, npairs};
  int W = ctx->tune_W > 0 ? ctx->tune_W : 2;
  double cost = -1;
  int rc = plan_units(ctx, D, exact, W, split_share(ctx), false,
                      [&](int R, int, std::vector<Unit> &u) { batch_units(P, Q, R, u); }, pl, &cost);
  if (rc) return rc;
  // short pairs, one per lane, when no launch shape is forced and the model
  // prefers it: the whole batch, or its short pairs in a launch before the
  // streaming kernel's for the rest
  if (ctx->tune_R == 0 && ctx->tune_W == 0 && ctx->split == 0.f) {
    Plan lanes;
    double lc = 0;
    std::vector<int32_t> rest;
    if (build_lanes(ctx, p_off, q_off, npairs, D, exact, lanes, lc, &rest) && lc < cost) {
      const size_t alt = ws_layout(pl, npairs, npairs, exact).total;  // the job-table plan for all
      if (rest.empty()) {
        pl = std::move(lanes);
        pl.alt_ws = alt;
      } else {
        Plan longp;
        double sc = -1;
        rc = plan_units(ctx, D, exact, W, split_share(ctx), false,
                        [&](int R, int, std::vector<Unit> &u) { batch_units_of(P, Q, R, rest, u); }, longp, &sc);
        if (rc == FFD_OK && lc + sc < cost) {
          longp.lanes = true;
          longp.lane_classes = lanes.lane_classes;
          std::copy(lanes.lane_cols, lanes.lane_cols + ffd::kLaneClasses, longp.lane_cols);
          std::copy(lanes.lane_first, lanes.lane_first + ffd::kLaneClasses + 1, longp.lane_first);
          longp.lane_order = std::move(lanes.lane_order);
          longp.lane_waves = lanes.nwaves;
          pl = std::move(longp);
          pl.alt_ws = alt;
        }
      }
    }
  }
  return FFD_OK;
}

int plan_cross(ffd_ctx *ctx, const int64_t *q_off, int64_t nq, const int64_t *db_off, int64_t ndb, int D,
               bool exact, Plan &pl) {
  CurveSet Qs{q_off, nq}, DB{db_off, ndb};
  int W = ctx->tune_W > 0 ? ctx->tune_W : 2;
  double cost = -1;
  int rc = plan_units(ctx, D, exact, W, split_share(ctx), false,
                      [&](int R, int Wv, std::vector<Unit> &u) {
                        // about eight units per wave
                        double total = 0, cols = 0;
                        for (int64_t k = 0; k < ndb; ++k) cols += (double)ffd::task_len(DB.len(k), false);
                        for (int64_t i = 0; i < nq; ++i) total += (double)ffd::bands_for(Qs.len(i), R) * cols;
                        double target = total / ((double)ctx->cus * 4 * Wv * 8.0);
                        cross_units(Qs, DB, R, std::max(target, 1.0), u);
                      },
                      pl, &cost);
  if (rc) return rc;
  // every (query, database curve) pair short: one pair per lane, when no
  // launch shape is forced and the model prefers it
  if (ctx->tune_R == 0 && ctx->tune_W == 0 && ctx->split == 0.f && nq * ndb <= INT32_MAX) {
    Plan lanes;
    double lc = 0;
    if (build_lanes(ctx, q_off, db_off, nq * ndb, D, exact, lanes, lc, nullptr, ndb) && lc < cost) {
      const size_t alt = ws_layout(pl, nq, ndb, exact).total;  // the job-table plan
      pl = std::move(lanes);
      pl.alt_ws = alt;
    }
  }
  return FFD_OK;
}

// One pair; a long pair is split into bands over waves when that pays.
int plan_pair(ffd_ctx *ctx, int64_t n, int64_t m, int D, bool exact, Plan &pl) {
  int64_t off0[2] = {0, n}, off1[2] = {0, m};
  CurveSet P{off0, 1}, Q{off1, 1};
  int W = ctx->tune_W > 0 ? ctx->tune_W : 1;
  double share = ctx->split < 0.f ? -1.0 : 0.0;
  double cost = -1;
  int rc = plan_units(ctx, D, exact, W, share, true,
                      [&](int R, int, std::vector<Unit> &u) { batch_units(P, Q, R, u); }, pl, &cost);
  if (rc) return rc;
  // the Frechet distance on squared cells may run on the pipelined kernel,
  // either curve holding the rows, when the model says it is faster
  // (waves_per_simd = -1 asks for it whenever it can run the pair)
  if (ctx->measure != 0 || share < 0 || ctx->tune_W > 0) return FFD_OK;
  const bool force = ctx->tune_W < 0;
  double best_pipe = -1;
  for (int R : {2, 4}) {
    if (ctx->tune_R && R != ctx->tune_R) continue;
    for (int swap = 0; swap < 2; ++swap) {
      Plan pp;
      double pc = 0;
      if (!build_pipe(ctx, swap ? m : n, swap ? n : m, R, D, exact, pp, pc)) continue;
      pp.pipe_swap = swap != 0;
      if ((force && (best_pipe < 0 || pc < best_pipe)) || (!force && pc < cost)) {
        best_pipe = cost = pc;
        pl = std::move(pp);
      }
    }
  }
  return FFD_OK;
}

// ---------------------------------------------------------------- workspace



// The staging buffer for plan uploads, at least `bytes` long.  Replacing
// its contents first waits until every upload has read it: the last one
// (the event), or, when uploads since the last rewrite went to several
// streams, all work on the device.
int ensure_pinned(ffd_ctx *ctx, size_t bytes) {
  if (ctx->upload_streams_mixed) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize (plan upload)");
  } else if (ctx->upload_done) {
    hipError_t e = hipEventSynchronize(ctx->upload_done);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize (plan upload)");
  }
  ctx->upload_streams_mixed = false;
  ctx->upload_stream = nullptr;
  ctx->staged_gen = 0;
  if (ctx->pinned_bytes >= bytes) return FFD_OK;
  if (ctx->pinned) {
    hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
  }
  hipError_t e = hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipHostMalloc");
  ctx->pinned_bytes = bytes;
  return FFD_OK;
}

// Whether work submitted to `st` is being recorded into a graph.
hipError_t capturing_on(hipStream_t st, bool &capturing) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  capturing = cs != hipStreamCaptureStatusNone;
  return e;
}

int use_begin(ffd_ctx *ctx, UseOrder &u, const void *ptr, hipStream_t st, bool capturing) {
  if (capturing || !u.pending || u.ptr != ptr || u.stream == st) return FFD_OK;
  hipError_t e = hipStreamWaitEvent(st, u.done, 0);
  return e == hipSuccess ? FFD_OK : hip_fail(ctx, e, "hipStreamWaitEvent");
}

int use_end(ffd_ctx *ctx, UseOrder &u, const void *ptr, hipStream_t st, bool capturing) {
  if (capturing) return FFD_OK;
  if (!u.done) {
    hipError_t e = hipEventCreateWithFlags(&u.done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
  }
  hipError_t e = hipEventRecord(u.done, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
  u.ptr = ptr;
  u.stream = st;
  u.pending = true;
  return FFD_OK;
}

// Run a planned launch.  Outside graph capture the plan (jobs, job ranges,
// offsets, zeroed flags and error word) is uploaded into the workspace on
// every call: the library never trusts what device memory it does not own
// held between calls.  The staging copy in pinned host memory is rebuilt
// only when the plan changes.  A launch recorded into a graph cannot
// upload (each replay would read the staging buffer as it is then); it
// requires the plan that the context's last eager upload put into this
// workspace, and the recorded work clears the flags and the error word
// first, since every replay reuses the recorded epoch.
// Copy the plan image of a launch (jobs, job ranges, offsets, zeroed flags
// and error word) into host memory at h.
void plan_image(const Plan &pl, const WsLayout &wl, const int64_t *off0, int64_t n0, const int64_t *off1,
                int64_t n1, unsigned char *h) {
  if (!pl.jobs.empty()) memcpy(h + wl.jobs, pl.jobs.data(), pl.jobs.size() * sizeof(Job));
  if (!pl.wave_jobs.empty()) memcpy(h + wl.wj, pl.wave_jobs.data(), pl.wave_jobs.size() * sizeof(int32_t));
  if (pl.lanes) {
    // 32-bit offsets (the planner checked that they fit)
    int32_t *o0 = reinterpret_cast<int32_t *>(h + wl.lo0), *o1 = reinterpret_cast<int32_t *>(h + wl.lo1);
    for (int64_t k = 0; k <= n0; ++k) o0[k] = (int32_t)off0[k];
    for (int64_t k = 0; k <= n1; ++k) o1[k] = (int32_t)off1[k];
  }
  if (!pl.lanes || !pl.jobs.empty()) {
    memcpy(h + wl.off0, off0, (size_t)(n0 + 1) * sizeof(int64_t));
    memcpy(h + wl.off1, off1, (size_t)(n1 + 1) * sizeof(int64_t));
  }
  if (!pl.lane_order.empty()) memcpy(h + wl.order, pl.lane_order.data(), pl.lane_order.size() * sizeof(int32_t));
  memset(h + wl.flags, 0, wl.links - wl.flags);  // flags and error word
}

// Kernel timing: an event on the launch stream before the first kernel and
// after the last one of a launch (never inside a graph capture).
constexpr size_t kMaxTimedLaunches = 1 << 16;

int time_mark(ffd_ctx *ctx, hipStream_t st, bool capturing) {
  if (!ctx->timing || capturing || ctx->tev_used >= 2 * kMaxTimedLaunches) return FFD_OK;
  if (ctx->tev_used == ctx->tev.size()) {
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate (timing)");
    ctx->tev.push_back(ev);
  }
  hipError_t e = hipEventRecord(ctx->tev[ctx->tev_used], st);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord (timing)");
  ++ctx->tev_used;
  return FFD_OK;
}

int run_plan(ffd_ctx *ctx, const Plan &pl, uint64_t gen, const void *X0, const int64_t *off0, int64_t n0,
             const void *X1, const int64_t *off1, int64_t n1, int D, bool exact, int metric, void *out, void *ws,
             size_t ws_bytes, hipStream_t st, UseOrder &use, bool noalloc = false) {
  WsLayout wl = ws_layout(pl, n0, n1, exact);
  ctx->last = ffd_launch_info{pl.R, pl.nwaves, pl.wpb, lds_bytes(pl.R, D, exact, pl.hcap, pl.rings, ctx->measure),
                              exact ? 1 : 0, D, 0, 0, pl.max_steps};
  if (noalloc && ws_bytes < wl.total) {
    std::string msg = "the request needs " + std::to_string(wl.total) +
                      " bytes of device scratch; ffd_batch_noalloc has " + std::to_string(ws_bytes);
    return fail(ctx, FFD_E_NOMEM, msg.c_str());
  }
  if (noalloc && ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot launch");
  if (!ws || ws_bytes < wl.total) return fail(ctx, FFD_E_NOMEM, "workspace too small (see ffd_workspace_size)");
  if (pl.max_steps + 4 * ffd::kRing > INT32_MAX) return fail(ctx, FFD_E_UNSUPPORTED, "stream too long");
  if (ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot launch");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  bool capturing = false;
  e = capturing_on(st, capturing);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamIsCapturing");
  unsigned char *w = (unsigned char *)ws;
  int rc = use_begin(ctx, use, ws, st, capturing);
  if (rc) return rc;
  if (noalloc && !capturing) {
    // pageable host memory, copied by the runtime's own staging before the
    // copy call returns, so the image may change again afterwards
    if (ctx->noalloc_gen != gen || ctx->noalloc_img.size() < wl.links) {
      ctx->noalloc_img.resize(wl.links);
      plan_image(pl, wl, off0, n0, off1, n1, ctx->noalloc_img.data());
      ctx->noalloc_gen = gen;
    }
    e = hipMemcpyAsync(w, ctx->noalloc_img.data(), wl.links, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync (plan)");
    ctx->plan_ws = ws;
    ctx->plan_ws_gen = gen;
  } else if (!capturing) {
    if (ctx->staged_gen != gen) {
      if ((rc = ensure_pinned(ctx, wl.links))) return rc;
      plan_image(pl, wl, off0, n0, off1, n1, (unsigned char *)ctx->pinned);
      ctx->staged_gen = gen;
    }
    e = hipMemcpyAsync(w, ctx->pinned, wl.links, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync (plan)");
    if (!ctx->upload_done) {
      e = hipEventCreateWithFlags(&ctx->upload_done, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
    }
    e = hipEventRecord(ctx->upload_done, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    if (ctx->upload_stream && ctx->upload_stream != st) ctx->upload_streams_mixed = true;
    ctx->upload_stream = st;
    ctx->plan_ws = ws;
    ctx->plan_ws_gen = gen;
  } else {
    if (!(ctx->plan_ws == ws && ctx->plan_ws_gen == gen))
      return fail(ctx, FFD_E_UNSUPPORTED,
                  "a launch recorded into a graph needs its plan in the workspace: make the same call on the same "
                  "workspace outside the capture just before");
    if (!(pl.lanes && pl.jobs.empty())) {  // the per-lane kernel alone reads no flags
      e = ffd::clear_words((uint64_t *)(w + wl.flags), (int64_t)((wl.links - wl.flags) / sizeof(uint64_t)), st);
      if (e != hipSuccess) return hip_fail(ctx, e, "flag clearing launch");
    }
  }
  if (pl.lanes) {
    // short pairs, one per lane: a launch per class of column count
    ffd::LaneArgs la;
    memset(&la, 0, sizeof la);
    la.X[0] = X0;
    la.X[1] = X1;
    la.off[0] = (const int32_t *)(w + wl.lo0);
    la.off[1] = (const int32_t *)(w + wl.lo1);
    la.order = (const int32_t *)(w + wl.order);
    la.out = out;
    la.col_count = (int32_t)pl.lane_cross;
    la.metric = metric;
    la.cell = ctx->measure >> 1;  // the planner took only ops 0 ... 8 but 2 (op 8: cell 4, Levenshtein)
    la.dtw = ctx->measure & 1;
    la.classes = pl.lane_classes;
    for (int c = 0; c < pl.lane_classes; ++c) {
      la.cols[c] = pl.lane_cols[c];
      la.first[c] = pl.lane_first[c];
      la.first[c + 1] = pl.lane_first[c + 1];
      la.block_first[c + 1] = la.block_first[c] + (pl.lane_first[c + 1] - pl.lane_first[c] + ffd::kLaneBlock - 1) /
                                                      ffd::kLaneBlock;
    }
    if (int rc = time_mark(ctx, st, capturing)) return rc;
    e = ffd::launch_lanes(exact, D, la, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
    if (pl.jobs.empty()) {
      if (int rc = time_mark(ctx, st, capturing)) return rc;
      ctx->last = ffd_launch_info{0, pl.nwaves, pl.wpb, 0, exact ? 1 : 0, D, 0, 0, pl.max_steps, 1};
      ctx->last_err = nullptr;  // the kernel waits on nothing and raises no error bits
      ctx->last_stream = st;
      return use_end(ctx, use, ws, st, capturing);
    }
    // the rest of the batch on the streaming kernel, after the lanes on the same stream
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
  a.lds_per_wave = lds_bytes(pl.R, D, exact, pl.hcap, pl.rings, ctx->measure);
  a.max_steps = (int32_t)(pl.max_steps + 4 * ffd::kRing);
  a.epoch = ++ctx->epoch;
  a.links = pl.nflags > 0 ? w + wl.links : nullptr;  // no links: the kernel skips their bookkeeping
  a.flags = pl.nflags > 0 ? (uint64_t *)(w + wl.flags) : nullptr;
  a.err = (uint64_t *)(w + wl.err);
  a.rings = pl.rings ? 1 : 0;
  a.dim = D;
  ctx->last = ffd_launch_info{pl.R, pl.nwaves, pl.wpb, a.lds_per_wave, exact ? 1 : 0, D, 0, 0, pl.max_steps,
                              pl.lanes ? 1 : 0};
  if (!pl.lanes)
    if (int rc = time_mark(ctx, st, capturing)) return rc;
  e = ffd::launch_stream(exact, pl.R, D, a, pl.wpb, pl.coop, st, ctx->measure);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  if (int rc = time_mark(ctx, st, capturing)) return rc;
  ctx->last_err = a.err;
  ctx->last_epoch = a.epoch;
  ctx->last_stream = st;
  return use_end(ctx, use, ws, st, capturing);
}

// A request: op, dim, type, measure and, unless `base`, the tuning and
// split settings (a plan depends on all of them), then both offset arrays.
struct Req {
  static constexpr int kHdr = 9;
  int64_t hdr[kHdr];
  const int64_t *a, *b;
  int64_t na, nb;
};

Req req_of(ffd_ctx *ctx, int op, int D, bool exact, const int64_t *a, int64_t na, const int64_t *b, int64_t nb,
           bool base = false) {
  Req r;
  float sp = base ? 0.f : ctx->split;
  int32_t spb;
  memcpy(&spb, &sp, sizeof spb);
  int64_t h[Req::kHdr] = {op, D, exact ? 1 : 0, base ? 0 : ctx->tune_R, base ? 0 : ctx->tune_W, ctx->measure,
                          spb, na, nb};
  memcpy(r.hdr, h, sizeof h);
  r.a = a;
  r.b = b;
  r.na = na;
  r.nb = nb;
  return r;
}

bool req_matches(const ReqKey &k, const Req &r) {
  const size_t nh = Req::kHdr, na = (size_t)r.na + 1, nb = (size_t)r.nb + 1;
  if (k.words.size() != nh + na + nb) return false;
  const int64_t *w = k.words.data();
  return memcmp(w, r.hdr, nh * 8) == 0 && memcmp(w + nh, r.a, na * 8) == 0 && memcmp(w + nh + na, r.b, nb * 8) == 0;
}

ReqKey req_key(const Req &r) {
  ReqKey k;
  k.words.reserve(Req::kHdr + r.na + r.nb + 2);
  k.words.insert(k.words.end(), r.hdr, r.hdr + Req::kHdr);
  k.words.insert(k.words.end(), r.a, r.a + r.na + 1);
  k.words.insert(k.words.end(), r.b, r.b + r.nb + 1);
  k.hash = mix_words(1469598103934665603ull, k.words.data(), k.words.size());
  return k;
}

constexpr int kOpPair = 100;  // internal plan kind of ffd_distance

// The measure of the call in progress (0 Frechet, 1 DTW of squared cells, 2
// DTW of Euclidean cells), read by the planner and the launcher.
struct MeasureScope {
  ffd_ctx *ctx;
  int saved;
  MeasureScope(ffd_ctx *c, int m) : ctx(c), saved(c->measure) { c->measure = m; }
  ~MeasureScope() { ctx->measure = saved; }
};

// The class of a request in the on-disk autotune cache: the target (gfx950
// and its compute units), the operation, the kernel (measure and ground
// distance), the value type and D, and log2 buckets of the mean row and
// column curve lengths and of the number of curves on each side.
std::string tune_class(const ffd_ctx *c, int op, int D, bool exact, const int64_t *a, int64_t na,
                       const int64_t *b, int64_t nb) {
  auto lg = [](double x) { return x < 1 ? 0 : (int)std::lround(std::log2(x)); };
  char buf[160];
  snprintf(buf, sizeof buf, "gfx950/cu%d/op%d/k%d/%s/D%d/L%d/M%d/N%d/Q%d", c->cus, op, c->measure,
           exact ? "i32" : "f32", D, lg((double)a[na] / (double)na), lg((double)b[nb] / (double)nb), lg((double)na),
           lg((double)nb));
  return buf;
}

// The cache file: a JSON object, one entry per line,
//   "class": {"rows_per_lane": R, "waves_per_simd": W, "split": S},
// R = W = S = 0 meaning that the model's own choice was the fastest.
void load_tune_cache(ffd_ctx *c) {
  c->tune_file.clear();
  FILE *f = c->tune_cache_path.empty() ? nullptr : fopen(c->tune_cache_path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char key[256];
    int R = 0, W = 0;
    float S = 0.f;
    if (sscanf(line, " \"%255[^\"]\": {\"rows_per_lane\": %d, \"waves_per_simd\": %d, \"split\": %f", key, &R, &W,
               &S) == 4) {
      if ((R == 0 || R == 1 || R == 2 || R == 4 || R == 8) && W >= 0 && W <= 8 && S == S)
        c->tune_file[key] = ffd_tuning{R, W, S, -1.f, -1.f, 0};
    }
  }
  fclose(f);
}

void save_tune_cache(const ffd_ctx *c) {
  if (c->tune_cache_path.empty()) return;
  std::string tmp = c->tune_cache_path + ".tmp";
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto &kv : c->tune_file)
    fprintf(f, "\"%s\": {\"rows_per_lane\": %d, \"waves_per_simd\": %d, \"split\": %.6g}%s\n", kv.first.c_str(),
            kv.second.rows_per_lane, kv.second.waves_per_simd, kv.second.split,
            ++i < c->tune_file.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
  std::rename(tmp.c_str(), c->tune_cache_path.c_str());
}

// With automatic settings, a launch shape the autotuner chose for this
// request (or, failing that, for its class in the cache file) replaces the
// model's choice for the duration of the call.
struct TunedScope {
  ffd_ctx *ctx;
  int R, W;
  float split;
  bool active = false;
  TunedScope(ffd_ctx *c, int op, int D, bool exact, const int64_t *a, int64_t na, const int64_t *b, int64_t nb)
      : ctx(c), R(c->tune_R), W(c->tune_W), split(c->split) {
    if (c->tune_R || c->tune_W || c->split != 0.f) return;
    const ffd_tuning *t = nullptr;
    if (!c->tuned.empty()) {
      ReqKey k = req_key(req_of(c, op, D, exact, a, na, b, nb, true));
      auto it = c->tuned.find(k.hash);
      if (it != c->tuned.end() && it->second.first.words == k.words) t = &it->second.second;
    }
    if (!t && !c->tune_file.empty() && na > 0 && nb > 0) {
      auto it = c->tune_file.find(tune_class(c, op, D, exact, a, na, b, nb));
      if (it != c->tune_file.end()) t = &it->second;
    }
    if (!t) return;
    c->tune_R = t->rows_per_lane;
    c->tune_W = t->waves_per_simd;
    c->split = t->split;
    active = true;
  }
  ~TunedScope() {
    if (active) {
      ctx->tune_R = R;
      ctx->tune_W = W;
      ctx->split = split;
    }
  }
};

// The Levenshtein kernels hold the table's values in float32, exact below
// 2^24: every value is at most n + m.
constexpr int64_t kLevMax = (int64_t)1 << 24;

static int64_t longest(const int64_t *off, int64_t count) {
  int64_t l = 0;
  if (!off) return 0;
  for (int64_t k = 0; k < count; ++k) l = std::max(l, off[k + 1] - off[k]);
  return l;
}

// (validate: check both offset arrays, unless they equal those of the
// cached plan, which were checked when it was made; a Levenshtein request's
// sequence lengths are checked against the float32 bound on the same terms)
int cached_plan(ffd_ctx *ctx, PlanCache &pc, int op, const int64_t *a_off, int64_t na, const int64_t *b_off,
                int64_t nb, int D, bool exact, const Plan **out, uint64_t &gen, bool validate = false) {
  Req r = req_of(ctx, op, D, exact, a_off, na, b_off, nb);
  if (pc.valid && req_matches(pc.key, r)) {
    *out = &pc.plan;
    gen = pc.gen;
    return FFD_OK;
  }
  Plan pl;
  int rc;
  if (validate) {
    if ((rc = check_offsets(ctx, a_off, na, "offsets are NULL"))) return rc;
    if ((rc = check_offsets(ctx, b_off, nb, "offsets are NULL"))) return rc;
  }
  if (ctx->measure == 8 && op != kOpPair && longest(a_off, na) + longest(b_off, nb) >= kLevMax)
    return fail(ctx, FFD_E_UNSUPPORTED, "Levenshtein sequences must have n + m < 2^24");
  if (op == FFD_OP_BATCH) rc = plan_batch(ctx, a_off, b_off, na, D, exact, pl);
  else if (op == FFD_OP_CROSS) rc = plan_cross(ctx, a_off, na, b_off, nb, D, exact, pl);
  else rc = plan_pair(ctx, a_off[1], b_off[1], D, exact, pl);
  if (rc) return rc;
  pc.plan = std::move(pl);
  pc.key = req_key(r);
  pc.gen = ++ctx->plan_gen;
  pc.valid = true;
  *out = &pc.plan;
  gen = pc.gen;
  return FFD_OK;
}

// Device scratch a single-pair plan needs (0: none).
size_t pair_scratch_bytes(const Plan &pl, bool exact) {
  if (pl.pipe) return pipe_layout(pl, exact).total;
  if (pl.nwaves == 1 && pl.link_elems == 0) return 0;
  return ws_layout(pl, 1, 1, exact).total;
}

// Launch a pipelined single-pair plan.
int run_pipe(ffd_ctx *ctx, const Plan &pl, const void *p, const void *q, int D, bool exact, int metric, void *out,
             hipStream_t st) {
  PipeLayout L = pipe_layout(pl, exact);
  size_t lds = pl.pipe_lds;
  ctx->last = ffd_launch_info{pl.R, pl.nwaves, ffd::kPipeWaves, (int32_t)(lds / ffd::kPipeWaves), exact ? 1 : 0, D,
                              1, 1, pl.max_steps};
  if (ctx->scratch_bytes < L.total)
    return fail(ctx, FFD_E_NOMEM,
                "a pair this long runs on many wavefronts and needs device scratch: register at least "
                "ffd_workspace_size(FFD_OP_PAIR) bytes with ffd_set_scratch");
  bool capturing = false;
  hipError_t e = capturing_on(st, capturing);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamIsCapturing");
  unsigned char *w = (unsigned char *)ctx->scratch;
  int rc;
  if (L.total > 0 && (rc = use_begin(ctx, ctx->scratch_use, w, st, capturing))) return rc;
  ffd::PipeArgs a;
  memset(&a, 0, sizeof a);
  a.X = pl.pipe_swap ? q : p;
  a.Y = pl.pipe_swap ? p : q;
  a.n = pl.pipe_rows;
  a.m = pl.pipe_cols;
  a.nb = pl.pipe_nb;
  a.nwg = pl.pipe_nwg;
  a.xcd_span = pl.pipe_xcd;
  a.metric = metric;
  a.links = L.total ? w + L.links : nullptr;
  a.link_stride = pl.pipe_stride;
  a.err = L.total ? (uint64_t *)(w + L.err) : nullptr;
  a.epoch = ++ctx->epoch;
  a.out = out;
  // a link wait may last ten times the modelled run time at 1 GHz, and at
  // least a second (real-time counter at 100 MHz)
  a.patience = (uint64_t)std::max(1e8, 10.0 * pl.makespan * pipe_step_clocks(pl.R, D, exact) / 1e9 * 1e8);
  if (L.total) {
    // every launch (and every graph replay) starts from unwritten link rows
    e = ffd::pipe_init(a.links, (int64_t)((L.total - L.links) / 4), a.err, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "link initialisation launch");
  }
  if (int rc2 = time_mark(ctx, st, capturing)) return rc2;
  e = ffd::launch_pipe(exact, pl.R, D, a, lds, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "pipelined kernel launch");
  if (int rc2 = time_mark(ctx, st, capturing)) return rc2;
  ctx->last_err = a.err;
  ctx->last_epoch = a.epoch;
  ctx->last_stream = st;
  if (L.total) return use_end(ctx, ctx->scratch_use, w, st, capturing);
  return FFD_OK;
}

int pair_common(ffd_ctx *ctx, const void *p, int64_t n, const void *q, int64_t m, int32_t dim, int32_t metric,
                void *out, hipStream_t st, bool exact) {
  int rc = check_common(ctx, dim, metric, exact);
  if (rc) return rc;
  if (!p || !q || !out) return fail(ctx, FFD_E_INVALID, "NULL pointer");
  if (n < 1 || m < 1) return fail(ctx, FFD_E_INVALID, "curves must have at least one point");
  int64_t off0[2] = {0, n}, off1[2] = {0, m};
  const Plan *pl;
  uint64_t key;
  rc = cached_plan(ctx, ctx->pair_plans, kOpPair, off0, 1, off1, 1, dim, exact, &pl, key);
  if (rc) return rc;
  if (pl->max_steps + 4 * ffd::kRing > INT32_MAX) return fail(ctx, FFD_E_UNSUPPORTED, "stream too long");
  ctx->last = ffd_launch_info{pl->R, pl->nwaves, pl->wpb, lds_bytes(pl->R, dim, exact, pl->hcap, false, ctx->measure),
                              exact ? 1 : 0, dim, 0, 0, pl->max_steps};
  if (ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot launch");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (pl->pipe) return run_pipe(ctx, *pl, p, q, dim, exact, metric, out, st);
  if (pl->nwaves == 1 && pl->link_elems == 0) {
    // one stream: the job travels in the kernel arguments, no device memory
    KernelArgs a;
    memset(&a, 0, sizeof a);
    a.X[0] = p;
    a.X[1] = q;
    a.inl_off[0][0] = 0;
    a.inl_off[0][1] = n;
    a.inl_off[1][0] = 0;
    a.inl_off[1][1] = m;
    a.jobs = nullptr;
    a.inl_job = pl->jobs[0];
    a.out = out;
    a.nwaves = 1;
    a.metric = metric;
    a.hcap = (int32_t)pl->hcap;
    a.lds_per_wave = lds_bytes(pl->R, dim, exact, pl->hcap, false, ctx->measure);
    a.max_steps = (int32_t)(pl->max_steps + 4 * ffd::kRing);
    a.epoch = ++ctx->epoch;
    a.dim = dim;
    e = ffd::launch_stream(exact, pl->R, dim, a, 1, false, st, ctx->measure);
    if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
    ctx->last_err = nullptr;
    return FFD_OK;
  }
  // bands split over waves: the plan and the links live in the scratch the
  // caller registered with ffd_set_scratch
  WsLayout wl = ws_layout(*pl, 1, 1, exact);
  if (ctx->scratch_bytes < wl.total)
    return fail(ctx, FFD_E_NOMEM,
                "a pair this long runs on many wavefronts and needs device scratch: register at least "
                "ffd_workspace_size(FFD_OP_PAIR) bytes with ffd_set_scratch");
  return run_plan(ctx, *pl, key, p, off0, 1, q, off1, 1, dim, exact, metric, out, ctx->scratch,
                  ctx->scratch_bytes, st, ctx->scratch_use);
}

int batch_common(ffd_ctx *ctx, const void *P, const int64_t *p_off, const void *Q, const int64_t *q_off,
                 int64_t npairs, int32_t dim, int32_t metric, void *out, void *ws, size_t ws_bytes, hipStream_t st,
                 bool exact, bool noalloc = false, UseOrder *use = nullptr) {
  int rc = check_common(ctx, dim, metric, exact);
  if (rc) return rc;
  if (npairs < 0) return fail(ctx, FFD_E_INVALID, "npairs < 0");
  if (npairs == 0) return FFD_OK;
  if (npairs > INT32_MAX / 2) return fail(ctx, FFD_E_UNSUPPORTED, "too many pairs");
  if (!P || !Q || !out) return fail(ctx, FFD_E_INVALID, "NULL pointer");
  if (!p_off) return fail(ctx, FFD_E_INVALID, "p_off is NULL");
  if (!q_off) return fail(ctx, FFD_E_INVALID, "q_off is NULL");
  TunedScope tuned(ctx, FFD_OP_BATCH, dim, exact, p_off, npairs, q_off, npairs);
  const Plan *pl;
  uint64_t key;
  rc = cached_plan(ctx, ctx->batch_plans, FFD_OP_BATCH, p_off, npairs, q_off, npairs, dim, exact, &pl, key, true);
  if (rc) return rc;
  return run_plan(ctx, *pl, key, P, p_off, npairs, Q, q_off, npairs, dim, exact, metric, out, ws, ws_bytes, st,
                  use ? *use : ctx->ws_use, noalloc);
}

int cross_common(ffd_ctx *ctx, const void *Qs, const int64_t *q_off, int64_t nq, const void *DB,
                 const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, void *out, void *ws,
                 size_t ws_bytes, hipStream_t st, bool exact) {
  int rc = check_common(ctx, dim, metric, exact);
  if (rc) return rc;
  if (nq < 0 || ndb < 0) return fail(ctx, FFD_E_INVALID, "negative count");
  if (nq == 0 || ndb == 0) return FFD_OK;
  if (nq > INT32_MAX / 2 || ndb > INT32_MAX / 2 || nq * ndb > ((int64_t)1 << 40))
    return fail(ctx, FFD_E_UNSUPPORTED, "too many curves");
  if (!Qs || !DB || !out) return fail(ctx, FFD_E_INVALID, "NULL pointer");
  if (!q_off) return fail(ctx, FFD_E_INVALID, "q_off is NULL");
  if (!db_off) return fail(ctx, FFD_E_INVALID, "db_off is NULL");
  TunedScope tuned(ctx, FFD_OP_CROSS, dim, exact, q_off, nq, db_off, ndb);
  const Plan *pl;
  uint64_t key;
  rc = cached_plan(ctx, ctx->batch_plans, FFD_OP_CROSS, q_off, nq, db_off, ndb, dim, exact, &pl, key, true);
  if (rc) return rc;
  return run_plan(ctx, *pl, key, Qs, q_off, nq, DB, db_off, ndb, dim, exact, metric, out, ws, ws_bytes, st,
                  ctx->ws_use);
}

// Time one launch of `call` (already planned and uploaded by a first call)
// between two events on the stream; < 0 when the shape cannot run.
template <typename Call>
float time_shape(ffd_ctx *ctx, hipStream_t st, Call call) {
  if (call() != FFD_OK) return -1.f;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return -1.f;
  }
  float best = -1.f;
  for (int rep = 0; rep < 2; ++rep) {
    hipEventRecord(e0, st);
    int rc = call();
    hipEventRecord(e1, st);
    float ms = -1.f;
    if (rc == FFD_OK && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
      best = best < 0 || ms < best ? ms : best;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  int32_t flags = 0;
  if (ffd_last_errors(ctx, &flags) != FFD_OK || flags != 0) return -1.f;
  return best;
}

// Try the launch shapes and keep the fastest for this request.
template <typename Call>
int autotune(ffd_ctx *ctx, int op, int D, bool exact, const int64_t *a, int64_t na, const int64_t *b, int64_t nb,
             hipStream_t st, Call call, ffd_tuning *best_out) {
  if (ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot launch");
  bool capturing = false;
  hipError_t ce = capturing_on(st, capturing);
  if (ce != hipSuccess) return hip_fail(ctx, ce, "hipStreamIsCapturing");
  if (capturing) return fail(ctx, FFD_E_UNSUPPORTED, "the autotuner times launches and cannot be captured");
  int R0 = ctx->tune_R, W0 = ctx->tune_W;
  float S0 = ctx->split;
  ReqKey base = req_key(req_of(ctx, op, D, exact, a, na, b, nb, true));
  ctx->tuned.erase(base.hash);
  // time the model's own choice, not a shape from the cache file
  std::map<std::string, ffd_tuning> file = std::move(ctx->tune_file);
  ctx->tune_file.clear();
  ffd_tuning best{0, 0, 0.f, -1.f, -1.f, 0};
  ctx->tune_R = ctx->tune_W = 0;
  ctx->split = 0.f;
  best.ms_planner = time_shape(ctx, st, call);
  const int Rs[3] = {2, 4, 8};
  const int Ws[2] = {1, 2};
  const float Ss[5] = {-1.f, 1.0f, 1.25f, 1.5f, 2.0f};
  for (int R : Rs)
    for (int W : Ws)
      for (float sp : Ss) {
        ctx->tune_R = R;
        ctx->tune_W = W;
        ctx->split = sp;
        float ms = time_shape(ctx, st, call);
        best.tried++;
        if (ms > 0 && (best.ms < 0 || ms < best.ms)) {
          best.ms = ms;
          best.rows_per_lane = R;
          best.waves_per_simd = W;
          best.split = sp;
        }
      }
  ctx->tune_R = R0;
  ctx->tune_W = W0;
  ctx->split = S0;
  ctx->tune_file = std::move(file);
  if (best.ms < 0) return fail(ctx, FFD_E_UNSUPPORTED, "no launch shape could run");
  if (best.ms_planner > 0 && best.ms_planner <= best.ms) {
    // the planner's own choice is as fast: keep using the model
    best.rows_per_lane = best.waves_per_simd = 0;
    best.split = 0.f;
    best.ms = best.ms_planner;
  } else {
    ctx->tuned[base.hash] = std::make_pair(base, best);
  }
  if (!ctx->tune_cache_path.empty()) {
    ctx->tune_file[tune_class(ctx, op, D, exact, a, na, b, nb)] = best;
    save_tune_cache(ctx);
  }
  if (best_out) *best_out = best;
  return FFD_OK;
}

}  // namespace ffdi

using namespace ffdi;

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
    case FFD_E_CANCELED: return "canceled";
    case FFD_E_EXPIRED: return "deadline passed before the request ran";
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
  c->lds_block_hw = prop.sharedMemPerBlock;
  c->lds_cu = prop.maxSharedMemoryPerMultiProcessor > 0 ? prop.maxSharedMemoryPerMultiProcessor : 65536;
  c->epoch = (uint32_t)std::chrono::steady_clock::now().time_since_epoch().count() | 1u;
  // events and the no-allocation scratch are set up here, so that no later
  // call needs to create or allocate anything on the device
  int prev = 0;
  bool ok = hipGetDevice(&prev) == hipSuccess && hipSetDevice(device) == hipSuccess;
  for (hipEvent_t *ev : {&c->upload_done, &c->ws_use.done, &c->scratch_use.done})
    ok = ok && hipEventCreateWithFlags(ev, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipSetDevice(prev) == hipSuccess;
  if (!ok || noalloc_setup(c, device) != FFD_OK) {
    ffd_destroy(c);
    return FFD_E_DEVICE;
  }
  if (const char *path = std::getenv("FFD_TUNE_CACHE")) {
    c->tune_cache_path = path;
    load_tune_cache(c);
  }
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
  c->lds_block_max = (size_t)std::min<int64_t>(lds_per_block, 65536);
  c->lds_block_hw = (size_t)lds_per_block;
  c->lds_cu = (size_t)lds_per_block;
  c->epoch = 1;
  *out = c;
  return FFD_OK;
}

void ffd_destroy(ffd_ctx *ctx) {
  if (!ctx) return;
  for (hipEvent_t ev : ctx->tev) {
    hipEventSynchronize(ev);
    hipEventDestroy(ev);
  }
  if (ctx->upload_done) {
    hipEventSynchronize(ctx->upload_done);
    hipEventDestroy(ctx->upload_done);
  }
  if (ctx->pinned) hipHostFree(ctx->pinned);
  for (UseOrder *u : {&ctx->scratch_use, &ctx->ws_use})
    if (u->done) {
      hipEventSynchronize(u->done);
      hipEventDestroy(u->done);
    }
  if (ctx->search_host) hipHostFree(ctx->search_host);
  delete ctx;
}

int ffd_set_scratch(ffd_ctx *ctx, void *scratch, size_t bytes) {
  if (!ctx) return FFD_E_INVALID;
  if (!scratch && bytes) return fail(ctx, FFD_E_INVALID, "NULL scratch with a nonzero size");
  if (ctx->plan_ws == ctx->scratch) ctx->plan_ws = nullptr;
  ctx->scratch = bytes ? scratch : nullptr;
  ctx->scratch_bytes = bytes ? bytes : 0;
  ctx->scratch_use.pending = false;  // the caller orders work on the memory it replaces
  ctx->scratch_use.ptr = ctx->scratch;
  return FFD_OK;
}

int ffd_last_launch(const ffd_ctx *ctx, ffd_launch_info *info) {
  if (!ctx || !info) return FFD_E_INVALID;
  *info = ctx->last;
  return FFD_OK;
}

int ffd_set_kernel_timing(ffd_ctx *ctx, int32_t enable) {
  if (!ctx) return FFD_E_INVALID;
  if (enable && ctx->device < 0) return fail(ctx, FFD_E_INVALID, "a planning-only context launches nothing");
  ctx->timing = enable != 0;
  ctx->tev_used = 0;
  return FFD_OK;
}

int ffd_kernel_time(ffd_ctx *ctx, double *total_ms, int64_t *launches) {
  if (!ctx || !total_ms || !launches) return FFD_E_INVALID;
  *total_ms = 0;
  *launches = 0;
  double sum = 0;
  for (size_t k = 0; k + 1 < ctx->tev_used; k += 2) {
    hipError_t e = hipEventSynchronize(ctx->tev[k + 1]);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize (timing)");
    float ms = 0;
    e = hipEventElapsedTime(&ms, ctx->tev[k], ctx->tev[k + 1]);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
    sum += ms;
  }
  *total_ms = sum;
  *launches = (int64_t)(ctx->tev_used / 2);
  ctx->tev_used = 0;
  return FFD_OK;
}

int ffd_last_errors(ffd_ctx *ctx, int32_t *flags) {
  if (!ctx || !flags) return FFD_E_INVALID;
  *flags = 0;
  if (!ctx->last_err) return FFD_OK;
  hipError_t e = hipStreamSynchronize(ctx->last_stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  uint64_t word = 0;
  e = hipMemcpy(&word, ctx->last_err, sizeof word, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy (error word)");
  if ((uint32_t)(word >> 32) == ctx->last_epoch) *flags = (int32_t)(uint32_t)word;
  return FFD_OK;
}

int ffd_set_tuning(ffd_ctx *ctx, int32_t rows_per_lane, int32_t waves_per_simd) {
  if (!ctx) return FFD_E_INVALID;
  if (rows_per_lane != 0 && rows_per_lane != 1 && rows_per_lane != 2 && rows_per_lane != 4 && rows_per_lane != 8)
    return fail(ctx, FFD_E_INVALID, "rows_per_lane must be 0, 1, 2, 4 or 8");
  if (waves_per_simd < -1 || waves_per_simd > 8)
    return fail(ctx, FFD_E_INVALID, "waves_per_simd must be -1 .. 8");
  ctx->tune_R = rows_per_lane;
  ctx->tune_W = waves_per_simd;
  return FFD_OK;
}

int ffd_set_tune_cache(ffd_ctx *ctx, const char *path) {
  if (!ctx) return FFD_E_INVALID;
  ctx->tune_cache_path = path ? path : "";
  load_tune_cache(ctx);
  return FFD_OK;
}

int ffd_set_split(ffd_ctx *ctx, float share) {
  if (!ctx) return FFD_E_INVALID;
  if (!(share == share) || share > 1e6f) return fail(ctx, FFD_E_INVALID, "share must be a finite number");
  ctx->split = share;
  return FFD_OK;
}

// Kernel op of a call: measure (0 Frechet, 1 DTW) + 2 * cell, where the
// cell is 0 squared Euclidean (the Frechet kernel also serves Euclidean: one
// root per pair), 1 Euclidean per cell (DTW), 2 Manhattan, 3 Chebyshev.
// Kernel op of a call; `geo` marks the float32 calls, the only ones that
// take FFD_HAVERSINE (elsewhere check_common refuses it).
static int op_of(bool dtw, int32_t metric, bool geo = false) {
  if (metric == FFD_HAVERSINE) return geo ? (dtw ? kOpGeoDtw : kOpGeo) : 0;
  int cell = metric == FFD_MANHATTAN ? 2 : metric == FFD_CHEBYSHEV ? 3 : (dtw && metric == FFD_EUCLIDEAN ? 1 : 0);
  return (dtw ? 1 : 0) + 2 * cell;
}

// Great-circle calls take (latitude, longitude) points and run the FP64
// unit-vector kernel: dim 2 of the call becomes the kernel's D = 3 and its
// value type FP64 (`exact`); the coordinates stay float32.
static int geo_shape(ffd_ctx *ctx, int32_t metric, int32_t &dim, bool &exact) {
  if (metric != FFD_HAVERSINE) return FFD_OK;
  if (dim != 2) return fail(ctx, FFD_E_INVALID, "great-circle curves take (latitude, longitude) points: dim must be 2");
  dim = 3;
  exact = true;
  return FFD_OK;
}

int ffd_distance(ffd_ctx *ctx, const float *p, int64_t n, const float *q, int64_t m, int32_t dim, int32_t metric,
                 float *out, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(false, metric, true));
  bool exact = false;
  if (int rc = geo_shape(ctx, metric, dim, exact)) return rc;
  return pair_common(ctx, p, n, q, m, dim, metric, out, (hipStream_t)stream, exact);
}

int ffd_distance_i32(ffd_ctx *ctx, const int32_t *p, int64_t n, const int32_t *q, int64_t m, int32_t dim,
                     int32_t metric, int64_t *out, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(false, metric));
  return pair_common(ctx, p, n, q, m, dim, metric, out, (hipStream_t)stream, true);
}

int ffd_batch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
              int64_t npairs, int32_t dim, int32_t metric, float *out, void *workspace, size_t ws_bytes,
              void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(false, metric, true));
  bool exact = false;
  if (int rc = geo_shape(ctx, metric, dim, exact)) return rc;
  return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, workspace, ws_bytes, (hipStream_t)stream,
                      exact);
}

}  // extern "C"

namespace ffdi {

int batch_noalloc(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
                  int64_t npairs, int32_t dim, int32_t metric, float *out, void *ws, size_t ws_bytes, hipStream_t st) {
  MeasureScope scope(ctx, op_of(false, metric, true));
  bool exact = false;
  if (int rc = geo_shape(ctx, metric, dim, exact)) return rc;
  return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, ws, ws_bytes, st, exact, true);
}

int batch_in_scratch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
                     int64_t npairs, int32_t dim, int32_t metric, float *out, hipStream_t st) {
  MeasureScope scope(ctx, op_of(false, metric, true));
  return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, ctx->scratch, ctx->scratch_bytes, st, false,
                      false, &ctx->scratch_use);
}

}  // namespace ffdi

extern "C" {

int ffd_batch_i32(ffd_ctx *ctx, const int32_t *P, const int64_t *p_off, const int32_t *Q, const int64_t *q_off,
                  int64_t npairs, int32_t dim, int32_t metric, int64_t *out, void *workspace, size_t ws_bytes,
                  void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(false, metric));
  return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, workspace, ws_bytes, (hipStream_t)stream,
                      true);
}

int ffd_cross(ffd_ctx *ctx, const float *Qs, const int64_t *q_off, int64_t nq, const float *DB,
              const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, float *out, void *workspace,
              size_t ws_bytes, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(false, metric, true));
  bool exact = false;
  if (int rc = geo_shape(ctx, metric, dim, exact)) return rc;
  return cross_common(ctx, Qs, q_off, nq, DB, db_off, ndb, dim, metric, out, workspace, ws_bytes,
                      (hipStream_t)stream, exact);
}

int ffd_cross_i32(ffd_ctx *ctx, const int32_t *Qs, const int64_t *q_off, int64_t nq, const int32_t *DB,
                  const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, int64_t *out, void *workspace,
                  size_t ws_bytes, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(false, metric));
  return cross_common(ctx, Qs, q_off, nq, DB, db_off, ndb, dim, metric, out, workspace, ws_bytes,
                      (hipStream_t)stream, true);
}

// Levenshtein distance (Appendix B, Algorithm B.2) of int32 symbol
// sequences: the same calls with the Levenshtein kernels (kernel op 8).
// The kernels hold the table's values in float32, exact below 2^24: every
// value is at most n + m.

int ffd_levenshtein_distance(ffd_ctx *ctx, const int32_t *p, int64_t n, const int32_t *q, int64_t m, int32_t dim,
                             int64_t *out, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  if (n + m >= kLevMax) return fail(ctx, FFD_E_UNSUPPORTED, "Levenshtein sequences must have n + m < 2^24");
  MeasureScope scope(ctx, 8);
  return pair_common(ctx, p, n, q, m, dim, FFD_SQEUCLIDEAN, out, (hipStream_t)stream, false);
}

int ffd_levenshtein_batch(ffd_ctx *ctx, const int32_t *P, const int64_t *p_off, const int32_t *Q,
                          const int64_t *q_off, int64_t npairs, int32_t dim, int64_t *out, void *workspace,
                          size_t ws_bytes, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, 8);  // the sequence lengths are checked with the offsets, when planned
  return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, FFD_SQEUCLIDEAN, out, workspace, ws_bytes,
                      (hipStream_t)stream, false);
}

int ffd_levenshtein_cross(ffd_ctx *ctx, const int32_t *Qs, const int64_t *q_off, int64_t nq, const int32_t *DB,
                          const int64_t *db_off, int64_t ndb, int32_t dim, int64_t *out, void *workspace,
                          size_t ws_bytes, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, 8);  // the sequence lengths are checked with the offsets, when planned
  return cross_common(ctx, Qs, q_off, nq, DB, db_off, ndb, dim, FFD_SQEUCLIDEAN, out, workspace, ws_bytes,
                      (hipStream_t)stream, false);
}

// Dynamic time warping (Appendix B): the same calls with the DTW kernels.

int ffd_dtw_distance(ffd_ctx *ctx, const float *p, int64_t n, const float *q, int64_t m, int32_t dim,
                     int32_t metric, float *out, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(true, metric, true));
  bool exact = false;
  if (int rc = geo_shape(ctx, metric, dim, exact)) return rc;
  return pair_common(ctx, p, n, q, m, dim, metric, out, (hipStream_t)stream, exact);
}

int ffd_dtw_distance_i32(ffd_ctx *ctx, const int32_t *p, int64_t n, const int32_t *q, int64_t m, int32_t dim,
                         int32_t metric, int64_t *out, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(true, metric));
  return pair_common(ctx, p, n, q, m, dim, metric, out, (hipStream_t)stream, true);
}

int ffd_dtw_batch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
                  int64_t npairs, int32_t dim, int32_t metric, float *out, void *workspace, size_t ws_bytes,
                  void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(true, metric, true));
  bool exact = false;
  if (int rc = geo_shape(ctx, metric, dim, exact)) return rc;
  return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, workspace, ws_bytes, (hipStream_t)stream,
                      exact);
}

int ffd_dtw_batch_i32(ffd_ctx *ctx, const int32_t *P, const int64_t *p_off, const int32_t *Q, const int64_t *q_off,
                      int64_t npairs, int32_t dim, int32_t metric, int64_t *out, void *workspace, size_t ws_bytes,
                      void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(true, metric));
  return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, workspace, ws_bytes, (hipStream_t)stream,
                      true);
}

int ffd_dtw_cross(ffd_ctx *ctx, const float *Qs, const int64_t *q_off, int64_t nq, const float *DB,
                  const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, float *out, void *workspace,
                  size_t ws_bytes, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(true, metric, true));
  bool exact = false;
  if (int rc = geo_shape(ctx, metric, dim, exact)) return rc;
  return cross_common(ctx, Qs, q_off, nq, DB, db_off, ndb, dim, metric, out, workspace, ws_bytes,
                      (hipStream_t)stream, exact);
}

int ffd_dtw_cross_i32(ffd_ctx *ctx, const int32_t *Qs, const int64_t *q_off, int64_t nq, const int32_t *DB,
                      const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, int64_t *out, void *workspace,
                      size_t ws_bytes, void *stream) {
  if (!ctx) return FFD_E_INVALID;
  MeasureScope scope(ctx, op_of(true, metric));
  return cross_common(ctx, Qs, q_off, nq, DB, db_off, ndb, dim, metric, out, workspace, ws_bytes,
                      (hipStream_t)stream, true);
}

static_assert(sizeof(ffd_plan_job) == sizeof(Job), "plan job layout");

int ffd_plan_describe(ffd_ctx *ctx, int32_t op, const int64_t *a_off, int64_t na, const int64_t *b_off, int64_t nb,
                      int32_t dim, int32_t exact, int32_t measure, int32_t metric, ffd_plan_summary *summary,
                      ffd_plan_job *jobs, int64_t jobs_cap, int32_t *wave_jobs, int64_t wave_jobs_cap) {
  if (!ctx || !summary) return FFD_E_INVALID;
  if (measure < 0 || measure > 2) return fail(ctx, FFD_E_INVALID, "unknown measure");
  if (measure == 2 && !exact) return fail(ctx, FFD_E_UNSUPPORTED, "Levenshtein takes int32 symbols");
  MeasureScope scope(ctx, measure == 2 ? 8 : op_of(measure == 1, metric, exact == 0));
  bool ex = exact != 0 && measure != 2;  // Levenshtein: int32 symbols, float32 values
  int rc = geo_shape(ctx, metric, dim, ex);
  if (rc) return rc;
  if ((rc = check_common(ctx, dim, metric, ex))) return rc;
  if (op != FFD_OP_BATCH && op != FFD_OP_CROSS && op != FFD_OP_PAIR) return fail(ctx, FFD_E_INVALID, "unknown op");
  if (na < 1 || nb < 1) return fail(ctx, FFD_E_INVALID, "nothing to plan");
  if ((op == FFD_OP_BATCH || op == FFD_OP_PAIR) && na != nb) return fail(ctx, FFD_E_INVALID, "na != nb");
  if (op == FFD_OP_PAIR && na != 1) return fail(ctx, FFD_E_INVALID, "a pair has one curve per side");
  if ((rc = check_offsets(ctx, a_off, na, "offsets are NULL"))) return rc;
  if ((rc = check_offsets(ctx, b_off, nb, "offsets are NULL"))) return rc;
  TunedScope tuned(ctx, op, dim, ex, a_off, na, b_off, nb);
  Plan pl;
  if (op == FFD_OP_BATCH) rc = plan_batch(ctx, a_off, b_off, na, dim, ex, pl);
  else if (op == FFD_OP_CROSS) rc = plan_cross(ctx, a_off, na, b_off, nb, dim, ex, pl);
  else rc = plan_pair(ctx, a_off[1], b_off[1], dim, ex, pl);
  if (rc) return rc;
  summary->rows_per_lane = pl.R;
  summary->waves = pl.nwaves;
  summary->waves_per_block = pl.wpb;
  summary->cooperative = pl.coop ? 1 : 0;
  summary->rings = pl.rings ? 1 : 0;
  summary->flags = pl.nflags;
  summary->link_elems = pl.link_elems;
  summary->stream_steps = pl.max_steps;
  summary->jobs = (int64_t)pl.jobs.size();
  summary->pipelined = pl.pipe ? 1 : 0;
  summary->per_lane = pl.lanes ? 1 : 0;
  if (jobs) {
    if (jobs_cap < (int64_t)pl.jobs.size()) return fail(ctx, FFD_E_NOMEM, "jobs_cap too small");
    if (!pl.jobs.empty()) memcpy(jobs, pl.jobs.data(), pl.jobs.size() * sizeof(Job));
  }
  if (wave_jobs) {
    if (wave_jobs_cap < (int64_t)pl.wave_jobs.size()) return fail(ctx, FFD_E_NOMEM, "wave_jobs too small");
    if (!pl.wave_jobs.empty()) memcpy(wave_jobs, pl.wave_jobs.data(), pl.wave_jobs.size() * sizeof(int32_t));
  }
  return FFD_OK;
}

int ffd_workspace_size(ffd_ctx *ctx, int32_t op, const int64_t *a_off, int64_t na, const int64_t *b_off, int64_t nb,
                       int32_t dim, size_t *bytes) {
  if (!ctx || !bytes) return FFD_E_INVALID;
  if (op != FFD_OP_BATCH && op != FFD_OP_CROSS && op != FFD_OP_PAIR && op != FFD_OP_DECIDE && op != FFD_OP_KNN)
    return fail(ctx, FFD_E_INVALID, "unknown op");
  if (dim < 1) return fail(ctx, FFD_E_INVALID, "dim must be >= 1");
  if (dim > FFD_MAX_DIM) return fail(ctx, FFD_E_UNSUPPORTED, "dim exceeds FFD_MAX_DIM");
  if (na < 0 || nb < 0) return fail(ctx, FFD_E_INVALID, "negative count");
  if ((op == FFD_OP_BATCH || op == FFD_OP_PAIR) && na != nb) return fail(ctx, FFD_E_INVALID, "needs na == nb");
  if (op == FFD_OP_PAIR && na > 1) return fail(ctx, FFD_E_INVALID, "a pair has one curve per side");
  *bytes = 0;
  if (na == 0 || nb == 0) return FFD_OK;
  int rc;
  if ((rc = check_offsets(ctx, a_off, na, "offsets are NULL"))) return rc;
  if ((rc = check_offsets(ctx, b_off, nb, "offsets are NULL"))) return rc;
  if (op == FFD_OP_DECIDE || op == FFD_OP_KNN) return search_scratch_size(ctx, op, a_off, na, b_off, nb, dim, bytes);
  // one size for every path: float and int32 coordinates, every measure and
  // ground distance (kernel ops 0, 1, 3, ..., 8, and 10, 11 for 2-D curves),
  // and for requests that run one pair per lane the job-table plan they were
  // weighed against as well (a forced launch shape or the autotuner uses it)
  size_t worst = 0;
  for (int ms = 0; ms <= kOpGeoDtw; ++ms)
    for (int ex = 0; ex < 2; ++ex) {
      if (ms == 2 || ms == 9 || (ms == 3 && ex == 1) || (ms == 8 && ex == 1)) continue;  // no such kernel
      if (ms >= kOpGeo && (ex == 0 || dim != 2)) continue;  // FP64 on (latitude, longitude) only
      MeasureScope scope(ctx, ms);
      const Plan *pl;
      uint64_t gen;
      PlanCache tmp;
      rc = cached_plan(ctx, tmp, op == FFD_OP_PAIR ? kOpPair : op, a_off, na, b_off, nb, ms >= kOpGeo ? 3 : dim,
                       ex == 1, &pl, gen);
      if (rc == FFD_E_UNSUPPORTED) continue;
      if (rc) return rc;
      if (op == FFD_OP_PAIR) worst = std::max(worst, pair_scratch_bytes(*pl, ex == 1));
      else worst = std::max({worst, ws_layout(*pl, na, nb, ex == 1).total, pl->alt_ws});
    }
  if (worst == 0 && op != FFD_OP_PAIR) return fail(ctx, FFD_E_UNSUPPORTED, "request not supported by any path");
  *bytes = worst;
  return FFD_OK;
}

}  // extern "C"

extern "C" {

int ffd_autotune_batch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
                       int64_t npairs, int32_t dim, int32_t metric, float *out, void *workspace, size_t ws_bytes,
                       void *stream, ffd_tuning *best) {
  if (!ctx) return FFD_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  MeasureScope scope(ctx, op_of(false, metric, true));
  bool exact = false;
  int rc = geo_shape(ctx, metric, dim, exact);
  if (rc) return rc;
  rc = batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, workspace, ws_bytes, st, exact);
  if (rc) return rc;  // argument errors, before any tuning
  if (npairs == 0) return FFD_OK;
  return autotune(ctx, FFD_OP_BATCH, dim, exact, p_off, npairs, q_off, npairs, st,
                  [&] { return batch_common(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, workspace, ws_bytes,
                                            st, exact); },
                  best);
}

int ffd_autotune_cross(ffd_ctx *ctx, const float *Qs, const int64_t *q_off, int64_t nq, const float *DB,
                       const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, float *out,
                       void *workspace, size_t ws_bytes, void *stream, ffd_tuning *best) {
  if (!ctx) return FFD_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  MeasureScope scope(ctx, op_of(false, metric, true));
  bool exact = false;
  int rc = geo_shape(ctx, metric, dim, exact);
  if (rc) return rc;
  rc = cross_common(ctx, Qs, q_off, nq, DB, db_off, ndb, dim, metric, out, workspace, ws_bytes, st, exact);
  if (rc) return rc;
  if (nq == 0 || ndb == 0) return FFD_OK;
  return autotune(ctx, FFD_OP_CROSS, dim, exact, q_off, nq, db_off, ndb, st,
                  [&] { return cross_common(ctx, Qs, q_off, nq, DB, db_off, ndb, dim, metric, out, workspace,
                                            ws_bytes, st, exact); },
                  best);
}

}  // extern "C"

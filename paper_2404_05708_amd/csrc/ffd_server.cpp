// Serving: query curves against a device-resident database, with continuous
// batching.
//
// The database is laid out once, at server creation, in "chunk order": its
// curves, sorted by length, are dealt to as many chunks as a launch has
// waves so that every chunk streams about the same number of steps
// (longest-first greedy), and each chunk's curves are stored contiguously
// in the arena.  A request (one query against the whole database, the
// batched form of Sec. 4 against one reference curve) then becomes one job
// per chunk -- the query's rows against the chunk's curves -- and a launch
// ("tick") runs the jobs of every request admitted with it, one chunk per
// wave, with no planning beyond filling in the job table.
//
// A request is swept in "items" of at most a few bands of its query rows
// (about four bands of 512 rows' worth of work), so that no launch holds
// the GPU for the whole of a long query and short queries that arrive
// meanwhile run between its items.  Between two items the bottom rows of
// the last band swept (one row per database curve) wait in a pair of
// boundary-row buffers of the request in the arena; a request needs them,
// and is admitted, only when a buffer pair is free (admission by the
// device memory the request needs; requests that fit one item need none).
// The next item of a request keeps the request's arrival position, so a
// long query is not passed over by later ones.
//
// A worker thread admits queued requests as soon as a slot and the memory
// they need are free, forms a tick from the items of admitted requests
// when a tick is free, uploads the queries and jobs, launches on the
// tick's own stream, and collects results when the tick's event completes;
// ticks on different streams overlap on the device.  The arena (caller
// device memory) holds the reordered database, the regions of the ticks
// and the boundary-row buffers; the library allocates no device memory for
// serving.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <queue>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ffd_internal.h"

using ffd::Job;
using ffd::KernelArgs;
using namespace ffdi;

struct ffd_db {
  ffd_ctx *ctx = nullptr;
  const float *X = nullptr;     // caller's device coordinates
  std::vector<int64_t> off;     // host copy of the offsets
  int64_t ndb = 0;
  int32_t dim = 0;
};

namespace {

constexpr int kServeR = 8;       // most rows per lane of a tick
constexpr int kServeRMulti = 3;  // fewest rows per lane of a tick whose queries span several bands
constexpr int kServeW = 2;       // LDS share of a wave: 1 / (4 kServeW) of a CU
#ifndef FFD_SERVE_TICKS
#define FFD_SERVE_TICKS 4
#endif
#ifndef FFD_SERVE_ITEM_BANDS
#define FFD_SERVE_ITEM_BANDS 4
#endif
constexpr int kTicks = FFD_SERVE_TICKS;  // launches in flight

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Chunk {
  int32_t first = 0, count = 0;  // curves [first, first + count) in chunk order
  int64_t sumL[2] = {0, 0};      // stream steps of one band: [0] single-band query, [1] chained
  int64_t maxL = 0;              // longest task (chained)
};

struct Request {
  uint64_t ticket = 0;
  std::vector<float> q;
  int64_t n = 0;
  int32_t metric = 0;
  float *out = nullptr;
  double t_submit = 0, t_done = 0;
  double deadline = 0;  // > 0: its last launch must be issued by then (seconds, now_s clock)
  bool cancel = false;  // ffd_server_cancel was called
  int state = 0;      // 0 queued, 1 ready for its next item, 3 item in flight, 2 done, < 0 error status
  int R = 0;          // rows per lane of its items (fixed once an item ran)
  int64_t nb = 0;     // bands at R
  int64_t next_band = 0;
  int32_t link = -1;  // boundary-row buffer pair (multi-item requests)
  int link_cur = 0;   // which buffer of the pair holds the rows of band next_band - 1
};

// One item of a tick: bands [b0, b0 + c) of a request's query.
struct Item {
  Request *r = nullptr;
  int64_t b0 = 0, c = 0;
  bool last = false;  // the query's last band is in this item (results)
};

// Byte layout of one tick's region; the same offsets are used in its pinned
// upload mirror (which covers [0, upload)).
struct TickLayout {
  size_t q, qo, jobs, wj, flags, err, upload, links, out, total;
};

struct Tick {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  unsigned char *dev = nullptr;   // region in the arena
  unsigned char *pin = nullptr;   // pinned upload mirror
  float *pin_out = nullptr;       // pinned results
  uint64_t *pin_err = nullptr;
  std::vector<Item> items;
  uint32_t epoch = 0;
};

constexpr int kFlagDone = 0;   // flag of every link written by an earlier launch: preset complete
constexpr int kFlagSink = 1;   // flag the last band of an item publishes to (nobody waits on it)
constexpr int kFlagFirst = 2;  // flags of links inside a launch

}  // namespace

struct ffd_server {
  ffd_ctx *ctx = nullptr;
  ffd_db *db = nullptr;
  int device = 0;
  int dim = 0;
  // launch shape (LDS is sized for R = kServeR; a tick runs the rows per
  // lane that fit its queries, see query_rows)
  int R = kServeR, nwaves = 0, wpb = 1, lds_per_wave = 0;
  int lds_rows[kServeR + 1] = {}; // LDS per wave for 1 ... kServeR rows per lane
  int lds_rows1[kServeR + 1] = {};  // the same without a hand-off row (ticks of single-band queries)
  int64_t hcap = 0;
  // database in chunk order
  std::vector<Chunk> chunks;
  std::vector<int32_t> perm;      // chunk-order position -> original curve index
  std::vector<int32_t> long_chunks;  // chunks whose longest task exceeds hcap
  int64_t long_sumL = 0;          // sum of their chained band lengths
  std::vector<int64_t> chunk_link;  // offset of each chunk's boundary rows in a row buffer
  int64_t link_row = 0;           // values of a boundary-row buffer (all chunks, chained lengths)
  int link_pairs = 0;             // boundary-row buffer pairs in the arena
  std::vector<int32_t> free_links;
  unsigned char *arena = nullptr;
  size_t links_at = 0;            // arena offset of the boundary-row buffers
  int64_t db_points = 0;
  const float *dbx = nullptr;     // reordered coordinates (arena)
  const int64_t *dbo = nullptr;   // their offsets (arena)
  // ticks
  int kmax = 1;                   // requests per tick
  int64_t qcap = 0;               // query points per tick
  int64_t max_query = 0;
  size_t jobs_cap = 0, flags_cap = 0, links_cap = 0;
  TickLayout lay{};
  Tick ticks[kTicks];
  uint32_t epoch = 1;
  // requests
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  int max_slots = 1;
  std::deque<Request *> pending;  // submitted, not admitted (arrival order)
  std::deque<Request *> active;   // admitted, not finished (arrival order)
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // statistics
  std::vector<double> lat;
  int64_t submitted = 0, completed = 0, deferred = 0, failed = 0, canceled = 0, expired = 0;
  int64_t deadline_us = 0;        // watchdog limit of newly submitted requests (0: none)
  int64_t launches_by_rows[kServeR] = {};
  double cells = 0, t_first = 0, t_last = 0;
  std::string last_error;
};

namespace {

// Fewest rows per lane of a tick whose queries span several bands: curves of
// more than four coordinates run on the wide kernels' R only.
int multi_rows(const ffd_server &s) { return s.dim > 4 ? ffd::wide_rows(s.dim) : kServeRMulti; }

int64_t job_count_bound(const ffd_server &s) {
  int64_t max_nb = ffd::bands_for(s.max_query, multi_rows(s));
  // per request: one job per chunk, or for a self-chained chunk a band job
  // and an idle job per band
  return (int64_t)s.chunks.size() + (int64_t)s.long_chunks.size() * (2 * max_nb);
}

TickLayout tick_layout(const ffd_server &s) {
  TickLayout t;
  size_t o = 0;
  t.q = o;     o = al256(o + (size_t)s.qcap * s.dim * sizeof(float));
  t.qo = o;    o = al256(o + (size_t)(s.kmax + 1) * sizeof(int64_t));
  t.jobs = o;  o = al256(o + s.jobs_cap * sizeof(Job));
  t.wj = o;    o = al256(o + (size_t)(s.nwaves + 1) * sizeof(int32_t));
  t.flags = o; o = al256(o + std::max<size_t>(s.flags_cap, 1) * sizeof(uint64_t));
  t.err = o;   o = al256(o + sizeof(uint64_t));
  t.upload = o;
  t.links = o; o = al256(o + std::max<size_t>(s.links_cap, 1) * sizeof(float));
  t.out = o;   o = al256(o + (size_t)s.kmax * s.db->ndb * sizeof(float));
  t.total = o;
  return t;
}

size_t db_bytes(const ffd_server &s) {
  return al256((size_t)s.db_points * s.dim * sizeof(float)) + al256((size_t)(s.db->ndb + 1) * sizeof(int64_t));
}

size_t link_pair_bytes(const ffd_server &s) { return al256((size_t)2 * s.link_row * sizeof(float)); }

size_t arena_total(const ffd_server &s) {
  return db_bytes(s) + (size_t)kTicks * s.lay.total + (size_t)s.link_pairs * link_pair_bytes(s);
}

// Shape of the launches and the chunk order of the database.
int plan_server(ffd_server &s, int32_t max_slots, int64_t max_query) {
  ffd_ctx *ctx = s.ctx;
  const ffd_db &db = *s.db;
  Resources rs = resources(ctx, s.R, s.dim, false, kServeW);
  s.nwaves = std::min<int>(rs.nwaves_max, ctx->cus * 4 * kServeW);
  s.nwaves = (int)std::min<int64_t>(s.nwaves, db.ndb);
  s.wpb = std::min(rs.wpb, s.nwaves);
  s.hcap = rs.hand_max;
  s.lds_per_wave = lds_bytes(s.R, s.dim, false, s.hcap);
  for (int r = 1; r <= kServeR; ++r) {
    s.lds_rows[r] = lds_bytes(r, s.dim, false, s.hcap);
    s.lds_rows1[r] = lds_bytes(r, s.dim, false, 0);
  }
  s.max_query = max_query;
  s.kmax = std::max(1, (max_slots + kTicks - 1) / kTicks);
  s.qcap = (int64_t)s.kmax * max_query;
  s.db_points = db.off[db.ndb];

  // longest first onto the least loaded chunk
  std::vector<int32_t> order(db.ndb);
  for (int64_t k = 0; k < db.ndb; ++k) order[k] = (int32_t)k;
  auto len = [&](int32_t k) { return db.off[k + 1] - db.off[k]; };
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return len(a) > len(b); });
  using Load = std::pair<int64_t, int32_t>;
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int32_t c = 0; c < s.nwaves; ++c) heap.push({0, c});
  std::vector<std::vector<int32_t>> members(s.nwaves);
  for (int32_t k : order) {
    Load l = heap.top();
    heap.pop();
    members[l.second].push_back(k);
    heap.push({l.first + ffd::task_len(len(k), true), l.second});
  }
  s.chunks.assign(s.nwaves, Chunk());
  s.perm.clear();
  s.perm.reserve(db.ndb);
  s.long_chunks.clear();
  s.long_sumL = 0;
  for (int32_t c = 0; c < s.nwaves; ++c) {
    Chunk &ch = s.chunks[c];
    ch.first = (int32_t)s.perm.size();
    ch.count = (int32_t)members[c].size();
    for (int32_t k : members[c]) {
      s.perm.push_back(k);
      ch.sumL[0] += ffd::task_len(len(k), false);
      ch.sumL[1] += ffd::task_len(len(k), true);
      ch.maxL = std::max<int64_t>(ch.maxL, ffd::task_len(len(k), true));
    }
    if (ch.maxL > s.hcap) {
      s.long_chunks.push_back(c);
      s.long_sumL += ch.sumL[1];
    }
  }
  int64_t max_nb = ffd::bands_for(max_query, multi_rows(s));
  s.jobs_cap = (size_t)s.kmax * (size_t)job_count_bound(s);
  s.flags_cap = kFlagFirst + (size_t)s.kmax * s.long_chunks.size() * (size_t)std::max<int64_t>(max_nb - 1, 0);
  s.links_cap = (size_t)s.kmax * (size_t)s.long_sumL;
  s.lay = tick_layout(s);
  // boundary-row buffers of multi-item requests: one row per database curve
  // (chained task lengths), chunk after chunk; a pair per request
  s.chunk_link.assign(s.nwaves, 0);
  int64_t o = 0;
  for (int32_t c = 0; c < s.nwaves; ++c) {
    s.chunk_link[c] = o;
    o += s.chunks[c].sumL[1];
  }
  s.link_row = (o + 63) / 64 * 64;
  s.max_slots = max_slots;
  s.link_pairs = std::max(1, std::min(max_slots, 64));
  return FFD_OK;
}

void release_link(ffd_server &s, Request *r) {
  if (r->link >= 0) s.free_links.push_back(r->link);
  r->link = -1;
}

void drop_active(ffd_server &s, Request *r) {
  auto it = std::find(s.active.begin(), s.active.end(), r);
  if (it != s.active.end()) s.active.erase(it);
}

void finish_tick(ffd_server &s, Tick &t) {
  const int64_t ndb = s.db->ndb;
  bool bad = false;
  uint64_t e = *t.pin_err;
  if (e != 0 && (uint32_t)(e >> 32) == t.epoch) bad = true;
  double tn = now_s();
  for (size_t i = 0; i < t.items.size(); ++i) {
    const Item &it = t.items[i];
    Request *r = it.r;
    if (bad) {
      r->state = FFD_E_DEVICE;
      s.failed++;
    } else if (!it.last) {
      // more bands to sweep: the rows just written are in the other buffer
      r->next_band = it.b0 + it.c;
      r->link_cur ^= 1;
      r->state = 1;
      continue;
    } else {
      const float *src = t.pin_out + i * (size_t)ndb;
      for (int64_t p = 0; p < ndb; ++p) r->out[s.perm[p]] = src[p];
      r->state = 2;
      s.completed++;
      s.cells += (double)r->n * (double)s.db_points;
      s.lat.push_back(tn - r->t_submit);
      s.t_last = tn;
    }
    r->t_done = tn;
    release_link(s, r);
    drop_active(s, r);
  }
  t.items.clear();
  t.busy = false;
  s.cv_done.notify_all();
}

void fail_tick(ffd_server &s, Tick &t, int code) {
  for (const Item &it : t.items) {
    it.r->state = code;
    s.failed++;
    release_link(s, it.r);
    drop_active(s, it.r);
  }
  t.items.clear();
  t.busy = false;
  s.cv_done.notify_all();
}

Job band_job(int32_t i, const Chunk &ch, int64_t ndb) {
  Job jb;
  memset(&jb, 0, sizeof jb);
  jb.out_base = (int64_t)i * ndb + ch.first;
  jb.row_sel = 0;
  jb.row_idx = i;
  jb.col_sel = 1;
  jb.col_first = ch.first;
  jb.col_count = ch.count;
  jb.out_stride = 1;
  jb.band_first = 0;
  jb.band_count = 0;
  jb.link_in = jb.link_out = -1;
  jb.flag_in = jb.flag_out = -1;
  return jb;
}

// Modelled cost of a query of n points at R rows per lane: its bands times
// the clocks of a stream step (the database side is the same for every R),
// or +inf where R is not allowed (several bands below kServeRMulti rows per
// lane: the tick's job and flag capacities are sized for that).
double query_cost(const ffd_server &s, int64_t n, int R) {
  int64_t nb = ffd::bands_for(n, R);
  if (s.dim > 4 && R != ffd::wide_rows(s.dim)) return HUGE_VAL;
  if (nb > 1 && R < multi_rows(s)) return HUGE_VAL;
  return (double)nb * step_clocks(R, s.dim, false, kServeW);
}

// Rows per lane for a query of n points: the R in 1 ... kServeR of least
// modelled cost.  A band's rows past the query's end are computed and
// dropped (a 300-point query uses 59 % of a 512-row band, 94 % of a 320-row
// one), while fewer rows per lane cost more clocks per row; ticks group
// queries that suit one R.
int query_rows(const ffd_server &s, int64_t n) {
  int best = kServeR;
  double bc = query_cost(s, n, kServeR);
  for (int R = kServeR - 1; R >= 1; --R) {
    double c = query_cost(s, n, R);
    if (c < bc) best = R, bc = c;
  }
  return best;
}

// A query joins a tick of Rt rows per lane when that costs at most this
// factor more than its own best R.
constexpr double kServeSlack = 1.10;

// Bands of one item at R rows per lane: about four bands of kServeR rows'
// worth of work (a band sweeps every database curve once).
int64_t item_bands(const ffd_server &s, int R) {
  double cap = (double)FFD_SERVE_ITEM_BANDS * step_clocks(kServeR, s.dim, false, kServeW);
  return std::max<int64_t>(1, (int64_t)(cap / step_clocks(R, s.dim, false, kServeW)));
}

// Whether request r needs boundary-row buffers (more than one item).
bool multi_item(const ffd_server &s, const Request &r) { return r.nb > item_bands(s, r.R); }

// Form tick t from the items of ready requests and launch it.  Called with
// the lock held; at least one admitted request is ready.
int launch_tick(ffd_server &s, Tick &t) {
  const TickLayout &L = s.lay;
  const int64_t ndb = s.db->ndb;
  // the oldest ready request sets the metric and the rows per lane; later
  // ones join if they suit them (a request with bands already swept only
  // at its own R; a fresh one at another R within the slack when all its
  // bands fit this item)
  Request *first = nullptr;
  for (Request *r : s.active)
    if (r->state == 1) {
      first = r;
      break;
    }
  if (!first) return FFD_OK;
  const int32_t metric = first->metric;
  const int Rt = first->R;
  const int64_t cap = item_bands(s, Rt);
  int64_t pts = 0;
  for (Request *r : s.active) {
    if ((int)t.items.size() >= s.kmax) break;
    if (r->state != 1 || r->metric != metric || pts + r->n > s.qcap) continue;
    Item it;
    it.r = r;
    if (r->R == Rt) {
      it.b0 = r->next_band;
      it.c = std::min(r->nb - r->next_band, cap);
    } else {
      int64_t nbt = ffd::bands_for(r->n, Rt);
      if (r->next_band > 0 || nbt > cap ||
          query_cost(s, r->n, Rt) > kServeSlack * query_cost(s, r->n, r->R))
        continue;
      r->R = Rt;  // runs whole in this tick
      r->nb = nbt;
      it.b0 = 0;
      it.c = nbt;
    }
    it.last = it.b0 + it.c == r->nb;
    pts += r->n;
    r->state = 3;
    t.items.push_back(it);
  }
  const int k = (int)t.items.size();
  unsigned char *h = t.pin;
  // queries and their offsets
  float *hq = reinterpret_cast<float *>(h + L.q);
  int64_t *hqo = reinterpret_cast<int64_t *>(h + L.qo);
  hqo[0] = 0;
  for (int i = 0; i < k; ++i) {
    const Request *r = t.items[i].r;
    memcpy(hq + hqo[i] * s.dim, r->q.data(), r->q.size() * sizeof(float));
    hqo[i + 1] = hqo[i] + r->n;
  }
  // jobs, wave by wave: the chunk of wave w against every item of the tick.
  // Link offsets count floats from the arena's start (a.links is the arena).
  const int64_t tick_links = (int64_t)((t.dev + L.links - s.arena) / sizeof(float));
  Job *hj = reinterpret_cast<Job *>(h + L.jobs);
  int32_t *hwj = reinterpret_cast<int32_t *>(h + L.wj);
  size_t nj = 0;
  int32_t nflags = kFlagFirst;
  int64_t nlinks = 0, max_steps = 0;
  bool chained = false;  // some item hands a band's bottom row on inside a wave
  for (int i = 0; i < k; ++i) chained = chained || t.items[i].c > 1;
  for (int w = 0; w < s.nwaves; ++w) {
    hwj[w] = (int32_t)nj;
    const Chunk &ch = s.chunks[w];
    int64_t steps = 0;
    for (int i = 0; i < k; ++i) {
      const Item &it = t.items[i];
      const Request *r = it.r;
      // the request's boundary rows: read from buffer link_cur, written to the other
      int64_t lin = -1, lout = -1;
      if (r->link >= 0) {
        int64_t pair = (int64_t)((s.links_at + (size_t)r->link * link_pair_bytes(s)) / sizeof(float));
        lin = pair + (int64_t)r->link_cur * s.link_row + s.chunk_link[w];
        lout = pair + (int64_t)(r->link_cur ^ 1) * s.link_row + s.chunk_link[w];
      }
      const bool from_link = it.b0 > 0, to_link = !it.last;
      Job jb = band_job(i, ch, ndb);
      int64_t sumL = ch.sumL[r->nb > 1 ? 1 : 0];
      if (it.c == 1 || ch.maxL <= s.hcap) {
        // the item's bands chained through LDS on this wave
        jb.band_first = (int32_t)it.b0;
        jb.band_count = (int32_t)it.c;
        if (from_link) {
          jb.link_in = lin;
          jb.flag_in = kFlagDone;
        }
        if (to_link) {
          jb.link_out = lout;
          jb.flag_out = kFlagSink;
        }
        hj[nj++] = jb;
        steps += it.c * sumL;
        continue;
      }
      // the chunk's boundary row does not fit LDS: the item's bands run in
      // order on this wave and pass the row on in place in the tick's region
      int64_t gap = self_gap(sumL);
      for (int64_t b = it.b0; b < it.b0 + it.c; ++b) {
        if (b > it.b0 && gap > 0) {
          Job idle;
          memset(&idle, 0, sizeof idle);
          idle.row_sel = ffd::kRowIdle;
          idle.col_count = (int32_t)gap;
          idle.link_in = idle.link_out = -1;
          idle.flag_in = idle.flag_out = -1;
          hj[nj++] = idle;
          steps += gap;
        }
        Job bj = jb;
        bj.band_first = (int32_t)b;
        bj.band_count = 1;
        int32_t fl = nflags + (int32_t)(b - it.b0);
        if (b > it.b0) {
          bj.link_in = tick_links + nlinks;
          bj.flag_in = fl - 1;
        } else if (from_link) {
          bj.link_in = lin;
          bj.flag_in = kFlagDone;
        }
        if (b + 1 < it.b0 + it.c) {
          bj.link_out = tick_links + nlinks;
          bj.flag_out = fl;
        } else if (to_link) {
          bj.link_out = lout;
          bj.flag_out = kFlagSink;
        }
        hj[nj++] = bj;
        steps += sumL;
      }
      nflags += (int32_t)(it.c - 1);
      nlinks += sumL;
    }
    max_steps = std::max(max_steps, steps);
  }
  hwj[s.nwaves] = (int32_t)nj;
  memset(h + L.flags, 0, L.upload - L.flags);  // flags and error word
  t.epoch = ++s.epoch;
  // links written by an earlier launch are complete: their flag says so
  reinterpret_cast<uint64_t *>(h + L.flags)[kFlagDone] = ffd::flag_word(t.epoch, 0xFFFFFFFFu);

  hipError_t e = hipMemcpyAsync(t.dev, h, L.upload, hipMemcpyHostToDevice, t.stream);
  if (e != hipSuccess) return FFD_E_DEVICE;
  KernelArgs a;
  memset(&a, 0, sizeof a);
  a.X[0] = t.dev + L.q;
  a.X[1] = s.dbx;
  a.off[0] = reinterpret_cast<const int64_t *>(t.dev + L.qo);
  a.off[1] = s.dbo;
  a.jobs = reinterpret_cast<const Job *>(t.dev + L.jobs);
  a.wave_jobs = reinterpret_cast<const int32_t *>(t.dev + L.wj);
  a.out = t.dev + L.out;
  a.nwaves = s.nwaves;
  a.metric = metric;
  // a tick whose items sweep one band each hands no row on inside a wave
  // (its tasks read the ghost row or a link and write to the sink or a
  // link), so its waves take no hand-off row in LDS and more of them fit a
  // CU, also from the other launches in flight
  a.hcap = chained ? (int32_t)s.hcap : 0;
  a.lds_per_wave = chained ? s.lds_rows[Rt] : s.lds_rows1[Rt];
  a.max_steps = (int32_t)(max_steps + 4 * ffd::kRing);
  a.epoch = t.epoch;
  a.links = s.arena;
  a.flags = reinterpret_cast<uint64_t *>(t.dev + L.flags);
  a.err = reinterpret_cast<uint64_t *>(t.dev + L.err);
  a.dim = s.dim;
  e = ffd::launch_stream(false, Rt, s.dim, a, s.wpb, false, t.stream);
  if (e != hipSuccess) return FFD_E_DEVICE;
  s.launches_by_rows[Rt - 1]++;
  e = hipMemcpyAsync(t.pin_out, t.dev + L.out, (size_t)k * ndb * sizeof(float), hipMemcpyDeviceToHost, t.stream);
  if (e != hipSuccess) return FFD_E_DEVICE;
  e = hipMemcpyAsync(t.pin_err, t.dev + L.err, sizeof(uint64_t), hipMemcpyDeviceToHost, t.stream);
  if (e != hipSuccess) return FFD_E_DEVICE;
  e = hipEventRecord(t.done, t.stream);
  if (e != hipSuccess) return FFD_E_DEVICE;
  t.busy = true;
  return FFD_OK;
}

// Admit queued requests in arrival order while slots are free; a request
// that needs boundary-row buffers waits for a free pair (later requests
// that need none may pass it).  Called with the lock held.
void admit(ffd_server &s) {
  for (auto it = s.pending.begin(); it != s.pending.end() && (int)s.active.size() < s.max_slots;) {
    Request *r = *it;
    if (multi_item(s, *r)) {
      if (s.free_links.empty()) {
        ++it;
        continue;
      }
      r->link = s.free_links.back();
      s.free_links.pop_back();
      r->link_cur = 0;
    }
    r->state = 1;
    s.active.push_back(r);
    it = s.pending.erase(it);
  }
}

// The watchdog and cancellation: drop every request that was canceled, or
// whose deadline has passed, while it is queued or between two of its
// items (an item in flight finishes first; a request whose last item is in
// flight completes).  Its out array is never written.  Called with the lock
// held.
void expire(ffd_server &s) {
  const double tn = now_s();
  auto verdict = [&](const Request *r) {
    if (r->cancel) return FFD_E_CANCELED;
    if (r->deadline > 0 && tn > r->deadline) return FFD_E_EXPIRED;
    return FFD_OK;
  };
  auto end = [&](Request *r, int v) {
    r->state = v;
    r->t_done = tn;
    (v == FFD_E_CANCELED ? s.canceled : s.expired)++;
  };
  bool any = false;
  for (auto it = s.pending.begin(); it != s.pending.end();) {
    int v = verdict(*it);
    if (v == FFD_OK) {
      ++it;
      continue;
    }
    end(*it, v);
    it = s.pending.erase(it);
    any = true;
  }
  for (auto it = s.active.begin(); it != s.active.end();) {
    Request *r = *it;
    int v = r->state == 1 ? verdict(r) : FFD_OK;
    if (v == FFD_OK) {
      ++it;
      continue;
    }
    release_link(s, r);
    end(r, v);
    it = s.active.erase(it);
    any = true;
  }
  if (any) s.cv_done.notify_all();
}

bool any_ready(const ffd_server &s) {
  for (const Request *r : s.active)
    if (r->state == 1) return true;
  return false;
}

void worker_loop(ffd_server *s) {
  hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progressed = false, busy = false;
    for (Tick &t : s->ticks) {
      if (!t.busy) continue;
      hipError_t q = hipEventQuery(t.done);
      if (q == hipSuccess) {
        finish_tick(*s, t);
        progressed = true;
      } else if (q != hipErrorNotReady) {
        fail_tick(*s, t, FFD_E_DEVICE);
        progressed = true;
      } else {
        busy = true;
      }
    }
    expire(*s);
    admit(*s);
    while (any_ready(*s)) {
      Tick *free_tick = nullptr;
      for (Tick &t : s->ticks)
        if (!t.busy && t.items.empty()) {
          free_tick = &t;
          break;
        }
      if (!free_tick) break;
      int rc = launch_tick(*s, *free_tick);
      if (rc != FFD_OK) fail_tick(*s, *free_tick, rc);
      progressed = true;
      busy = true;
    }
    if (s->stop && s->pending.empty() && s->active.empty() && !busy) break;
    if (!progressed) {
      if (busy) s->cv_work.wait_for(lk, std::chrono::microseconds(20));
      else s->cv_work.wait(lk);
    }
  }
}

int sfail(ffd_server *s, int code, const char *msg) {
  if (s) s->last_error = msg;
  return code;
}

void destroy_server(ffd_server *s) {
  if (!s) return;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->worker.join();
  }
  for (Tick &t : s->ticks) {
    if (t.stream) hipStreamSynchronize(t.stream);
    if (t.done) hipEventDestroy(t.done);
    if (t.stream) hipStreamDestroy(t.stream);
    if (t.pin) hipHostFree(t.pin);
    if (t.pin_out) hipHostFree(t.pin_out);
    if (t.pin_err) hipHostFree(t.pin_err);
  }
  delete s;
}

int make_server(ffd_db *db, int32_t max_slots, int64_t max_query, ffd_server *s) {
  s->ctx = db->ctx;
  s->db = db;
  s->device = db->ctx->device;
  s->dim = db->dim;
  if (s->dim > 4) s->R = ffd::wide_rows(s->dim);  // LDS sized for the wide kernels' only shape
  return plan_server(*s, max_slots, max_query);
}

}  // namespace

extern "C" {

int ffd_db_create(ffd_ctx *ctx, const float *DB, const int64_t *db_off, int64_t ndb, int32_t dim, ffd_db **out) {
  if (!out) return FFD_E_INVALID;
  *out = nullptr;
  if (!ctx) return FFD_E_INVALID;
  int rc = check_common(ctx, dim, FFD_EUCLIDEAN, false);
  if (rc) return rc;
  if (!DB) return fail(ctx, FFD_E_INVALID, "NULL pointer");
  if (ndb < 1 || ndb > INT32_MAX / 2) return fail(ctx, FFD_E_INVALID, "database must hold 1 .. 2^30 curves");
  if ((rc = check_offsets(ctx, db_off, ndb, "db_off is NULL"))) return rc;
  ffd_db *d = new (std::nothrow) ffd_db();
  if (!d) return FFD_E_NOMEM;
  d->ctx = ctx;
  d->X = DB;
  d->off.assign(db_off, db_off + ndb + 1);
  d->ndb = ndb;
  d->dim = dim;
  *out = d;
  return FFD_OK;
}

void ffd_db_destroy(ffd_db *db) { delete db; }

int ffd_server_arena_size(ffd_db *db, int32_t max_slots, int64_t max_query, size_t *bytes) {
  if (!db || !bytes) return FFD_E_INVALID;
  if (max_slots < 1 || max_slots > 4096) return fail(db->ctx, FFD_E_INVALID, "max_slots must be 1 .. 4096");
  if (max_query < 1 || max_query > (1 << 20)) return fail(db->ctx, FFD_E_INVALID, "max_query must be 1 .. 2^20");
  ffd_server s;
  int rc = make_server(db, max_slots, max_query, &s);
  if (rc) return rc;
  *bytes = arena_total(s);
  return FFD_OK;
}

int ffd_server_create(ffd_db *db, void *arena, size_t arena_bytes, int32_t max_slots, int64_t max_query,
                      ffd_server **out) {
  if (!out) return FFD_E_INVALID;
  *out = nullptr;
  if (!db) return FFD_E_INVALID;
  ffd_ctx *ctx = db->ctx;
  size_t need = 0;
  int rc = ffd_server_arena_size(db, max_slots, max_query, &need);
  if (rc) return rc;
  if (!arena) return fail(ctx, FFD_E_INVALID, "NULL arena");
  if (arena_bytes < need) return fail(ctx, FFD_E_NOMEM, "arena too small (see ffd_server_arena_size)");
  if (ctx->device < 0) return fail(ctx, FFD_E_DEVICE, "planning-only context cannot serve");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  ffd_server *s = new (std::nothrow) ffd_server();
  if (!s) return FFD_E_NOMEM;
  make_server(db, max_slots, max_query, s);
  unsigned char *A = static_cast<unsigned char *>(arena);
  // reordered database: coordinates and offsets
  float *dbx = reinterpret_cast<float *>(A);
  int64_t *dbo = reinterpret_cast<int64_t *>(A + al256((size_t)s->db_points * s->dim * sizeof(float)));
  std::vector<int64_t> hoff(db->ndb + 1, 0);
  hipStream_t st = nullptr;
  e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) {
    destroy_server(s);
    return hip_fail(ctx, e, "hipStreamCreate");
  }
  for (int64_t p = 0; p < db->ndb; ++p) {
    int32_t k = s->perm[p];
    int64_t n = db->off[k + 1] - db->off[k];
    hoff[p + 1] = hoff[p] + n;
    e = hipMemcpyAsync(dbx + hoff[p] * s->dim, db->X + db->off[k] * s->dim, (size_t)n * s->dim * sizeof(float),
                       hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) break;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(dbo, hoff.data(), hoff.size() * sizeof(int64_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipStreamDestroy(st);
  if (e != hipSuccess) {
    destroy_server(s);
    return hip_fail(ctx, e, "copying the database into the arena");
  }
  s->dbx = dbx;
  s->dbo = dbo;
  s->arena = A;
  s->links_at = db_bytes(*s) + (size_t)kTicks * s->lay.total;
  for (int i = s->link_pairs - 1; i >= 0; --i) s->free_links.push_back(i);
  // ticks
  size_t base = db_bytes(*s);
  for (int i = 0; i < kTicks; ++i) {
    Tick &t = s->ticks[i];
    t.dev = A + base + (size_t)i * s->lay.total;
    if ((e = hipStreamCreateWithFlags(&t.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&t.done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipHostMalloc((void **)&t.pin, s->lay.upload, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&t.pin_out, (size_t)s->kmax * db->ndb * sizeof(float),
                           hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&t.pin_err, sizeof(uint64_t), hipHostMallocDefault)) != hipSuccess) {
      destroy_server(s);
      return hip_fail(ctx, e, "creating the serving streams and staging buffers");
    }
  }
  try {
    s->worker = std::thread(worker_loop, s);
  } catch (...) {
    destroy_server(s);
    return fail(ctx, FFD_E_NOMEM, "cannot start the serving thread");
  }
  *out = s;
  return FFD_OK;
}

void ffd_server_destroy(ffd_server *s) { destroy_server(s); }

int ffd_server_submit(ffd_server *s, const float *q, int64_t n, int32_t metric, float *out, uint64_t *ticket) {
  if (!s || !q || !out || !ticket) return FFD_E_INVALID;
  if (n < 1) return sfail(s, FFD_E_INVALID, "query must have at least one point");
  if (n > s->max_query) return sfail(s, FFD_E_UNSUPPORTED, "query longer than the server's max_query");
  if (metric == FFD_MANHATTAN || metric == FFD_CHEBYSHEV)
    return sfail(s, FFD_E_UNSUPPORTED, "serving takes the Euclidean and squared Euclidean metrics");
  if (metric != FFD_EUCLIDEAN && metric != FFD_SQEUCLIDEAN) return sfail(s, FFD_E_INVALID, "unknown metric");
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return FFD_E_NOMEM;
  r->q.assign(q, q + n * s->dim);
  r->n = n;
  r->metric = metric;
  r->R = query_rows(*s, n);
  r->nb = ffd::bands_for(n, r->R);
  r->out = out;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->deadline_us > 0) r->deadline = r->t_submit + (double)s->deadline_us * 1e-6;
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    bool slot_free = s->pending.empty();
    if (slot_free) {
      slot_free = false;
      for (Tick &t : s->ticks)
        if (!t.busy && t.items.empty()) slot_free = true;
    }
    if (!slot_free) s->deferred++;
    if (s->submitted == 0) s->t_first = r->t_submit;
    s->submitted++;
    s->pending.push_back(r.get());
    s->reqs.emplace(r->ticket, std::move(r));
  }
  s->cv_work.notify_one();
  return FFD_OK;
}

int ffd_server_poll(ffd_server *s, uint64_t ticket, int32_t *done) {
  if (!s || !done) return FFD_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return sfail(s, FFD_E_INVALID, "unknown or already collected ticket");
  int st = it->second->state;
  if (st == 2 || st < 0) {
    *done = 1;
    s->reqs.erase(it);
    return st < 0 ? st : FFD_OK;
  }
  *done = 0;
  return FFD_OK;
}

int ffd_server_wait(ffd_server *s, uint64_t ticket, int64_t timeout_us) {
  if (!s) return FFD_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return sfail(s, FFD_E_INVALID, "unknown or already collected ticket");
  Request *r = it->second.get();
  auto ready = [&] { return r->state == 2 || r->state < 0; };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return FFD_E_TIMEOUT;
  }
  int st = r->state;
  s->reqs.erase(it);
  return st < 0 ? st : FFD_OK;
}

int ffd_server_cancel(ffd_server *s, uint64_t ticket) {
  if (!s) return FFD_E_INVALID;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(s, FFD_E_INVALID, "unknown or already collected ticket");
    it->second->cancel = true;
  }
  s->cv_work.notify_one();
  return FFD_OK;
}

int ffd_server_set_deadline(ffd_server *s, int64_t timeout_us) {
  if (!s) return FFD_E_INVALID;
  if (timeout_us < 0) return sfail(s, FFD_E_INVALID, "timeout_us < 0");
  std::lock_guard<std::mutex> g(s->mu);
  s->deadline_us = timeout_us;
  return FFD_OK;
}

int ffd_server_get_stats(ffd_server *s, ffd_server_stats *out) {
  if (!s || !out) return FFD_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->deferred = s->deferred;
  out->failed = s->failed;
  out->queued = (int64_t)s->pending.size();
  std::vector<double> l = s->lat;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) { return l[std::min(l.size() - 1, (size_t)std::floor(p * (double)(l.size() - 1) + 0.5))]; };
    out->p50_ms = pct(0.50) * 1e3;
    out->p99_ms = pct(0.99) * 1e3;
    out->max_ms = l.back() * 1e3;
    double sum = 0;
    for (double x : l) sum += x;
    out->mean_ms = sum / (double)l.size() * 1e3;
  }
  double span = s->t_last - s->t_first;
  if (span > 0) {
    out->qps = (double)s->completed / span;
    out->cells_per_s = s->cells / span;
  }
  out->requests_per_launch = s->kmax;
  out->waves = s->nwaves;
  for (int r = 0; r < kServeR; ++r) out->launches_by_rows[r] = s->launches_by_rows[r];
  out->canceled = s->canceled;
  out->expired = s->expired;
  return FFD_OK;
}

int ffd_server_reset_stats(ffd_server *s) {
  if (!s) return FFD_E_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  s->lat.clear();
  s->submitted = s->completed = s->deferred = s->failed = s->canceled = s->expired = 0;
  s->cells = 0;
  s->t_first = s->t_last = 0;
  for (int64_t &c : s->launches_by_rows) c = 0;
  return FFD_OK;
}

const char *ffd_server_last_error(const ffd_server *s) { return s ? s->last_error.c_str() : "NULL server"; }

}  // extern "C"

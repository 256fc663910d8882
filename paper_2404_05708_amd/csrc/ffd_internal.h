// Internal declarations shared by the host files of the library (planner,
// launcher and the serving loop).  Not part of the C ABI.
#ifndef FFD_INTERNAL_H
#define FFD_INTERNAL_H

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "ffd.h"
#include "ffd_plan.h"
#include "ffd_pipe_args.h"
#include "ffd_lanes.h"

namespace ffd {
hipError_t launch_stream_plain(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st);
hipError_t launch_stream_rings(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st);
hipError_t occupancy_stream_plain(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu);
hipError_t occupancy_stream_rings(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu);
// Float Frechet launches (no rings, not cooperative) with R in {3, 5, 6, 7}.
hipError_t launch_stream_serve(int R, int D, const KernelArgs &a, int wpb, hipStream_t st);
#define FFD_DECLARE_OP(n)                                                                                   \
  hipError_t launch_op_##n(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st); \
  hipError_t occupancy_op_##n(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu);
FFD_DECLARE_OP(1)
FFD_DECLARE_OP(3)
FFD_DECLARE_OP(4)
FFD_DECLARE_OP(5)
FFD_DECLARE_OP(6)
FFD_DECLARE_OP(7)
FFD_DECLARE_OP(8)
FFD_DECLARE_OP(10)
FFD_DECLARE_OP(11)
#undef FFD_DECLARE_OP
hipError_t clear_words(uint64_t *p, int64_t n, hipStream_t st);
// The pipelined single-pair kernel (ffd_kernels_pipe.hip): R in {2, 4}.
hipError_t launch_pipe(bool exact, int R, int D, const PipeArgs &a, size_t lds, hipStream_t st);
hipError_t occupancy_pipe(bool exact, int R, int D, size_t lds, int *blocks);
hipError_t pipe_init(void *links, int64_t nwords32, uint64_t *err, hipStream_t st);
size_t pipe_lds(bool exact, int D);  // LDS of a workgroup

// The kernel variant with LDS rings between waves serves launches whose
// plan uses them (a.rings); every other launch takes the plain variant.
// `op` = measure + 2 * cell (measure 0 Frechet, 1 DTW; cell 0 squared
// Euclidean, 1 Euclidean per cell, 2 Manhattan, 3 Chebyshev); op 8 is the
// Levenshtein distance (int32 symbols), ops 10 and 11 the Frechet distance
// and DTW on great-circle cells (FP64 unit vectors, D = 3).  Op 0 is the
// Frechet kernel on squared cells (with or without LDS rings); every other
// op has its own kernel family and never uses rings.  R is 1, 2, 4 or 8,
// or for op 0 with float coordinates, no rings and no cooperative launch
// also 3, 5, 6 or 7 (the serving shapes).
// D is the curves' coordinates per point (a.dim), run on the kernel of
// kernel_dim(D) coordinates.
inline hipError_t launch_stream(bool exact, int R, int D, const KernelArgs &a, int wpb, bool coop, hipStream_t st,
                                int op = 0) {
  if (a.dim != D) return hipErrorInvalidValue;
  D = kernel_dim(D);
  if ((R & (R - 1)) != 0) {
    if (op != 0 || exact || a.rings || coop) return hipErrorInvalidValue;
    return launch_stream_serve(R, D, a, wpb, st);
  }
  switch (op) {
    case 0: return a.rings ? launch_stream_rings(exact, R, D, a, wpb, coop, st)
                           : launch_stream_plain(exact, R, D, a, wpb, coop, st);
    case 1: return launch_op_1(exact, R, D, a, wpb, coop, st);
    case 3: return launch_op_3(exact, R, D, a, wpb, coop, st);
    case 4: return launch_op_4(exact, R, D, a, wpb, coop, st);
    case 5: return launch_op_5(exact, R, D, a, wpb, coop, st);
    case 6: return launch_op_6(exact, R, D, a, wpb, coop, st);
    case 7: return launch_op_7(exact, R, D, a, wpb, coop, st);
    case 8: return launch_op_8(exact, R, D, a, wpb, coop, st);
    case 10: return launch_op_10(exact, R, D, a, wpb, coop, st);
    case 11: return launch_op_11(exact, R, D, a, wpb, coop, st);
  }
  return hipErrorInvalidValue;
}
inline hipError_t occupancy_stream(bool exact, int R, int D, int wpb, size_t lds, int *blocks_per_cu,
                                   bool rings = false, int op = 0) {
  D = kernel_dim(D);
  switch (op) {
    case 0: return rings ? occupancy_stream_rings(exact, R, D, wpb, lds, blocks_per_cu)
                         : occupancy_stream_plain(exact, R, D, wpb, lds, blocks_per_cu);
    case 1: return occupancy_op_1(exact, R, D, wpb, lds, blocks_per_cu);
    case 3: return occupancy_op_3(exact, R, D, wpb, lds, blocks_per_cu);
    case 4: return occupancy_op_4(exact, R, D, wpb, lds, blocks_per_cu);
    case 5: return occupancy_op_5(exact, R, D, wpb, lds, blocks_per_cu);
    case 6: return occupancy_op_6(exact, R, D, wpb, lds, blocks_per_cu);
    case 7: return occupancy_op_7(exact, R, D, wpb, lds, blocks_per_cu);
    case 8: return occupancy_op_8(exact, R, D, wpb, lds, blocks_per_cu);
    case 10: return occupancy_op_10(exact, R, D, wpb, lds, blocks_per_cu);
    case 11: return occupancy_op_11(exact, R, D, wpb, lds, blocks_per_cu);
  }
  return hipErrorInvalidValue;
}
}  // namespace ffd

namespace ffdi {

using ffd::Job;
using ffd::KernelArgs;


// A planned launch.
struct Plan {
  int R = 4;
  int nwaves = 0;
  int wpb = 1;
  int64_t hcap = 0;            // LDS hand-off entries per wave
  int64_t max_steps = 0;       // longest stream of any wave
  int64_t link_elems = 0;      // elements of all link buffers
  int32_t nflags = 0;          // progress flags
  bool coop = false;           // some link joins two waves: cooperative launch
  bool rings = false;          // some bands hand rows on through LDS rings of their workgroup
  double makespan = 0;         // modelled, in steps
  std::vector<Job> jobs;       // grouped by wave, in placement order
  std::vector<int32_t> wave_jobs;
  // a single long pair on the pipelined kernel (no jobs): bands, workgroups,
  // XCD span of the chain order, orientation and link rows
  bool pipe = false;
  int32_t pipe_nb = 0, pipe_nwg = 0, pipe_xcd = 0;
  bool pipe_swap = false;      // the second curve holds the rows
  int64_t pipe_rows = 0, pipe_cols = 0;
  int64_t pipe_stride = 0;     // values per link row
  int64_t pipe_nlinks = 0;     // link rows
  size_t pipe_lds = 0;         // LDS requested per workgroup
  // a batch of short pairs on the one-pair-per-lane kernel (no jobs): class
  // c holds lane_order[lane_first[c], lane_first[c + 1]), column curves of at
  // most lane_cols[c] points, the widest class first
  bool lanes = false;
  int32_t lane_classes = 0;
  int32_t lane_cols[ffd::kLaneClasses] = {};
  int64_t lane_first[ffd::kLaneClasses + 1] = {};
  std::vector<int32_t> lane_order;  // pair index; the top bit: the second set holds the rows
  int32_t lane_waves = 0;           // with jobs as well: wavefronts of the lane launch
  int64_t lane_cross = 0;           // > 0: (query, database curve) pairs, this many database curves
  size_t alt_ws = 0;                // workspace of the job-table plan this one was chosen over
};

// A request as the planner sees it: header words (operation, dimension,
// value type, measure, tuning) and both offset arrays, compared in full
// (the hash only speeds up mismatches).
struct ReqKey {
  uint64_t hash = 0;
  std::vector<int64_t> words;
};

struct PlanCache {
  ReqKey key;
  uint64_t gen = 0;            // unique id of the cached (request, plan), never reused by a context
  Plan plan;
  bool valid = false;
};

// Device memory used by successive calls of a context (the caller's scratch
// or a workspace): the end of the last use, so that a use on another stream
// waits for it on the device.
struct UseOrder {
  const void *ptr = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool pending = false;
};

}  // namespace ffdi

struct ffd_ctx {
  int device = 0;
  int cus = 0;
  size_t lds_block_max = 0;   // LDS per workgroup the planner uses
  size_t lds_block_hw = 0;    // LDS a workgroup may request (device limit)
  size_t lds_cu = 0;          // LDS per compute unit
  int tune_R = 0;
  int tune_W = 0;
  float split = 0.f;          // 0 auto, < 0 split only when needed, > 0 split above this share
  int measure = 0;            // kernel op of the call in progress (measure + 2 * cell, see launch_stream)
  uint32_t epoch = 0;
  std::string last_error;
  uint64_t plan_gen = 0;      // last generation id handed out to a cached plan
  // plan most recently uploaded to device memory (a recorded launch needs it there)
  const void *plan_ws = nullptr;
  uint64_t plan_ws_gen = 0;
  void *pinned = nullptr;     // host staging buffer for plan uploads (pinned)
  size_t pinned_bytes = 0;
  uint64_t staged_gen = 0;    // plan whose bytes the staging buffer holds (0: none)
  hipEvent_t upload_done = nullptr;   // end of the last plan upload
  // kernel timing (ffd_set_kernel_timing): an event pair per launch around its kernels
  bool timing = false;
  std::vector<hipEvent_t> tev;  // pool, two per recorded launch
  size_t tev_used = 0;          // events recorded since the last ffd_kernel_time
  hipStream_t upload_stream = nullptr;
  bool upload_streams_mixed = false;  // uploads on more than one stream since the staging was written
  // plan image of the no-allocation entry point (pageable host memory)
  std::vector<unsigned char> noalloc_img;
  uint64_t noalloc_gen = 0;
  ffdi::PlanCache batch_plans, pair_plans;
  // launch shapes chosen by the autotuner, by request (offsets, op, dim, type)
  std::unordered_map<uint64_t, std::pair<ffdi::ReqKey, ffd_tuning>> tuned;
  // autotune results kept on disk by request class (ffd_set_tune_cache or
  // FFD_TUNE_CACHE): used for requests with no tuned shape of their own
  std::string tune_cache_path;
  std::map<std::string, ffd_tuning> tune_file;
  // device scratch registered by the caller (ffd_set_scratch): long single
  // pairs and the search calls; not owned
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  ffdi::UseOrder scratch_use, ws_use;
  void *search_host = nullptr;  // pinned host staging of the k-nearest search (owned)
  size_t search_host_bytes = 0;
  ffd_search_info last_search{};
  ffd_launch_info last{};
  uint64_t *last_err = nullptr; // device error word of the last launch (workspace)
  uint32_t last_epoch = 0;
  hipStream_t last_stream = nullptr;
};


namespace ffdi {

int fail(ffd_ctx *ctx, int code, const char *msg);
int hip_fail(ffd_ctx *ctx, hipError_t e, const char *what);
int check_offsets(ffd_ctx *ctx, const int64_t *off, int64_t count, const char *name);
int check_common(ffd_ctx *ctx, int32_t dim, int32_t metric, bool exact);
int lds_bytes(int R, int D, bool exact, int64_t hcap, bool rings = false, int measure = 0);
int64_t self_gap(int64_t sumL);

struct Resources {
  int nwaves_max;   // waves resident at once
  int nwaves_coop;  // waves surely resident at once (cooperative launches)
  int wpb;          // waves per workgroup
  int64_t hand_max; // longest LDS hand-off row
};
Resources resources(ffd_ctx *ctx, int R, int D, bool exact, int W);
// Modelled clocks of one stream step of a wave (R rows per lane, D
// coordinates, kernel op) with `waves_per_simd` waves sharing its SIMD.
double step_clocks(int R, int D, bool exact, double waves_per_simd, int op = 0);

// Make work on `st` that uses `ptr` wait for the previous use of the same
// memory on another stream (eager calls only: a recorded launch must not
// overlap other users of that memory), and record the end of this use.
int use_begin(ffd_ctx *ctx, UseOrder &u, const void *ptr, hipStream_t st, bool capturing);
int use_end(ffd_ctx *ctx, UseOrder &u, const void *ptr, hipStream_t st, bool capturing);
// Scratch bytes of the search calls (FFD_OP_DECIDE, FFD_OP_KNN; ffd_search.cpp).
int search_scratch_size(ffd_ctx *ctx, int32_t op, const int64_t *a_off, int64_t na, const int64_t *b_off,
                        int64_t nb, int32_t dim, size_t *bytes);

// The no-allocation entry point (ffd_noalloc.hip): resolve the device
// address of its static scratch on `device` (ffd_create), and run a batch
// with it as the workspace (ffd_host.cpp).
int noalloc_setup(ffd_ctx *ctx, int device);
size_t noalloc_bytes();
int batch_noalloc(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
                  int64_t npairs, int32_t dim, int32_t metric, float *out, void *ws, size_t ws_bytes, hipStream_t st);

// ffd_batch (float32, Euclidean or squared) with the registered scratch as
// the workspace: the decider at eps = +inf, where no pair can be dropped.
int batch_in_scratch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
                     int64_t npairs, int32_t dim, int32_t metric, float *out, hipStream_t st);

int plan_cross(ffd_ctx *ctx, const int64_t *q_off, int64_t nq, const int64_t *db_off, int64_t ndb, int D,
               bool exact, Plan &pl);
int cross_common(ffd_ctx *ctx, const void *Qs, const int64_t *q_off, int64_t nq, const void *DB,
                 const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, void *out, void *ws,
                 size_t ws_bytes, hipStream_t st, bool exact);

}  // namespace ffdi

#endif  // FFD_INTERNAL_H

/*
 * ffd.h -- C ABI of the MI355X (gfx950) discrete Frechet distance library.
 *
 * The library computes the discrete Frechet distance of Eiter and Mannila
 * between polygonal curves p in R^{P x D} and q in R^{Q x D} (Meinert,
 * "Walking Your Frog Fast in 4 LoC", arXiv 2404.05708, Sec. 2), i.e. M_PQ of
 * the recurrence of Eq. (1)
 *
 *     M_ij = max{ min{ M_{i-1,j}, M_{i-1,j-1}, M_{i,j-1} }, d_ij },
 *
 * with the first row and column given by running maxima (Algorithms 3-5).
 * It evaluates d_ij lazily, keeps O(Q) state per pair (Theorem 1) and never
 * branches per cell.  Ground distances: Euclidean ||p_i - q_j||_2 and squared
 * Euclidean (Sec. 4 names the Euclidean distance; Sec. 3 notes that the
 * method makes no assumption about the metric).
 *
 * Conventions for every call
 * --------------------------
 *  - Curves are row-major arrays of points: point i of a D-dimensional curve
 *    is x[i*D .. i*D+D).  Indices in this header are 0-based.
 *  - Coordinate, output and workspace pointers are DEVICE pointers (memory of
 *    the context's GPU); offset arrays are HOST pointers (the host plans the
 *    work from them).  The caller owns all of them; the library never frees
 *    or keeps a caller pointer beyond the completion of the call's work on
 *    `stream`, except the scratch registered with ffd_set_scratch (kept
 *    until it is replaced or the context is destroyed) and an ffd_db, which
 *    refers to its database until ffd_db_destroy.  The library allocates no
 *    device memory: device scratch comes from the caller (workspaces,
 *    ffd_set_scratch, the serving arena).
 *  - Workspaces and the scratch: a call writes its plan (job table,
 *    offsets, cleared progress flags) into the workspace before its kernel,
 *    on `stream`, every time it runs outside graph capture, so nothing the
 *    memory held before the call is trusted.  Successive calls of one
 *    context that use the same workspace, or the scratch, on different
 *    streams are ordered on the device (the later stream waits for the
 *    earlier call's work).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous: results are valid once the stream has completed.
 *  - Return value: FFD_OK or a negative FFD_E_* status.  All argument checks
 *    happen on the host before anything is launched; a failed call launches
 *    nothing and leaves the outputs untouched.  Device faults surface as
 *    FFD_E_DEVICE from a later call that synchronises.
 *  - Preconditions (documented, not checked): coordinates are finite; float
 *    coordinates satisfy |x| < 1e18 so that squares do not overflow; int32
 *    coordinates satisfy |x| < 2^24 (dim <= 4) or |x| < 2^23 (dim 5 to 16)
 *    so that every intermediate is exact.
 *  - Float32 results of the Frechet calls agree with the exact real-number
 *    result to a relative error of 2e-6 (each d_ij is evaluated in float32
 *    in a fixed order, with at most 2 D - 1 roundings; the recurrence only
 *    selects values; for FFD_EUCLIDEAN the square root is taken once per
 *    pair and correctly rounded).  Int32 results are exact.
 *  - A context may be used by one host thread at a time.
 *  - Graph capture: ffd_distance, ffd_batch and ffd_cross (and their int32
 *    forms) may be recorded into a hipGraph by stream capture when the
 *    context's last call outside the capture that used this workspace (or,
 *    for a single long pair, the registered scratch) was the same call (same
 *    offsets, dimension, type, tuning and memory): the plan is then in that
 *    memory, and the recorded work is a small kernel that clears the
 *    launch's progress flags followed by the distance kernel.  Otherwise the
 *    call returns FFD_E_UNSUPPORTED and records nothing.  The memory then
 *    belongs to the graph: the caller promises that nothing writes to it
 *    between replays (a later eager call with other offsets on the same
 *    workspace replaces the plan the replays read).  Replays of one graph
 *    must not overlap each other or other work on the same memory.  The
 *    autotuner, the search and the serving calls cannot be captured.
 */
#ifndef FFD_H
#define FFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define FFD_OK 0
#define FFD_E_INVALID (-1)     /* bad argument (NULL, empty curve, bad offsets ...) */
#define FFD_E_UNSUPPORTED (-2) /* valid request outside what the library supports */
#define FFD_E_NOMEM (-3)       /* workspace or arena too small                      */
#define FFD_E_DEVICE (-4)      /* HIP runtime error                                 */
#define FFD_E_BUSY (-5)        /* serving: no free slot right now                   */
#define FFD_E_TIMEOUT (-6)     /* serving: wait timed out                           */
#define FFD_E_CANCELED (-7)    /* serving: request canceled (ffd_server_cancel)     */
#define FFD_E_EXPIRED (-8)     /* serving: request deadline passed before it ran    */

/* Ground distances (Sec. 2: f(p_i, q_j); Sec. 3: the method makes no
 * assumption about it).  int32 calls take every metric but FFD_EUCLIDEAN
 * and FFD_HAVERSINE; the serving calls take FFD_EUCLIDEAN and
 * FFD_SQEUCLIDEAN.
 * FFD_HAVERSINE is the great-circle distance on the unit sphere (the
 * central angle, in radians; multiply by the sphere's radius for a length)
 * between points given as (latitude, longitude) in radians, dim = 2.  The
 * float32 Frechet and DTW calls take it (ffd_distance, ffd_batch, ffd_cross,
 * their DTW forms and the autotuners; not the int32, serving or search
 * calls).  Internally each point becomes its FP64 unit vector and the cell
 * is its squared chord: the Frechet sweep selects on chords (the angle
 * 2 asin(chord / 2) increases with the chord, so Eq. (1) selects the same
 * cells) and takes the angle once per pair; DTW takes the angle in every
 * cell (float32 square root and arcsine of the FP64 chord) and sums in FP64.  ffd_last_launch then reports dim 3 and the FP64
 * value type. */
#define FFD_EUCLIDEAN 0   /* ||p_i - q_j||_2                          */
#define FFD_SQEUCLIDEAN 1 /* ||p_i - q_j||_2^2                        */
#define FFD_MANHATTAN 2   /* sum_k |p_ik - q_jk|                      */
#define FFD_CHEBYSHEV 3   /* max_k |p_ik - q_jk|                      */
#define FFD_HAVERSINE 4   /* central angle of (lat, lon) points       */

/* Largest supported dimension D (coordinates per point).  Curves of up to
 * four coordinates run on kernels of their own; curves of 5 to 16 on kernels
 * for 8 or 16 coordinates that hold zeros past the curves' own (the same
 * results, bit for bit, at the cost of the padded coordinates' arithmetic,
 * with 2 rows per lane and no pipelined single-pair kernel). */
#define FFD_MAX_DIM 16

/* Operation codes for ffd_workspace_size (and ffd_plan_describe). */
#define FFD_OP_BATCH 0
#define FFD_OP_CROSS 1
#define FFD_OP_PAIR 2
#define FFD_OP_DECIDE 3
#define FFD_OP_KNN 4

typedef struct ffd_ctx ffd_ctx;

/* Create a context on HIP device `device`.  The context owns host-side plans
 * and launch settings only; it allocates no device memory.
 * Errors: FFD_E_INVALID (out == NULL), FFD_E_DEVICE (no such device or the
 * device is not gfx950). */
int ffd_create(int device, ffd_ctx **out);
void ffd_destroy(ffd_ctx *ctx);

/* Create a planning-only context without a device, describing a GPU with
 * `compute_units` CUs and `lds_per_block` bytes of LDS per workgroup.  It
 * checks arguments and sizes workspaces exactly like a device context; every
 * call that would launch work returns FFD_E_DEVICE after its checks pass.
 * Errors: FFD_E_INVALID (out == NULL, compute_units < 1, lds_per_block <
 * 16384). */
int ffd_create_planner(int32_t compute_units, int64_t lds_per_block, ffd_ctx **out);

/* Static text for a status code. */
const char *ffd_strerror(int status);
/* Text of the last error reported on this context ("" if none). */
const char *ffd_last_error(const ffd_ctx *ctx);
/* Library version string. */
const char *ffd_version(void);

/* One pair (Eq. (1), result M_PQ; Algorithm 5 / Algorithm 2 form).
 *   p   [n * dim] float32, device;  q [m * dim] float32, device;
 *   out [1] float32, device: delta_dF(p, q) under `metric`.
 * A pair short enough for one wavefront needs no device memory; a long pair
 * is split into bands over many wavefronts, whose plan and boundary rows go
 * into the scratch registered with ffd_set_scratch (its size from
 * ffd_workspace_size with FFD_OP_PAIR; 0 for a pair that needs none).
 * Errors: FFD_E_INVALID for NULL pointers, n < 1, m < 1, dim < 1, an
 * unknown metric or FFD_HAVERSINE with dim != 2; FFD_E_UNSUPPORTED for
 * dim > FFD_MAX_DIM; FFD_E_NOMEM for a long pair without enough registered
 * scratch. */
int ffd_distance(ffd_ctx *ctx, const float *p, int64_t n, const float *q, int64_t m,
                 int32_t dim, int32_t metric, float *out, void *stream);

/* One pair with int32 coordinates, exact: out [1] int64, device.  metric is
 *   FFD_SQEUCLIDEAN, FFD_MANHATTAN or FFD_CHEBYSHEV (FFD_EUCLIDEAN and
 *   FFD_HAVERSINE: FFD_E_UNSUPPORTED).  Other errors as ffd_distance. */
int ffd_distance_i32(ffd_ctx *ctx, const int32_t *p, int64_t n, const int32_t *q, int64_t m,
                     int32_t dim, int32_t metric, int64_t *out, void *stream);

/* Many independent pairs in one launch (Sec. 4: batches of curves; here
 * each pair has its own lengths).
 *   Pair k is (P[p_off[k] .. p_off[k+1]), Q[q_off[k] .. q_off[k+1])), offsets
 *   in points, HOST int64 arrays of npairs + 1 entries starting at 0 and
 *   strictly increasing (every curve has at least one point).
 *   P, Q: device float32 coordinates; out [npairs] float32, device.
 *   workspace: device memory of ws_bytes >= ffd_workspace_size(FFD_OP_BATCH).
 *   Contents of the workspace are overwritten; it may be reused across calls
 *   once the previous call on it has completed.
 *   Many short pairs (a curve of at most 64 points; 32 for dim 3 and 4) may
 *   run one pair per GPU lane, alone or in a launch before the streaming
 *   kernel's for the batch's other pairs, when that is modelled faster
 *   (ffd_last_launch reports per_lane = 1): the same results, bit for bit.
 * npairs == 0 is a no-op.  Errors: FFD_E_INVALID (bad offsets, NULL, metric),
 * FFD_E_UNSUPPORTED (dim), FFD_E_NOMEM (workspace too small). */
int ffd_batch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q,
              const int64_t *q_off, int64_t npairs, int32_t dim, int32_t metric, float *out,
              void *workspace, size_t ws_bytes, void *stream);

/* ffd_batch for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same launch and results, with no workspace argument.  Its workspace is a
 * static device array of the library, 32 MiB on each GPU, held until the
 * process ends; the call allocates no device or pinned memory and creates
 * no runtime objects (its events and the array's device address are set up
 * by ffd_create).  The plan is copied from pageable host memory of the
 * context.  Every call on one GPU shares that GPU's array, from any
 * context: calls that overlap on one GPU race (calls of one context on
 * different streams are ordered by the library; calls of different contexts
 * are not).  Results are valid once the stream has completed.
 * Errors: as ffd_batch; FFD_E_NOMEM when the request needs more than the
 * 32 MiB (the message gives the size it needs), checked before any launch;
 * FFD_E_DEVICE when the array could not be resolved on the device. */
int ffd_batch_noalloc(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q,
                      const int64_t *q_off, int64_t npairs, int32_t dim, int32_t metric, float *out,
                      void *stream);

/* Int32 version of ffd_batch: exact int64 out[npairs]; metrics as
 * ffd_distance_i32. */
int ffd_batch_i32(ffd_ctx *ctx, const int32_t *P, const int64_t *p_off, const int32_t *Q,
                  const int64_t *q_off, int64_t npairs, int32_t dim, int32_t metric,
                  int64_t *out, void *workspace, size_t ws_bytes, void *stream);

/* Query set x database set (Sec. 4: a batch of curves against a reference
 * curve, generalised to many references):
 *   out[i * ndb + k] = delta_dF(query i, database curve k), row-major,
 *   out [nq * ndb] float32 device.  q_off [nq + 1] and db_off [ndb + 1] are
 *   HOST offsets as in ffd_batch.  Errors as ffd_batch. */
int ffd_cross(ffd_ctx *ctx, const float *Qs, const int64_t *q_off, int64_t nq,
              const float *DB, const int64_t *db_off, int64_t ndb, int32_t dim,
              int32_t metric, float *out, void *workspace, size_t ws_bytes, void *stream);

/* Int32 version of ffd_cross: exact int64 out[nq * ndb]; metrics as
 * ffd_distance_i32. */
int ffd_cross_i32(ffd_ctx *ctx, const int32_t *Qs, const int64_t *q_off, int64_t nq,
                  const int32_t *DB, const int64_t *db_off, int64_t ndb, int32_t dim,
                  int32_t metric, int64_t *out, void *workspace, size_t ws_bytes,
                  void *stream);

/* Dynamic time warping (Appendix B, Algorithm B.1): the recurrence of Eq. (1)
 * with the outer max replaced by a sum,
 *     M_ij = min{ M_{i-1,j}, M_{i-1,j-1}, M_{i,j-1} } + d_ij,   DTW = M_PQ,
 * whose first row and column are running sums of d.  Each call takes the
 * arguments of its Frechet counterpart (ffd_distance, ffd_batch, ffd_cross
 * and their int32 forms) with the same layouts, ownership, workspace sizes
 * (ffd_workspace_size covers both) and errors.  The ground distance is
 * summed per cell, so FFD_EUCLIDEAN takes the hardware float32 square root
 * (within 1 ulp) in every cell, FFD_SQEUCLIDEAN sums squared distances and
 * FFD_MANHATTAN / FFD_CHEBYSHEV their cell distances, FFD_HAVERSINE the
 * angles (float32 in every cell, summed in FP64); the result is the sum
 * itself.  Float32 results agree with the exact result to a relative error
 * of (n + m + 2 D + 2) 2^-24 (each cell carries at most 2 D + 1 rounding
 * errors, the sum along the selected coupling one per addition), for
 * Euclidean cells whose squared distance is not below 2^-126; great-circle
 * results to 2e-6 relative.  Int32 calls
 * (every metric but FFD_EUCLIDEAN) are exact while the sums stay below 2^53
 * (for example |x| < 2^15 and n + m < 2^19). */
int ffd_dtw_distance(ffd_ctx *ctx, const float *p, int64_t n, const float *q, int64_t m,
                     int32_t dim, int32_t metric, float *out, void *stream);
int ffd_dtw_distance_i32(ffd_ctx *ctx, const int32_t *p, int64_t n, const int32_t *q,
                         int64_t m, int32_t dim, int32_t metric, int64_t *out, void *stream);
int ffd_dtw_batch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q,
                  const int64_t *q_off, int64_t npairs, int32_t dim, int32_t metric, float *out,
                  void *workspace, size_t ws_bytes, void *stream);
int ffd_dtw_batch_i32(ffd_ctx *ctx, const int32_t *P, const int64_t *p_off, const int32_t *Q,
                      const int64_t *q_off, int64_t npairs, int32_t dim, int32_t metric,
                      int64_t *out, void *workspace, size_t ws_bytes, void *stream);
int ffd_dtw_cross(ffd_ctx *ctx, const float *Qs, const int64_t *q_off, int64_t nq,
                  const float *DB, const int64_t *db_off, int64_t ndb, int32_t dim,
                  int32_t metric, float *out, void *workspace, size_t ws_bytes, void *stream);
int ffd_dtw_cross_i32(ffd_ctx *ctx, const int32_t *Qs, const int64_t *q_off, int64_t nq,
                      const int32_t *DB, const int64_t *db_off, int64_t ndb, int32_t dim,
                      int32_t metric, int64_t *out, void *workspace, size_t ws_bytes,
                      void *stream);

/* Levenshtein distance (Appendix B, Algorithm B.2) of sequences of int32
 * symbols (a symbol is `dim` int32 values; two symbols are equal when every
 * value is): the minimum number of insertions, deletions and substitutions,
 * the recurrence
 *     M_ij = min{ M_{i-1,j} + 1, M_{i,j-1} + 1, M_{i-1,j-1} + [p_i != q_j] }
 * with M_{-1,j} = j + 1, M_{i,-1} = i + 1, M_{-1,-1} = 0 (0-based; the
 * algorithm's index vectors read 0-based), result M_PQ, exact int64.  The
 * calls take the arguments of ffd_distance_i32, ffd_batch_i32 and
 * ffd_cross_i32 without the metric, with the same layouts, workspace sizes
 * and errors, and FFD_E_UNSUPPORTED when a pair's lengths reach n + m >=
 * 2^24 (the table's values are held as float32 integers, exact below 2^24;
 * any int32 symbol values are allowed). */
int ffd_levenshtein_distance(ffd_ctx *ctx, const int32_t *p, int64_t n, const int32_t *q,
                             int64_t m, int32_t dim, int64_t *out, void *stream);
int ffd_levenshtein_batch(ffd_ctx *ctx, const int32_t *P, const int64_t *p_off,
                          const int32_t *Q, const int64_t *q_off, int64_t npairs, int32_t dim,
                          int64_t *out, void *workspace, size_t ws_bytes, void *stream);
int ffd_levenshtein_cross(ffd_ctx *ctx, const int32_t *Qs, const int64_t *q_off, int64_t nq,
                          const int32_t *DB, const int64_t *db_off, int64_t ndb, int32_t dim,
                          int64_t *out, void *workspace, size_t ws_bytes, void *stream);

/* Device memory needed by a call.  Workspaces: ffd_batch (op =
 * FFD_OP_BATCH: a_off = p_off, na = npairs, b_off = q_off, nb = npairs) or
 * ffd_cross (op = FFD_OP_CROSS: a_off = q_off, na = nq, b_off = db_off, nb =
 * ndb), and their int32, DTW and Levenshtein forms: the size covers all of
 * them.  Scratch (ffd_set_scratch): ffd_distance of a pair (op =
 * FFD_OP_PAIR: a_off = {0, n}, b_off = {0, m}, na = nb = 1; every form and
 * metric), ffd_decide_batch (op = FFD_OP_DECIDE, arguments as FFD_OP_BATCH)
 * and ffd_knn / ffd_knn_batch (op = FFD_OP_KNN: a_off = the queries'
 * offsets ({0, n} for one), na = nq, b_off = db_off, nb = ndb).  Writes
 * *bytes (0: the call needs none).
 * Errors: FFD_E_INVALID for a bad op, NULL or bad offsets. */
int ffd_workspace_size(ffd_ctx *ctx, int32_t op, const int64_t *a_off, int64_t na,
                       const int64_t *b_off, int64_t nb, int32_t dim, size_t *bytes);

/* Register device memory of `bytes` bytes (caller-owned; NULL and 0
 * unregister) as the context's scratch for ffd_distance of long pairs and
 * for the search calls (ffd_decide_batch, ffd_knn).  The context keeps the
 * pointer until it is replaced or the context is destroyed; the caller
 * keeps the memory alive that long and, before freeing memory it replaces,
 * waits for the calls that used it.  Calls that need more than the
 * registered size return FFD_E_NOMEM and launch nothing.
 * Errors: FFD_E_INVALID (NULL ctx, NULL scratch with bytes > 0). */
int ffd_set_scratch(ffd_ctx *ctx, void *scratch, size_t bytes);

/* Introspection (tests and tools): the plan that a call would launch.
 *   op: FFD_OP_BATCH (a_off = p_off, b_off = q_off, na = nb = npairs),
 *   FFD_OP_CROSS (a_off = q_off, b_off = db_off) or FFD_OP_PAIR (a_off =
 *   {0, n}, b_off = {0, m}, na = nb = 1: ffd_distance); measure 0 for the
 *   Frechet calls, 1 for DTW, 2 for Levenshtein (exact = 1); metric,
 *   dim and exact (int32 coordinates) as in the calls (FFD_HAVERSINE:
 *   dim 2, exact 0, measure 0).  HOST
 *   arrays only; nothing is launched, and a planning-only context works.
 *   *summary receives the launch shape; jobs (ffd_plan_job[jobs_cap], may be
 *   NULL) receives the job table grouped by wave, wave_jobs (int32
 *   [waves + 1], may be NULL) the first job of each wave.  Stream positions
 *   follow from the jobs: each job runs its column curves in order, each
 *   column curve's bands in order; a task lasts 16 + m steps (at least 16
 *   separators, then the m columns) rounded up to a multiple of 16 and to
 *   at least 80; an idle job (row_sel 2) lasts col_count steps.
 * Errors: as ffd_batch / ffd_cross / ffd_distance; FFD_E_NOMEM when jobs_cap
 * or the wave_jobs array is too small (the summary is filled first). */
typedef struct ffd_plan_summary {
  int32_t rows_per_lane;   /* R                                              */
  int32_t waves;           /* wavefronts                                     */
  int32_t waves_per_block; /* wavefronts per workgroup                       */
  int32_t cooperative;     /* 1: waves wait on each other (global links)     */
  int32_t rings;           /* 1: bands hand rows on through LDS rings        */
  int32_t flags;           /* progress flags (global links)                  */
  int64_t link_elems;      /* elements of all link buffers                   */
  int64_t stream_steps;    /* longest stream of any wave                     */
  int64_t jobs;            /* entries of the job table                       */
  int32_t pipelined;       /* 1: a single long pair on the pipelined kernel:
                              no job table; waves = 4 x workgroups, one band
                              of 64 R rows per wave and pass, link_elems
                              values of boundary rows between workgroups   */
  int32_t per_lane;        /* 1: short pairs one per lane.  With no job table
                              the whole batch (rows_per_lane 0; waves =
                              pairs / 64 rounded up per class of column
                              count, stream_steps = the most rows of any
                              lane); with one, the batch's short pairs, in a
                              launch before the job table's for the rest  */
} ffd_plan_summary;
typedef struct ffd_plan_job { /* 64 bytes */
  int64_t out_base;   /* output index of the first column curve              */
  int64_t link_in;    /* first element of the incoming boundary rows          */
  int64_t link_out;   /* first element of the outgoing boundary rows          */
  int32_t row_sel;    /* 0: row curve from the first set (P, queries), 1:
                         from the second (Q, database), 2: idle job           */
  int32_t row_idx;    /* row curve index                                      */
  int32_t col_sel;    /* set of the column curves                             */
  int32_t col_first;  /* first column curve                                   */
  int32_t col_count;  /* column curves (idle job: steps)                      */
  int32_t out_stride; /* output index step between column curves            */
  int32_t band_first; /* bands [band_first, band_first + band_count) of 64 R  */
  int32_t band_count; /* rows (<= 0: to the last band)                        */
  int32_t flag_in;    /* flag of the incoming link; -1 none; <= -2: LDS ring
                         of wave (-2 - flag_in) of the same workgroup         */
  int32_t flag_out;   /* flag of the outgoing link; -1 none; -2: LDS ring     */
} ffd_plan_job;
int ffd_plan_describe(ffd_ctx *ctx, int32_t op, const int64_t *a_off, int64_t na,
                      const int64_t *b_off, int64_t nb, int32_t dim, int32_t exact,
                      int32_t measure, int32_t metric, ffd_plan_summary *summary,
                      ffd_plan_job *jobs, int64_t jobs_cap, int32_t *wave_jobs,
                      int64_t wave_jobs_cap);

/* Tuning knobs (0 = automatic).  rows_per_lane in {1, 2, 4, 8}: points of the
 * row curve each GPU lane holds; waves_per_simd: resident waves per SIMD the
 * batch planner targets, or -1: a single Frechet pair (ffd_distance) runs on
 * the pipelined single-pair kernel whenever that kernel can run it, whatever
 * the cost model prefers.  Curves of 5 to 16 coordinates run with one rows
 * per lane only (2 up to 8 coordinates, 1 above): a forced other value makes
 * their calls return FFD_E_UNSUPPORTED.  Returns FFD_E_INVALID for values out
 * of range. */
int ffd_set_tuning(ffd_ctx *ctx, int32_t rows_per_lane, int32_t waves_per_simd);

/* Shape of the most recent launch on this context, for reporting and tuning.
 * Fields are 0 if nothing has been launched.  Errors: FFD_E_INVALID (NULL). */
typedef struct ffd_launch_info {
  int32_t rows_per_lane;   /* points of the row curve per lane (R)          */
  int32_t waves;           /* wavefronts launched                           */
  int32_t waves_per_block; /* wavefronts per workgroup                      */
  int32_t lds_per_wave;    /* bytes of LDS per wavefront                    */
  int32_t exact;           /* 1: int32 path with FP64-exact values          */
  int32_t dim;             /* D                                             */
  int32_t pipelined;       /* 1: the pipelined single-pair kernel           */
  int32_t helper_waves;    /* waves per workgroup that compute no band      */
  int64_t stream_steps;    /* longest per-wave stream (steps)               */
  int32_t per_lane;        /* 1: short pairs one per lane: the whole batch
                              (rows_per_lane 0) or, before this streaming
                              launch, the batch's short pairs             */
} ffd_launch_info;

int ffd_last_launch(const ffd_ctx *ctx, ffd_launch_info *info);

/* Kernel timing, for measurement.  While enabled, every ffd_batch,
 * ffd_cross (all their variants, eager calls only) and ffd_distance that
 * runs on many wavefronts records a HIP event on its stream just before its
 * first kernel and one just after its last: the time between them leaves
 * out the plan upload.  The first time a launch is timed the context
 * creates the events it needs (kept until ffd_destroy); at most 65536
 * launches are recorded between two reads, later ones are not.  Enabling
 * or disabling clears the record.
 * Errors: FFD_E_INVALID (NULL, or a planning-only context). */
int ffd_set_kernel_timing(ffd_ctx *ctx, int32_t enable);

/* Waits for the launches recorded since the last read or ffd_set_kernel_timing
 * and returns their summed kernel time (milliseconds, `*total_ms`) and their
 * number (`*launches`, 0 when none), then clears the record.
 * Errors: FFD_E_INVALID (NULL), FFD_E_DEVICE. */
int ffd_kernel_time(ffd_ctx *ctx, double *total_ms, int64_t *launches);

/* Error bits the most recent launch on this context raised on the device
 * (waits for it to finish): bit 0 = a wavefront hit its step bound, bit 1 =
 * a wavefront gave up waiting for a boundary row from another wavefront
 * (possible only when other work occupies the GPU so long that the
 * producing wavefront cannot start).  Results of such a launch are not
 * valid: a wavefront that abandons a wait stores every later result as NaN
 * (float results) or -1 (int64 results), and waits no more.  0 for
 * launches that use no workspace.
 * Errors: FFD_E_INVALID (NULL), FFD_E_DEVICE. */
int ffd_last_errors(ffd_ctx *ctx, int32_t *flags);

/* How eagerly long pairs are split into bands that run on different
 * wavefronts (their boundary rows pass through the workspace): a pair whose
 * modelled work exceeds `share` times a wavefront's fair share of the launch
 * is split; a negative value = never (a pair whose boundary row does not fit
 * in LDS then keeps its bands on one wavefront, chained through the
 * workspace); 0 = automatic: share 1.25 for ffd_batch and ffd_cross, and
 * ffd_distance splits a long pair whenever the model says it pays.  A
 * launch with split pairs is cooperative (all its workgroups resident at
 * once).  Results do not depend on the setting.
 * Errors: FFD_E_INVALID (NaN or huge share). */
int ffd_set_split(ffd_ctx *ctx, float share);

/* ----------------------------------------------------------- autotune --- */
typedef struct ffd_tuning {
  int32_t rows_per_lane;   /* chosen launch shape */
  int32_t waves_per_simd;
  float split;             /* band-split share (see ffd_set_split) */
  float ms;                /* kernel time of the chosen shape */
  float ms_planner;        /* kernel time of the planner's own choice */
  int32_t tried;           /* shapes timed */
} ffd_tuning;

/* Time the launch shapes the planner can produce for this request (rows per
 * lane 2, 4, 8; one or two waves per SIMD; band-split shares) on the given
 * data, on `stream`, and keep the fastest: later ffd_batch (ffd_cross)
 * calls with the same offsets, dim and coordinate type, made while the
 * context's tuning and split settings are automatic, use it.  Arguments as
 * for ffd_batch (ffd_cross); `out` receives the results; shapes whose
 * workspace exceeds ws_bytes are skipped.  Synchronises the stream.
 * Errors: as ffd_batch (ffd_cross). */
int ffd_autotune_batch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
                       int64_t npairs, int32_t dim, int32_t metric, float *out, void *workspace, size_t ws_bytes,
                       void *stream, ffd_tuning *best);
int ffd_autotune_cross(ffd_ctx *ctx, const float *Qs, const int64_t *q_off, int64_t nq, const float *DB,
                       const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, float *out,
                       void *workspace, size_t ws_bytes, void *stream, ffd_tuning *best);

/* Keep autotune results on disk: `path` names a JSON file (NULL or "": none,
 * the default; a context made by ffd_create takes the environment variable
 * FFD_TUNE_CACHE).  Its entries are read now.  Every later autotune call
 * adds its choice to the file, under the class of the request: gfx950 and
 * its compute units, the operation, the kernel (measure and ground
 * distance), the value type, D, and log2 buckets of the mean lengths and
 * the curve counts of both sides.  A request that has no tuned shape of its
 * own and runs with automatic settings uses the file's shape for its class;
 * an entry of zeros keeps the model's choice.  A missing file counts as
 * empty, and lines that do not parse are skipped.  Errors: FFD_E_INVALID
 * (NULL ctx). */
int ffd_set_tune_cache(ffd_ctx *ctx, const char *path);

/* ------------------------------------------- decider and k-nearest search ---
 * Early abandoning (Eq. (1): M_ij is the smallest, over monotone paths to
 * (i, j), of the largest cell on the path, so delta is at least the smallest
 * M over any set of cells that every full path must cross).  A wavefront
 * sweeps one pair at a time and, every 16 columns, tests such a set -- its
 * current anti-diagonal staircase, the cells just above it, the rest of the
 * band above and, when bands follow, the band's own bottom row so far --
 * against a threshold; once every cell of the set exceeds it the pair is
 * dropped.  Float32 coordinates, FFD_EUCLIDEAN or
 * FFD_SQEUCLIDEAN (other metrics: FFD_E_UNSUPPORTED); the values that are
 * kept have the same bits as ffd_batch's.  The calls use the scratch
 * registered with ffd_set_scratch (sizes from ffd_workspace_size with
 * FFD_OP_DECIDE or FFD_OP_KNN; FFD_E_NOMEM without it); the k-nearest
 * calls also use pinned host staging of about 12 bytes per (query, database
 * curve) pair that the context allocates on first need and keeps until
 * ffd_destroy.  They cannot be recorded into a graph (FFD_E_UNSUPPORTED). */

/* Decider: out[k] = delta(P_k, Q_k) when it is <= eps (the same value as
 * ffd_batch), else +inf, so that out[k] <= eps answers "is delta <= eps?".
 * Arguments as ffd_batch without the workspace; eps is a distance in the
 * metric's units (+inf: no pair can be dropped, and the call runs ffd_batch
 * in the registered scratch; below 0: every pair is dropped).  Each pair is
 * swept with the curve whose bands waste fewer rows as the row curve (the
 * distance is symmetric).
 * Asynchronous on `stream`; offsets are HOST arrays, read before return.
 * Errors: FFD_E_INVALID (NULL, bad offsets, NaN eps, unknown metric, dim <
 * 1), FFD_E_UNSUPPORTED (metric, dim > FFD_MAX_DIM, a column curve of 2^31
 * or more values), FFD_E_NOMEM (registered scratch too small), FFD_E_DEVICE. */
int ffd_decide_batch(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q, const int64_t *q_off,
                     int64_t npairs, int32_t dim, int32_t metric, float eps, float *out, void *stream);

/* The k database curves nearest to the query q (n points) under the
 * discrete Frechet distance, exactly: out_idx[i] (int64, device) and
 * out_dist[i] (float32, device) for i < min(k, ndb), in increasing
 * distance, ties by the smaller index; entries past ndb get index -1 and
 * distance +inf.  Stages: the larger of the first-point and last-point
 * distances bounds each curve's distance from below; 128 curves (at least
 * k) with the smallest bounds, taken from those at most four times the
 * median length when there are enough, are evaluated exactly and the k-th
 * smallest distance becomes the threshold; every other curve whose bound
 * does not exceed it runs through the early-abandoning sweep at that
 * threshold.  Database layout as ffd_cross (device coordinates, HOST
 * offsets).  Synchronises the stream.
 * Errors: FFD_E_INVALID (NULL, k < 1, n < 1, ndb < 1, bad offsets, unknown
 * metric), FFD_E_UNSUPPORTED (metric, dim, too many or too long curves),
 * FFD_E_NOMEM (registered scratch too small),
 * FFD_E_DEVICE. */
int ffd_knn(ffd_ctx *ctx, const float *q, int64_t n, const float *DB, const int64_t *db_off, int64_t ndb,
            int32_t dim, int32_t metric, int32_t k, int64_t *out_idx, float *out_dist, void *stream);

/* ffd_knn for nq queries in one call (CSR: Q device coordinates, q_off HOST
 * offsets, every query at least one point): the results of query i are
 * out_idx[i * k + j] and out_dist[i * k + j], each query's exactly as
 * ffd_knn gives them.  The stages run for all queries at once: one launch
 * of the bounds, one of the 128-curve first stages, one of the thresholded
 * sweeps, so the host work and the GPU's fill are shared.
 * Errors: as ffd_knn; FFD_E_INVALID for nq < 1 or an empty query,
 * FFD_E_UNSUPPORTED when nq * ndb exceeds 2^30. */
int ffd_knn_batch(ffd_ctx *ctx, const float *Q, const int64_t *q_off, int64_t nq, const float *DB,
                  const int64_t *db_off, int64_t ndb, int32_t dim, int32_t metric, int32_t k, int64_t *out_idx,
                  float *out_dist, void *stream);

typedef struct ffd_search_info {
  int64_t exact;     /* curves evaluated before the threshold was set */
  int64_t bounded;   /* curves swept against the threshold */
  int64_t rejected;  /* of those, curves beyond the threshold (dropped) */
} ffd_search_info;
/* Counts of the context's last ffd_knn call.  Errors: FFD_E_INVALID. */
int ffd_last_search(const ffd_ctx *ctx, ffd_search_info *info);

/* ------------------------------------------------------------ serving ---
 * Queries against a device-resident database of curves (the batched form
 * of Sec. 4 against one reference curve, turned around: one query against
 * every database curve).  Requests are submitted from the host at any time;
 * a worker thread admits them into launches as soon as a launch slot and
 * its arena region are free, so requests that arrive while others run on
 * the GPU join the next launch and their work overlaps on the device
 * (continuous batching).  Each result equals, bit for bit, what ffd_cross
 * gives for the same query and database, whatever else runs with it. */
typedef struct ffd_db ffd_db;
typedef struct ffd_server ffd_server;

/* A database of ndb float32 curves: DB[db_off[k]*dim .. db_off[k+1]*dim) is
 * curve k (device pointer, kept referenced until ffd_db_destroy; db_off is a
 * host array, copied).  The database must outlive every server made from
 * it and must not change while a server exists.
 * Errors: FFD_E_INVALID (NULL, ndb < 1, bad offsets or dim), FFD_E_UNSUPPORTED
 * (dim > FFD_MAX_DIM). */
int ffd_db_create(ffd_ctx *ctx, const float *DB, const int64_t *db_off, int64_t ndb, int32_t dim, ffd_db **out);
void ffd_db_destroy(ffd_db *db);

/* Device bytes of the arena a server needs: a reordered copy of the
 * database plus the regions of its launch slots, sized for max_slots
 * requests in flight and queries of up to max_query points.
 * Errors: FFD_E_INVALID (NULL, max_slots outside 1..4096, max_query outside
 * 1..2^20). */
int ffd_server_arena_size(ffd_db *db, int32_t max_slots, int64_t max_query, size_t *bytes);

/* Start a server on the database's context device.  `arena` is caller
 * device memory of arena_bytes >= ffd_server_arena_size(...); it stays in
 * use until ffd_server_destroy.  The server owns a worker thread, four HIP
 * streams and pinned host staging buffers.  The HIP runtime maps a
 * process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 by default,
 * round robin in creation order); where two of the server's streams share
 * a queue their launches run one after the other.  A serving process may
 * set the variable higher before the runtime starts (with 8 the saturation
 * on a 10,000-curve database measured 1,620-1,650 requests/s, against
 * 1,200-1,490 with 4, depending on the streams created before the server).
 * Errors: FFD_E_INVALID, FFD_E_NOMEM (arena too small), FFD_E_DEVICE. */
int ffd_server_create(ffd_db *db, void *arena, size_t arena_bytes, int32_t max_slots, int64_t max_query,
                      ffd_server **out);
/* Waits for every submitted request, then stops the worker. */
void ffd_server_destroy(ffd_server *s);

/* Submit one query: q is a HOST array of n*dim floats (copied before the
 * call returns); out is a HOST array of ndb floats that receives
 * delta(query, database curve k) in out[k] and must stay valid until the
 * request is collected by ffd_server_poll or ffd_server_wait.  Returns at
 * once with a ticket.  Thread-safe.
 * Errors: FFD_E_INVALID (NULL, n < 1, unknown metric), FFD_E_UNSUPPORTED
 * (n > max_query). */
int ffd_server_submit(ffd_server *s, const float *q, int64_t n, int32_t metric, float *out, uint64_t *ticket);
/* *done = 1 once the request has finished; the ticket is then collected
 * and the request's status returned (FFD_OK or FFD_E_DEVICE).  Thread-safe.
 * Errors: FFD_E_INVALID (unknown or collected ticket). */
int ffd_server_poll(ffd_server *s, uint64_t ticket, int32_t *done);
/* Block until the request has finished (timeout_us < 0: no limit), then
 * collect it.  Thread-safe.
 * Errors: FFD_E_TIMEOUT, FFD_E_INVALID (unknown ticket), FFD_E_DEVICE. */
int ffd_server_wait(ffd_server *s, uint64_t ticket, int64_t timeout_us);

/* Cancel a submitted request.  A request that is still waiting, or that is
 * between two of its launches (a long query swept in several), is dropped
 * at the worker's next scheduling pass: its launch slot and boundary-row
 * buffers are reclaimed, `out` is left untouched, and poll / wait then
 * report FFD_E_CANCELED and collect the ticket.  A request whose last
 * launch is already in flight completes normally.  Thread-safe.
 * Errors: FFD_E_INVALID (unknown or collected ticket). */
int ffd_server_cancel(ffd_server *s, uint64_t ticket);

/* Watchdog: every request submitted after this call must have its last
 * launch issued within timeout_us of its submission (0: no limit, the
 * default).  One that has not is dropped as ffd_server_cancel drops it and
 * reports FFD_E_EXPIRED.  Thread-safe.  Errors: FFD_E_INVALID (NULL,
 * timeout_us < 0). */
int ffd_server_set_deadline(ffd_server *s, int64_t timeout_us);

typedef struct ffd_server_stats {
  int64_t submitted, completed, failed;
  int64_t deferred;     /* submissions that found no free launch slot */
  int64_t queued;       /* waiting for a launch slot now */
  double p50_ms, p99_ms, mean_ms, max_ms;  /* submit-to-result latency */
  double qps;           /* completed requests per second, first submit to last result */
  double cells_per_s;   /* DP cells of completed requests per second, same span */
  int32_t requests_per_launch, waves;
  int64_t launches_by_rows[8];  /* launches run with r + 1 rows per lane (r = 0 ... 7) */
  int64_t canceled, expired;    /* requests dropped by ffd_server_cancel / the deadline */
} ffd_server_stats;

/* Statistics since creation or the last reset.  Thread-safe. */
int ffd_server_get_stats(ffd_server *s, ffd_server_stats *out);
int ffd_server_reset_stats(ffd_server *s);
const char *ffd_server_last_error(const ffd_server *s);

#ifdef __cplusplus
}
#endif

#endif /* FFD_H */

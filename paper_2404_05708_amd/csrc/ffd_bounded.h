// Arguments and launchers of the early-abandoning sweep (ffd_bounded.hip).
#ifndef FFD_BOUNDED_H
#define FFD_BOUNDED_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffd {

struct BoundedArgs {
  const float *X0, *X1;        // coordinates of the row curves and of the column curves
  const int64_t *off0, *off1;  // their offsets in points (device)
  const int32_t *order;        // work item k -> pair index (the output index); the top bit set:
                               // the pair's curves swap roles (decider: no fixed row or mapping)
  int32_t fixed_row;           // >= 0: row curve of every pair; -1: the pair index (or, with
                               // col_count > 0, pair / col_count)
  int64_t col_count;           // > 0: pair p is row curve p / col_count against column curve
                               // p % col_count; 0: column curve = pair index
  const float *row_eps2;       // non-null: the threshold of each row curve (replaces eps2)
  int32_t metric;              // 0: store sqrt(delta^2) rounded once; 1: delta^2
  int64_t npairs;              // work items
  float eps2;                  // drop a pair once every cell of a crossing set exceeds this (squared)
  float *out;                  // per pair: its value when delta^2 <= eps2, else +inf
  float *rows;                 // per wave: 3 * row_cap floats (two bottom rows, suffix minima)
  int64_t row_cap;             // > the longest column curve when some row curve has several bands
  uint32_t *counter;           // work counter, zero at launch
  int32_t dim;                 // coordinates per point (the launch's D)
};

// nwaves wavefronts (workgroups of 4) take pairs from the counter.  D is the
// curves' coordinates per point (a.dim); D > 4 runs with R = wide_rows(D) only.
hipError_t launch_bounded(int R, int D, const BoundedArgs &a, int nwaves, hipStream_t st);
// lb[c] = larger of the squared first-point and last-point distances between
// the query and curve c.
hipError_t launch_endpoint_bound(int D, const float *q, int64_t n, const float *X, const int64_t *off, int64_t count,
                                 float *lb, hipStream_t st);
// The same for nq queries (CSR offsets q_off, device) against every curve:
// lb[i * count + c].
hipError_t launch_endpoint_bound_batch(int D, const float *Q, const int64_t *q_off, int64_t nq, const float *X,
                                       const int64_t *off, int64_t count, float *lb, hipStream_t st);

}  // namespace ffd

#endif  // FFD_BOUNDED_H

// Launch arguments and shape constants of the pipelined single-pair kernel
// (ffd_pipe.h), shared by the kernel and the host planner.
#ifndef FFD_PIPE_ARGS_H
#define FFD_PIPE_ARGS_H

#include <stdint.h>

namespace ffd {

constexpr int kPipeWaves = 4;   // computing waves per workgroup, one per SIMD
constexpr int kPipeThreads = (kPipeWaves + 1) * 64;  // and a helper wave (loads and links)
constexpr int kPipeLag = 5;     // groups a wave runs behind the wave above it in the workgroup
constexpr int kPipeRing = 256;  // column ring and hand-off ring entries (power of two, multiple of 16)
constexpr int kPipeGroup = 16;  // steps per phase

struct PipeArgs {
  const void *X;        // row curve, n points (float32, or int32 for FP64-exact values)
  const void *Y;        // column curve, m points
  int64_t n, m;
  int32_t nb;           // bands of 64 R rows
  int32_t nwg;          // workgroups launched (kPipeWaves computing waves and a helper each)
  int32_t xcd_span;     // > 0: workgroups per XCD in the chain order (nwg is a multiple of 8)
  int32_t metric;       // float: 0 Euclidean (one root of the result), 1 squared
  void *links;          // link rows of link_stride values (value bits; all ones = not written yet)
  int64_t link_stride;  // a multiple of 64, at least m
  uint64_t *err;        // (epoch << 32) | bits: bit 1 = a link wait was abandoned
  uint64_t patience;    // ticks of the 100 MHz real-time counter a link wait may last
  uint32_t epoch;
  void *out;            // one result
};

}  // namespace ffd

#endif  // FFD_PIPE_ARGS_H

// The pipelined single-pair kernel (ffd_pipe.h): instantiations for R = 2
// and 4 rows per lane, D = 1 ... 4, float32 values and FP64-exact values of
// int32 coordinates, its launcher and the link initialisation.
#include "ffd_pipe.h"

namespace ffd {

namespace {

template <int R, int D, typename V>
hipError_t pipe_one(const PipeArgs &a, size_t lds, hipStream_t st) {
  const void *k = reinterpret_cast<const void *>(&pipe_kernel<R, D, V>);
  if (lds > 65536) {
    // more than 64 KiB of dynamic LDS per workgroup (the device allows 160 KiB)
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  PipeArgs copy = a;
  void *args[] = {&copy};
  return hipLaunchCooperativeKernel(k, dim3((unsigned)a.nwg), dim3(kPipeThreads), args, (unsigned)lds, st);
}

template <int R, int D, typename V>
hipError_t pipe_occ(size_t lds, int *blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, &pipe_kernel<R, D, V>, kPipeThreads, lds);
}

template <typename V>
hipError_t pipe_v(int R, int D, const PipeArgs &a, size_t lds, hipStream_t st) {
  switch (R * 8 + D) {
#define FFD_PIPE_CASE(r, d) \
  case r * 8 + d: return pipe_one<r, d, V>(a, lds, st);
    FFD_PIPE_CASE(2, 1) FFD_PIPE_CASE(2, 2) FFD_PIPE_CASE(2, 3) FFD_PIPE_CASE(2, 4)
    FFD_PIPE_CASE(4, 1) FFD_PIPE_CASE(4, 2) FFD_PIPE_CASE(4, 3) FFD_PIPE_CASE(4, 4)
#undef FFD_PIPE_CASE
  }
  return hipErrorInvalidValue;
}

template <typename V>
hipError_t pipe_occ_v(int R, int D, size_t lds, int *blocks) {
  switch (R * 8 + D) {
#define FFD_PIPE_CASE(r, d) \
  case r * 8 + d: return pipe_occ<r, d, V>(lds, blocks);
    FFD_PIPE_CASE(2, 1) FFD_PIPE_CASE(2, 2) FFD_PIPE_CASE(2, 3) FFD_PIPE_CASE(2, 4)
    FFD_PIPE_CASE(4, 1) FFD_PIPE_CASE(4, 2) FFD_PIPE_CASE(4, 3) FFD_PIPE_CASE(4, 4)
#undef FFD_PIPE_CASE
  }
  return hipErrorInvalidValue;
}

// Link rows start as all ones (the "not written" pattern) and the error
// word as 0; 32-bit words, a grid-stride loop.
__global__ void pipe_init_kernel(uint32_t *links, int64_t nwords, uint64_t *err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && err) *err = 0;
  for (; i < nwords; i += (int64_t)gridDim.x * blockDim.x) links[i] = 0xFFFFFFFFu;
}

}  // namespace

size_t pipe_lds(bool exact, int D) {
  switch (D) {
    case 1: return exact ? PipeLds<1, double>::kTotal : PipeLds<1, float>::kTotal;
    case 2: return exact ? PipeLds<2, double>::kTotal : PipeLds<2, float>::kTotal;
    case 3: return exact ? PipeLds<3, double>::kTotal : PipeLds<3, float>::kTotal;
    case 4: return exact ? PipeLds<4, double>::kTotal : PipeLds<4, float>::kTotal;
  }
  return 0;
}

hipError_t launch_pipe(bool exact, int R, int D, const PipeArgs &a, size_t lds, hipStream_t st) {
  return exact ? pipe_v<double>(R, D, a, lds, st) : pipe_v<float>(R, D, a, lds, st);
}

hipError_t occupancy_pipe(bool exact, int R, int D, size_t lds, int *blocks) {
  return exact ? pipe_occ_v<double>(R, D, lds, blocks) : pipe_occ_v<float>(R, D, lds, blocks);
}

hipError_t pipe_init(void *links, int64_t nwords32, uint64_t *err, hipStream_t st) {
  int64_t blocks = (nwords32 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(pipe_init_kernel, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<uint32_t *>(links),
                     nwords32, err);
  return hipGetLastError();
}

}  // namespace ffd

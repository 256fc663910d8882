// ffd_batch_noalloc: the launches of ffd_batch with their workspace in a
// file-scope device array instead of caller memory, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// Each GPU holds its own copy of `scratch` for as long as the library is
// loaded.  Host code never uses the array's name as an address (on the
// host it is only a stand-in for the symbol): ffd_create resolves the
// device address of the copy on its device once, with that device current,
// and every call uses that address.  All calls on one GPU share the array,
// so calls that overlap on one GPU (from several contexts, or from one
// context on streams the library does not know to order) race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ffd.h"
#include "ffd_internal.h"

namespace {

constexpr size_t kNoAllocBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void *g_addr[kMaxDevices];  // device address of `scratch` on each device (nullptr: not resolved)

}  // namespace

namespace ffdi {

size_t noalloc_bytes() { return kNoAllocBytes; }

// Resolve the device address of the array on `device` (once per device,
// with that device current).  Called by ffd_create.
int noalloc_setup(ffd_ctx *ctx, int device) {
  if (device < 0 || device >= kMaxDevices) return FFD_OK;  // the entry point then reports FFD_E_DEVICE
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_addr[device]) return FFD_OK;
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipGetDevice");
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  void *p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  hipError_t e2 = hipSetDevice(prev);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipGetSymbolAddress (no-allocation scratch)");
  if (e2 != hipSuccess) return hip_fail(ctx, e2, "hipSetDevice");
  g_addr[device] = p;
  return FFD_OK;
}

}  // namespace ffdi

extern "C" int ffd_batch_noalloc(ffd_ctx *ctx, const float *P, const int64_t *p_off, const float *Q,
                                 const int64_t *q_off, int64_t npairs, int32_t dim, int32_t metric, float *out,
                                 void *stream) {
  if (!ctx) return FFD_E_INVALID;
  void *ws = nullptr;
  if (ctx->device >= 0 && ctx->device < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_mu);
    ws = g_addr[ctx->device];
  }
  if (ctx->device >= 0 && !ws) return ffdi::fail(ctx, FFD_E_DEVICE, "no-allocation scratch not resolved on this device");
  return ffdi::batch_noalloc(ctx, P, p_off, Q, q_off, npairs, dim, metric, out, ws, kNoAllocBytes,
                             (hipStream_t)stream);
}

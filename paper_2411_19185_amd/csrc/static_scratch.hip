// hope_rk_step_static: the Runge-Kutta step of hope_rk_step with its
// workspace (two padded stage states and the panel-edge traces) in a static
// device array instead of a caller's buffer, for callers that cannot
// allocate device memory.  Declared in include/hope.h.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hope.h"
#include "grid_internal.hpp"

using namespace hope;

namespace {

constexpr size_t kStaticScratchBytes = HOPE_STATIC_SCRATCH_BYTES;   // per GPU
constexpr int kMaxDevices = 64;

// The workspace of hope_rk_step_static.  Each GPU the library runs on holds
// its own copy until the process ends.  In host code this name is only a
// stand-in for the symbol: the device address comes from
// hipGetSymbolAddress, once per device (scratch_ptr).
__device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// the device address of device dev's copy of scratch; dev must be current
int scratch_ptr(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (static scratch)");
    if (!p) return fail(HOPE_ERR_HIP, "hipGetSymbolAddress returned no address for the static scratch");
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return HOPE_OK;
}

}  // namespace

extern "C" int hope_rk_step_static(const hope_grid* G, double* q, double dt, int32_t scheme, void* stream) {
  if (!G || !q) return fail(HOPE_ERR_INVALID, "null argument");
  const size_t need = rk_workspace_bytes(G);
  if (need > kStaticScratchBytes)
    return fail(HOPE_ERR_INVALID, "this grid's Runge-Kutta workspace needs " + std::to_string(need) +
                                      " bytes, more than the " + std::to_string(kStaticScratchBytes) +
                                      " bytes of the static scratch; use hope_rk_step with a workspace");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(HOPE_ERR_INVALID, "device index beyond the static scratch table");
  if (stream) {
    int sdev = -1;
    e = hipStreamGetDevice(static_cast<hipStream_t>(stream), &sdev);
    if (e != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
    if (sdev != dev) return fail(HOPE_ERR_INVALID, "the stream is not on the current device");
  }
  double* ws = nullptr;
  if (int st = scratch_ptr(dev, &ws)) return st;
  // every word of the workspace a step reads is written earlier in the same
  // step (stage states: interior by the stage kernel, ghost rings by the
  // fill; traces by the trace kernel), so nothing needs clearing
  return rk_step_ws(G, q, dt, scheme, ws, kStaticScratchBytes, stream);
}

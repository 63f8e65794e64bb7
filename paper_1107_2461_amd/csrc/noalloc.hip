// helm_solve_noalloc: the solve with its workspace in a file-scope device array instead of a
// caller-provided buffer, for callers that cannot allocate (include/helm.h).
//
// `scratch` is one array per GPU, created when the code object is loaded on that device and
// held until the process ends.  In host code its name is only a stand-in for the symbol, so
// its device address is looked up once per device (hipGetSymbolAddress, with that device
// current) and that address is what the kernels receive.  Every call on one GPU uses the same
// array: calls that overlap on one GPU race.  No kernel of the solve reads a workspace word
// before writing it in the same call (the refinement norms are cleared by the residual kernel
// of each sweep), so nothing is cleared between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/helm.h"
#include "solve_impl.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // HELM_NOALLOC_MAX_WORKSPACE
static_assert(kScratchBytes == HELM_NOALLOC_MAX_WORKSPACE, "header and library disagree on the size");

__attribute__((used)) static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch` per device, resolved once

// The device address of `scratch` on the current device (looked up on the first call there).
hipError_t scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" helm_status helm_solve_noalloc(helm_plan* plan, const double* f, double* u, int nrhs,
                                          const double* sigma_per_rhs, void* stream, helm_info* info) {
  size_t need = 0;
  helm_status st = helm_workspace_size(plan, nrhs, &need);
  if (st != HELM_OK) return st;
  if (need > kScratchBytes) return HELM_EINVAL;
  // the plan's device is the one whose array is used (helm_solve switches to it as well)
  int cur = -1, dev = -1;
  if (hipGetDevice(&cur) != hipSuccess) return HELM_EDEVICE;
  if ((dev = helm::plan_device(plan)) < 0) return HELM_EINVAL;
  if (dev != cur && hipSetDevice(dev) != hipSuccess) return HELM_EDEVICE;
  void* ws = nullptr;
  const hipError_t e = scratch_ptr(&ws);
  if (dev != cur) (void)hipSetDevice(cur);
  if (e != hipSuccess) return HELM_EDEVICE;
  return helm::solve_impl(plan, f, u, nrhs, sigma_per_rhs, ws, stream, info, true);
}

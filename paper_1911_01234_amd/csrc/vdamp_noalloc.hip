// vdamp_solve for callers that cannot allocate: the workspace is a file-scope device
// array of fixed size, one copy per GPU, held until the process ends.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "vdamp.h"
#include "vdamp_host.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // VDAMP_NOALLOC_MAX_WORKSPACE
static_assert(kScratchBytes == VDAMP_NOALLOC_MAX_WORKSPACE, "header and library disagree");

// The workspace of every vdamp_solve_noalloc call on a GPU.  In host code this name is
// only a stand-in for the symbol: its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, void*> g_scratch_of_device;

// Device address of this GPU's copy of the array (looked up on the first call made with
// that device current).
vdamp_status scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_scratch_of_device.find(dev);
  if (it != g_scratch_of_device.end()) {
    *out = it->second;
    return VDAMP_OK;
  }
  void* ptr = nullptr;
  HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return vdamp::fail(VDAMP_ERR_HIP, "hipGetSymbolAddress returned a null address");
  g_scratch_of_device[dev] = ptr;
  *out = ptr;
  return VDAMP_OK;
}

}  // namespace

extern "C" vdamp_status vdamp_solve_noalloc(vdamp_plan_h plan, hipStream_t stream, const float* y,
                                            const uint8_t* mask, const float* p,
                                            const float* sigma2, int32_t iters, float* x_hat,
                                            float* trace) {
  vdamp::g_err.clear();
  if (!plan) return vdamp::fail(VDAMP_ERR_ARG, "plan is null");
  if (plan->ws_bytes > kScratchBytes)
    return vdamp::fail(VDAMP_ERR_WORKSPACE,
                       "the plan needs a workspace of " + std::to_string(plan->ws_bytes) +
                           " bytes, more than the " + std::to_string(kScratchBytes) +
                           " bytes vdamp_solve_noalloc holds; use vdamp_solve with a workspace");
  void* ws = nullptr;
  vdamp_status s = scratch_address(&ws);
  if (s != VDAMP_OK) return s;
  return vdamp::solve_eager(plan, stream, ws, kScratchBytes, y, mask, p, sigma2, iters, x_hat, trace);
}

// Small gfx950 kernels around the solve: the m/p weights with optional data checks,
// a flag reset and a zero fill (used instead of memset so that captured graphs hold
// kernels only).
#include "vdamp_internal.h"

namespace vdamp {

// wgt = m / p on Omega, 0 elsewhere (p == nullptr: p = 1, the FISTA weights m);
// bad[0] |= 1 for p outside (0, 1] on Omega or a non-finite y (only when check != 0).
__global__ void __launch_bounds__(kThreads) k_prep(const uint8_t* __restrict__ mask,
                                                   const float* __restrict__ p,
                                                   const float2* __restrict__ y,
                                                   float* __restrict__ wgt, long long n,
                                                   int check, int* bad) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  int flag = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const bool m = mask[i] != 0;
    float w = 0.f;
    if (m) {
      const float pv = p ? p[i] : 1.0f;
      if (check && !(pv > 0.f && pv <= 1.f)) flag = 1;
      w = (pv > 0.f) ? 1.0f / pv : 0.f;
    }
    if (check) {
      const float2 v = y[i];
      if (!isfinite(v.x) || !isfinite(v.y)) flag = 1;
    }
    wgt[i] = w;
  }
  if (check && flag) atomicOr(bad, 1);
}

__global__ void k_fill_int(int* p, int v) { *p = v; }

__global__ void __launch_bounds__(kThreads) k_zero(float2* __restrict__ x, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    x[i] = make_float2(0.f, 0.f);
}

hipError_t launch_prep(const uint8_t* mask, const float* p, const float2* y, float* wgt,
                       long long n, int check, int* bad, hipStream_t st) {
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  if (check) hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, st, bad, 0);
  hipLaunchKernelGGL(k_prep, dim3((unsigned)blocks), dim3(kThreads), 0, st, mask, p, y, wgt, n,
                     check, bad);
  return hipGetLastError();
}

hipError_t launch_zero(float2* x, long long n, hipStream_t st) {
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kThreads), 0, st, x, n);
  return hipGetLastError();
}

}  // namespace vdamp

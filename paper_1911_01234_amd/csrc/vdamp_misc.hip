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

// Plan-time tuning data (no part of any solve): iterate-like values for timing the
// passes' alternatives.  r, X, y get components with a standard normal distribution (so
// |r|^2 / tau is Exp(1) with tau = 1, the distribution of noise-only coefficients the
// threshold search sees most), wgt = 4 on about a quarter of k-space and 0 elsewhere.
// Normal values by Box-Muller from a 64-bit integer hash of (stream, index).
__device__ __forceinline__ unsigned long long tune_hash(unsigned long long z) {
  z ^= z >> 33;
  z *= 0xff51afd7ed558ccdull;
  z ^= z >> 33;
  z *= 0xc4ceb9fe1a85ec53ull;
  return z ^ (z >> 33);
}
__device__ __forceinline__ float2 tune_normal2(unsigned long long key) {
  const unsigned long long h = tune_hash(key);
  const float u1 = ((float)(h >> 40) + 0.5f) * (1.0f / 16777216.0f);
  const float u2 = (float)((h >> 16) & 0xFFFFFF) * (1.0f / 16777216.0f);
  const float rr = sqrtf(-2.0f * logf(u1));
  float sn, cs;
  sincosf(6.283185307f * u2, &sn, &cs);
  return make_float2(rr * cs, rr * sn);
}
__global__ void __launch_bounds__(kThreads) k_tune_fill(float2* __restrict__ r, float2* __restrict__ X,
                                                        float2* __restrict__ y, float* __restrict__ wgt,
                                                        long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const unsigned long long k = (unsigned long long)i * 4ull;
    r[i] = tune_normal2(k);
    X[i] = tune_normal2(k + 1);
    y[i] = tune_normal2(k + 2);
    wgt[i] = (tune_hash(k + 3) & 3ull) == 0 ? 4.0f : 0.0f;
  }
}
__global__ void k_fill_f32(float* __restrict__ x, long long n, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
hipError_t launch_tune_fill(float2* r, float2* X, float2* y, float* wgt, long long n, hipStream_t st) {
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)blocks), dim3(kThreads), 0, st, r, X, y, wgt, n);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* x, long long n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, v);
  return hipGetLastError();
}

// Per-slice input scale of the learned denoiser: s0^2 = (1/N) sum_j w_j |y_j|^2 with
// w = m / p (an unbiased estimate of the mean |x0|^2 plus noise, since E[m/p] = 1);
// s0 = 1 when that sum is not positive.  One block per slice, fixed-order reduction.
__global__ void __launch_bounds__(kThreads) k_scale(const SliceDev* __restrict__ slices,
                                                    const float2* __restrict__ y,
                                                    const float* __restrict__ wgt,
                                                    float* __restrict__ s0) {
  __shared__ double red[kThreads];
  const SliceDev S = slices[blockIdx.x];
  const long long n = (long long)S.ny * S.nx;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += kThreads) {
    const float2 v = y[S.off + i];
    acc += (double)wgt[S.off + i] * ((double)v.x * v.x + (double)v.y * v.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = red[0] / (double)n;
    s0[blockIdx.x] = (m > 0.0 && m < 1e300) ? (float)sqrt(m) : 1.0f;
  }
}

// Judge of the learned denoiser against soft thresholding, per slice and subband: from
// the strip partial sums D = sum |w_cnn - r|^2 and J = sum Re(conj(b) (J_g b)), the
// divergence estimate alpha = J / N_b (mean Wirtinger derivative) and the denoiser's
// SURE = D + (2 alpha - 1) N_b tau; the learned output is used (sel = 1, alpha replaced)
// when its SURE is below soft thresholding's minimum and alpha <= 1 - 1/N_b (the range
// soft thresholding's alpha has, which keeps the Onsager correction's division bounded).  always != 0:
// no SURE comparison, only the bound on alpha.
__global__ void k_judge(KArgs a, int nrowstrips, int always, int* __restrict__ sel,
                        float* __restrict__ jout) {
  const int sl = blockIdx.x, b = threadIdx.x;
  if (sl >= a.batch || b >= a.nbands) return;
  const SliceDev S = a.slices[sl];
  const int s = a.levels, nstr = S.ny >> s;
  double D = 0.0, J = 0.0;
  for (int i = 0; i < nstr; ++i) {
    D += (double)a.jpart[((long long)S.rowstrip0 + i) * kMaxBands + b];
    J += (double)a.jpart[((long long)nrowstrips + S.rowstrip0 + i) * kMaxBands + b];
  }
  const int l = (b == 0) ? s : s - (b - 1) / 3;
  const double Nb = (double)(S.ny >> l) * (double)(S.nx >> l);
  const double tau = (double)a.tau[sl * kMaxBands + b];
  const double al = J / Nb;
  const double sure = D + (2.0 * al - 1.0) * Nb * tau;
  const bool use = (always || sure < (double)a.smin[sl * kMaxBands + b]) && (al <= 1.0 - 1.0 / Nb);
  sel[sl * kMaxBands + b] = use ? 1 : 0;
  jout[sl * kMaxBands + b] = (float)sure;                             // the denoiser's SURE
  jout[(a.batch + sl) * kMaxBands + b] = (float)al;                   // its alpha
  jout[(2 * a.batch + sl) * kMaxBands + b] = a.smin[sl * kMaxBands + b];  // soft's SURE
  if (use) a.alpha[sl * kMaxBands + b] = (float)al;
}

// State import of a resumed solve: per slice and band the threshold theta, its key
// (the FP32 squared magnitude thresholding compares |r|^2 against; fl(theta * theta)
// when th2 is null) and alpha, from dense [B][nb] arrays into the plan's [B][kMaxBands]
// slots.  With check != 0, bad[0] |= 1 for a non-finite or negative theta or an alpha
// outside [0, 1) (Onsager correction divides by 1 - alpha).
__global__ void k_import_state(const float* __restrict__ th, const float* __restrict__ th2,
                               const float* __restrict__ al, int batch, int nb,
                               float* __restrict__ theta, float* __restrict__ thr2,
                               float* __restrict__ alpha, int check, int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch * nb) return;
  const int sl = i / nb, b = i - sl * nb;
  const float t = th[i], a = al[i];
  const float t2 = th2 ? th2[i] : __fmul_rn(t, t);
  if (check && !(t >= 0.f && isfinite(t) && t2 >= 0.f && isfinite(t2) && a >= 0.f && a < 1.f))
    atomicOr(bad, 1);
  theta[sl * kMaxBands + b] = t;
  thr2[sl * kMaxBands + b] = t2;
  alpha[sl * kMaxBands + b] = a;
}

hipError_t launch_import_state(const float* th, const float* th2, const float* al, int batch,
                               int nb, float* theta, float* thr2, float* alpha, int check, int* bad,
                               hipStream_t st) {
  const int n = batch * nb;
  hipLaunchKernelGGL(k_import_state, dim3((n + 255) / 256), dim3(256), 0, st, th, th2, al, batch, nb,
                     theta, thr2, alpha, check, bad);
  return hipGetLastError();
}

// FISTA objective of eq. 2 at w_k, per slice: 1/2 ||y - M F Psi^H w_k||^2 + lambda ||w_k||_1,
// from the column strips' residual sums (slot 0 of tau_part) and the row strips' sums of
// |w| (jpart), added in a fixed order in FP64.
__global__ void k_fista_obj(KArgs a, float* __restrict__ obj) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= a.batch) return;
  const SliceDev S = a.slices[sl];
  double res = 0.0, l1 = 0.0;
  for (int i = 0; i < S.ncs; ++i) res += (double)a.tau_part[(long long)(S.colstrip0 + i) * kMaxBands];
  for (int i = 0; i < (S.ny >> a.levels); ++i) l1 += (double)a.jpart[S.rowstrip0 + i];
  obj[(long long)a.iter * a.batch + sl] = (float)(0.5 * res + (double)a.lambda[sl] * l1);
}

hipError_t launch_fista_obj(const KArgs& a, float* obj, hipStream_t st) {
  hipLaunchKernelGGL(k_fista_obj, dim3((a.batch + 63) / 64), dim3(64), 0, st, a, obj);
  return hipGetLastError();
}

hipError_t launch_scale(const SliceDev* slices, int batch, const float2* y, const float* wgt,
                        float* s0, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(batch), dim3(kThreads), 0, st, slices, y, wgt, s0);
  return hipGetLastError();
}

hipError_t launch_judge(const KArgs& a, int nrowstrips, int always, int* sel, float* jout,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_judge, dim3(a.batch), dim3(64), 0, st, a, nrowstrips, always, sel, jout);
  return hipGetLastError();
}

}  // namespace vdamp

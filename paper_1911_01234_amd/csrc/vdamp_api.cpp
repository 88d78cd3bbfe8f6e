// Host side of libvdamp: argument checks, the plan (initialisation's tau weights, FFT twiddles
// and radix plans, work lists), workspace layout, the pass schedule of Algorithm 1 and
// of FISTA, optional hipGraph capture and per-pass event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "vdamp.h"
#include "vdamp_host.h"


using namespace vdamp;

namespace {


// Radix plan: radix-4 stages first, then 5, 3, 4 and 2 for the remaining factor.
bool radix_plan(int n, std::vector<int>& rad) {
  rad.clear();
  int m = n;
  while (m % 4 == 0 && m > 4) { rad.push_back(4); m /= 4; }
  for (int r : {5, 3, 4, 2})
    while (m % r == 0) { rad.push_back(r); m /= r; }
  return m == 1 && (int)rad.size() <= kMaxRadices;
}

// |unitary DFT of a 1D Haar basis function of length n|^2 at every k, by direct summation
// over its support: the scaling function of level m is 2^(-m/2) on 2^m samples; the
// wavelet of level l is +2^(-l/2) on 2^(l-1) samples then -2^(-l/2) on 2^(l-1) samples.
void haar_power(int n, int level, bool wavelet, std::vector<double>& out) {
  out.assign(n, 0.0);
  const int len = 1 << level;
  const double h = std::pow(2.0, -0.5 * level);
  for (int k = 0; k < n; ++k) {
    double re = 0.0, im = 0.0;
    for (int t = 0; t < len; ++t) {
      const double sgn = (wavelet && t >= len / 2) ? -1.0 : 1.0;
      const double ang = -2.0 * M_PI * double((long long)k * t % n) / double(n);
      re += sgn * h * std::cos(ang);
      im += sgn * h * std::sin(ang);
    }
    out[k] = (re * re + im * im) / double(n);
  }
}


// n-point DFTs of the level-l scaling function and wavelet of the periodic filter bank
// (lowpass h, highpass g[t] = (-1)^t h[L-1-t]): F_{A_l}(k) = prod_{i<l} H(2^i k) and
// F_{D_l}(k) = prod_{i<l-1} H(2^i k) G(2^(l-1) k), with H, G the n-point DFTs of h and g
// (a level-l basis function is the level-(l-1) scaling function filtered by the
// 2^(l-1)-upsampled h or g).  Out: 2 s rows of n values, A_1..A_s then D_1..D_s, in FP64.
void filter_responses(const std::vector<double>& h, int n, int s,
                      std::vector<std::complex<double>>& out) {
  const int L = (int)h.size();
  std::vector<std::complex<double>> H(n), G(n);
  for (int k = 0; k < n; ++k) {
    std::complex<double> hs = 0.0, gs = 0.0;
    for (int t = 0; t < L; ++t) {
      const double ang = -2.0 * M_PI * double((long long)k * t % n) / double(n);
      const std::complex<double> e(std::cos(ang), std::sin(ang));
      hs += h[t] * e;
      gs += ((t % 2) ? -1.0 : 1.0) * h[L - 1 - t] * e;
    }
    H[k] = hs;
    G[k] = gs;
  }
  out.assign((size_t)2 * s * n, 0.0);
  for (int k = 0; k < n; ++k) {
    std::complex<double> acc = 1.0;  // prod_{i<l-1} H(2^i k)
    for (int l = 1; l <= s; ++l) {
      const int k2 = (int)(((long long)k << (l - 1)) % n);
      out[(size_t)(l - 1) * n + k] = acc * H[k2];
      out[(size_t)(s + l - 1) * n + k] = acc * G[k2];
      acc *= H[k2];
    }
  }
}

// max |sum_t h[t] h[t + 2j] - delta_j| and |sum h - sqrt 2|: zero for an orthonormal
// two-channel lowpass filter.
double orthonormality_error(const double* h, int L) {
  double s = 0.0;
  for (int t = 0; t < L; ++t) s += h[t];
  double err = std::fabs(s - std::sqrt(2.0));
  for (int j = 0; 2 * j < L; ++j) {
    double acc = 0.0;
    for (int t = 0; t + 2 * j < L; ++t) acc += h[t] * h[t + 2 * j];
    err = std::max(err, std::fabs(acc - (j == 0 ? 1.0 : 0.0)));
  }
  return err;
}

// Group rows of one work item of the general-wavelet passes (the same rule as the kernels).
int ortho_rows_per_item(int ng) { return (ng % 8 == 0) ? 8 : (ng % 4 == 0) ? 4 : (ng % 2 == 0) ? 2 : 1; }

}  // namespace


namespace {

void free_plan(vdamp_plan_t* P) {
  if (!P) return;
  if (P->gexec) hipGraphExecDestroy(P->gexec);
  if (P->graph) hipGraphDestroy(P->graph);
  for (auto e : P->ev_pool) hipEventDestroy(e);
  for (int i = 0; i < vdamp_plan_t::kForks; ++i) {
    if (P->side[i]) hipStreamDestroy(P->side[i]);
    if (P->ev_join[i]) hipEventDestroy(P->ev_join[i]);
  }
  if (P->ev_fork) hipEventDestroy(P->ev_fork);
  hipFree(P->d_slices);
  hipFree(P->d_ffts);
  hipFree(P->d_tw);
  hipFree(P->d_tables);
  hipFree(P->d_work_rows);
  hipFree(P->d_work_cols);
  hipFree(P->d_work_sure);
  hipFree(P->d_tiles);
  hipFree(P->d_tile_off);
  hipFree(P->d_resp);
  hipFree(P->d_work_orows);
  hipFree(P->d_work_img);
  hipFree(P->d_work_bricks);
  hipFree(P->d_work_rows3);
  hipFree(P->d_work_ystrips);
  hipFree(P->d_work_zstrips);
  delete P;
}


}  // namespace

namespace vdamp {
thread_local std::string g_err;

vdamp_status fail(vdamp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

// Threshold-search size classes (launch shapes in launch_sure): 0 = 256 threads x 16
// keys, 1 = 512 x 8, 2 = 1024 x 16, 3 = 1024 x 32, kSureBigClass = the large-band search.
int sure_class_capacity(int cls) {
  return cls <= 1 ? kSureSmall : cls == 2 ? 4 * kSureSmall : cls == 3 ? kSureMaxKeys : kSureBigMaxKeys;
}
int sure_default_class(long long nb) {
  return nb > kSureMaxKeys ? kSureBigClass
         : nb > 4 * kSureSmall ? 3
         : nb > kSureSmall / 2 ? 2
                               : 0;
}

std::vector<int2> sure_work_list(vdamp_plan_t* P) {
  std::vector<std::pair<long long, int2>> wsc[kSureClasses];
  for (int b = 0; b < P->B; ++b)
    for (int band = 0; band < P->nbands; ++band) {
      const int l = band == 0 ? P->levels : P->levels - (band - 1) / (P->dim3 ? 7 : 3);
      const long long nb = (long long)(P->ny[b] >> l) * (P->nx[b] >> l) * (P->dim3 ? (P->nz[b] >> l) : 1) / P->grp;
      auto it = P->sure_cls_of_size.find(nb);
      int cls = it != P->sure_cls_of_size.end() ? it->second : sure_default_class(nb);
      if (cls < 0 || cls >= kSureClasses || nb > sure_class_capacity(cls)) cls = sure_default_class(nb);
      wsc[cls].push_back({nb, make_int2(b, band)});
    }
  std::vector<int2> out;
  for (int c = kSureClasses - 1; c >= 0; --c) {  // largest class first, as launched
    std::stable_sort(wsc[c].begin(), wsc[c].end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    P->nsure_cls[c] = (int)wsc[c].size();
    for (auto& e : wsc[c]) out.push_back(e.second);
  }
  return out;
}

Ws layout(const vdamp_plan_t* P, void* ws) {
  char* b = static_cast<char*>(ws);
  Ws w;
  w.wgt = reinterpret_cast<float*>(b + P->o_wgt);
  w.r = reinterpret_cast<float2*>(b + P->o_r);
  w.X = reinterpret_cast<float2*>(b + P->o_X);
  w.r2 = reinterpret_cast<float2*>(b + P->o_r2);
  w.theta = reinterpret_cast<float*>(b + P->o_theta);
  w.thr2 = reinterpret_cast<float*>(b + P->o_thr2);
  w.alpha = reinterpret_cast<float*>(b + P->o_alpha);
  w.tau = reinterpret_cast<float*>(b + P->o_tau);
  w.taup = reinterpret_cast<float*>(b + P->o_taup);
  w.rpart = reinterpret_cast<float*>(b + P->o_rpart);
  w.bad = reinterpret_cast<int*>(b + P->o_bad);
  w.big = P->o_big ? reinterpret_cast<float*>(b + P->o_big) : nullptr;
  w.Z = P->o_Z ? reinterpret_cast<float2*>(b + P->o_Z) : nullptr;
  return w;
}
}  // namespace vdamp

namespace {

vdamp_status check_common(vdamp_plan_h plan, void* ws, size_t wsb, const void* y,
                          const void* mask, int iters, const void* x_hat) {
  if (!plan) return fail(VDAMP_ERR_ARG, "plan is null");
  if (!ws) return fail(VDAMP_ERR_WORKSPACE, "workspace is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(VDAMP_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (wsb < plan->ws_bytes)
    return fail(VDAMP_ERR_WORKSPACE, "workspace has " + std::to_string(wsb) + " bytes, needs " +
                                         std::to_string(plan->ws_bytes));
  if (!y || !mask || !x_hat) return fail(VDAMP_ERR_ARG, "y, mask and x_hat must be non-null");
  if (iters < 0) return fail(VDAMP_ERR_ARG, "iters must be >= 0");
  return VDAMP_OK;
}

// State a resumed solve starts from (all null: a fresh start with r_tilde_0 = 0).
struct Resume {
  const float2* r = nullptr;
  const float *theta = nullptr, *theta2 = nullptr, *alpha = nullptr;
};

// Algorithm 1 on volumes: per iteration the 3D Haar synthesis of the Onsager-corrected
// r_tilde, the forward DFTs along x, y and z, the k-space step between the z DFTs, the
// inverse DFTs along y and x, the 3D Haar analysis with the back-projection's + r_tilde,
// and the threshold search of the denoising and alpha steps.  Timing classes: Haar
// synthesis = rows_synth, the DFT and k-space passes = cols, Haar analysis = rows_anal.
vdamp_status enqueue_vdamp3d(vdamp_plan_t* P, hipStream_t st, void* ws, const float2* y,
                             const uint8_t* mask, const float* p, const float* sigma2, int iters,
                             float2* x_hat, float* trace, bool timing, const Resume& rs,
                             float2* x_monitor) {
  const Ws w = layout(P, ws);
  Launcher L{P, st, timing};
  const int check = (P->flags & VDAMP_FLAG_CHECK_FINITE) ? 1 : 0;
  const bool resume = rs.r != nullptr;
  LAUNCH(L, VDAMP_PASS_PREP, launch_prep(mask, p, y, w.wgt, P->ntot, check, w.bad, st));
  if (resume) {
    HIP_TRY(hipMemcpyAsync(w.r, rs.r, sizeof(float2) * (size_t)P->ntot, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_import_state(rs.theta, rs.theta2, rs.alpha, P->B, P->nbands, w.theta, w.thr2,
                                w.alpha, check, w.bad, st));
  }
  KArgs a = base_args(P, w);
  a.y = y;
  a.sigma2 = sigma2;
  a.trace = trace;
  // the output step into out: F^H [ (1 - m) F Psi^H w + m y ] (w = eta(r; theta)), or F^H y
  auto output = [&](float2* out, bool has_w) -> vdamp_status {
    KArgs m = a;
    m.out = out;
    if (has_w) {
      m.mode = RS_WHAT;
      LAUNCH(L, VDAMP_PASS_ROWS_SYNTH, pass3_haar(P, m, true, st));
      LAUNCH(L, VDAMP_PASS_COLS, pass3_rows(P, m, false, false, st));
      m.mode = AX_Y_FWD;
      LAUNCH(L, VDAMP_PASS_COLS, pass3_axis(P, m, st));
    }
    m.mode = has_w ? CM_OUTPUT : CM_ZEROFILL;
    LAUNCH(L, VDAMP_PASS_COLS, pass3_axis(P, m, st));
    m.mode = AX_Y_INV;
    LAUNCH(L, VDAMP_PASS_COLS, pass3_axis(P, m, st));
    LAUNCH(L, VDAMP_PASS_ROWS_ANAL, pass3_rows(P, m, true, true, st));
    return VDAMP_OK;
  };
  for (int k = 0; k < iters; ++k) {
    a.iter = k;
    const bool has_prev = k > 0 || resume;
    if (has_prev) {
      a.mode = RS_RTILDE;
      LAUNCH(L, VDAMP_PASS_ROWS_SYNTH, pass3_haar(P, a, true, st));
      LAUNCH(L, VDAMP_PASS_COLS, pass3_rows(P, a, false, false, st));
      a.mode = AX_Y_FWD;
      LAUNCH(L, VDAMP_PASS_COLS, pass3_axis(P, a, st));
    }
    a.mode = has_prev ? CM_VDAMP : CM_VDAMP_FIRST;
    LAUNCH(L, VDAMP_PASS_COLS, pass3_axis(P, a, st));
    a.mode = AX_Y_INV;
    LAUNCH(L, VDAMP_PASS_COLS, pass3_axis(P, a, st));
    LAUNCH(L, VDAMP_PASS_COLS, pass3_rows(P, a, true, false, st));
    a.mode = has_prev ? RA_VDAMP : RA_VDAMP_FIRST;
    LAUNCH(L, VDAMP_PASS_ROWS_ANAL, pass3_haar(P, a, false, st));
    LAUNCH(L, VDAMP_PASS_SURE, launch_sure_all(P, a, w.big, st));
    if (x_monitor) {
      const vdamp_status s = output(x_monitor + (long long)k * P->ntot, true);
      if (s != VDAMP_OK) return s;
    }
  }
  return output(x_hat, iters > 0 || resume);
}

vdamp_status enqueue_vdamp(vdamp_plan_t* P, hipStream_t st, void* ws, const float2* y,
                           const uint8_t* mask, const float* p, const float* sigma2, int iters,
                           float2* x_hat, float* trace, bool timing, const Resume& rs,
                           float2* x_monitor) {
  if (P->dim3)
    return enqueue_vdamp3d(P, st, ws, y, mask, p, sigma2, iters, x_hat, trace, timing, rs, x_monitor);
  const Ws w = layout(P, ws);
  Launcher L{P, st, timing};
  const int check = (P->flags & VDAMP_FLAG_CHECK_FINITE) ? 1 : 0;
  const bool resume = rs.r != nullptr;
  LAUNCH(L, VDAMP_PASS_PREP, launch_prep(mask, p, y, w.wgt, P->ntot, check, w.bad, st));
  if (resume) {  // r_k, theta_k, alpha_k of an earlier iteration: the Onsager correction
                 // starts from them
    HIP_TRY(hipMemcpyAsync(w.r, rs.r, sizeof(float2) * (size_t)P->ntot, hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_import_state(rs.theta, rs.theta2, rs.alpha, P->B, P->nbands, w.theta, w.thr2,
                                w.alpha, check, w.bad, st));
  }
  KArgs a = base_args(P, w);
  a.y = y;
  a.sigma2 = sigma2;
  a.out = x_hat;
  a.trace = trace;
  for (int k = 0; k < iters; ++k) {
    a.iter = k;
    const bool has_prev = k > 0 || resume;  // r_tilde_k from the previous r, theta, alpha
    if (has_prev) {
      a.mode = P->grp > 1 ? RS_RTILDE_G : RS_RTILDE;
      LAUNCH(L, VDAMP_PASS_ROWS_SYNTH, pass_synth(P, a, st));
    }
    a.mode = has_prev ? CM_VDAMP : CM_VDAMP_FIRST;
    LAUNCH(L, VDAMP_PASS_COLS, pass_cols(P, a, st));
    a.mode = has_prev ? (P->grp > 1 ? RA_VDAMP_G : RA_VDAMP) : RA_VDAMP_FIRST;
    LAUNCH(L, VDAMP_PASS_ROWS_ANAL, pass_anal(P, a, st));
    LAUNCH(L, VDAMP_PASS_SURE, launch_sure_all(P, a, w.big, st));
    if (x_monitor) {  // the output step at this iteration (X is free between iterations)
      KArgs m = a;
      m.out = x_monitor + (long long)k * P->ntot;
      m.mode = P->grp > 1 ? RS_WHAT_G : RS_WHAT;
      LAUNCH(L, VDAMP_PASS_ROWS_SYNTH, pass_synth(P, m, st));
      m.mode = CM_OUTPUT;
      LAUNCH(L, VDAMP_PASS_COLS, pass_cols(P, m, st));
      m.mode = RA_IMAGE;
      LAUNCH(L, VDAMP_PASS_ROWS_ANAL, pass_anal(P, m, st));
    }
  }
  // the output step: x_hat = F^H [ (1 - m) F Psi^H w + m y ]
  const bool has_w = iters > 0 || resume;
  if (has_w) {
    a.mode = P->grp > 1 ? RS_WHAT_G : RS_WHAT;
    LAUNCH(L, VDAMP_PASS_ROWS_SYNTH, pass_synth(P, a, st));
  }
  a.mode = has_w ? CM_OUTPUT : CM_ZEROFILL;
  LAUNCH(L, VDAMP_PASS_COLS, pass_cols(P, a, st));
  a.mode = RA_IMAGE;
  LAUNCH(L, VDAMP_PASS_ROWS_ANAL, pass_anal(P, a, st));
  return VDAMP_OK;
}

vdamp_status enqueue_fista(vdamp_plan_t* P, hipStream_t st, void* ws, const float2* y,
                           const uint8_t* mask, const float* lambda, int iters, float2* x_hat,
                           float* objective, bool timing) {
  const Ws w = layout(P, ws);
  Launcher L{P, st, timing};
  // weights: m (p taken as 1)
  LAUNCH(L, VDAMP_PASS_PREP, launch_prep(mask, nullptr, y, w.wgt, P->ntot, 0, w.bad, st));
  KArgs a = base_args(P, w);
  a.y = y;
  a.lambda = lambda;
  a.out = x_hat;
  a.jpart = objective ? w.rpart : nullptr;  // per row strip ||w_k||_1 for the objective
  double t = 1.0;
  for (int k = 0; k < iters; ++k) {
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    a.beta = (float)((t - 1.0) / tn);
    a.iter = k;
    t = tn;
    if (k > 0) {
      a.mode = RS_PLAIN;
      LAUNCH(L, VDAMP_PASS_ROWS_SYNTH, launch_rows_synth_all(P, a, st));
    }
    a.mode = k ? CM_FISTA : CM_FISTA_FIRST;
    LAUNCH(L, VDAMP_PASS_COLS, launch_cols_all(P, a, st));
    a.mode = k ? RA_FISTA : RA_FISTA_FIRST;
    LAUNCH(L, VDAMP_PASS_ROWS_ANAL, launch_rows_anal_all(P, a, st));
    if (objective) {  // eq. 2 at w_k (in r2): forward transform of w_k, residual on Omega
      KArgs o = a;
      o.r = w.r2;
      o.mode = RS_PLAIN;
      LAUNCH(L, VDAMP_PASS_ROWS_SYNTH, launch_rows_synth_all(P, o, st));
      o.mode = CM_FISTA_OBJ;
      LAUNCH(L, VDAMP_PASS_COLS, launch_cols_all(P, o, st));
      LAUNCH(L, VDAMP_PASS_PREP, launch_fista_obj(o, objective, st));
    }
  }
  // x_hat = Psi^H w_K (w_K lives in r2); K = 0 gives zeros (a fill kernel, so that a
  // captured graph holds no memset node)
  if (iters == 0) {
    HIP_TRY(launch_zero(x_hat, P->ntot, st));
    return VDAMP_OK;
  }
  a.work = P->d_work_rows; a.nwork = P->nrows; a.mode = RS_PLAIN;
  a.r = w.r2;
  LAUNCH(L, VDAMP_PASS_ROWS_SYNTH, launch_rows_synth(a, P->ept, 0, P->lds_rows, st));
  return VDAMP_OK;
}

}  // namespace

namespace vdamp {
// vdamp_solve's schedule on a given workspace, always launched eagerly (no graph capture,
// no timing events): nothing here allocates.
vdamp_status solve_eager(vdamp_plan_t* plan, hipStream_t stream, void* workspace,
                         size_t workspace_bytes, const float* y, const uint8_t* mask,
                         const float* p, const float* sigma2, int32_t iters, float* x_hat,
                         float* trace) {
  vdamp_status s = check_common(plan, workspace, workspace_bytes, y, mask, iters, x_hat);
  if (s != VDAMP_OK) return s;
  if (!p || !sigma2) return fail(VDAMP_ERR_ARG, "p and sigma2 must be non-null");
  s = enqueue_vdamp(plan, stream, workspace, reinterpret_cast<const float2*>(y), mask, p, sigma2, iters,
                    reinterpret_cast<float2*>(x_hat), trace, false, Resume(), nullptr);
  if (s != VDAMP_OK) return s;
  if (plan->flags & VDAMP_FLAG_CHECK_FINITE) {
    int bad = 0;
    const Ws w = layout(plan, workspace);
    HIP_TRY(hipMemcpyAsync(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (bad) return fail(VDAMP_ERR_NONFINITE, "p outside (0, 1] on the mask or non-finite y");
  }
  plan->state_ws = workspace;
  plan->has_state = iters > 0;
  return VDAMP_OK;
}
}  // namespace vdamp

extern "C" {

const char* vdamp_status_string(vdamp_status s) {
  switch (s) {
    case VDAMP_OK: return "ok";
    case VDAMP_ERR_ARG: return "invalid argument";
    case VDAMP_ERR_SHAPE: return "invalid shape";
    case VDAMP_ERR_UNSUPPORTED: return "unsupported";
    case VDAMP_ERR_WORKSPACE: return "bad workspace";
    case VDAMP_ERR_HIP: return "HIP error";
    case VDAMP_ERR_NONFINITE: return "invalid data";
    case VDAMP_ERR_STATE: return "no state";
    case VDAMP_STATUS_MAX_ENUM: break;
  }
  return "unknown status";
}

const char* vdamp_last_error(void) { return g_err.c_str(); }

static vdamp_status make_plan(vdamp_plan_h* plan, int32_t batch, const int32_t* ny,
                              const int32_t* nx, int32_t levels, const double* filt, int32_t flen,
                              uint32_t flags, size_t* workspace_bytes) {
  g_err.clear();
  if (!plan || !ny || !nx || !workspace_bytes) return fail(VDAMP_ERR_ARG, "null pointer argument");
  *plan = nullptr;
  if (batch < 1) return fail(VDAMP_ERR_ARG, "batch must be >= 1");
  if (levels < 1 || levels > 4) return fail(VDAMP_ERR_UNSUPPORTED, "levels must be in 1..4");
  const bool ortho = filt != nullptr;
  if (ortho) {
    if (flen < 2 || flen > kMaxFilter || flen % 2)
      return fail(VDAMP_ERR_ARG, "filter length must be even, in 2.." + std::to_string(kMaxFilter));
    for (int t = 0; t < flen; ++t)
      if (!std::isfinite(filt[t])) return fail(VDAMP_ERR_ARG, "filter taps must be finite");
    const double oe = orthonormality_error(filt, flen);
    if (!(oe <= 1e-9))
      return fail(VDAMP_ERR_ARG, "filter is not an orthonormal lowpass filter (error " + std::to_string(oe) + ")");
    if (flags & VDAMP_FLAG_AUTOTUNE)
      return fail(VDAMP_ERR_UNSUPPORTED, "VDAMP_FLAG_AUTOTUNE tunes the Haar passes only");
  }
  const uint32_t known = VDAMP_FLAG_DETERMINISTIC | VDAMP_FLAG_USE_GRAPH | VDAMP_FLAG_CHECK_FINITE |
                         VDAMP_FLAG_TIMING | VDAMP_FLAG_AUTOTUNE | VDAMP_FLAG_SURE_CONTINUOUS |
                         VDAMP_FLAG_GROUP_PAIRS;
  if (flags & ~known) return fail(VDAMP_ERR_ARG, "unknown flag bits");
  if (ortho && (flags & VDAMP_FLAG_GROUP_PAIRS))
    return fail(VDAMP_ERR_UNSUPPORTED, "VDAMP_FLAG_GROUP_PAIRS runs on Haar plans only");
  const int H = 1 << levels;
  std::vector<int> rad;
  for (int b = 0; b < batch; ++b) {
    for (int n : {ny[b], nx[b]}) {
      if (n < H || n % H || n > kMaxN)
        return fail(VDAMP_ERR_SHAPE, "slice " + std::to_string(b) + ": size " + std::to_string(n) +
                                         " must be a multiple of 2^levels in [2^levels, 512]");
      if (!radix_plan(n, rad))
        return fail(VDAMP_ERR_UNSUPPORTED, "size " + std::to_string(n) + " is not 2^a 3^b 5^c");
    }
    if (nx[b] % kColW)
      return fail(VDAMP_ERR_UNSUPPORTED, "nx must be a multiple of 16 (column strip width)");
    if ((nx[b] >> levels) % 2)
      return fail(VDAMP_ERR_UNSUPPORTED,
                  "nx / 2^levels must be even (both coefficients of an 8-byte pair lie in one subband)");
    if (H * nx[b] > kMaxElems || ny[b] * kColW > kMaxElems)
      return fail(VDAMP_ERR_UNSUPPORTED, "strip does not fit the LDS tile");
    const long long finest = (long long)(ny[b] >> 1) * (nx[b] >> 1);
    if (finest > kSureBigMaxKeys)
      return fail(VDAMP_ERR_UNSUPPORTED, "finest subband larger than the threshold search (" +
                                             std::to_string(kSureBigMaxKeys) + " coefficients)");
  }

  vdamp_plan_t* P = new vdamp_plan_t();
  P->B = batch;
  P->levels = levels;
  P->nbands = 1 + 3 * levels;
  P->flags = flags;
  P->ny.assign(ny, ny + batch);
  P->nx.assign(nx, nx + batch);
  P->off.resize(batch);
  P->ortho = ortho;
  if (ortho) P->filt.assign(filt, filt + flen);
  P->grp = (flags & VDAMP_FLAG_GROUP_PAIRS) ? 2 : 1;

  // FFT plans and twiddles, one per distinct length
  std::map<int, int> fft_index;
  std::vector<FftPlanDev> ffts;
  std::vector<float2> tw;
  auto get_fft = [&](int n) {
    auto it = fft_index.find(n);
    if (it != fft_index.end()) return it->second;
    FftPlanDev f;
    std::memset(&f, 0, sizeof(f));
    std::vector<int> rr;
    radix_plan(n, rr);
    f.n = n;
    f.nst = (int)rr.size();
    for (size_t i = 0; i < rr.size(); ++i) f.rad[i] = rr[i];
    f.tw_off = (int)tw.size();
    for (int k = 0; k < n; ++k) {
      const double ang = -2.0 * M_PI * double(k) / double(n);
      tw.push_back(make_float2((float)std::cos(ang), (float)std::sin(ang)));
    }
    ffts.push_back(f);
    fft_index[n] = (int)ffts.size() - 1;
    return (int)ffts.size() - 1;
  };
  // tau-weight tables (initialisation), one set per distinct length: L_1..L_s then H_1..H_s
  std::map<int, int> tab_index;
  std::vector<float> tables;
  auto get_tab = [&](int n) {
    auto it = tab_index.find(n);
    if (it != tab_index.end()) return it->second;
    const int o = (int)tables.size();
    std::vector<double> pw;
    if (ortho) {  // |F_{A_l}|^2 / n, then |F_{D_l}|^2 / n
      std::vector<std::complex<double>> F;
      filter_responses(P->filt, n, levels, F);
      for (size_t i = 0; i < F.size(); ++i) tables.push_back((float)(std::norm(F[i]) / n));
    } else {
      for (int wv = 0; wv < 2; ++wv)
        for (int l = 1; l <= levels; ++l) {
          haar_power(n, l, wv == 1, pw);
          for (int k = 0; k < n; ++k) tables.push_back((float)pw[k]);
        }
    }
    // then (cos^2, sin^2)(pi k / n) per k: the factors the four-step column pass builds
    // the same products from (D_{2^m}(k) = 2^m prod_{j<m} cos(pi k 2^j / n))
    for (int k = 0; k < n; ++k) {
      const double t = M_PI * (double)k / (double)n;
      tables.push_back((float)(std::cos(t) * std::cos(t)));
      tables.push_back((float)(std::sin(t) * std::sin(t)));
    }
    tab_index[n] = o;
    return o;
  };

  // complex filter responses (general wavelets), one set per distinct length
  std::map<int, int> resp_index;
  std::vector<float2> resp;
  auto get_resp = [&](int n) {
    auto it = resp_index.find(n);
    if (it != resp_index.end()) return it->second;
    const int o = (int)resp.size();
    std::vector<std::complex<double>> F;
    filter_responses(P->filt, n, levels, F);
    for (auto& f : F) resp.push_back(make_float2((float)f.real(), (float)f.imag()));
    resp_index[n] = o;
    return o;
  };

  std::vector<SliceDev> sl(batch);
  long long off = 0, zoff = 0;
  int colstrip = 0, rowstrip = 0;
  for (int b = 0; b < batch; ++b) {
    SliceDev& S = sl[b];
    std::memset(&S, 0, sizeof(S));
    S.off = off;
    S.ny = ny[b];
    S.nx = nx[b];
    S.fft_y = get_fft(ny[b]);
    S.fft_x = get_fft(nx[b]);
    S.ytab_off = get_tab(ny[b]);
    S.xtab_off = get_tab(nx[b]);
    S.colstrip0 = colstrip;
    S.rowstrip0 = rowstrip;
    S.nd = 1;
    S.ncs = nx[b] / kColW;
    if (ortho) {
      for (int l = 0; l <= levels; ++l) {
        S.fft_yl[l] = get_fft(ny[b] >> l);
        S.fft_xl[l] = get_fft(nx[b] >> l);
      }
      S.zoff = zoff;
      S.zrows = 0;
      for (int l = 1; l <= levels; ++l) S.zrows += 2 * (ny[b] >> l);
      zoff += (long long)S.zrows * nx[b];
      S.yresp_off = get_resp(ny[b]);
      S.xresp_off = get_resp(nx[b]);
    }
    P->off[b] = off;
    off += (long long)ny[b] * nx[b];
    colstrip += nx[b] / kColW;
    rowstrip += ny[b] / H;
  }
  P->ntot = off;
  P->ncolstrips = colstrip;
  P->nrowstrips = rowstrip;

  // 16x16 pixel tiles of the learned denoiser, slice-major (only when every size allows)
  std::vector<int2> tiles;
  P->tiles_ok = true;
  for (int b = 0; b < batch; ++b) P->tiles_ok = P->tiles_ok && ny[b] % 16 == 0 && nx[b] % 16 == 0;
  P->tile_off.assign(1, 0);
  if (P->tiles_ok)
    for (int b = 0; b < batch; ++b) {
      const int nt = (ny[b] / 16) * (nx[b] / 16);
      for (int t = 0; t < nt; ++t) tiles.push_back(make_int2(b, t));
      P->tile_off.push_back((int)tiles.size());
    }
  P->ntiles = (int)tiles.size();

  // work lists, heaviest items first
  std::vector<std::pair<long long, int2>> wr, wc;
  int maxnx = 0, maxny = 0;
  for (int b = 0; b < batch; ++b) {
    maxnx = std::max(maxnx, nx[b]);
    maxny = std::max(maxny, ny[b]);
    for (int i = 0; i < ny[b] / H; ++i) wr.push_back({(long long)nx[b], make_int2(b, i)});
    for (int i = 0; i < nx[b] / kColW; ++i) wc.push_back({(long long)ny[b], make_int2(b, i)});
  }
  auto sort_items = [](std::vector<std::pair<long long, int2>>& v) {
    std::stable_sort(v.begin(), v.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    std::vector<int2> out;
    for (auto& e : v) out.push_back(e.second);
    return out;
  };
  std::vector<int2> vr = sort_items(wr), vc = sort_items(wc), vs = sure_work_list(P);
  P->nrows = (int)vr.size();
  P->ncols = (int)vc.size();
  for (int i = 0; i < P->nrows;) {
    const int n = nx[vr[i].x];
    int j = i;
    while (j < P->nrows && nx[vr[j].x] == n) ++j;
    P->row_groups.push_back({i, j - i, cols4_supported(n) ? n / 16 : 0, n});
    i = j;
  }
  for (int i = 0; i < P->ncols;) {
    const int n = ny[vc[i].x];
    int j = i;
    while (j < P->ncols && ny[vc[j].x] == n) ++j;
    P->col_groups.push_back({i, j - i, cols4_supported(n) ? n / 16 : 0, n});
    i = j;
  }
  // general wavelets: group-row items (slice, first group row) and image-row items
  // (slice, first image row), heaviest (widest) first
  std::vector<int2> vor, vimg;
  if (ortho) {
    std::vector<std::pair<long long, int2>> wo, wi;
    for (int b = 0; b < batch; ++b) {
      int goff = 0;
      for (int l = 1; l <= levels; ++l)
        for (int kind = 0; kind < 2; ++kind) {
          const int ng = ny[b] >> l, rpi = ortho_rows_per_item(ng);
          for (int i = 0; i < ng; i += rpi) wo.push_back({(long long)nx[b] * rpi, make_int2(b, goff + i)});
          goff += ng;
        }
      const int rpi = ortho_rows_per_item(ny[b]);
      for (int i = 0; i < ny[b]; i += rpi) wi.push_back({(long long)nx[b] * rpi, make_int2(b, i)});
    }
    vor = sort_items(wo);
    vimg = sort_items(wi);
    P->n_orows = (int)vor.size();
    P->n_img = (int)vimg.size();
    P->lds_osynth = sizeof(float2) * (size_t)10 * maxnx;  // 8 rows + 2 responses
    P->lds_oanal = sizeof(float2) * (size_t)18 * maxnx;   // 8 group rows + 8 band rows + 2 responses
    P->lds_ocols = ocols_lds_bytes(maxny, levels);
    P->ocols_ept = maxny * kColW <= 16 * kThreads ? 16 : 32;
    P->ocols_ny = std::all_of(ny, ny + batch, [&](int v) { return v == ny[0]; }) ? ny[0] : 0;
  }
  P->lds_rows = sizeof(float2) * (size_t)H * maxnx;
  P->lds_cols = sizeof(float2) * (size_t)maxny * kColW;
  P->ept = (H * maxnx <= 16 * kThreads && maxny * kColW <= 16 * kThreads) ? 16 : 32;

  // workspace layout
  size_t o = 0;
  const size_t N = (size_t)P->ntot;
  P->o_wgt = o; o = align256(o + 4 * N);
  P->o_r = o; o = align256(o + 8 * N);
  P->o_X = o; o = align256(o + 8 * N);
  P->o_r2 = o; o = align256(o + 8 * N);
  P->o_theta = o; o = align256(o + 4 * (size_t)batch * kMaxBands);
  P->o_thr2 = o; o = align256(o + 4 * (size_t)batch * kMaxBands);
  P->o_alpha = o; o = align256(o + 4 * (size_t)batch * kMaxBands);
  P->o_tau = o; o = align256(o + 4 * (size_t)batch * kMaxBands);
  P->o_taup = o; o = align256(o + 4 * (size_t)colstrip * kMaxBands);
  P->o_rpart = o; o = align256(o + 4 * (size_t)rowstrip);
  P->o_bad = o; o = align256(o + 4);
  if (ortho) {
    P->o_Z = o;
    o = align256(o + sizeof(float2) * (size_t)zoff);
  }
  if (P->nsure_cls[kSureBigClass]) {
    P->o_big = o;
    o = align256(o + 4 * (size_t)P->nsure_cls[kSureBigClass] * kSureBigStride);
  }
  P->ws_bytes = o;

  auto upload = [&](auto*& dst, const auto& vec) -> hipError_t {
    using T = typename std::decay_t<decltype(vec)>::value_type;
    hipError_t e = hipMalloc((void**)&dst, sizeof(T) * std::max<size_t>(vec.size(), 1));
    if (e != hipSuccess) return e;
    return hipMemcpy(dst, vec.data(), sizeof(T) * vec.size(), hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(P->d_slices, sl);
  if (e == hipSuccess) e = upload(P->d_ffts, ffts);
  if (e == hipSuccess) e = upload(P->d_tw, tw);
  if (e == hipSuccess) e = upload(P->d_tables, tables);
  if (e == hipSuccess) e = upload(P->d_work_rows, vr);
  if (e == hipSuccess) e = upload(P->d_work_cols, vc);
  if (e == hipSuccess) e = upload(P->d_work_sure, vs);
  if (e == hipSuccess) e = upload(P->d_tiles, tiles);
  if (e == hipSuccess) e = upload(P->d_tile_off, P->tile_off);
  if (e == hipSuccess) e = set_lds_limits_passes(sizeof(float2) * kMaxElems, sizeof(float2) * kMaxElems);
  if (e == hipSuccess && ortho) {
    e = upload(P->d_resp, resp);
    if (e == hipSuccess) e = upload(P->d_work_orows, vor);
    if (e == hipSuccess) e = upload(P->d_work_img, vimg);
    if (e == hipSuccess) e = set_lds_limits_ortho(P->lds_osynth, P->lds_ocols, P->lds_oanal);
  }
  if (e == hipSuccess && (P->row_groups.size() > 1 || P->col_groups.size() > 1)) {
    for (int i = 0; i < vdamp_plan_t::kForks && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&P->side[i], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    free_plan(P);
    return fail(VDAMP_ERR_HIP, std::string("plan upload: ") + hipGetErrorString(e));
  }
  if (flags & VDAMP_FLAG_AUTOTUNE) {
    e = autotune(P);
    if (e != hipSuccess) {
      free_plan(P);
      return fail(VDAMP_ERR_HIP, std::string("plan autotune: ") + hipGetErrorString(e));
    }
  }
  *plan = P;
  *workspace_bytes = P->ws_bytes;
  return VDAMP_OK;
}

vdamp_status vdamp_plan(vdamp_plan_h* plan, int32_t batch, const int32_t* ny, const int32_t* nx,
                        int32_t levels, int32_t wavelet, uint32_t flags, size_t* workspace_bytes) {
  if (wavelet != VDAMP_WAVELET_HAAR) {
    g_err.clear();
    if (plan) *plan = nullptr;
    return fail(VDAMP_ERR_UNSUPPORTED, "wavelet must be VDAMP_WAVELET_HAAR (other wavelets: vdamp_plan_ortho)");
  }
  return make_plan(plan, batch, ny, nx, levels, nullptr, 0, flags, workspace_bytes);
}

static vdamp_status make_plan3d(vdamp_plan_h* plan, int32_t batch, const int32_t* nz, const int32_t* ny,
                                const int32_t* nx, int32_t levels, uint32_t flags, size_t* workspace_bytes) {
  g_err.clear();
  if (!plan || !nz || !ny || !nx || !workspace_bytes) return fail(VDAMP_ERR_ARG, "null pointer argument");
  *plan = nullptr;
  if (batch < 1) return fail(VDAMP_ERR_ARG, "batch must be >= 1");
  if (levels < 1 || levels > 4) return fail(VDAMP_ERR_UNSUPPORTED, "levels must be in 1..4");
  const uint32_t known = VDAMP_FLAG_DETERMINISTIC | VDAMP_FLAG_USE_GRAPH | VDAMP_FLAG_CHECK_FINITE |
                         VDAMP_FLAG_TIMING | VDAMP_FLAG_AUTOTUNE | VDAMP_FLAG_SURE_CONTINUOUS |
                         VDAMP_FLAG_GROUP_PAIRS;
  if (flags & ~known) return fail(VDAMP_ERR_ARG, "unknown flag bits");
  if (flags & VDAMP_FLAG_AUTOTUNE) return fail(VDAMP_ERR_UNSUPPORTED, "VDAMP_FLAG_AUTOTUNE tunes 2D plans only");
  if (flags & VDAMP_FLAG_GROUP_PAIRS) return fail(VDAMP_ERR_UNSUPPORTED, "VDAMP_FLAG_GROUP_PAIRS runs on 2D plans only");
  const int C = 1 << levels;
  std::vector<int> rad;
  for (int b = 0; b < batch; ++b) {
    for (int n : {nz[b], ny[b], nx[b]}) {
      if (n < C || n % C || n > kMaxN)
        return fail(VDAMP_ERR_SHAPE, "volume " + std::to_string(b) + ": size " + std::to_string(n) +
                                         " must be a multiple of 2^levels in [2^levels, 512]");
      if (!radix_plan(n, rad))
        return fail(VDAMP_ERR_UNSUPPORTED, "size " + std::to_string(n) + " is not 2^a 3^b 5^c");
    }
    if (nx[b] % kColW) return fail(VDAMP_ERR_UNSUPPORTED, "nx must be a multiple of 16 (strip width)");
    const long long finest = (long long)(nz[b] >> 1) * (ny[b] >> 1) * (nx[b] >> 1);
    if (finest > kSureBigMaxKeys)
      return fail(VDAMP_ERR_UNSUPPORTED, "finest subband larger than the threshold search (" +
                                             std::to_string(kSureBigMaxKeys) + " coefficients)");
  }
  vdamp_plan_t* P = new vdamp_plan_t();
  P->dim3 = true;
  P->B = batch;
  P->levels = levels;
  P->nbands = 1 + 7 * levels;
  P->flags = flags;
  P->nz.assign(nz, nz + batch);
  P->ny.assign(ny, ny + batch);
  P->nx.assign(nx, nx + batch);
  P->off.resize(batch);
  std::map<int, int> fft_index, tab_index;
  std::vector<FftPlanDev> ffts;
  std::vector<float2> tw;
  std::vector<float> tables;
  auto get_fft = [&](int n) {
    auto it = fft_index.find(n);
    if (it != fft_index.end()) return it->second;
    FftPlanDev f;
    std::memset(&f, 0, sizeof(f));
    std::vector<int> rr;
    radix_plan(n, rr);
    f.n = n;
    f.nst = (int)rr.size();
    for (size_t i = 0; i < rr.size(); ++i) f.rad[i] = rr[i];
    f.tw_off = (int)tw.size();
    for (int k = 0; k < n; ++k) {
      const double ang = -2.0 * M_PI * double(k) / double(n);
      tw.push_back(make_float2((float)std::cos(ang), (float)std::sin(ang)));
    }
    ffts.push_back(f);
    return fft_index[n] = (int)ffts.size() - 1;
  };
  auto get_tab = [&](int n) {  // the initialisation's 1D factors: L_1..L_s then H_1..H_s
    auto it = tab_index.find(n);
    if (it != tab_index.end()) return it->second;
    const int o = (int)tables.size();
    std::vector<double> pw;
    for (int wv = 0; wv < 2; ++wv)
      for (int l = 1; l <= levels; ++l) {
        haar_power(n, l, wv == 1, pw);
        for (int k = 0; k < n; ++k) tables.push_back((float)pw[k]);
      }
    return tab_index[n] = o;
  };
  std::vector<SliceDev> sl(batch);
  std::vector<std::pair<long long, int2>> wb, wr, wy, wz;
  long long off = 0;
  int colstrip = 0, maxn = 0, maxnd = 0, maxnx = 0;
  size_t haar_elems = 0;
  for (int b = 0; b < batch; ++b) {
    SliceDev& S = sl[b];
    std::memset(&S, 0, sizeof(S));
    S.off = off;
    S.nd = nz[b];
    S.ny = ny[b];
    S.nx = nx[b];
    S.fft_x = get_fft(nx[b]);
    S.fft_y = get_fft(ny[b]);
    S.fft_z = get_fft(nz[b]);
    S.xtab_off = get_tab(nx[b]);
    S.ytab_off = get_tab(ny[b]);
    S.ztab_off = get_tab(nz[b]);
    S.colstrip0 = colstrip;
    S.ncs = ny[b] * (nx[b] / kColW);
    // bricks of m whole 2^s cubes along x: the largest m dividing nx / 2^s with
    // m 2^(3s) <= 4096 complex (32 KB of LDS)
    int m = 1;
    for (int q = 1; q <= nx[b] / C; ++q)
      if ((nx[b] / C) % q == 0 && (long long)q * C * C * C <= 4096) m = q;
    S.bw3 = m * C;
    haar_elems = std::max(haar_elems, (size_t)C * C * S.bw3);
    const long long cost = (long long)nz[b] * ny[b] * nx[b];
    const int nbrick = (nz[b] / C) * (ny[b] / C) * (nx[b] / S.bw3);
    for (int i = 0; i < nbrick; ++i) wb.push_back({cost, make_int2(b, i)});
    const int rows = nz[b] * ny[b];
    const int rpi = (rows % 8 == 0) ? 8 : (rows % 4 == 0) ? 4 : (rows % 2 == 0) ? 2 : 1;
    for (int i = 0; i < rows; i += rpi) wr.push_back({cost, make_int2(b, i)});
    for (int i = 0; i < nz[b] * (nx[b] / kColW); ++i) wy.push_back({cost, make_int2(b, i)});
    for (int i = 0; i < S.ncs; ++i) wz.push_back({cost, make_int2(b, i)});
    P->off[b] = off;
    off += cost;
    colstrip += S.ncs;
    maxn = std::max(maxn, std::max(ny[b], nz[b]));
    maxnd = std::max(maxnd, nz[b]);
    maxnx = std::max(maxnx, nx[b]);
  }
  P->ntot = off;
  P->ncolstrips = colstrip;
  auto sort_items = [](std::vector<std::pair<long long, int2>>& v) {
    std::stable_sort(v.begin(), v.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    std::vector<int2> out;
    for (auto& e : v) out.push_back(e.second);
    return out;
  };
  std::vector<int2> vb = sort_items(wb), vr = sort_items(wr), vy = sort_items(wy), vz = sort_items(wz);
  std::vector<int2> vs = sure_work_list(P);
  P->n_bricks = (int)vb.size();
  P->n_rows3 = (int)vr.size();
  P->n_ystrips = (int)vy.size();
  P->n_zstrips = (int)vz.size();
  P->lds_k3haar = sizeof(float2) * haar_elems;
  P->lds_k3rows = sizeof(float2) * (size_t)8 * maxnx;
  P->lds_k3axis = k3_axis_lds_bytes(maxn, maxnd, levels);
  P->k3_ept = maxn * kColW <= 16 * kThreads ? 16 : 32;
  // workspace layout
  size_t o = 0;
  const size_t N = (size_t)P->ntot;
  P->o_wgt = o; o = align256(o + 4 * N);
  P->o_r = o; o = align256(o + 8 * N);
  P->o_X = o; o = align256(o + 8 * N);
  P->o_r2 = P->o_X;  // (no FISTA or learned denoiser on volumes)
  P->o_theta = o; o = align256(o + 4 * (size_t)batch * kMaxBands);
  P->o_thr2 = o; o = align256(o + 4 * (size_t)batch * kMaxBands);
  P->o_alpha = o; o = align256(o + 4 * (size_t)batch * kMaxBands);
  P->o_tau = o; o = align256(o + 4 * (size_t)batch * kMaxBands);
  P->o_taup = o; o = align256(o + 4 * (size_t)colstrip * kMaxBands);
  P->o_rpart = o;
  P->o_bad = o; o = align256(o + 4);
  if (P->nsure_cls[kSureBigClass]) {
    P->o_big = o;
    o = align256(o + 4 * (size_t)P->nsure_cls[kSureBigClass] * kSureBigStride);
  }
  P->ws_bytes = o;
  auto upload = [&](auto*& dst, const auto& vec) -> hipError_t {
    using T = typename std::decay_t<decltype(vec)>::value_type;
    hipError_t e = hipMalloc((void**)&dst, sizeof(T) * std::max<size_t>(vec.size(), 1));
    if (e != hipSuccess) return e;
    return hipMemcpy(dst, vec.data(), sizeof(T) * vec.size(), hipMemcpyHostToDevice);
  };
  hipError_t e = upload(P->d_slices, sl);
  if (e == hipSuccess) e = upload(P->d_ffts, ffts);
  if (e == hipSuccess) e = upload(P->d_tw, tw);
  if (e == hipSuccess) e = upload(P->d_tables, tables);
  if (e == hipSuccess) e = upload(P->d_work_bricks, vb);
  if (e == hipSuccess) e = upload(P->d_work_rows3, vr);
  if (e == hipSuccess) e = upload(P->d_work_ystrips, vy);
  if (e == hipSuccess) e = upload(P->d_work_zstrips, vz);
  if (e == hipSuccess) e = upload(P->d_work_sure, vs);
  if (e == hipSuccess) e = set_lds_limits_3d(P->lds_k3haar, P->lds_k3rows, P->lds_k3axis);
  if (e != hipSuccess) {
    free_plan(P);
    return fail(VDAMP_ERR_HIP, std::string("plan upload: ") + hipGetErrorString(e));
  }
  *plan = P;
  *workspace_bytes = P->ws_bytes;
  return VDAMP_OK;
}

vdamp_status vdamp_plan_3d(vdamp_plan_h* plan, int32_t batch, const int32_t* nz, const int32_t* ny,
                           const int32_t* nx, int32_t levels, uint32_t flags, size_t* workspace_bytes) {
  return make_plan3d(plan, batch, nz, ny, nx, levels, flags, workspace_bytes);
}

vdamp_status vdamp_plan_ortho(vdamp_plan_h* plan, int32_t batch, const int32_t* ny, const int32_t* nx,
                              int32_t levels, const double* lowpass, int32_t filter_len,
                              uint32_t flags, size_t* workspace_bytes) {
  if (!lowpass) {
    g_err.clear();
    if (plan) *plan = nullptr;
    return fail(VDAMP_ERR_ARG, "lowpass is null");
  }
  return make_plan(plan, batch, ny, nx, levels, lowpass, filter_len, flags, workspace_bytes);
}

vdamp_status vdamp_plan_describe(vdamp_plan_h plan, char* buf, size_t len, size_t* needed) {
  g_err.clear();
  if (!plan) return fail(VDAMP_ERR_ARG, "plan is null");
  const vdamp_plan_t* P = plan;
  std::string s = std::string(P->dim3 ? "volumes: 3D Haar, 3D DFT; "
                              : P->ortho ? "wavelet: orthonormal filter of " + std::to_string(P->filt.size()) +
                                               " taps (Fourier-domain passes); "
                                         : "wavelet: Haar; ") +
                  "slices " + std::to_string(P->B) + ", levels " + std::to_string(P->levels) + ", pixels " +
                  std::to_string(P->ntot) + ", workspace " + std::to_string(P->ws_bytes) + " bytes;";
  auto group = [&](const char* what, const std::array<int, 4>& g) {
    s += std::string(" ") + what + std::to_string(g[3]) + ": " + std::to_string(g[1]) + " strips, " +
         (g[2] ? "four-step M=" + std::to_string(g[2]) : std::string("Stockham")) + ";";
  };
  for (const auto& g : P->row_groups) group("rows nx=", g);
  for (const auto& g : P->col_groups) group("cols ny=", g);
  for (int c = kSureClasses - 1; c >= 0; --c)
    if (P->nsure_cls[c])
      s += " sure class " + std::to_string(c) + ": " + std::to_string(P->nsure_cls[c]) + " bands;";
  if (!P->tune_log.empty()) s += " " + P->tune_log;
  if (needed) *needed = s.size() + 1;
  if (buf && len) {
    const size_t n = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return VDAMP_OK;
}

vdamp_status vdamp_plan_destroy(vdamp_plan_h plan) {
  g_err.clear();
  if (!plan) return fail(VDAMP_ERR_ARG, "plan is null");
  free_plan(plan);
  return VDAMP_OK;
}

namespace {
vdamp_status solve_common(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                          size_t workspace_bytes, const float* y, const uint8_t* mask,
                          const float* p, const float* sigma2, const Resume& rs, int32_t iters,
                          float* x_hat, float* trace, float* x_monitor) {
  vdamp_status s = check_common(plan, workspace, workspace_bytes, y, mask, iters, x_hat);
  if (s != VDAMP_OK) return s;
  if (!p || !sigma2) return fail(VDAMP_ERR_ARG, "p and sigma2 must be non-null");
  if (rs.r && (!rs.theta || !rs.alpha))
    return fail(VDAMP_ERR_ARG, "r_init needs theta_init and alpha_init");
  if (!rs.r && (rs.theta || rs.theta2 || rs.alpha))
    return fail(VDAMP_ERR_ARG, "theta_init, theta2_init and alpha_init are read only with r_init");
  GraphKey key;
  key.kind = 0; key.ws = workspace; key.y = y; key.mask = mask; key.p = p; key.sig = sigma2;
  key.x = x_hat; key.trace = trace; key.iters = iters; key.stream = stream;
  key.r_init = rs.r; key.th_init = rs.theta; key.th2_init = rs.theta2; key.al_init = rs.alpha;
  key.mon = x_monitor;
  s = run_maybe_graph(plan, stream, key, [&](bool timing) {
    return enqueue_vdamp(plan, stream, workspace, reinterpret_cast<const float2*>(y), mask, p,
                         sigma2, iters, reinterpret_cast<float2*>(x_hat), trace, timing, rs,
                         reinterpret_cast<float2*>(x_monitor));
  });
  if (s != VDAMP_OK) return s;
  if (plan->flags & VDAMP_FLAG_CHECK_FINITE) {
    int bad = 0;
    const Ws w = layout(plan, workspace);
    HIP_TRY(hipMemcpyAsync(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (bad)
      return fail(VDAMP_ERR_NONFINITE,
                  "p outside (0, 1] on the mask, non-finite y, or an imported theta/alpha out of range");
  }
  plan->state_ws = workspace;
  plan->has_state = iters > 0 || rs.r;
  return VDAMP_OK;
}
}  // namespace


vdamp_status vdamp_solve(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                         size_t workspace_bytes, const float* y, const uint8_t* mask,
                         const float* p, const float* sigma2, int32_t iters, float* x_hat,
                         float* trace) {
  g_err.clear();
  return solve_common(plan, stream, workspace, workspace_bytes, y, mask, p, sigma2, Resume(), iters,
                      x_hat, trace, nullptr);
}

vdamp_status vdamp_solve_resume(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                                size_t workspace_bytes, const float* y, const uint8_t* mask,
                                const float* p, const float* sigma2, const float* r_init,
                                const float* theta_init, const float* theta2_init,
                                const float* alpha_init, int32_t iters, float* x_hat, float* trace,
                                float* x_monitor) {
  g_err.clear();
  Resume rs;
  rs.r = reinterpret_cast<const float2*>(r_init);
  rs.theta = theta_init;
  rs.theta2 = theta2_init;
  rs.alpha = alpha_init;
  return solve_common(plan, stream, workspace, workspace_bytes, y, mask, p, sigma2, rs, iters, x_hat,
                      trace, x_monitor);
}

vdamp_status fista_solve(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                         size_t workspace_bytes, const float* y, const uint8_t* mask,
                         const float* lambda, int32_t iters, float* x_hat, float* objective) {
  g_err.clear();
  vdamp_status s = check_common(plan, workspace, workspace_bytes, y, mask, iters, x_hat);
  if (s != VDAMP_OK) return s;
  if (!lambda) return fail(VDAMP_ERR_ARG, "lambda must be non-null");
  if (plan->ortho || plan->dim3) return fail(VDAMP_ERR_UNSUPPORTED, "fista_solve runs on 2D Haar plans only");
  if (plan->grp > 1) return fail(VDAMP_ERR_UNSUPPORTED, "fista_solve thresholds single coefficients (no VDAMP_FLAG_GROUP_PAIRS)");
  GraphKey key;
  key.kind = 1; key.ws = workspace; key.y = y; key.mask = mask; key.lam = lambda;
  key.x = x_hat; key.iters = iters; key.stream = stream; key.obj = objective;
  s = run_maybe_graph(plan, stream, key, [&](bool timing) {
    return enqueue_fista(plan, stream, workspace, reinterpret_cast<const float2*>(y), mask,
                         lambda, iters, reinterpret_cast<float2*>(x_hat), objective, timing);
  });
  if (s != VDAMP_OK) return s;
  plan->has_state = false;
  return VDAMP_OK;
}

vdamp_status vdamp_state_export(vdamp_plan_h plan, hipStream_t stream, const void* workspace,
                                float* r, float* theta, float* theta2, float* alpha, float* tau) {
  g_err.clear();
  if (!plan || !workspace) return fail(VDAMP_ERR_ARG, "plan and workspace must be non-null");
  if (!plan->has_state || plan->state_ws != workspace)
    return fail(VDAMP_ERR_STATE, "no vdamp_solve with iters >= 1 on this workspace");
  const Ws w = layout(plan, const_cast<void*>(workspace));
  if (r)
    HIP_TRY(hipMemcpyAsync(r, w.r, sizeof(float2) * (size_t)plan->ntot, hipMemcpyDeviceToDevice, stream));
  const int nb = plan->nbands;
  float* outs[4] = {theta, theta2, alpha, tau};
  float* srcs[4] = {w.theta, w.thr2, w.alpha, w.tau};
  for (int i = 0; i < 4; ++i) {
    if (!outs[i]) continue;
    HIP_TRY(hipMemcpy2DAsync(outs[i], sizeof(float) * nb, srcs[i], sizeof(float) * kMaxBands,
                             sizeof(float) * nb, plan->B, hipMemcpyDeviceToDevice, stream));
  }
  return VDAMP_OK;
}

vdamp_status vdamp_wavelet_ws(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                              size_t workspace_bytes, int32_t inverse, const float* in, float* out) {
  g_err.clear();
  if (!plan || !in || !out) return fail(VDAMP_ERR_ARG, "null pointer argument");
  if (in == out) return fail(VDAMP_ERR_ARG, "in and out must not overlap");
  if (!plan->ortho && !plan->dim3) return vdamp_wavelet(plan, stream, inverse, in, out);
  if (!workspace) return fail(VDAMP_ERR_WORKSPACE, "workspace is null");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(VDAMP_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (workspace_bytes < plan->ws_bytes)
    return fail(VDAMP_ERR_WORKSPACE, "workspace has " + std::to_string(workspace_bytes) + " bytes, needs " +
                                         std::to_string(plan->ws_bytes));
  const Ws w = layout(plan, workspace);
  KArgs a = base_args(plan, w);
  if (plan->state_ws == workspace) plan->has_state = false;  // the workspace's state is overwritten
  if (plan->dim3) {  // the 3D Haar bricks read in and write out directly
    if (inverse) {
      a.r = reinterpret_cast<float2*>(const_cast<float*>(in));
      a.X = reinterpret_cast<float2*>(out);
      a.mode = RS_PLAIN;
      HIP_TRY(pass3_haar(plan, a, true, stream));
    } else {
      a.X = reinterpret_cast<float2*>(const_cast<float*>(in));
      a.out = reinterpret_cast<float2*>(out);
      a.mode = OA_COEF;
      HIP_TRY(pass3_haar(plan, a, false, stream));
    }
    return VDAMP_OK;
  }
  if (inverse) {  // Psi^H: coefficient rows -> group rows -> image rows of X -> image
    a.r = reinterpret_cast<float2*>(const_cast<float*>(in));
    a.mode = RS_PLAIN;
    HIP_TRY(pass_synth(plan, a, stream));
    a.mode = OC_SYNTH;
    HIP_TRY(pass_cols(plan, a, stream));
    a.mode = RA_IMAGE;
    a.out = reinterpret_cast<float2*>(out);
    HIP_TRY(pass_anal(plan, a, stream));
  } else {  // Psi: image rows -> row DFTs in X -> group rows -> coefficients
    a.r = reinterpret_cast<float2*>(const_cast<float*>(in));
    a.mode = OS_IMAGE;
    HIP_TRY(pass_synth(plan, a, stream));
    a.mode = OC_ANAL;
    HIP_TRY(pass_cols(plan, a, stream));
    a.mode = OA_COEF;
    a.out = reinterpret_cast<float2*>(out);
    HIP_TRY(pass_anal(plan, a, stream));
  }
  return VDAMP_OK;
}

vdamp_status vdamp_pass_times(vdamp_plan_h plan, double* ms, int64_t* launches, int32_t npass) {
  g_err.clear();
  if (!plan || !ms || !launches || npass < 0) return fail(VDAMP_ERR_ARG, "null pointer or npass < 0");
  for (int i = 0; i < npass; ++i) { ms[i] = 0.0; launches[i] = 0; }
  for (auto& u : plan->ev_used) {
    hipEvent_t a = plan->ev_pool[u.second], b = plan->ev_pool[u.second + 1];
    HIP_TRY(hipEventSynchronize(b));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, a, b));
    if (u.first < npass) { ms[u.first] += t; launches[u.first] += 1; }
  }
  plan->ev_used.clear();
  plan->ev_next = 0;
  return VDAMP_OK;
}

}  // extern "C"

// Plan-time tuning of the launch configuration (VDAMP_FLAG_AUTOTUNE).  Every size group
// of a plan has kernels to choose from: the row and column passes a four-step register
// FFT or the in-LDS Stockham FFT (both the unitary DFT, rounded differently), the
// threshold search any size class whose LDS holds the band (the same sorted keys and
// argmin; only the FP64 chunk sums of the walk are grouped differently).  The tuner times
// each alternative on synthetic data in buffers of its own (iterate-like values; the
// threshold search sees noise-only keys, its most common case) and keeps the fastest,
// with a 3 % margin in favour of the default.  It runs once, when the plan is built;
// solves then use the recorded choice, so results stay reproducible for the plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "vdamp_host.h"

namespace vdamp {

namespace {

struct TuneBuffers {
  void* ws = nullptr;
  float2* y = nullptr;
  int2* work = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~TuneBuffers() {
    if (st) hipStreamSynchronize(st);
    hipFree(ws);
    hipFree(y);
    hipFree(work);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (st) hipStreamDestroy(st);
  }
};

// Median of `reps` timed runs after one untimed run, in milliseconds.
template <class F>
hipError_t time_ms(TuneBuffers& T, F&& run, double& ms, int reps = 5) {
  hipError_t e = run();
  if (e != hipSuccess) return e;
  std::vector<double> t;
  for (int i = 0; i < reps; ++i) {
    if ((e = hipEventRecord(T.e0, T.st)) != hipSuccess) return e;
    if ((e = run()) != hipSuccess) return e;
    if ((e = hipEventRecord(T.e1, T.st)) != hipSuccess) return e;
    if ((e = hipEventSynchronize(T.e1)) != hipSuccess) return e;
    float f = 0.f;
    if ((e = hipEventElapsedTime(&f, T.e0, T.e1)) != hipSuccess) return e;
    t.push_back(f);
  }
  std::sort(t.begin(), t.end());
  ms = t[t.size() / 2];
  return hipSuccess;
}

// Fresh tuning data: iterate-like r, X, y and weights; theta = 1 (key 1), alpha = 1/2
// for the Onsager correction; column-strip tau partials 1/16 each (tau = nx/256 per band).
hipError_t fill(const vdamp_plan_t* P, TuneBuffers& T, const Ws& w) {
  hipError_t e = launch_tune_fill(w.r, w.X, T.y, w.wgt, P->ntot, T.st);
  if (e == hipSuccess) e = launch_fill_f32(w.theta, (long long)P->B * kMaxBands, 1.0f, T.st);
  if (e == hipSuccess) e = launch_fill_f32(w.thr2, (long long)P->B * kMaxBands, 1.0f, T.st);
  if (e == hipSuccess) e = launch_fill_f32(w.alpha, (long long)P->B * kMaxBands, 0.5f, T.st);
  if (e == hipSuccess) e = launch_fill_f32(w.taup, (long long)P->ncolstrips * kMaxBands, 1.0f / 16, T.st);
  return e;
}

std::string fmt(const char* f, double a, double b) {
  char buf[96];
  std::snprintf(buf, sizeof(buf), f, a, b);
  return buf;
}
std::string fmt1(const char* f, double a) {
  char buf[64];
  std::snprintf(buf, sizeof(buf), f, a);
  return buf;
}

}  // namespace

hipError_t autotune(vdamp_plan_t* P) {
  TuneBuffers T;
  hipError_t e = hipStreamCreateWithFlags(&T.st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&T.e0);
  if (e == hipSuccess) e = hipEventCreate(&T.e1);
  if (e == hipSuccess) e = hipMalloc(&T.ws, P->ws_bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&T.y, sizeof(float2) * (size_t)P->ntot);
  if (e != hipSuccess) return e;
  const Ws w = layout(P, T.ws);
  if ((e = fill(P, T, w)) != hipSuccess) return e;
  KArgs base = base_args(P, w);
  base.y = T.y;
  const int H = 1 << P->levels;
  std::string log = "autotune:";

  // row passes: the Onsager correction + Psi^H + row FFT, then row IFFT + Psi + the
  // back-projection, per run of equal nx
  for (auto& g : P->row_groups) {
    if (!g[2]) continue;
    const int m4 = g[2];
    auto run = [&](int m) {
      KArgs a = base;
      a.work = P->d_work_rows + g[0];
      a.nwork = g[1];
      a.mode = P->grp > 1 ? RS_RTILDE_G : RS_RTILDE;
      hipError_t r = m ? launch_rows_synth4(a, m, rows4_lds_bytes(m, H), T.st)
                       : launch_rows_synth(a, P->ept, 1, P->lds_rows, T.st);
      if (r != hipSuccess) return r;
      a.mode = P->grp > 1 ? RA_VDAMP_G : RA_VDAMP;
      return m ? launch_rows_anal4(a, m, rows4_lds_bytes(m, H), T.st) : launch_rows_anal(a, P->ept, P->lds_rows, T.st);
    };
    double t4 = 0, ts = 0;
    if ((e = time_ms(T, [&] { return run(m4); }, t4)) != hipSuccess) return e;
    if ((e = time_ms(T, [&] { return run(0); }, ts)) != hipSuccess) return e;
    const bool stock = ts < 0.97 * t4;
    log += " rows nx=" + std::to_string(g[3]) + fmt(" (four-step %.4f ms, Stockham %.4f ms)", t4, ts) +
           (stock ? " Stockham;" : " four-step;");
    if (stock) g[2] = 0;
  }
  if ((e = fill(P, T, w)) != hipSuccess) return e;
  // column pass: column FFT, the k-space step, column IFFT, per run of equal ny
  for (auto& g : P->col_groups) {
    if (!g[2]) continue;
    const int m4 = g[2];
    auto run = [&](int m) {
      KArgs a = base;
      a.work = P->d_work_cols + g[0];
      a.nwork = g[1];
      a.mode = CM_VDAMP;
      return m ? launch_cols4(a, m, T.st) : launch_cols(a, P->ept, P->lds_cols, T.st);
    };
    double t4 = 0, ts = 0;
    if ((e = time_ms(T, [&] { return run(m4); }, t4)) != hipSuccess) return e;
    if ((e = time_ms(T, [&] { return run(0); }, ts)) != hipSuccess) return e;
    const bool stock = ts < 0.97 * t4;
    log += " cols ny=" + std::to_string(g[3]) + fmt(" (four-step %.4f ms, Stockham %.4f ms)", t4, ts) +
           (stock ? " Stockham;" : " four-step;");
    if (stock) g[2] = 0;
  }
  if ((e = fill(P, T, w)) != hipSuccess) return e;
  // threshold search: per band size, every LDS class that holds it
  std::map<long long, std::vector<int2>> by_size;
  for (int b = 0; b < P->B; ++b)
    for (int band = 0; band < P->nbands; ++band) {
      const int l = band == 0 ? P->levels : P->levels - (band - 1) / 3;
      by_size[(long long)(P->ny[b] >> l) * (P->nx[b] >> l) / P->grp].push_back(make_int2(b, band));
    }
  size_t most = 0;
  for (auto& kv : by_size) most = std::max(most, kv.second.size());
  if ((e = hipMalloc((void**)&T.work, sizeof(int2) * std::max<size_t>(most, 1))) != hipSuccess) return e;
  bool changed = false;
  for (auto& kv : by_size) {
    const long long nb = kv.first;
    const int def = sure_default_class(nb);
    if (def == kSureBigClass) continue;
    if ((e = hipMemcpy(T.work, kv.second.data(), sizeof(int2) * kv.second.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return e;
    std::vector<std::pair<int, double>> times;
    double tdef = 0;
    for (int c = 0; c < kSureBigClass; ++c) {
      if (nb > sure_class_capacity(c)) continue;
      KArgs a = base;
      a.work = T.work;
      a.nwork = (int)kv.second.size();
      double t = 0;
      if ((e = time_ms(T, [&] { return launch_sure(a, c, w.big, T.st); }, t)) != hipSuccess) return e;
      times.push_back({c, t});
      if (c == def) tdef = t;
    }
    int best = def;
    double tb = tdef;
    std::string cand;
    for (auto& ct : times) {
      if (ct.first != def && ct.second < 0.97 * tdef && ct.second < tb) {
        best = ct.first;
        tb = ct.second;
      }
      cand += (cand.empty() ? "class " : ", class ") + std::to_string(ct.first) + fmt1(" %.4f ms", ct.second);
    }
    log += " sure N_b=" + std::to_string(nb) + " (" + cand + ") class " + std::to_string(best) + ";";
    if (best != def) {
      P->sure_cls_of_size[nb] = best;
      changed = true;
    }
  }
  if (changed) {
    std::vector<int2> vs = sure_work_list(P);
    if ((e = hipMemcpy(P->d_work_sure, vs.data(), sizeof(int2) * vs.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return e;
  }
  if ((e = hipStreamSynchronize(T.st)) != hipSuccess) return e;
  P->tune_log = log;
  return hipSuccess;
}

}  // namespace vdamp

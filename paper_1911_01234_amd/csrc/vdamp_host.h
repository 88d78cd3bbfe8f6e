// Host-side internals shared by the library's translation units: the plan, the
// workspace layout, error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "vdamp.h"
#include "vdamp_internal.h"

namespace vdamp {

struct GraphKey {
  int kind = -1;
  const void *ws = nullptr, *y = nullptr, *mask = nullptr, *p = nullptr, *sig = nullptr,
             *lam = nullptr, *x = nullptr, *trace = nullptr;
  const void* aux_ws = nullptr;  // learned solve: the denoiser's workspace
  unsigned long long aux_id = 0; // learned solve: the denoiser's unique id (never reused)
  int judge = -1;
  // resumed solve: the imported state; monitor output; FISTA objective
  const void *r_init = nullptr, *th_init = nullptr, *th2_init = nullptr, *al_init = nullptr,
             *mon = nullptr, *obj = nullptr;
  unsigned long long seed = 0;
  int extra = 0;
  int iters = -1;
  hipStream_t stream = nullptr;
  bool operator==(const GraphKey& o) const {
    return kind == o.kind && ws == o.ws && y == o.y && mask == o.mask && p == o.p &&
           sig == o.sig && lam == o.lam && x == o.x && trace == o.trace && aux_ws == o.aux_ws &&
           aux_id == o.aux_id && judge == o.judge && r_init == o.r_init && th_init == o.th_init &&
           th2_init == o.th2_init && al_init == o.al_init && mon == o.mon && obj == o.obj &&
           seed == o.seed && extra == o.extra && iters == o.iters && stream == o.stream;
  }
};

struct Ws {
  float* wgt;
  float2 *r, *X, *r2;
  float *theta, *thr2, *alpha, *tau, *taup, *rpart;
  int* bad;
  float* big;  // full-sort scratch of the bands larger than the LDS search (or null)
  float2* Z;   // group rows of the general-wavelet passes (or null)
};

extern thread_local std::string g_err;  // detail of the last failure on this thread
vdamp_status fail(vdamp_status st, const std::string& msg);
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return ::vdamp::fail(VDAMP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace vdamp

struct vdamp_plan_t {
  using GraphKey = vdamp::GraphKey;
  int B = 0, levels = 0, nbands = 0;
  uint32_t flags = 0;
  std::vector<int> ny, nx;
  std::vector<long long> off;
  long long ntot = 0;
  int ncolstrips = 0;
  // device constants
  vdamp::SliceDev* d_slices = nullptr;
  vdamp::FftPlanDev* d_ffts = nullptr;
  float2* d_tw = nullptr;
  float* d_tables = nullptr;
  int2* d_work_rows = nullptr;
  int2* d_work_cols = nullptr;
  int2* d_work_sure = nullptr;      // bands grouped by threshold-search class, largest class first
  int nrows = 0, ncols = 0, nsure_cls[vdamp::kSureClasses] = {};
  int nrowstrips = 0;
  // column launches: runs of the column work list with one ny each (first, count, M, ny),
  // M = ny / 16 for the four-step kernel, 0 for the LDS Stockham kernel
  std::vector<std::array<int, 4>> col_groups;
  // row launches: runs of the row work list with one nx each (first, count, M, nx),
  // M = nx / 16 for the four-step row kernels, 0 for the LDS Stockham ones
  std::vector<std::array<int, 4>> row_groups;
  // learned denoiser: 16x16 tiles (slice, tile index), slice-major; tile_off[b] = first
  // tile of slice b
  bool tiles_ok = false;
  int ntiles = 0;
  std::vector<int> tile_off;
  int2* d_tiles = nullptr;
  int* d_tile_off = nullptr;
  // threshold-search size class chosen per band size (absent: the default by size)
  std::map<long long, int> sure_cls_of_size;
  std::string tune_log;             // what the plan-time tuner measured and chose
  int ept = 16;                     // complex elements per thread of the LDS passes
  size_t lds_rows = 0, lds_cols = 0;
  // general orthonormal wavelet (plans made with a filter): lowpass filter, complex filter
  // responses, group-row and image-row work lists, LDS sizes of its passes
  bool ortho = false;
  int grp = 1;  // coefficients per thresholding group (VDAMP_FLAG_GROUP_PAIRS: 2)
  std::vector<double> filt;
  float2* d_resp = nullptr;
  int2* d_work_orows = nullptr;
  int n_orows = 0;
  int2* d_work_img = nullptr;
  int n_img = 0;
  size_t lds_osynth = 0, lds_ocols = 0, lds_oanal = 0;
  int ocols_ept = 16;
  int ocols_ny = 0;  // the rows of every slice when they agree, else 0
  size_t o_Z = 0;
  // volumes (plans made by vdamp_plan_3d): depths, Haar bricks, x-row items, y and z
  // strips, LDS sizes and elements a thread of the strip kernel
  bool dim3 = false;
  std::vector<int> nz;
  int2 *d_work_bricks = nullptr, *d_work_rows3 = nullptr, *d_work_ystrips = nullptr,
       *d_work_zstrips = nullptr;
  int n_bricks = 0, n_rows3 = 0, n_ystrips = 0, n_zstrips = 0;
  size_t lds_k3haar = 0, lds_k3rows = 0, lds_k3axis = 0;
  int k3_ept = 16;
  // workspace layout (byte offsets)
  size_t o_wgt = 0, o_r = 0, o_X = 0, o_r2 = 0, o_theta = 0, o_thr2 = 0, o_alpha = 0, o_tau = 0,
         o_taup = 0, o_rpart = 0, o_bad = 0, o_big = 0, ws_bytes = 0;
  // last solve
  const void* state_ws = nullptr;
  bool has_state = false;
  // side streams (default priority) on which the launches of a pass's other size groups
  // run beside the first group's, forked from and joined back into the caller's stream
  // with events; created at plan time only for plans with more than one size group
  static constexpr int kForks = 3;
  hipStream_t side[kForks] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kForks] = {};
  // graph cache
  GraphKey gkey;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  // timing
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_used;  // (pass, index of start event in ev_pool)
  size_t ev_next = 0;
};

namespace vdamp {
Ws layout(const vdamp_plan_t* P, void* ws);
vdamp_status solve_eager(vdamp_plan_t* plan, hipStream_t stream, void* workspace,
                         size_t workspace_bytes, const float* y, const uint8_t* mask,
                         const float* p, const float* sigma2, int32_t iters, float* x_hat,
                         float* trace);
// Threshold-search work list of the plan's bands grouped by size class (largest class
// first, heaviest bands first within a class), with P->nsure_cls set; classes from
// P->sure_cls_of_size where present, else by size.
std::vector<int2> sure_work_list(vdamp_plan_t* P);
int sure_default_class(long long nb);
int sure_class_capacity(int cls);
// Plan-time tuning (VDAMP_FLAG_AUTOTUNE): times the alternatives of every size group on
// synthetic data and keeps the fastest; rewrites P's groups and threshold-search list.
hipError_t autotune(vdamp_plan_t* P);
hipError_t launch_rows_synth(const KArgs& a, int ept, int do_fft, size_t lds, hipStream_t st);
hipError_t launch_cols(const KArgs& a, int ept, size_t lds, hipStream_t st);
hipError_t launch_rows_anal(const KArgs& a, int ept, size_t lds, hipStream_t st);
hipError_t launch_sure(const KArgs& a, int cls, float* scratch, hipStream_t st);
hipError_t launch_prep(const uint8_t* mask, const float* p, const float2* y, float* wgt,
                       long long n, int check, int* bad, hipStream_t st);
hipError_t launch_zero(float2* x, long long n, hipStream_t st);
hipError_t launch_import_state(const float* th, const float* th2, const float* al, int batch,
                               int nb, float* theta, float* thr2, float* alpha, int check, int* bad,
                               hipStream_t st);
hipError_t launch_fista_obj(const KArgs& a, float* obj, hipStream_t st);
hipError_t launch_tune_fill(float2* r, float2* X, float2* y, float* wgt, long long n, hipStream_t st);
hipError_t launch_fill_f32(float* x, long long n, float v, hipStream_t st);
hipError_t set_lds_limits_passes(size_t rows, size_t cols);
hipError_t launch_cols4(const KArgs& a, int m, hipStream_t st);
hipError_t launch_rows_synth4(const KArgs& a, int m, size_t lds, hipStream_t st);
hipError_t launch_rows_anal4(const KArgs& a, int m, size_t lds, hipStream_t st);
size_t rows4_lds_bytes(int m, int H);
bool cols4_supported(int ny);
hipError_t launch_wave_anal(const KArgs& a, int ept, int jmode, size_t lds, hipStream_t st);
hipError_t launch_scale(const SliceDev* slices, int batch, const float2* y, const float* wgt,
                        float* s0, hipStream_t st);
hipError_t launch_judge(const KArgs& a, int nrowstrips, int always, int* sel, float* jout,
                        hipStream_t st);
// general orthonormal wavelets
size_t ocols_lds_bytes(int maxny, int s);
hipError_t set_lds_limits_ortho(size_t synth, size_t cols, size_t anal);
hipError_t launch_osynth(const KArgs& a, size_t lds, hipStream_t st);
hipError_t launch_ocols(const KArgs& a, int ept, int ny_all, size_t lds, hipStream_t st);
hipError_t launch_oanal(const KArgs& a, size_t lds, hipStream_t st);
// volumes
size_t k3_axis_lds_bytes(int maxn, int maxnd, int s);
hipError_t set_lds_limits_3d(size_t haar, size_t rows, size_t axis);
hipError_t launch_k3_haar(const KArgs& a, bool synth, size_t lds, hipStream_t st);
hipError_t launch_k3_rows(const KArgs& a, bool inv, bool to_out, size_t lds, hipStream_t st);
hipError_t launch_k3_axis(const KArgs& a, int ept, size_t lds, hipStream_t st);

// Launch helper that records timing events around each kernel when asked.
struct Launcher {
  vdamp_plan_t* P;
  hipStream_t st;
  bool timing;
  hipError_t begin(int pass) {
    if (!timing) return hipSuccess;
    if (P->ev_next + 2 > P->ev_pool.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        P->ev_pool.push_back(e);
      }
    }
    P->ev_used.emplace_back(pass, (int)P->ev_next);
    hipError_t err = hipEventRecord(P->ev_pool[P->ev_next], st);
    P->ev_next += 2;
    return err;
  }
  hipError_t end() {
    if (!timing) return hipSuccess;
    return hipEventRecord(P->ev_pool[P->ev_used.back().second + 1], st);
  }
};

#define LAUNCH(L, pass, call)                                                           \
  do {                                                                                  \
    HIP_TRY((L).begin(pass));                                                           \
    HIP_TRY(call);                                                                      \
    HIP_TRY((L).end());                                                                 \
  } while (0)

// The launches of a pass, one per size group, with group i on stream i mod (1 + kForks)
// (stream 0 the caller's): the side streams wait for everything enqueued before the
// pass and the caller's stream waits for them after it, so the groups of a ragged batch
// fill each other's tails while the pass as a whole stays ordered; under graph capture
// the same events make parallel branches.  With one group (or no side streams) every
// launch goes to the caller's stream.
template <class F>
inline hipError_t launch_groups(const vdamp_plan_t* P, int ngroups, hipStream_t st, F&& launch) {
  const int nside = (ngroups > 1 && P->side[0]) ? std::min(ngroups - 1, (int)vdamp_plan_t::kForks) : 0;
  hipError_t e = hipSuccess;
  if (nside) {
    if ((e = hipEventRecord(P->ev_fork, st)) != hipSuccess) return e;
    for (int i = 0; i < nside; ++i)
      if ((e = hipStreamWaitEvent(P->side[i], P->ev_fork, 0)) != hipSuccess) return e;
  }
  for (int g = 0; g < ngroups; ++g) {
    const int lane = nside ? g % (nside + 1) : 0;
    if ((e = launch(g, lane ? P->side[lane - 1] : st)) != hipSuccess) return e;
  }
  for (int i = 0; i < nside; ++i) {
    if ((e = hipEventRecord(P->ev_join[i], P->side[i])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st, P->ev_join[i], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Every column strip of the plan: one launch per run of equal ny.
inline hipError_t launch_cols_all(const vdamp_plan_t* P, KArgs a, hipStream_t st) {
  return launch_groups(P, (int)P->col_groups.size(), st, [&](int i, hipStream_t s) {
    const auto& g = P->col_groups[i];
    KArgs b = a;
    b.work = P->d_work_cols + g[0];
    b.nwork = g[1];
    return g[2] ? launch_cols4(b, g[2], s) : launch_cols(b, P->ept, P->lds_cols, s);
  });
}

// Every row strip of the plan through the transform passes: one launch per run of equal
// nx (Onsager correction + Psi^H + row FFT, and row IFFT + Psi + the back-projection).
inline hipError_t launch_rows_synth_all(const vdamp_plan_t* P, KArgs a, hipStream_t st) {
  return launch_groups(P, (int)P->row_groups.size(), st, [&](int i, hipStream_t s) {
    const auto& g = P->row_groups[i];
    KArgs b = a;
    b.work = P->d_work_rows + g[0];
    b.nwork = g[1];
    return g[2] ? launch_rows_synth4(b, g[2], rows4_lds_bytes(g[2], 1 << P->levels), s)
                : launch_rows_synth(b, P->ept, 1, P->lds_rows, s);
  });
}
inline hipError_t launch_rows_anal_all(const vdamp_plan_t* P, KArgs a, hipStream_t st) {
  return launch_groups(P, (int)P->row_groups.size(), st, [&](int i, hipStream_t s) {
    const auto& g = P->row_groups[i];
    KArgs b = a;
    b.work = P->d_work_rows + g[0];
    b.nwork = g[1];
    return g[2] ? launch_rows_anal4(b, g[2], rows4_lds_bytes(g[2], 1 << P->levels), s)
                : launch_rows_anal(b, P->ept, P->lds_rows, s);
  });
}

// Every band's threshold search (denoising step): one launch per size class, largest first.
inline hipError_t launch_sure_all(const vdamp_plan_t* P, KArgs a, float* scratch, hipStream_t st) {
  for (int c = kSureClasses - 1, first = 0; c >= 0; --c) {
    if (!P->nsure_cls[c]) continue;
    a.work = P->d_work_sure + first;
    a.nwork = P->nsure_cls[c];
    hipError_t e = launch_sure(a, c, scratch, st);
    if (e != hipSuccess) return e;
    first += P->nsure_cls[c];
  }
  return hipSuccess;
}

inline KArgs base_args(const vdamp_plan_t* P, const Ws& w) {
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.slices = P->d_slices;
  a.ffts = P->d_ffts;
  a.twiddles = P->d_tw;
  a.tables = P->d_tables;
  a.levels = P->levels;
  a.nbands = P->nbands;
  a.batch = P->B;
  a.wgt = w.wgt;
  a.r = w.r;
  a.r2 = w.r2;
  a.X = w.X;
  a.theta = w.theta;
  a.thr2 = w.thr2;
  a.alpha = w.alpha;
  a.tau = w.tau;
  a.tau_part = w.taup;
  a.sure_cont = (P->flags & VDAMP_FLAG_SURE_CONTINUOUS) ? 1 : 0;
  a.grp = P->grp;
  a.resp = P->d_resp;
  a.Z = w.Z;
  return a;
}

// The three transform passes of an iteration, for either wavelet: Haar plans run the
// strip kernels (one launch per size group), general-wavelet plans the Fourier-domain
// kernels (one launch over the plan's group rows or column strips; OS_IMAGE and RA_IMAGE
// work on image rows).
inline hipError_t pass_synth(const vdamp_plan_t* P, KArgs a, hipStream_t st) {
  if (!P->ortho) return launch_rows_synth_all(P, a, st);
  const bool img = a.mode == OS_IMAGE;
  a.work = img ? P->d_work_img : P->d_work_orows;
  a.nwork = img ? P->n_img : P->n_orows;
  return launch_osynth(a, P->lds_osynth, st);
}
inline hipError_t pass_cols(const vdamp_plan_t* P, KArgs a, hipStream_t st) {
  if (!P->ortho) return launch_cols_all(P, a, st);
  a.work = P->d_work_cols;
  a.nwork = P->ncols;
  return launch_ocols(a, P->ocols_ept, P->ocols_ny, P->lds_ocols, st);
}
// Volumes: Haar bricks (Psi^H into X, or Psi from X), x-row DFTs, y or z strip DFTs.
inline hipError_t pass3_haar(const vdamp_plan_t* P, KArgs a, bool synth, hipStream_t st) {
  a.work = P->d_work_bricks;
  a.nwork = P->n_bricks;
  return launch_k3_haar(a, synth, P->lds_k3haar, st);
}
inline hipError_t pass3_rows(const vdamp_plan_t* P, KArgs a, bool inv, bool to_out, hipStream_t st) {
  a.work = P->d_work_rows3;
  a.nwork = P->n_rows3;
  return launch_k3_rows(a, inv, to_out, P->lds_k3rows, st);
}
inline hipError_t pass3_axis(const vdamp_plan_t* P, KArgs a, hipStream_t st) {
  const bool y = a.mode == AX_Y_FWD || a.mode == AX_Y_INV;
  a.work = y ? P->d_work_ystrips : P->d_work_zstrips;
  a.nwork = y ? P->n_ystrips : P->n_zstrips;
  return launch_k3_axis(a, P->k3_ept, P->lds_k3axis, st);
}

inline hipError_t pass_anal(const vdamp_plan_t* P, KArgs a, hipStream_t st) {
  if (!P->ortho) return launch_rows_anal_all(P, a, st);
  const bool img = a.mode == RA_IMAGE;
  a.work = img ? P->d_work_img : P->d_work_orows;
  a.nwork = img ? P->n_img : P->n_orows;
  return launch_oanal(a, P->lds_oanal, st);
}


template <class F>
inline vdamp_status run_maybe_graph(vdamp_plan_t* P, hipStream_t st, const GraphKey& key, F&& enqueue) {
  const bool timing = (P->flags & VDAMP_FLAG_TIMING) != 0;
  if (timing || !(P->flags & VDAMP_FLAG_USE_GRAPH)) return enqueue(timing);
  if (!(P->gexec && P->gkey == key)) {
    if (P->gexec) { hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
    if (P->graph) { hipGraphDestroy(P->graph); P->graph = nullptr; }
    P->gkey = GraphKey();
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    vdamp_status s = enqueue(false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != VDAMP_OK) {
      if (g) hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(VDAMP_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    P->graph = g;
    HIP_TRY(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0));
    P->gkey = key;
  }
  HIP_TRY(hipGraphLaunch(P->gexec, st));
  return VDAMP_OK;
}

}  // namespace vdamp

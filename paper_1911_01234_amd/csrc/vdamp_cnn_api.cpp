// Host side of the learned denoiser: parameters and their BF16 packings, the forward
// pass with its Jacobian-vector product, one training step (backpropagation and Adam),
// the learned variant of Algorithm 1 with its per-subband SURE judge, and the plain
// wavelet transform.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <string>
#include <vector>

#include "vdamp.h"
#include "vdamp_cnn_args.h"
#include "vdamp_host.h"

namespace vdamp {
namespace cnn {
hipError_t launch_conv(const ConvArgs& a, int cin, int mt, int mode, int grid, hipStream_t st);
hipError_t launch_wgrad(const WgradArgs& a, int layer, int grid, hipStream_t st);
hipError_t launch_reduce_wgrad(const float* part, const float* part_bias, int nwg, int rows,
                               int cols, int cinp, int cout, int cin, float* stage, float* gW,
                               float* gb, hipStream_t st);
hipError_t launch_pack_input(const SliceDev* slices, int batch, const float2* x, const float* s0,
                             long long npx, u16* out, hipStream_t st);
hipError_t launch_slice_bias(const float* b1, const float* wt, const float* tau, const float* s0,
                             int nb, int batch, int tau_stride, float* sb, hipStream_t st);
hipError_t launch_loss_grad(const SliceDev* slices, int batch, const float2* xo, const float2* x0,
                            const float* s0, long long npx, u16* go, float* part, float* loss,
                            hipStream_t st);
hipError_t launch_wt_grad(const float* tile_sums, const int* tile_off, const float* tau,
                          const float* s0, int nb, int batch, int tau_stride, float* dwt, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float c1,
                       float c2, hipStream_t st);
hipError_t launch_pack_w(const float* W, int cout, int cin, int cinp, int coutp, int kpad, u16* wf,
                         int dcoutp, int dkpad, u16* wd, hipStream_t st);
}  // namespace cnn
}  // namespace vdamp

using namespace vdamp;
using vdamp::cnn::u16;

namespace {

constexpr int kC = 48;        // hidden channels
constexpr int kLayers = 6;
constexpr int kConvGrid = 512;   // persistent convolution workgroups (two per CU)
constexpr int kWgradGrid = 512;  // weight-gradient workgroups (two per CU)

// Geometry of layer l (1..6): channels, the padded channel stride of its input, the
// rows of its forward weight matrix (16 per MFMA tile) and the padded K of the forward
// and input-gradient matrices (9 taps x channels, rounded up to 32).
struct LayerGeom {
  int cin, cout, cinp, rows, kpad, dcoutp, dkpad;
};
LayerGeom geom(int l) {
  if (l == 1) return {2, kC, 8, kC, 96, 0, 0};
  if (l == kLayers) return {kC, 2, kC, 16, 448, 8, 96};
  return {kC, kC, kC, kC, 448, kC, 448};
}

}  // namespace

struct vdamp_cnn_t {
  int nb = 0;
  long long n = 0;
  long long oW[kLayers + 1] = {}, ob[kLayers + 1] = {}, oWt = 0;
  float *d_p = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr;
  u16* d_wf[kLayers + 1] = {};
  u16* d_wd[kLayers + 1] = {};
  int step = 0;
  unsigned long long id = 0;  // unique per denoiser object, never reused (graph cache key)
};

namespace {

void free_cnn(vdamp_cnn_t* C) {
  if (!C) return;
  hipFree(C->d_p);
  hipFree(C->d_g);
  hipFree(C->d_m);
  hipFree(C->d_v);
  for (int l = 1; l <= kLayers; ++l) {
    hipFree(C->d_wf[l]);
    hipFree(C->d_wd[l]);
  }
  delete C;
}

// Workspace layout of the denoiser on a plan (byte offsets; 0 = absent).
struct CnnWs {
  size_t a0 = 0, t0 = 0, act[kLayers] = {}, ta = 0, tb = 0, g6 = 0, ga = 0, gb = 0;
  size_t sbias = 0, lpart = 0, part = 0, pbias = 0, rstage = 0, tsums = 0, xo = 0;
  size_t xi = 0, ti = 0, xo2 = 0, to = 0, jpart = 0, sel = 0, smin = 0, s0 = 0, jout = 0;
  size_t bits = 0;  // ReLU pattern of the current layer (forward and solve kinds)
  size_t bytes = 0;
};

CnnWs cnn_layout(const vdamp_plan_t* P, int kind) {
  CnnWs L;
  size_t o = 256;  // offset 0 marks an absent buffer
  const size_t N = (size_t)P->ntot;
  auto take = [&](size_t& field, size_t bytes) { field = o; o = align256(o + bytes); };
  take(L.a0, 2 * 8 * N);
  take(L.sbias, 4 * (size_t)P->B * kC);
  if (kind == VDAMP_CNN_WS_TRAIN) {
    for (int l = 1; l < kLayers; ++l) take(L.act[l], 2 * (size_t)kC * N);
    take(L.g6, 2 * 8 * N);
    take(L.ga, 2 * (size_t)kC * N);
    take(L.gb, 2 * (size_t)kC * N);
    take(L.xo, 8 * N);
    take(L.lpart, 4 * ((N + 255) / 256));
    take(L.part, 4 * (size_t)kWgradGrid * kC * 432);
    take(L.pbias, 4 * (size_t)kWgradGrid * kC);
    take(L.rstage, 4 * (size_t)cnn::kWgradReduceGroups * (kC * 432 + kC));  // first-stage group sums
    take(L.tsums, 4 * (size_t)std::max(P->ntiles, 1) * kC);
  } else {
    take(L.t0, 2 * 8 * N);
    take(L.act[1], 2 * (size_t)kC * N);  // ping-pong activations
    take(L.act[2], 2 * (size_t)kC * N);
    take(L.ta, 2 * (size_t)kC * N);      // ping-pong tangents
    take(L.tb, 2 * (size_t)kC * N);
    take(L.bits, 8 * N);
  }
  if (kind == VDAMP_CNN_WS_SOLVE) {
    take(L.xi, 8 * N);
    take(L.ti, 8 * N);
    take(L.xo2, 8 * N);
    take(L.to, 8 * N);
    take(L.jpart, 4 * 2 * (size_t)P->nrowstrips * kMaxBands);
    take(L.sel, 4 * (size_t)P->B * kMaxBands);
    take(L.smin, 4 * (size_t)P->B * kMaxBands);
    take(L.s0, 4 * (size_t)P->B);
    take(L.jout, 4 * 3 * (size_t)P->B * kMaxBands);
  }
  L.bytes = o;
  return L;
}

template <class T>
T* at(void* ws, size_t off) {
  return off ? reinterpret_cast<T*>(static_cast<char*>(ws) + off) : nullptr;
}

vdamp_status check_cnn_ws(const vdamp_plan_t* P, int kind, void* ws, size_t wsb) {
  if (P->ortho || P->dim3 || P->grp > 1)
    return fail(VDAMP_ERR_UNSUPPORTED, "the learned denoiser runs on 2D Haar plans without groups only");
  if (!P->tiles_ok) return fail(VDAMP_ERR_UNSUPPORTED, "the learned denoiser needs ny and nx multiples of 16");
  if (!ws) return fail(VDAMP_ERR_WORKSPACE, "denoiser workspace is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(VDAMP_ERR_WORKSPACE, "denoiser workspace not 256-byte aligned");
  const size_t need = cnn_layout(P, kind).bytes;
  if (wsb < need)
    return fail(VDAMP_ERR_WORKSPACE, "denoiser workspace has " + std::to_string(wsb) + " bytes, needs " +
                                         std::to_string(need));
  return VDAMP_OK;
}

vdamp_status repack(vdamp_cnn_t* C, hipStream_t st) {
  for (int l = 1; l <= kLayers; ++l) {
    const LayerGeom g = geom(l);
    HIP_TRY(cnn::launch_pack_w(C->d_p + C->oW[l], g.cout, g.cin, g.cinp, g.rows, g.kpad, C->d_wf[l],
                               g.dcoutp, g.dkpad, l > 1 ? C->d_wd[l] : nullptr, st));
  }
  return VDAMP_OK;
}

cnn::ConvArgs conv_args(const vdamp_plan_t* P) {
  cnn::ConvArgs a;
  std::memset(&a, 0, sizeof(a));
  a.slices = P->d_slices;
  a.tiles = P->d_tiles;
  a.ntiles = P->ntiles;
  return a;
}

int conv_grid(const vdamp_plan_t* P) { return std::max(1, std::min(P->ntiles, kConvGrid)); }

// Forward pass (and, with tangent, the JVP interleaved layer by layer: the tangent of
// layer l needs only the ReLU pattern of the same layer).
vdamp_status enqueue_forward(const vdamp_cnn_t* C, const vdamp_plan_t* P, const CnnWs& L, void* ws,
                             const float2* x, const float* tau, int tau_stride, const float* s0,
                             float2* x_out, const float2* tangent, float2* jvp_out, hipStream_t st) {
  const long long N = P->ntot;
  u16* a0 = at<u16>(ws, L.a0);
  u16* t0 = at<u16>(ws, L.t0);
  float* sbias = at<float>(ws, L.sbias);
  HIP_TRY(cnn::launch_pack_input(P->d_slices, P->B, x, s0, N, a0, st));
  HIP_TRY(cnn::launch_slice_bias(C->d_p + C->ob[1], C->d_p + C->oWt, tau, s0, C->nb, P->B, tau_stride,
                                 sbias, st));
  if (tangent) HIP_TRY(cnn::launch_pack_input(P->d_slices, P->B, tangent, nullptr, N, t0, st));
  u16* act[2] = {at<u16>(ws, L.act[1]), at<u16>(ws, L.act[2])};
  u16* tan[2] = {at<u16>(ws, L.ta), at<u16>(ws, L.tb)};
  const int grid = conv_grid(P);
  const u16* cur = a0;
  const u16* tcur = t0;
  for (int l = 1; l <= kLayers; ++l) {
    cnn::ConvArgs a = conv_args(P);
    const int cin = l == 1 ? 8 : kC;
    a.in = cur;
    a.w = C->d_wf[l];
    if (l < kLayers) {
      u16* out = act[l & 1];
      a.bias = l == 1 ? nullptr : C->d_p + C->ob[l];
      a.sbias = l == 1 ? sbias : nullptr;
      a.out = out;
      // with a tangent the layer also writes its ReLU pattern, which the tangent's
      // masked convolution reads (8 bytes a pixel instead of the 96-byte activation)
      uint2* bits = tangent ? at<uint2>(ws, L.bits) : nullptr;
      a.bits_out = bits;
      HIP_TRY(cnn::launch_conv(a, cin, 3, cnn::CV_RELU, grid, st));
      if (tangent) {
        cnn::ConvArgs t = conv_args(P);
        t.in = tcur;
        t.w = C->d_wf[l];
        t.mask = out;
        t.bits = bits;
        t.out = tan[l & 1];
        HIP_TRY(cnn::launch_conv(t, cin, 3, cnn::CV_MASK, grid, st));
        tcur = tan[l & 1];
      }
      cur = out;
    } else {
      a.bias = C->d_p + C->ob[l];
      a.resid = x;
      a.s0 = s0;
      a.img_out = x_out;
      HIP_TRY(cnn::launch_conv(a, cin, 1, cnn::CV_LAST, grid, st));
      if (tangent) {
        cnn::ConvArgs t = conv_args(P);
        t.in = tcur;
        t.w = C->d_wf[l];
        t.resid = tangent;
        t.img_out = jvp_out;
        HIP_TRY(cnn::launch_conv(t, cin, 1, cnn::CV_LAST_TAN, grid, st));
      }
    }
  }
  return VDAMP_OK;
}

vdamp_status enqueue_train(vdamp_cnn_t* C, const vdamp_plan_t* P, const CnnWs& L, void* ws,
                           const float2* x, const float* tau, const float* s0, const float2* x0,
                           float lr, float* loss, hipStream_t st) {
  const long long N = P->ntot;
  u16* A[kLayers] = {at<u16>(ws, L.a0)};
  for (int l = 1; l < kLayers; ++l) A[l] = at<u16>(ws, L.act[l]);
  float* sbias = at<float>(ws, L.sbias);
  float2* xo = at<float2>(ws, L.xo);
  HIP_TRY(cnn::launch_pack_input(P->d_slices, P->B, x, s0, N, A[0], st));
  HIP_TRY(cnn::launch_slice_bias(C->d_p + C->ob[1], C->d_p + C->oWt, tau, s0, C->nb, P->B, kCnnTauStride,
                                 sbias, st));
  const int grid = conv_grid(P);
  for (int l = 1; l <= kLayers; ++l) {
    cnn::ConvArgs a = conv_args(P);
    a.in = A[l - 1];
    a.w = C->d_wf[l];
    a.bias = l == 1 ? nullptr : C->d_p + C->ob[l];
    if (l < kLayers) {
      a.sbias = l == 1 ? sbias : nullptr;
      a.out = A[l];
      HIP_TRY(cnn::launch_conv(a, l == 1 ? 8 : kC, 3, cnn::CV_RELU, grid, st));
    } else {
      a.resid = x;
      a.s0 = s0;
      a.img_out = xo;
      HIP_TRY(cnn::launch_conv(a, kC, 1, cnn::CV_LAST, grid, st));
    }
  }
  u16* g6 = at<u16>(ws, L.g6);
  HIP_TRY(cnn::launch_loss_grad(P->d_slices, P->B, xo, x0, s0, N, g6, at<float>(ws, L.lpart), loss, st));
  float* part = at<float>(ws, L.part);
  float* pbias = at<float>(ws, L.pbias);
  float* tsums = at<float>(ws, L.tsums);
  const int wgrid = std::max(1, std::min(P->ntiles, kWgradGrid));
  u16* G[2] = {at<u16>(ws, L.ga), at<u16>(ws, L.gb)};
  const u16* gcur = g6;
  for (int l = kLayers; l >= 1; --l) {
    const LayerGeom g = geom(l);
    cnn::WgradArgs w;
    std::memset(&w, 0, sizeof(w));
    w.slices = P->d_slices;
    w.tiles = P->d_tiles;
    w.ntiles = P->ntiles;
    w.dz = gcur;
    w.dzc = l == kLayers ? 8 : kC;
    w.cout = g.cout;
    w.h = A[l - 1];
    w.part = part;
    w.part_bias = pbias;
    w.tile_sums = l == 1 ? tsums : nullptr;
    HIP_TRY(cnn::launch_wgrad(w, l, wgrid, st));
    const int rows = l == kLayers ? 16 : kC;
    const int cols = l == 1 ? 80 : 432;
    HIP_TRY(cnn::launch_reduce_wgrad(part, pbias, wgrid, rows, cols, g.cinp, g.cout, g.cin,
                                     at<float>(ws, L.rstage), C->d_g + C->oW[l], C->d_g + C->ob[l], st));
    if (l == 1) {
      HIP_TRY(cnn::launch_wt_grad(tsums, P->d_tile_off, tau, s0, C->nb, P->B, kCnnTauStride, C->d_g + C->oWt,
                                  st));
      break;
    }
    // input gradient of layer l, masked by the ReLU pattern of layer l-1
    cnn::ConvArgs a = conv_args(P);
    a.in = gcur;
    a.w = C->d_wd[l];
    a.mask = A[l - 1];
    a.out = G[l & 1];
    HIP_TRY(cnn::launch_conv(a, l == kLayers ? 8 : kC, 3, cnn::CV_MASK, grid, st));
    gcur = G[l & 1];
  }
  C->step += 1;
  const double c1 = 1.0 - std::pow(0.9, C->step), c2 = 1.0 - std::pow(0.999, C->step);
  HIP_TRY(cnn::launch_adam(C->d_p, C->d_g, C->d_m, C->d_v, (int)C->n, lr, (float)c1, (float)c2, st));
  return repack(C, st);
}

// Algorithm 1 with the judged learned denoiser.
vdamp_status enqueue_learned(vdamp_plan_t* P, const vdamp_cnn_t* C, hipStream_t st, void* ws,
                             void* cws, const float2* y, const uint8_t* mask, const float* p,
                             const float* sigma2, int iters, int learned_from, int judge,
                             unsigned long long seed, float2* x_hat, float* trace, bool timing) {
  const Ws w = layout(P, ws);
  const CnnWs L = cnn_layout(P, VDAMP_CNN_WS_SOLVE);
  Launcher Lr{P, st, timing};
  const int check = (P->flags & VDAMP_FLAG_CHECK_FINITE) ? 1 : 0;
  float* s0 = at<float>(cws, L.s0);
  int* sel = at<int>(cws, L.sel);
  float2* xi = at<float2>(cws, L.xi);
  float2* ti = at<float2>(cws, L.ti);
  float2* xo = at<float2>(cws, L.xo2);
  float2* to = at<float2>(cws, L.to);
  LAUNCH(Lr, VDAMP_PASS_PREP, launch_prep(mask, p, y, w.wgt, P->ntot, check, w.bad, st));
  HIP_TRY(launch_scale(P->d_slices, P->B, y, w.wgt, s0, st));
  KArgs a = base_args(P, w);
  a.y = y;
  a.sigma2 = sigma2;
  a.out = x_hat;
  a.trace = trace;
  a.smin = at<float>(cws, L.smin);
  a.sel = sel;
  a.jpart = at<float>(cws, L.jpart);
  a.seed = seed;
  a.r2 = w.r2;  // w_cnn of the current iteration
  for (int k = 0; k < iters; ++k) {
    a.iter = k;
    const bool prev_learned = k > 0 && k - 1 >= learned_from;  // the Onsager correction used the judge
    if (k > 0) {
      a.mode = prev_learned ? RS_RTILDE_L : RS_RTILDE;
      LAUNCH(Lr, VDAMP_PASS_ROWS_SYNTH, launch_rows_synth_all(P, a, st));
    }
    a.mode = k ? CM_VDAMP : CM_VDAMP_FIRST;
    LAUNCH(Lr, VDAMP_PASS_COLS, launch_cols_all(P, a, st));
    a.mode = k == 0 ? RA_VDAMP_FIRST : (prev_learned ? RA_LEARNED : RA_VDAMP);
    LAUNCH(Lr, VDAMP_PASS_ROWS_ANAL, launch_rows_anal_all(P, a, st));
    LAUNCH(Lr, VDAMP_PASS_SURE, launch_sure_all(P, a, w.big, st));
    if (k < learned_from) continue;  // soft thresholding only in this iteration
    // learned denoiser on r_k: x = Psi^H r, t = Psi^H b, f(x), J_f t
    KArgs s = a;
    s.work = P->d_work_rows; s.nwork = P->nrows;
    s.mode = RS_PLAIN; s.out = xi;
    LAUNCH(Lr, VDAMP_PASS_DENOISER, launch_rows_synth(s, P->ept, 0, P->lds_rows, st));
    s.mode = RS_PROBE; s.out = ti;
    LAUNCH(Lr, VDAMP_PASS_DENOISER, launch_rows_synth(s, P->ept, 0, P->lds_rows, st));
    HIP_TRY(Lr.begin(VDAMP_PASS_CNN));
    vdamp_status e = enqueue_forward(C, P, L, cws, xi, w.tau, kMaxBands, s0, xo, ti, to, st);
    if (e != VDAMP_OK) return e;
    HIP_TRY(Lr.end());
    // coefficients of f(x) into r2 with the judge's partial sums, then the judge
    s.X = xo;
    LAUNCH(Lr, VDAMP_PASS_DENOISER, launch_wave_anal(s, P->ept, 0, P->lds_rows, st));
    s.X = to;
    LAUNCH(Lr, VDAMP_PASS_DENOISER, launch_wave_anal(s, P->ept, 1, P->lds_rows, st));
    LAUNCH(Lr, VDAMP_PASS_DENOISER, launch_judge(a, P->nrowstrips, judge, sel, at<float>(cws, L.jout), st));
  }
  if (iters > 0) {
    a.mode = iters - 1 >= learned_from ? RS_WHAT_L : RS_WHAT;
    LAUNCH(Lr, VDAMP_PASS_ROWS_SYNTH, launch_rows_synth_all(P, a, st));
  }
  a.mode = iters > 0 ? CM_OUTPUT : CM_ZEROFILL;
  LAUNCH(Lr, VDAMP_PASS_COLS, launch_cols_all(P, a, st));
  a.mode = RA_IMAGE;
  LAUNCH(Lr, VDAMP_PASS_ROWS_ANAL, launch_rows_anal_all(P, a, st));
  return VDAMP_OK;
}

vdamp_status check_cnn(vdamp_cnn_h cnn, vdamp_plan_h plan) {
  if (!cnn || !plan) return fail(VDAMP_ERR_ARG, "denoiser and plan must be non-null");
  if (plan->ortho || plan->dim3 || plan->grp > 1)
    return fail(VDAMP_ERR_UNSUPPORTED, "the learned denoiser runs on 2D Haar plans without groups only");
  if (cnn->nb != plan->nbands)
    return fail(VDAMP_ERR_ARG, "denoiser built for " + std::to_string(cnn->nb) + " bands, plan has " +
                                   std::to_string(plan->nbands));
  return VDAMP_OK;
}

}  // namespace

extern "C" {

vdamp_status vdamp_cnn_create(vdamp_cnn_h* cnn, int32_t nbands) {
  g_err.clear();
  if (!cnn) return fail(VDAMP_ERR_ARG, "null pointer argument");
  *cnn = nullptr;
  if (nbands < 4 || nbands > 13 || (nbands - 1) % 3)
    return fail(VDAMP_ERR_ARG, "nbands must be 1 + 3 levels with levels in 1..4");
  vdamp_cnn_t* C = new vdamp_cnn_t();
  static std::atomic<unsigned long long> next_id{1};
  C->id = next_id.fetch_add(1);
  C->nb = nbands;
  long long o = 0;
  for (int l = 1; l <= kLayers; ++l) {
    const LayerGeom g = geom(l);
    C->oW[l] = o; o += (long long)g.cout * g.cin * 9;
    C->ob[l] = o; o += g.cout;
    if (l == 1) { C->oWt = o; o += (long long)kC * nbands; }
  }
  C->n = o;
  hipError_t e = hipSuccess;
  for (float** pp : {&C->d_p, &C->d_g, &C->d_m, &C->d_v})
    if (e == hipSuccess) e = hipMalloc((void**)pp, sizeof(float) * (size_t)o);
  for (int l = 1; l <= kLayers && e == hipSuccess; ++l) {
    const LayerGeom g = geom(l);
    e = hipMalloc((void**)&C->d_wf[l], sizeof(u16) * (size_t)g.rows * g.kpad);
    if (e == hipSuccess && l > 1) e = hipMalloc((void**)&C->d_wd[l], sizeof(u16) * (size_t)g.cin * g.dkpad);
  }
  for (float* q : {C->d_p, C->d_g, C->d_m, C->d_v})
    if (e == hipSuccess) e = hipMemset(q, 0, sizeof(float) * (size_t)o);
  if (e == hipSuccess && repack(C, nullptr) != VDAMP_OK) e = hipErrorUnknown;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_cnn(C);
    return fail(VDAMP_ERR_HIP, std::string("denoiser allocation: ") + hipGetErrorString(e));
  }
  *cnn = C;
  return VDAMP_OK;
}

vdamp_status vdamp_cnn_destroy(vdamp_cnn_h cnn) {
  g_err.clear();
  if (!cnn) return fail(VDAMP_ERR_ARG, "denoiser is null");
  free_cnn(cnn);
  return VDAMP_OK;
}

vdamp_status vdamp_cnn_param_count(vdamp_cnn_h cnn, int64_t* count) {
  g_err.clear();
  if (!cnn || !count) return fail(VDAMP_ERR_ARG, "null pointer argument");
  *count = cnn->n;
  return VDAMP_OK;
}

vdamp_status vdamp_cnn_set_params(vdamp_cnn_h cnn, hipStream_t stream, const float* params) {
  g_err.clear();
  if (!cnn || !params) return fail(VDAMP_ERR_ARG, "null pointer argument");
  const size_t bytes = sizeof(float) * (size_t)cnn->n;
  HIP_TRY(hipMemcpyAsync(cnn->d_p, params, bytes, hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipMemsetAsync(cnn->d_m, 0, bytes, stream));
  HIP_TRY(hipMemsetAsync(cnn->d_v, 0, bytes, stream));
  HIP_TRY(hipMemsetAsync(cnn->d_g, 0, bytes, stream));
  cnn->step = 0;
  return repack(cnn, stream);
}

vdamp_status vdamp_cnn_get_params(vdamp_cnn_h cnn, hipStream_t stream, float* params, float* grad) {
  g_err.clear();
  if (!cnn) return fail(VDAMP_ERR_ARG, "denoiser is null");
  const size_t bytes = sizeof(float) * (size_t)cnn->n;
  if (params) HIP_TRY(hipMemcpyAsync(params, cnn->d_p, bytes, hipMemcpyDeviceToDevice, stream));
  if (grad) HIP_TRY(hipMemcpyAsync(grad, cnn->d_g, bytes, hipMemcpyDeviceToDevice, stream));
  return VDAMP_OK;
}

vdamp_status vdamp_cnn_workspace(vdamp_cnn_h cnn, vdamp_plan_h plan, int32_t kind, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(VDAMP_ERR_ARG, "null pointer argument");
  vdamp_status s = check_cnn(cnn, plan);
  if (s != VDAMP_OK) return s;
  if (kind < VDAMP_CNN_WS_FORWARD || kind > VDAMP_CNN_WS_SOLVE) return fail(VDAMP_ERR_ARG, "unknown workspace kind");
  if (!plan->tiles_ok) return fail(VDAMP_ERR_UNSUPPORTED, "the learned denoiser needs ny and nx multiples of 16");
  *bytes = cnn_layout(plan, kind).bytes;
  return VDAMP_OK;
}

vdamp_status vdamp_cnn_forward(vdamp_cnn_h cnn, vdamp_plan_h plan, hipStream_t stream,
                               void* workspace, size_t workspace_bytes, const float* x,
                               const float* tau, const float* s0, float* x_out,
                               const float* tangent, float* jvp_out) {
  g_err.clear();
  vdamp_status s = check_cnn(cnn, plan);
  if (s != VDAMP_OK) return s;
  if (!x || !tau || !s0 || !x_out) return fail(VDAMP_ERR_ARG, "x, tau, s0 and x_out must be non-null");
  if ((tangent == nullptr) != (jvp_out == nullptr))
    return fail(VDAMP_ERR_ARG, "tangent and jvp_out must be given together");
  s = check_cnn_ws(plan, VDAMP_CNN_WS_FORWARD, workspace, workspace_bytes);
  if (s != VDAMP_OK) return s;
  return enqueue_forward(cnn, plan, cnn_layout(plan, VDAMP_CNN_WS_FORWARD), workspace,
                         reinterpret_cast<const float2*>(x), tau, kCnnTauStride, s0, reinterpret_cast<float2*>(x_out),
                         reinterpret_cast<const float2*>(tangent), reinterpret_cast<float2*>(jvp_out), stream);
}

vdamp_status vdamp_cnn_train_step(vdamp_cnn_h cnn, vdamp_plan_h plan, hipStream_t stream,
                                  void* workspace, size_t workspace_bytes, const float* x,
                                  const float* tau, const float* s0, const float* x0, float lr,
                                  float* loss) {
  g_err.clear();
  vdamp_status s = check_cnn(cnn, plan);
  if (s != VDAMP_OK) return s;
  if (!x || !tau || !s0 || !x0 || !loss) return fail(VDAMP_ERR_ARG, "x, tau, s0, x0 and loss must be non-null");
  if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(VDAMP_ERR_ARG, "lr must be finite and >= 0");
  s = check_cnn_ws(plan, VDAMP_CNN_WS_TRAIN, workspace, workspace_bytes);
  if (s != VDAMP_OK) return s;
  return enqueue_train(cnn, plan, cnn_layout(plan, VDAMP_CNN_WS_TRAIN), workspace,
                       reinterpret_cast<const float2*>(x), tau, s0, reinterpret_cast<const float2*>(x0),
                       lr, loss, stream);
}

vdamp_status vdamp_solve_learned(vdamp_plan_h plan, vdamp_cnn_h cnn, hipStream_t stream,
                                 void* workspace, size_t workspace_bytes, void* cnn_workspace,
                                 size_t cnn_workspace_bytes, const float* y, const uint8_t* mask,
                                 const float* p, const float* sigma2, int32_t iters,
                                 int32_t learned_from, int32_t judge, uint64_t seed, float* x_hat,
                                 float* trace) {
  g_err.clear();
  if (judge != VDAMP_JUDGE_SURE && judge != VDAMP_JUDGE_NONE) return fail(VDAMP_ERR_ARG, "unknown judge");
  vdamp_status s = check_cnn(cnn, plan);
  if (s != VDAMP_OK) return s;
  if (!plan->ws_bytes || !workspace) return fail(VDAMP_ERR_WORKSPACE, "workspace is null");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(VDAMP_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (workspace_bytes < plan->ws_bytes)
    return fail(VDAMP_ERR_WORKSPACE, "workspace has " + std::to_string(workspace_bytes) + " bytes, needs " +
                                         std::to_string(plan->ws_bytes));
  if (!y || !mask || !p || !sigma2 || !x_hat) return fail(VDAMP_ERR_ARG, "y, mask, p, sigma2 and x_hat must be non-null");
  if (iters < 0) return fail(VDAMP_ERR_ARG, "iters must be >= 0");
  if (learned_from < 0) return fail(VDAMP_ERR_ARG, "learned_from must be >= 0");
  s = check_cnn_ws(plan, VDAMP_CNN_WS_SOLVE, cnn_workspace, cnn_workspace_bytes);
  if (s != VDAMP_OK) return s;
  GraphKey key;
  key.kind = 2;
  key.ws = workspace;
  key.y = y;
  key.mask = mask;
  key.p = p;
  key.sig = sigma2;
  key.x = x_hat;
  key.trace = trace;
  // the captured graph holds the denoiser's device buffers: key on its unique id, not on
  // the handle's address (which a destroyed and re-created denoiser may reuse)
  key.aux_id = cnn->id;
  key.aux_ws = cnn_workspace;
  key.seed = seed;
  key.judge = judge;
  key.iters = iters;
  key.extra = learned_from;
  key.stream = stream;
  s = run_maybe_graph(plan, stream, key, [&](bool timing) {
    return enqueue_learned(plan, cnn, stream, workspace, cnn_workspace, reinterpret_cast<const float2*>(y),
                           mask, p, sigma2, iters, learned_from, judge == VDAMP_JUDGE_NONE ? 1 : 0, seed,
                           reinterpret_cast<float2*>(x_hat), trace, timing);
  });
  if (s != VDAMP_OK) return s;
  plan->state_ws = workspace;
  plan->has_state = iters > 0;
  if (plan->flags & VDAMP_FLAG_CHECK_FINITE) {
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, layout(plan, workspace).bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (bad) return fail(VDAMP_ERR_NONFINITE, "p outside (0, 1] on the sampled set, or non-finite y");
  }
  return VDAMP_OK;
}

vdamp_status vdamp_learned_export(vdamp_cnn_h cnn, vdamp_plan_h plan, hipStream_t stream,
                                  const void* cnn_workspace, int32_t* sel, float* s0,
                                  float* sure_cnn, float* alpha_cnn, float* sure_soft) {
  g_err.clear();
  vdamp_status s = check_cnn(cnn, plan);
  if (s != VDAMP_OK) return s;
  if (!cnn_workspace) return fail(VDAMP_ERR_ARG, "denoiser workspace is null");
  if (!plan->tiles_ok) return fail(VDAMP_ERR_UNSUPPORTED, "the learned denoiser needs ny and nx multiples of 16");
  const CnnWs L = cnn_layout(plan, VDAMP_CNN_WS_SOLVE);
  void* ws = const_cast<void*>(cnn_workspace);
  if (sel)
    HIP_TRY(hipMemcpy2DAsync(sel, sizeof(int) * plan->nbands, at<int>(ws, L.sel), sizeof(int) * kMaxBands,
                             sizeof(int) * plan->nbands, plan->B, hipMemcpyDeviceToDevice, stream));
  if (s0)
    HIP_TRY(hipMemcpyAsync(s0, at<float>(ws, L.s0), sizeof(float) * plan->B, hipMemcpyDeviceToDevice, stream));
  float* outs[3] = {sure_cnn, alpha_cnn, sure_soft};
  for (int i = 0; i < 3; ++i)
    if (outs[i])
      HIP_TRY(hipMemcpy2DAsync(outs[i], sizeof(float) * plan->nbands,
                               at<float>(ws, L.jout) + (size_t)i * plan->B * kMaxBands, sizeof(float) * kMaxBands,
                               sizeof(float) * plan->nbands, plan->B, hipMemcpyDeviceToDevice, stream));
  return VDAMP_OK;
}

vdamp_status vdamp_wavelet(vdamp_plan_h plan, hipStream_t stream, int32_t inverse,
                           const float* in, float* out) {
  g_err.clear();
  if (!plan || !in || !out) return fail(VDAMP_ERR_ARG, "null pointer argument");
  if (in == out) return fail(VDAMP_ERR_ARG, "in and out must not overlap");
  if (plan->ortho || plan->dim3)
    return fail(VDAMP_ERR_UNSUPPORTED, "general-wavelet and volume plans need a workspace: vdamp_wavelet_ws");
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.slices = plan->d_slices;
  a.ffts = plan->d_ffts;
  a.twiddles = plan->d_tw;
  a.levels = plan->levels;
  a.nbands = plan->nbands;
  a.batch = plan->B;
  a.work = plan->d_work_rows;
  a.nwork = plan->nrows;
  if (inverse) {
    a.mode = RS_PLAIN;
    a.r = reinterpret_cast<float2*>(const_cast<float*>(in));
    a.out = reinterpret_cast<float2*>(out);
    HIP_TRY(launch_rows_synth(a, plan->ept, 0, plan->lds_rows, stream));
  } else {
    a.X = reinterpret_cast<float2*>(const_cast<float*>(in));
    a.r2 = reinterpret_cast<float2*>(out);
    HIP_TRY(launch_wave_anal(a, plan->ept, 2, plan->lds_rows, stream));
  }
  return VDAMP_OK;
}

}  // extern "C"

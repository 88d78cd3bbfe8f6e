// Internal structures shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vdamp {

constexpr int kThreads = 256;      // threads per workgroup for every pass
constexpr int kEpt = 32;           // max complex elements per thread held by an LDS pass
constexpr int kMaxElems = kThreads * kEpt;  // complex elements an LDS tile may hold
constexpr int kMaxBands = 32;      // per-slice band slots (2D: 1 + 3 s <= 13; 3D: 1 + 7 s <= 29)
constexpr int kCnnTauStride = 16;  // row stride of the tau arrays the denoiser's entry points take
constexpr int kColW = 16;          // columns per column strip (16 complex = 128 B per row)
constexpr int kMaxRadices = 8;
constexpr int kMaxN = 512;         // largest ny / nx
constexpr int kSureSmall = 4096;   // capacity of the 256- and 512-thread search classes
constexpr int kSureClasses = 5;  // LDS classes 0..3 and the large-band search
constexpr int kSureBigClass = kSureClasses - 1;
constexpr int kSureBigMaxKeys = 65536;  // largest subband (the finest band of 512 x 512)
constexpr int kSureBigStride = kSureBigMaxKeys + kSureBigMaxKeys / 16 + 1;  // scratch floats per band
constexpr int kSureMaxKeys = 27648;// largest subband the LDS threshold search holds
constexpr int kMaxFilter = 64;     // longest lowpass filter of a general-wavelet plan

struct FftPlanDev {
  int n;                 // transform length
  int nst;               // number of Stockham stages
  int rad[kMaxRadices];  // radix of each stage (2, 3, 4 or 5)
  int tw_off;            // offset of exp(-2 pi i k / n), k < n, in the twiddle pool
};

struct SliceDev {
  long long off;         // pixel offset in packed arrays
  int ny, nx;
  int fft_y, fft_x;      // FFT plan index for column (length ny) / row (length nx)
  int ytab_off;          // 2 s tables of ny floats: L_1..L_s, H_1..H_s (y axis), then
                         // ny pairs (cos^2, sin^2)(pi k / ny)
  int xtab_off;          // 2 s tables of nx floats (x axis)
  int colstrip0;         // index of this slice's first column strip in tau_part
  int rowstrip0;         // index of this slice's first row strip (learned-denoiser partials)
  // general orthonormal wavelets (plans with a filter): FFT plans of the lengths n >> l
  // (l = 0..s), the slice's group rows in Z, and the filter responses
  int fft_yl[5], fft_xl[5];
  long long zoff;        // offset of the slice's group rows in Z (complex elements)
  int zrows;             // group rows: sum over l = 1..s of 2 (ny >> l)
  int yresp_off;         // 2 s tables of ny complex: F_{A_1..A_s}, F_{D_1..D_s} (y axis)
  int xresp_off;         // the same for nx (x axis)
  // volumes (3D plans): depth nd (1 for a 2D slice), the z-axis FFT plan and tau tables,
  // the width of the Haar bricks (2^s x 2^s x bw3); ncs = the slice's tau partial strips
  // (nx / 16 for a slice, ny nx / 16 for a volume)
  int nd;
  int fft_z;
  int ztab_off;
  int bw3;
  int ncs;
};

// Modes of the row-synthesis pass (Psi^H on row strips, then row FFT).
enum RowSynthMode : int {
  RS_RTILDE = 0,   // the Onsager correction: r_tilde = (eta(r; theta) - alpha r) / (1 - alpha)
  RS_WHAT = 1,     // eta(r; theta) (denoising step, used by the output step)
  RS_PLAIN = 2,    // r as is (FISTA momentum iterate; learned denoiser input)
  RS_RTILDE_L = 3, // the Onsager correction with the learned denoiser where the judge chose it (sel = 1)
  RS_WHAT_L = 4,   // the denoising step output with the learned denoiser where chosen
  RS_PROBE = 5,    // the Rademacher probe b of the divergence estimate (no input read)
  RS_RTILDE_G = 6, // RS_RTILDE with group soft thresholding of horizontal pairs
  RS_WHAT_G = 7    // RS_WHAT with group soft thresholding of horizontal pairs
};

// Modes of the column k-space pass.
enum ColMode : int {
  CM_VDAMP = 0,        // z = y - X on Omega, v = z / p, tau partials
  CM_VDAMP_FIRST = 1,  // same with X = 0 (r_tilde_0 = 0)
  CM_OUTPUT = 2,       // (1 - m) X + m y (output step)
  CM_ZEROFILL = 3,     // y (iters = 0)
  CM_FISTA = 4,        // m (y - X)
  CM_FISTA_FIRST = 5,  // m y
  CM_FISTA_OBJ = 6     // forward column FFT only: sum over Omega of |y - X|^2 per strip
};

// Modes of the row-analysis pass (row IFFT, then Psi on row strips).
enum RowAnalMode : int {
  RA_VDAMP = 0,        // r_k = r_tilde_k + coefficients (r_tilde from r_{k-1})
  RA_VDAMP_FIRST = 1,  // r_0 = coefficients
  RA_IMAGE = 2,        // no wavelet: write the image rows (the output step's image)
  RA_FISTA = 3,        // w = eta(v + g; lambda); v' = w + beta (w - w_prev)
  RA_FISTA_FIRST = 4,
  RA_LEARNED = 5,      // as RA_VDAMP with r_tilde from the judged denoiser (RS_RTILDE_L)
  RA_VDAMP_G = 6       // as RA_VDAMP with r_tilde from group soft thresholding of pairs
};

// Extra modes of the general-wavelet passes (Psi and Psi^H on their own).
enum OrthoMode : int {
  OS_IMAGE = 10,   // synthesis pass: row DFTs of image rows (a.r) into X
  OC_SYNTH = 11,   // column pass: from the group rows to the image rows of X (no k-space step)
  OC_ANAL = 12,    // column pass: from the row DFTs in X to the group rows (no k-space step)
  OA_COEF = 13,    // analysis pass: the coefficients themselves, into a.out
  AX_Y_FWD = 14,   // volumes: DFTs along y of a strip
  AX_Y_INV = 15    // volumes: inverse DFTs along y
};

struct KArgs {
  const SliceDev* slices;
  const FftPlanDev* ffts;
  const float2* twiddles;
  const float* tables;       // tau weight tables
  const int2* work;          // work items of this launch
  int nwork;
  int levels;
  int nbands;
  int batch;
  // data
  const float2* y;
  const float* wgt;          // m / p (0 off Omega)
  const float* sigma2;       // [B]
  const float* lambda;       // [B] (FISTA)
  float2* r;                 // wavelet iterate (VDAMP r_k; FISTA v_k)
  float2* r2;                // FISTA w_{k-1}
  float2* X;                 // image / k-space scratch
  float2* out;               // x_hat for image-writing modes
  float* theta;              // [B][kMaxBands] threshold theta_b
  float* thr2;               // [B][kMaxBands] its key: the FP32 squared magnitude
  float* alpha;
  float* tau;
  float* tau_part;           // [total column strips][kMaxBands]
  float* trace;              // nullable [iters][B][nb][3]
  float* smin;               // nullable [B][kMaxBands]: minimum SURE of soft thresholding
  const int* sel;            // [B][kMaxBands]: 1 where the learned denoiser is used
  float* jpart;              // [2][total row strips][kMaxBands] learned-denoiser partial sums;
                             // FISTA with an objective trace: [total row strips] sums of |w|
  unsigned long long seed;   // probe generator seed
  int iter;
  float beta;                // FISTA momentum factor for this iteration
  int mode;
  int sure_cont;             // threshold search over every theta > 0, not only the keys
  int grp;                   // coefficients per thresholding group: 1, or 2 (horizontal pairs)
  // general orthonormal wavelets
  const float2* resp;        // filter responses (SliceDev yresp_off / xresp_off)
  float2* Z;                 // group rows: every band's row DFT times its x filter response
};

}  // namespace vdamp

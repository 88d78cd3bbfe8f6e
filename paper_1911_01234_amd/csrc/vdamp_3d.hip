// Volumes: Algorithm 1 with a 3D DFT (Section 1 allows Phi = M_Omega F with F the 2D or
// 3D DFT) and the s-level periodic orthonormal 3D Haar transform.
//
// Per iteration (arrays [nz][ny][nx] per volume, row-major, packed volume after volume):
//   k3_haar<synth>: the Onsager correction on the coefficients of a brick of 2^s x 2^s x W voxels (whole
//                   2^s cubes: the 3D Haar transform never couples different cubes), the
//                   s-level synthesis in LDS, the image brick -> X;
//   k3_rows:        DFTs of the x rows of X (in place);
//   k3_axis (y):    DFTs along y of 16-column strips (stride nx);
//   k3_axis (z):    DFTs along z of 16-column strips (stride ny nx), the k-space step of
//                   the k-space step with its tau partials, the inverse DFTs;
//   k3_axis (y), k3_rows: the inverse DFTs;
//   k3_haar<anal>:  analysis of each brick of X, + r_tilde (back-projection), -> r.
// Unnormalised DFTs; the z pass applies (nz ny nx)^(-1/2) into and out of k-space.
#include "vdamp_device.hpp"
#include "vdamp_host.h"

namespace vdamp {
namespace {

// Position (cz, cy, cx) of a 2^s cube's own s-level layout, in the cube at (gz, gy, gx)
// (cube units): the band it belongs to and its offset in the volume's 3D Mallat layout.
// Level l's octants fill [0, 2h)^3 minus [0, h)^3 with h = 2^(s-l); the kind bits say
// which coordinates lie in the upper half; each cube contributes an h^3 block of the
// band at (gz h, gy h, gx h).  The cube's (0, 0, 0) is its LLL_s coefficient.
__device__ __forceinline__ long long cube_to_global(int cz, int cy, int cx, int gz, int gy, int gx,
                                                    int s, int nd, int ny, int nx, int& band) {
  const int C = 1 << s;
  int l = 0, k = 0;
  for (int L = 1; L <= s; ++L) {
    const int h = C >> L;
    if (l == 0 && (cz >= h || cy >= h || cx >= h)) {
      l = L;
      k = (cz >= h ? 4 : 0) | (cy >= h ? 2 : 0) | (cx >= h ? 1 : 0);
    }
  }
  if (l == 0) {
    band = 0;
    return ((long long)gz * ny + gy) * nx + gx;
  }
  const int h = C >> l, bd = nd >> l, bh = ny >> l, bw = nx >> l;
  band = 1 + 7 * (s - l) + (k - 1);
  const int z = ((k & 4) ? bd : 0) + gz * h + (cz - ((k & 4) ? h : 0));
  const int y = ((k & 2) ? bh : 0) + gy * h + (cy - ((k & 2) ? h : 0));
  const int x = ((k & 1) ? bw : 0) + gx * h + (cx - ((k & 1) ? h : 0));
  return ((long long)z * ny + y) * nx + x;
}

// One level of the 3D Haar transform on every cube of a brick held in LDS as
// buf[(cz C + cy) W + j C + cx] (cube j).  Each group of 8 (a 2x2x2 block of the
// approximation, or one position of the 8 octants) is a 3D Walsh-Hadamard butterfly
// scaled by 2^(-3/2): out_k = 2^(-3/2) sum_d (-1)^popcount(k & d) in_d, bit 0 = x,
// bit 1 = y, bit 2 = z.  The transform is its own inverse, so analysis (2x2x2 block ->
// octants) and synthesis (octants -> block) differ only in where they read and write.
// Every thread reads all its groups before the workgroup writes any.
// CC, WC > 0: the cube and brick widths at compile time (then l must be a constant too
// for the index arithmetic to fold; the callers unroll the level loop).
template <bool SYNTH, int CC = 0, int WC = 0>
__device__ __forceinline__ void haar3_level(float2* buf, int C_, int W_, int l) {
  const int C = CC ? CC : C_, W = WC ? WC : W_;
  const int h = C >> l, m = W / C, h3 = h * h * h, cnt = m * h3;
  constexpr int G = 2;  // groups a thread: m h^3 <= 512 for every brick the plan builds
  float2 v[G][8];
  int gp[G];
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const int g = threadIdx.x + u * kThreads;
    gp[u] = g;
    if (g < cnt) {
      const int j = g / h3, rem = g - j * h3, pz = rem / (h * h), py = (rem / h) % h, px = rem % h;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int dz = (d >> 2) & 1, dy = (d >> 1) & 1, dx = d & 1;
        const int cz = SYNTH ? dz * h + pz : 2 * pz + dz;
        const int cy = SYNTH ? dy * h + py : 2 * py + dy;
        const int cx = SYNTH ? dx * h + px : 2 * px + dx;
        v[u][d] = buf[(cz * C + cy) * W + j * C + cx];
      }
    }
  }
  __syncthreads();
  const float q = 0.35355339059327373f;  // 2^(-3/2)
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const int g = gp[u];
    if (g < cnt) {
#pragma unroll
      for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (!(i & bit)) {
            const float2 x0 = v[u][i], x1 = v[u][i | bit];
            v[u][i] = cadd(x0, x1);
            v[u][i | bit] = csub(x0, x1);
          }
      const int j = g / h3, rem = g - j * h3, pz = rem / (h * h), py = (rem / h) % h, px = rem % h;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int dz = (d >> 2) & 1, dy = (d >> 1) & 1, dx = d & 1;
        const int cz = SYNTH ? 2 * pz + dz : dz * h + pz;
        const int cy = SYNTH ? 2 * py + dy : dy * h + py;
        const int cx = SYNTH ? 2 * px + dx : dx * h + px;
        buf[(cz * C + cy) * W + j * C + cx] = cscale(v[u][d], q);
      }
    }
  }
  __syncthreads();
}

// Synthesis (SYNTH): coefficients a.r (RS_RTILDE: the Onsager correction, RS_WHAT: the
// denoising step, RS_PLAIN: as they are) -> image brick -> a.X.  Analysis: image a.X -> coefficients; RA_VDAMP:
// r = r_tilde(r) + coefficients, RA_VDAMP_FIRST: r = coefficients, OA_COEF: a.out.
// Dynamic LDS: the brick, 2^s x 2^s x W complex (at most 4096).
template <bool SYNTH, int SL, int WC>
__device__ __forceinline__ void k3_haar_body(const KArgs& a, float2* buf, float* th_s, float* t2_s, float* al_s);

template <bool SYNTH>
__global__ void __launch_bounds__(kThreads) k3_haar(KArgs a) {
  extern __shared__ float4 lds4[];
  float2* buf = reinterpret_cast<float2*>(lds4);
  __shared__ float th_s[kMaxBands], t2_s[kMaxBands], al_s[kMaxBands];
  const int2 item = a.work[blockIdx.x];
  const int sl = item.x, s = a.levels, W = a.slices[sl].bw3;
  // the bricks of 64^3 volumes at 3 levels and 32^3 volumes at 2 levels (64 and 32 wide):
  // levels and widths at compile time
  if (s == 3 && W == 64) k3_haar_body<SYNTH, 3, 64>(a, buf, th_s, t2_s, al_s);
  else if (s == 2 && W == 32) k3_haar_body<SYNTH, 2, 32>(a, buf, th_s, t2_s, al_s);
  else k3_haar_body<SYNTH, 0, 0>(a, buf, th_s, t2_s, al_s);
}

// The brick's work: SL, WC > 0 fix the level count and the brick width at compile time.
template <bool SYNTH, int SL, int WC>
__device__ __forceinline__ void k3_haar_body(const KArgs& a, float2* buf, float* th_s, float* t2_s, float* al_s) {
  const int2 item = a.work[blockIdx.x];
  const int sl = item.x;
  const SliceDev S = a.slices[sl];
  const int nd = S.nd, ny = S.ny, nx = S.nx, s = SL ? SL : a.levels, C = 1 << s, W = WC ? WC : S.bw3;
  const int nbx = nx / W, nby = ny / C, m = W / C;
  const int bx = item.y % nbx, by = (item.y / nbx) % nby, bz = item.y / (nbx * nby);
  const int tid = threadIdx.x, mode = a.mode;
  const bool state = SYNTH ? (mode == RS_RTILDE || mode == RS_WHAT) : (mode == RA_VDAMP);
  if (state && tid < kMaxBands) {
    th_s[tid] = a.theta[sl * kMaxBands + tid];
    t2_s[tid] = a.thr2[sl * kMaxBands + tid];
    al_s[tid] = a.alpha[sl * kMaxBands + tid];
  }
  __syncthreads();
  const int n = C * C * W;
  for (int e = tid; e < n; e += kThreads) {
    const int lx = e % W, cy = (e / W) % C, cz = e / (W * C);
    if (SYNTH) {
      int band;
      const long long g = cube_to_global(cz, cy, lx % C, bz, by, bx * m + lx / C, s, nd, ny, nx, band);
      float2 v = a.r[S.off + g];
      if (mode == RS_RTILDE) v = rtilde_c(v, th_s[band], t2_s[band], al_s[band]);
      else if (mode == RS_WHAT) v = soft_c(v, th_s[band], t2_s[band]);
      buf[e] = v;
    } else {
      buf[e] = a.X[S.off + ((long long)(bz * C + cz) * ny + (by * C + cy)) * nx + bx * W + lx];
    }
  }
  __syncthreads();
  if constexpr (SL > 0 && WC > 0) {
    static_for<SL>([&](auto li) __attribute__((always_inline)) {
      constexpr int l = SYNTH ? SL - decltype(li)::value : decltype(li)::value + 1;
      haar3_level<SYNTH, (1 << SL), WC>(buf, C, W, l);
    });
  } else if (SYNTH) {
    for (int l = s; l >= 1; --l) haar3_level<true>(buf, C, W, l);
  } else {
    for (int l = 1; l <= s; ++l) haar3_level<false>(buf, C, W, l);
  }
  for (int e = tid; e < n; e += kThreads) {
    const int lx = e % W, cy = (e / W) % C, cz = e / (W * C);
    if (SYNTH) {
      a.X[S.off + ((long long)(bz * C + cz) * ny + (by * C + cy)) * nx + bx * W + lx] = buf[e];
    } else {
      int band;
      const long long g = S.off + cube_to_global(cz, cy, lx % C, bz, by, bx * m + lx / C, s, nd, ny, nx, band);
      const float2 c = buf[e];
      if (mode == RA_VDAMP) a.r[g] = cadd(rtilde_c(a.r[g], th_s[band], t2_s[band], al_s[band]), c);
      else if (mode == RA_VDAMP_FIRST) a.r[g] = c;
      else a.out[g] = c;  // OA_COEF
    }
  }
}

__device__ __forceinline__ int rows_per_item3(int rows) {
  return (rows % 8 == 0) ? 8 : (rows % 4 == 0) ? 4 : (rows % 2 == 0) ? 2 : 1;
}

// DFTs (INV: inverse) of the x rows item.y .. item.y + rpi - 1 of a.X, written back to
// a.X, or to a.out when TO_OUT (output step's image).  Dynamic LDS: rpi x nx complex.
template <bool INV, bool TO_OUT>
__global__ void __launch_bounds__(kThreads) k3_rows(KArgs a) {
  extern __shared__ float4 lds4[];
  float2* buf = reinterpret_cast<float2*>(lds4);
  __shared__ float2 tw_s[kMaxN];
  const int2 item = a.work[blockIdx.x];
  const SliceDev S = a.slices[item.x];
  const int nx = S.nx, rpi = rows_per_item3(S.nd * S.ny), tid = threadIdx.x;
  const FftPlanDev& P = a.ffts[S.fft_x];
  load_twiddles(tw_s, P, a.twiddles);
  const long long base = S.off + (long long)item.y * nx;
  for (int e = tid; e < rpi * nx; e += kThreads) buf[e] = a.X[base + e];
  __syncthreads();
  fft_lines<INV, false, 16>(buf, P, rpi, nx, 1, tw_s);
  float2* dst = TO_OUT ? a.out : a.X;
  for (int e = tid; e < rpi * nx; e += kThreads) dst[base + e] = buf[e];
}

// DFTs along y (AXIS_Y_FWD / AXIS_Y_INV) or z of a 16-column strip.  Along z the modes
// are those of the 2D column pass: CM_VDAMP (forward DFT, the k-space step with tau partials,
// inverse DFT), CM_VDAMP_FIRST (the same with r_tilde_0 = 0: no forward DFT), CM_OUTPUT
// (output step: (1 - m) X + m y), CM_ZEROFILL (y).  Strip item.y: (outer, 16-column block)
// with outer = z for y strips, y for z strips.  Dynamic LDS: the strip (n x 16 complex)
// and, for the tau partials, the 2 s z-axis tables (nz floats each).
template <int EPT>
__global__ void __launch_bounds__(kThreads) k3_axis(KArgs a) {
  extern __shared__ float4 lds4[];
  __shared__ float2 tw_s[kMaxN];
  __shared__ float red[kThreads / 64][kMaxBands];
  const int2 item = a.work[xcd_item(blockIdx.x, gridDim.x)];
  const int sl = item.x;
  const SliceDev S = a.slices[sl];
  const int nd = S.nd, ny = S.ny, nx = S.nx, s = a.levels, tid = threadIdx.x, mode = a.mode;
  const int nxs = nx / kColW, outer = item.y / nxs, x0 = (item.y - outer * nxs) * kColW;
  const bool yaxis = (mode == AX_Y_FWD || mode == AX_Y_INV);
  const int n = yaxis ? ny : nd;
  const long long stride = yaxis ? (long long)nx : (long long)ny * nx;
  const long long base = S.off + (yaxis ? (long long)outer * ny * nx : (long long)outer * nx) + x0;
  const FftPlanDev& P = a.ffts[yaxis ? S.fft_y : S.fft_z];
  load_twiddles(tw_s, P, a.twiddles);
  float2* V = reinterpret_cast<float2*>(lds4);
  float* ztab_s = reinterpret_cast<float*>(V + n * kColW);
  const bool vd = (mode == CM_VDAMP || mode == CM_VDAMP_FIRST);
  const bool first = (mode == CM_VDAMP_FIRST || mode == CM_ZEROFILL);
  if (vd)
    for (int i = tid; i < 2 * s * nd; i += kThreads) ztab_s[i] = a.tables[S.ztab_off + i];
  const int n16 = n * kColW;
  if (!first)
    for (int e = tid; e < n16; e += kThreads) V[e] = a.X[base + (long long)(e >> 4) * stride + (e & 15)];
  __syncthreads();
  if (yaxis) {
    if (mode == AX_Y_FWD) fft_cols16<false, EPT>(V, P, tw_s);
    else fft_cols16<true, EPT>(V, P, tw_s);
    for (int e = tid; e < n16; e += kThreads) a.X[base + (long long)(e >> 4) * stride + (e & 15)] = V[e];
    return;
  }
  if (!first) fft_cols16<false, EPT>(V, P, tw_s);
  // k-space step at (kz, ky = outer, kx = x0 + c); thread t always has column c = t mod 16
  const float isq = rsqrtf((float)nd * (float)ny * (float)nx);
  const float sig2 = a.sigma2 ? a.sigma2[sl] : 0.f;
  const int c = tid & (kColW - 1), ky = outer, kx = x0 + c;
  float Q[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) Q[t] = 0.f;
  for (int e = tid; e < n16; e += kThreads) {
    const int kz = e >> 4;
    const float2 X = first ? make_float2(0.f, 0.f) : cscale(V[e], isq);
    const long long g = S.off + ((long long)kz * ny + ky) * nx + kx;
    const float2 yy = a.y[g];
    const float w = a.wgt[g];
    float2 o;
    if (vd) {
      o = make_float2(0.f, 0.f);
      if (w > 0.f) {
        const float2 z = csub(yy, X);
        o = cscale(z, w);
        const float cc = w * ((w - 1.0f) * (z.x * z.x + z.y * z.y) + sig2);
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (t < 2 * s) Q[t] = fmaf(ztab_s[t * nd + kz], cc, Q[t]);
      }
    } else if (mode == CM_OUTPUT) {
      o = (w > 0.f) ? yy : X;
    } else {  // CM_ZEROFILL
      o = yy;
    }
    V[e] = cscale(o, isq);
  }
  if (vd) {
    // tau_b partial = sum over the strip's columns of Ztab_b-weighted sums times
    // Ytab_b(ky) Xtab_b(kx) (S_b is separable: S_b = Z_b(kz) Y_b(ky) X_b(kx))
    const float* ytab = a.tables + S.ytab_off;
    const float* xtab = a.tables + S.xtab_off;
    const int lane = tid & 63, wid = tid >> 6;
    float vb[32];  // this lane's term of every band (1 + 7 s <= 29 bands)
#pragma unroll
    for (int b = 0; b < 32; ++b) {
      vb[b] = 0.f;
      if (b < a.nbands) {
        int tz, ty, tx;
        if (b == 0) { tz = ty = tx = s - 1; }
        else {
          const int l = s - (b - 1) / 7, k = (b - 1) % 7 + 1;
          tz = (k & 4) ? s + l - 1 : l - 1;
          ty = (k & 2) ? s + l - 1 : l - 1;
          tx = (k & 1) ? s + l - 1 : l - 1;
        }
        float qv = 0.f;
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (t == tz) qv = Q[t];
        vb[b] = qv * ytab[ty * ny + ky] * xtab[tx * nx + kx];
      }
    }
    const float part = wave_sum_rs<32>(vb);  // band (lane >> 1) & 31
    const int bl = (lane >> 1) & 31;
    if ((lane & 1) == 0 && bl < a.nbands) red[wid][bl] = part;
  }
  __syncthreads();
  if (vd && tid < a.nbands) {
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) sum += red[w][tid];
    a.tau_part[(S.colstrip0 + item.y) * kMaxBands + tid] = sum;
  }
  fft_cols16<true, EPT>(V, P, tw_s);
  for (int e = tid; e < n16; e += kThreads) a.X[base + (long long)(e >> 4) * stride + (e & 15)] = V[e];
}

}  // namespace

size_t k3_axis_lds_bytes(int maxn, int maxnd, int s) {
  return sizeof(float2) * (size_t)maxn * kColW + sizeof(float) * (size_t)2 * s * maxnd;
}

hipError_t set_lds_limits_3d(size_t haar, size_t rows, size_t axis) {
  hipError_t e = hipSuccess;
  const void* hk[] = {(const void*)k3_haar<true>, (const void*)k3_haar<false>};
  for (const void* f : hk)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)haar);
  const void* rk[] = {(const void*)k3_rows<false, false>, (const void*)k3_rows<true, false>,
                      (const void*)k3_rows<true, true>};
  for (const void* f : rk)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rows);
  const void* ak[] = {(const void*)k3_axis<16>, (const void*)k3_axis<32>};
  for (const void* f : ak)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)axis);
  return e;
}

hipError_t launch_k3_haar(const KArgs& a, bool synth, size_t lds, hipStream_t st) {
  if (a.nwork <= 0) return hipSuccess;
  if (synth)
    hipLaunchKernelGGL((k3_haar<true>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  else
    hipLaunchKernelGGL((k3_haar<false>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_k3_rows(const KArgs& a, bool inv, bool to_out, size_t lds, hipStream_t st) {
  if (a.nwork <= 0) return hipSuccess;
  if (!inv)
    hipLaunchKernelGGL((k3_rows<false, false>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  else if (!to_out)
    hipLaunchKernelGGL((k3_rows<true, false>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  else
    hipLaunchKernelGGL((k3_rows<true, true>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_k3_axis(const KArgs& a, int ept, size_t lds, hipStream_t st) {
  if (a.nwork <= 0) return hipSuccess;
  if (ept == 16)
    hipLaunchKernelGGL((k3_axis<16>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  else
    hipLaunchKernelGGL((k3_axis<32>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

}  // namespace vdamp

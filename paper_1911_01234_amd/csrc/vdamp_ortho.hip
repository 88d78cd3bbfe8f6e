// General orthonormal wavelets (Algorithm 1 needs only an orthogonal Psi), applied in
// the Fourier domain and fused with the passes of the iteration.
//
// For a periodic two-channel orthonormal filter bank (lowpass h, highpass g), the
// level-l basis functions of a band are the 2^l-shifts of one function whose n-point
// (unnormalised) DFT is F_{A_l}(k) = prod_{i<l} H(2^i k) for the scaling function and
// F_{D_l}(k) = prod_{i<l-1} H(2^i k) G(2^(l-1) k) for the wavelet, H and G the n-point
// DFTs of h and g.  Synthesis along one axis is therefore
//     X(k) = sum_b F_b(k) W_b(k mod m_b)      (W_b: m_b-point DFT of band b's samples),
// and analysis, its adjoint up to the factor 1/n, folds the 2^l aliases of a band:
//     W_b(k') = sum_{j < 2^l} conj(F_b(k' + j m_b)) X(k' + j m_b).
// Any filter length works, the periodic wrap included, and no strip needs a halo.
//
// In 2D every band of the Mallat layout is a y-filter times an x-filter of one level.
// Bands sharing a y-filter form a group: A_l = {LH_l} (plus LL_s when l = s) and
// D_l = {HL_l, HH_l}.  A group row i is the sum over the group's bands of
// F^x_b(kx) x (DFT of row i of band b)(kx mod m): a full row of x frequencies.
//   k_osynth: the Onsager correction (or the denoising step) on the coefficients,
//             band-row DFTs, group rows -> Z;
//   k_ocols:  per 16-column strip, each group column's DFT times its y response summed
//             into k-space, the k-space step with its tau partials, then
//             the fold back into group columns and their inverse DFTs -> Z (or, for
//             the output step, the full inverse column DFT -> X);
//   k_oanal:  each group row folded back into its bands, inverse DFTs, + r_tilde (back-projection).
// Scaling: every DFT here is unnormalised; the column pass applies (ny nx)^(-1/2) once
// on the way into k-space and once on the way out, so the round trip is unitary.
#include "vdamp_device.hpp"
#include "vdamp_host.h"

namespace vdamp {
namespace {

// Group rows of one work item: the largest of 8, 4, 2, 1 that divides the group's rows.
__device__ __forceinline__ int rows_per_item(int ng) {
  return (ng % 8 == 0) ? 8 : (ng % 4 == 0) ? 4 : (ng % 2 == 0) ? 2 : 1;
}

// Group of group row `grow` of a slice (groups in the order A_1, D_1, A_2, ..., D_s):
// level l, kind (0: y filter A_l, 1: D_l), its rows ng = ny >> l, its first row goff.
__device__ __forceinline__ void group_of(int grow, int ny, int s, int& l, int& kind, int& ng,
                                         int& goff) {
  int off = 0;
  l = s; kind = 1; ng = ny >> s; goff = 0;
  for (int L = 1; L <= s; ++L)
    for (int k = 0; k < 2; ++k) {
      const int n = ny >> L;
      if (grow >= off && grow < off + n) { l = L; kind = k; ng = n; goff = off; }
      off += n;
    }
}

// Segment j of a group row: j = 0 lies at column 0 with x filter A_l, j = 1 at column
// m = nx >> l with x filter D_l.  Group A_l (l < s) has only segment 1 (LH_l); group
// A_s has LL_s and LH_s; group D_l has HL_l and HH_l.
__device__ __forceinline__ int seg_band(int l, int kind, int j, int s) {
  const int base = 1 + 3 * (s - l);
  return kind ? base + 1 + j : (j ? base : 0);
}
// response / tau-table index of a filter: A_l -> l - 1, D_l -> s + l - 1
__device__ __forceinline__ int filt_index(int l, int hi, int s) { return hi ? s + l - 1 : l - 1; }

__device__ __forceinline__ float2 conj_mul(float2 f, float2 v) {  // conj(f) v
  return make_float2(f.x * v.x + f.y * v.y, f.x * v.y - f.y * v.x);
}


// ------------------------------------------------------------------ synthesis
template <int NXC, int LC>
__device__ __forceinline__ void osynth_group(const KArgs& a, const SliceDev& S, float2* buf, float2* tw_s, int sl,
                                             int item_y, int l_, int kind, int ng, int goff);

__global__ void __launch_bounds__(kThreads) k_osynth(KArgs a) {
  extern __shared__ float4 lds4[];
  float2* buf = reinterpret_cast<float2*>(lds4);
  __shared__ float2 tw_s[kMaxN];
  const int2 item = a.work[blockIdx.x];
  const int sl = item.x;
  const SliceDev S = a.slices[sl];
  const int ny = S.ny, nx = S.nx, s = a.levels, tid = threadIdx.x, mode = a.mode;
  if (mode == OS_IMAGE) {  // row DFTs of image rows item.y .. item.y + rpi - 1, into X
    const int rpi = rows_per_item(ny);
    const FftPlanDev& P = a.ffts[S.fft_x];
    load_twiddles(tw_s, P, a.twiddles);
    const long long base = S.off + (long long)item.y * nx;
    for (int e = tid; e < rpi * nx; e += kThreads) buf[e] = a.r[base + e];
    __syncthreads();
    fft_lines<false, false, 16>(buf, P, rpi, nx, 1, tw_s);
    for (int e = tid; e < rpi * nx; e += kThreads) a.X[base + e] = buf[e];
    return;
  }
  int l, kind, ng, goff;
  group_of(item.y, ny, s, l, kind, ng, goff);
  // 256-wide slices of 4-level plans: the level's lengths fixed at compile time
  if (nx == 256 && s == 4) {
    if (l == 1) osynth_group<256, 1>(a, S, buf, tw_s, sl, item.y, l, kind, ng, goff);
    else if (l == 2) osynth_group<256, 2>(a, S, buf, tw_s, sl, item.y, l, kind, ng, goff);
    else if (l == 3) osynth_group<256, 3>(a, S, buf, tw_s, sl, item.y, l, kind, ng, goff);
    else osynth_group<256, 4>(a, S, buf, tw_s, sl, item.y, l, kind, ng, goff);
  } else {
    osynth_group<0, 0>(a, S, buf, tw_s, sl, item.y, l, kind, ng, goff);
  }
}

// The group-row work of the synthesis pass: the Onsager correction on the band rows of the group rows,
// their DFTs, times the x responses, into Z.  NXC, LC > 0: the slice width and the level
// at compile time.
template <int NXC, int LC>
__device__ __forceinline__ void osynth_group(const KArgs& a, const SliceDev& S, float2* buf, float2* tw_s, int sl,
                                             int item_y, int l_, int kind, int ng, int goff) {
  const int ny = S.ny, nx = NXC ? NXC : S.nx, s = LC ? 4 : a.levels, tid = threadIdx.x, mode = a.mode;
  const int l = LC ? LC : l_;
  const int rpi = rows_per_item(ng), i0 = item_y - goff;
  const int mx = nx >> l, nseg = (kind || l == s) ? 2 : 1, j0 = 2 - nseg, seglen = nseg * mx;
  const int row0 = (kind ? (ny >> l) : 0) + i0;  // coefficient row of group row i0
  const FftPlanDev& P = a.ffts[a.slices[sl].fft_xl[l]];  // (indexing the local copy would put it in scratch)
  load_twiddles(tw_s, P, a.twiddles);
  float2* Fx = buf + 8 * nx;  // x responses of A_l and D_l
  for (int i = tid; i < 2 * nx; i += kThreads)
    Fx[i] = a.resp[S.xresp_off + filt_index(l, i >= nx, s) * nx + (i >= nx ? i - nx : i)];
  const float* th = a.theta + sl * kMaxBands;
  const float* t2 = a.thr2 + sl * kMaxBands;
  const float* al = a.alpha + sl * kMaxBands;
  for (int e = tid; e < rpi * seglen; e += kThreads) {
    const int rr = e / seglen, rem = e - rr * seglen, js = rem / mx, c = rem - js * mx;
    const int j = j0 + js, b = seg_band(l, kind, j, s);
    const float2 v = a.r[S.off + (long long)(row0 + rr) * nx + j * mx + c];
    float2 o = v;
    if (mode == RS_RTILDE) o = rtilde_c(v, th[b], t2[b], al[b]);
    else if (mode == RS_WHAT) o = soft_c(v, th[b], t2[b]);
    buf[e] = o;  // line rr * nseg + js, sample c
  }
  __syncthreads();
  if constexpr (NXC > 0 && LC > 0)
    fft_rows_n<false, 16, (NXC >> LC)>(buf, rpi * nseg, mx, tw_s);
  else
    fft_lines<false, false, 16>(buf, P, rpi * nseg, mx, 1, tw_s);
  for (int e = tid; e < rpi * nx; e += kThreads) {
    const int rr = e / nx, kx = e - rr * nx, k = kx % mx;
    float2 acc = make_float2(0.f, 0.f);
    for (int js = 0; js < nseg; ++js)
      acc = cadd(acc, cmul(Fx[(j0 + js) * nx + kx], buf[(rr * nseg + js) * mx + k]));
    a.Z[S.zoff + (long long)(item_y + rr) * nx + kx] = acc;
  }
}

// ------------------------------------------------------------------ columns
// Thread t owns column c = t mod 16 of the strip and the k-space rows q + 16 j (q = t / 16,
// j < ny / 16): the sum over groups accumulates in its registers, and the strip goes to
// LDS once, after the k-space step, for the folds.  Dynamic LDS: the k-space strip V
// (ny x 16), one group column block G (ny/2 x 16; during the k-space step it holds the
// 2 s y-axis tau tables instead, ny floats each) and the y responses (2 s x ny complex).
// SL > 0, NYC > 0: every slice of the launch has NYC rows (a power of two) and the plan
// SL levels, so the group loops unroll and every DFT runs with its length fixed at
// compile time.
template <int EPT, int SL = 0, int NYC = 0>
__global__ void __launch_bounds__(kThreads) k_ocols(KArgs a) {
  extern __shared__ float4 lds4[];
  __shared__ float2 tw_s[2 * kMaxN];
  __shared__ float red[kThreads / 64][kMaxBands];
  const int2 item = a.work[xcd_item(blockIdx.x, gridDim.x)];
  const int sl = item.x;
  const SliceDev S = a.slices[sl];
  const int ny = NYC ? NYC : S.ny, nx = S.nx, c0 = item.y * kColW, s = SL ? SL : a.levels;
  const int tid = threadIdx.x, mode = a.mode;
  float2* V = reinterpret_cast<float2*>(lds4);
  float2* G = V + ny * kColW;
  float2* Fy = G + (ny / 2) * kColW;
  float* ytab_s = reinterpret_cast<float*>(G);  // 2 s ny floats <= the ny/2 x 16 block
  const bool vd = (mode == CM_VDAMP || mode == CM_VDAMP_FIRST);
  const bool in_zero = (mode == CM_VDAMP_FIRST || mode == CM_ZEROFILL);
  const bool in_plain = (mode == OC_ANAL);
  const bool out_plain = (mode == CM_OUTPUT || mode == CM_ZEROFILL || mode == OC_SYNTH);
  // twiddles of the lengths ny >> l, l = 0..s, one after another: those of length
  // ny >> l start at twoff(l) = sum_{j<l} ny >> j.  The plans are read from the slice
  // descriptor in global memory (indexing the local copy by l would put it in scratch).
  const int* fyl = a.slices[sl].fft_yl;
  auto twoff = [ny](int l) { return l ? 2 * ny - (ny >> (l - 1)) : 0; };
  for (int l = 0; l <= s; ++l) {
    const FftPlanDev& P = a.ffts[fyl[l]];
    for (int i = tid; i < P.n; i += kThreads) tw_s[twoff(l) + i] = a.twiddles[P.tw_off + i];
  }
  // the column DFT of level l (length ny >> l) on buf: NG > 0 is that length at compile time
  auto col_fft = [&](auto inv, auto ngc, float2* buf, int l) __attribute__((always_inline)) {
    constexpr bool INV = decltype(inv)::value;
    constexpr int NG = decltype(ngc)::value;
    if constexpr (NG > 0)
      fft_cols16_n<INV, EPT, NG>(buf, tw_s + twoff(l));
    else
      fft_cols16<INV, EPT>(buf, a.ffts[fyl[l]], tw_s + twoff(l));
  };
  // group loops: (l, kind) for l = 1 .. s, kind = 0, 1, in that order
  auto for_groups = [&](auto&& body) __attribute__((always_inline)) {
    if constexpr (SL > 0 && NYC > 0) {
      // a loop over the levels (unrolled, it would keep all groups' values live), each
      // level's body with its lengths fixed at compile time
      static_assert(SL <= 4, "levels");
#pragma unroll 1
      for (int l = 1; l <= SL; ++l)
#pragma unroll 1
        for (int kind = 0; kind < 2; ++kind) {
          if (l == 1) body(1, kind, std::integral_constant<int, (NYC >> 1)>{});
          else if (l == 2) body(2, kind, std::integral_constant<int, (NYC >> 2)>{});
          else if (l == 3) body(3, kind, std::integral_constant<int, (NYC >> 3)>{});
          else body(4, kind, std::integral_constant<int, (NYC >> 4)>{});
        }
    } else {
      for (int l = 1; l <= s; ++l)
        for (int kind = 0; kind < 2; ++kind) body(l, kind, std::integral_constant<int, 0>{});
    }
  };
  using FwdT = std::false_type;
  using InvT = std::true_type;
  using FullN = std::integral_constant<int, (SL > 0 && NYC > 0) ? NYC : 0>;
  for (int i = tid; i < 2 * s * ny; i += kThreads) Fy[i] = a.resp[S.yresp_off + i];
  const int n16 = ny * kColW;
  const int c = tid & (kColW - 1), q = tid >> 4;
  float2 acc[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) acc[j] = make_float2(0.f, 0.f);
  // ---- into k-space
  if (in_plain) {
    for (int e = tid; e < n16; e += kThreads) V[e] = a.X[S.off + (long long)(e >> 4) * nx + c0 + (e & 15)];
    __syncthreads();
    col_fft(FwdT{}, FullN{}, V, 0);
#pragma unroll
    for (int j = 0; j < EPT; ++j)
      if (q + 16 * j < ny) acc[j] = V[(q + 16 * j) * kColW + c];
  } else if (!in_zero) {
    int goff = 0;
    for_groups([&](int l, int kind, auto ngc) __attribute__((always_inline)) {
      const int ng = ny >> l;
      __syncthreads();  // G is free (and the tables are in)
      for (int e = tid; e < ng * kColW; e += kThreads)
        G[e] = a.Z[S.zoff + (long long)(goff + (e >> 4)) * nx + c0 + (e & 15)];
      __syncthreads();
      col_fft(FwdT{}, ngc, G, l);
      const float2* F = Fy + filt_index(l, kind, s) * ny;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int ky = q + 16 * j;
        if (ky < ny) acc[j] = cadd(acc[j], cmul(F[ky], G[(ky % ng) * kColW + c]));
      }
      goff += ng;
    });
  }
  __syncthreads();  // V and G free
  if (vd) {
    for (int i = tid; i < 2 * s * ny; i += kThreads) ytab_s[i] = a.tables[S.ytab_off + i];
    __syncthreads();
  }
  // ---- the k-space step (or the output step, or nothing) on the strip
  const float isq = rsqrtf((float)ny * (float)nx);
  const float sig2 = a.sigma2 ? a.sigma2[sl] : 0.f;
  const int kx = c0 + c;
  float Q[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) Q[t] = 0.f;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int ky = q + 16 * j;
    if (ky >= ny) continue;
    const float2 X = cscale(acc[j], isq);
    float2 o = X;
    if (mode != OC_SYNTH && mode != OC_ANAL) {
      const long long g = S.off + (long long)ky * nx + kx;
      const float2 yy = a.y[g];
      const float w = a.wgt[g];
      if (vd) {
        o = make_float2(0.f, 0.f);
        if (w > 0.f) {
          const float2 z = csub(yy, X);
          o = cscale(z, w);
          const float cc = w * ((w - 1.0f) * (z.x * z.x + z.y * z.y) + sig2);
#pragma unroll
          for (int t = 0; t < 8; ++t)
            if (t < 2 * s) Q[t] = fmaf(ytab_s[t * ny + ky], cc, Q[t]);
        }
      } else if (mode == CM_OUTPUT) {
        o = (w > 0.f) ? yy : X;
      } else {  // CM_ZEROFILL
        o = yy;
      }
    }
    V[ky * kColW + c] = cscale(o, isq);
  }
  if (vd) {
    // tau_b partial = sum over this strip's columns of Xtab_b(kx) sum_ky Ytab_b(ky) c
    const float* xtab = a.tables + S.xtab_off;
    const int lane = tid & 63, wid = tid >> 6;
    float vb[16];  // this lane's term of every band (1 + 3 s <= 13 bands)
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      vb[b] = 0.f;
      if (b < a.nbands) {
        int ty, tx;
        if (b == 0) { ty = s - 1; tx = s - 1; }
        else {
          const int l = s - (b - 1) / 3, k3 = (b - 1) % 3;
          ty = (k3 == 0) ? l - 1 : s + l - 1;
          tx = (k3 == 1) ? l - 1 : s + l - 1;
        }
        float qv = 0.f;
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (t == ty) qv = Q[t];
        vb[b] = qv * xtab[tx * nx + kx];
      }
    }
    const float part = wave_sum_rs<16>(vb);  // band (lane >> 2) & 15
    const int bl = (lane >> 2) & 15;
    if ((lane & 3) == 0 && bl < a.nbands) red[wid][bl] = part;
  }
  __syncthreads();
  if (vd && tid < a.nbands) {
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) sum += red[w][tid];
    a.tau_part[(S.colstrip0 + item.y) * kMaxBands + tid] = sum;
  }
  // ---- out of k-space
  if (out_plain) {
    col_fft(InvT{}, FullN{}, V, 0);
    for (int e = tid; e < n16; e += kThreads) a.X[S.off + (long long)(e >> 4) * nx + c0 + (e & 15)] = V[e];
    return;
  }
  int goff = 0;
  for_groups([&](int l, int kind, auto ngc) __attribute__((always_inline)) {
    const int ng = ny >> l, nal = 1 << l;
    const float2* F = Fy + filt_index(l, kind, s) * ny;
    for (int e = tid; e < ng * kColW; e += kThreads) {
      const int k = e >> 4, cc = e & 15;
      float2 sum = make_float2(0.f, 0.f);
      for (int j = 0; j < nal; ++j) {
        const int ky = k + j * ng;
        sum = cadd(sum, conj_mul(F[ky], V[ky * kColW + cc]));
      }
      G[e] = sum;
    }
    __syncthreads();
    col_fft(InvT{}, ngc, G, l);
    for (int e = tid; e < ng * kColW; e += kThreads)
      a.Z[S.zoff + (long long)(goff + (e >> 4)) * nx + c0 + (e & 15)] = G[e];
    __syncthreads();  // G is read before the next group overwrites it
    goff += ng;
  });
}

// ------------------------------------------------------------------ analysis
// Dynamic LDS: the item's group rows (rpi x nx), its band rows (rpi x nseg x m) and the
// x responses of A_l and D_l.
template <int NXC, int LC>
__device__ __forceinline__ void oanal_group(const KArgs& a, const SliceDev& S, float2* Zs, float2* tw_s, int sl,
                                            int item_y, int l_, int kind, int ng, int goff);

__global__ void __launch_bounds__(kThreads) k_oanal(KArgs a) {
  extern __shared__ float4 lds4[];
  float2* Zs = reinterpret_cast<float2*>(lds4);
  __shared__ float2 tw_s[kMaxN];
  const int2 item = a.work[blockIdx.x];
  const int sl = item.x;
  const SliceDev S = a.slices[sl];
  const int ny = S.ny, nx = S.nx, s = a.levels, tid = threadIdx.x, mode = a.mode;
  if (mode == RA_IMAGE) {  // inverse row DFTs of X rows item.y .. item.y + rpi - 1
    const int rpi = rows_per_item(ny);
    const FftPlanDev& P = a.ffts[S.fft_x];
    load_twiddles(tw_s, P, a.twiddles);
    const long long base = S.off + (long long)item.y * nx;
    for (int e = tid; e < rpi * nx; e += kThreads) Zs[e] = a.X[base + e];
    __syncthreads();
    fft_lines<true, false, 16>(Zs, P, rpi, nx, 1, tw_s);
    for (int e = tid; e < rpi * nx; e += kThreads) a.out[base + e] = Zs[e];
    return;
  }
  int l, kind, ng, goff;
  group_of(item.y, ny, s, l, kind, ng, goff);
  // 256-wide slices of 4-level plans: the level's lengths fixed at compile time
  if (nx == 256 && s == 4) {
    if (l == 1) oanal_group<256, 1>(a, S, Zs, tw_s, sl, item.y, l, kind, ng, goff);
    else if (l == 2) oanal_group<256, 2>(a, S, Zs, tw_s, sl, item.y, l, kind, ng, goff);
    else if (l == 3) oanal_group<256, 3>(a, S, Zs, tw_s, sl, item.y, l, kind, ng, goff);
    else oanal_group<256, 4>(a, S, Zs, tw_s, sl, item.y, l, kind, ng, goff);
  } else {
    oanal_group<0, 0>(a, S, Zs, tw_s, sl, item.y, l, kind, ng, goff);
  }
}

// The group-row work of the analysis pass: fold each group row into its bands, inverse
// DFTs of the band rows, the back-projection.  NXC, LC > 0: the slice width and the level at compile
// time (band rows of NXC >> LC samples).
template <int NXC, int LC>
__device__ __forceinline__ void oanal_group(const KArgs& a, const SliceDev& S, float2* Zs, float2* tw_s, int sl,
                                            int item_y, int l_, int kind, int ng, int goff) {
  const int ny = S.ny, nx = NXC ? NXC : S.nx, s = LC ? 4 : a.levels, tid = threadIdx.x, mode = a.mode;
  const int l = LC ? LC : l_;
  const int rpi = rows_per_item(ng), i0 = item_y - goff;
  const int mx = nx >> l, nseg = (kind || l == s) ? 2 : 1, j0 = 2 - nseg, seglen = nseg * mx;
  const int row0 = (kind ? (ny >> l) : 0) + i0, nal = 1 << l;
  float2* Ss = Zs + 8 * nx;
  float2* Fx = Ss + 8 * nx;  // x responses of A_l and D_l
  const FftPlanDev& P = a.ffts[a.slices[sl].fft_xl[l]];  // (indexing the local copy would put it in scratch)
  load_twiddles(tw_s, P, a.twiddles);
  for (int i = tid; i < 2 * nx; i += kThreads)
    Fx[i] = a.resp[S.xresp_off + filt_index(l, i >= nx, s) * nx + (i >= nx ? i - nx : i)];
  for (int e = tid; e < rpi * nx; e += kThreads) Zs[e] = a.Z[S.zoff + (long long)item_y * nx + e];
  __syncthreads();
  for (int e = tid; e < rpi * seglen; e += kThreads) {
    const int rr = e / seglen, rem = e - rr * seglen, js = rem / mx, k = rem - js * mx;
    const float2* F = Fx + (j0 + js) * nx;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < (LC ? (1 << LC) : nal); ++j)
      acc = cadd(acc, conj_mul(F[k + j * mx], Zs[rr * nx + k + j * mx]));
    Ss[e] = acc;
  }
  __syncthreads();
  if constexpr (NXC > 0 && LC > 0)
    fft_rows_n<true, 16, (NXC >> LC)>(Ss, rpi * nseg, mx, tw_s);
  else
    fft_lines<true, false, 16>(Ss, P, rpi * nseg, mx, 1, tw_s);
  const float* th = a.theta + sl * kMaxBands;
  const float* t2 = a.thr2 + sl * kMaxBands;
  const float* al = a.alpha + sl * kMaxBands;
  for (int e = tid; e < rpi * seglen; e += kThreads) {
    const int rr = e / seglen, rem = e - rr * seglen, js = rem / mx, c = rem - js * mx;
    const int j = j0 + js, b = seg_band(l, kind, j, s);
    const long long gi = S.off + (long long)(row0 + rr) * nx + j * mx + c;
    const float2 coef = Ss[e];
    if (mode == RA_VDAMP) a.r[gi] = cadd(rtilde_c(a.r[gi], th[b], t2[b], al[b]), coef);
    else if (mode == RA_VDAMP_FIRST) a.r[gi] = coef;
    else a.out[gi] = coef;  // OA_COEF
  }
}

}  // namespace

size_t ocols_lds_bytes(int maxny, int s) {
  return sizeof(float2) * (size_t)maxny * kColW + sizeof(float2) * (size_t)(maxny / 2) * kColW +
         sizeof(float2) * (size_t)2 * s * maxny;
}

hipError_t set_lds_limits_ortho(size_t synth, size_t cols, size_t anal) {
  hipError_t e = hipFuncSetAttribute((const void*)k_osynth, hipFuncAttributeMaxDynamicSharedMemorySize, (int)synth);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_ocols<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cols);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_ocols<16, 4, 256>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cols);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_ocols<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cols);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_oanal, hipFuncAttributeMaxDynamicSharedMemorySize, (int)anal);
  return e;
}

hipError_t launch_osynth(const KArgs& a, size_t lds, hipStream_t st) {
  if (a.nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_osynth, dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_ocols(const KArgs& a, int ept, int ny_all, size_t lds, hipStream_t st) {
  if (a.nwork <= 0) return hipSuccess;
  if (ept == 16 && ny_all == 256 && a.levels == 4)  // the 256-row slices of 4-level plans
    hipLaunchKernelGGL((k_ocols<16, 4, 256>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  else if (ept == 16)
    hipLaunchKernelGGL((k_ocols<16>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  else
    hipLaunchKernelGGL((k_ocols<32>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_oanal(const KArgs& a, size_t lds, hipStream_t st) {
  if (a.nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_oanal, dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

}  // namespace vdamp

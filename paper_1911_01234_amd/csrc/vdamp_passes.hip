// gfx950 kernels of the three transform passes of one iteration (Algorithm 1):
//   rows_synth  (row strip of 2^s image rows): the Onsager correction applied to r_{k-1}, Psi^H on the
//               strip (Haar never couples strips of 2^s rows), then the row FFTs.
//   cols        (column strip of 16 columns): column FFT, k-space residual,
//               density compensation P^-1, the tau estimate's partial sums
//               (S is separable per band for Haar), column IFFT.
//   rows_anal   (row strip): row IFFTs, Psi on the strip, add r_tilde_k (back-projection).
// One workgroup of 256 threads per work item; every tile is staged in LDS and moved
// with 16-byte accesses (two complex values), all of a thread's loads issued before
// the first use.  EPT (8 B elements per thread) is 16 when every tile of the plan
// holds at most 4096 complex values, else 32.
#include <vector>

#include "vdamp_device.hpp"

namespace vdamp {

// ------------------------------------------------------------------ rows_synth
// do_fft = 0 writes the image rows Psi^H r (the FISTA output).
// SL > 0: the plan's level count, fixed at compile time (four-step kernels, nx = 16 M).
template <int EPT, int M, int NT = kThreads, int SL = 0>
__global__ void __launch_bounds__(NT) k_rows_synth(KArgs a, int do_fft) {
  extern __shared__ float4 lds4[];
  float2* lds = reinterpret_cast<float2*>(lds4);
  __shared__ float2 tw_s[kMaxN];
  __shared__ float th_s[kMaxBands], t2_s[kMaxBands], al_s[kMaxBands], ia_s[kMaxBands];
  const int2 item = a.work[blockIdx.x];
  const SliceDev S = a.slices[item.x];
  constexpr int NXC = M > 0 ? 16 * M : 0;
  const int strip = item.y, s = SL ? SL : a.levels, H = 1 << s, nx = NXC ? NXC : S.nx, ny = S.ny;
  const int tid = threadIdx.x, mode = a.mode;
  if (tid < kMaxBands && a.theta) {  // null for the plain transform Psi^H
    th_s[tid] = a.theta[item.x * kMaxBands + tid];
    t2_s[tid] = a.thr2[item.x * kMaxBands + tid];
    al_s[tid] = a.alpha[item.x * kMaxBands + tid];
    ia_s[tid] = 1.0f / (1.0f - al_s[tid]);
  }
  const FftPlanDev& P = a.ffts[S.fft_x];
  if (do_fft) load_twiddles<NT>(tw_s, P, a.twiddles);
  constexpr int U = EPT / 2;
  const int half = nx >> 1, npairs = H * half;
  const float2* r = a.r + S.off;
  const bool learned = (mode == RS_RTILDE_L || mode == RS_WHAT_L);
  const float2* wc = learned ? a.r2 + S.off : nullptr;
  float4 v[U], c4[U];
  int bnd[U];
  long long gi[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * NT;
    bnd[u] = 0;
    gi[u] = 0;
    v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    c4[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p < npairs) {
      const int lr = p / half, lc = 2 * (p - lr * half);
      int b;
      const int gr = strip_to_global_t<SL, NXC>(lr, lc, strip, s, ny, nx, b);
      bnd[u] = b;
      gi[u] = (long long)gr * nx + lc;
      if (mode != RS_PROBE) v[u] = *reinterpret_cast<const float4*>(r + gi[u]);
      if (learned) c4[u] = *reinterpret_cast<const float4*>(wc + gi[u]);
    }
  }
  __shared__ int sel_s[kMaxBands];
  if (learned && tid < kMaxBands) sel_s[tid] = a.sel[item.x * kMaxBands + tid];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * NT;
    if (p < npairs) {
      const int b = bnd[u];
      float2 x0 = lo2(v[u]), x1 = hi2(v[u]);
      if (mode == RS_RTILDE) {
        x0 = rtilde_ci(x0, th_s[b], t2_s[b], al_s[b], ia_s[b]);
        x1 = rtilde_ci(x1, th_s[b], t2_s[b], al_s[b], ia_s[b]);
      } else if (mode == RS_WHAT) {
        x0 = soft_c(x0, th_s[b], t2_s[b]);
        x1 = soft_c(x1, th_s[b], t2_s[b]);
      } else if (mode == RS_RTILDE_L) {
        if (sel_s[b]) {
          x0 = rtilde_w(lo2(c4[u]), x0, al_s[b]);
          x1 = rtilde_w(hi2(c4[u]), x1, al_s[b]);
        } else {
          x0 = rtilde_ci(x0, th_s[b], t2_s[b], al_s[b], ia_s[b]);
          x1 = rtilde_ci(x1, th_s[b], t2_s[b], al_s[b], ia_s[b]);
        }
      } else if (mode == RS_WHAT_L) {
        x0 = sel_s[b] ? lo2(c4[u]) : soft_c(x0, th_s[b], t2_s[b]);
        x1 = sel_s[b] ? hi2(c4[u]) : soft_c(x1, th_s[b], t2_s[b]);
      } else if (mode == RS_PROBE) {
        x0 = probe_c(a.seed, a.iter, item.x, gi[u]);
        x1 = probe_c(a.seed, a.iter, item.x, gi[u] + 1);
      } else if (mode == RS_RTILDE_G) {  // (x0, x1): a pair x = 2j, 2j + 1 of one band row
        rtilde_pair(x0, x1, th_s[b], t2_s[b], al_s[b], ia_s[b]);
      } else if (mode == RS_WHAT_G) {
        soft_pair(x0, x1, th_s[b], t2_s[b]);
      }
      lds4[p] = pack4(x0, x1);  // LDS index lr * nx + lc = 2 p
    }
  }
  __syncthreads();
  haar_strip_synth<EPT, NT, SL, NXC>(lds, H, nx, s);
  if constexpr (M > 0) {
    if (do_fft) {  // four-step row FFT, outputs straight to X
      using F = RowFft4<M, NT>;
      float2 v[M];
      const int a16 = tid & 15, line = tid >> 4;
      if (line < H) {
#pragma unroll
        for (int b = 0; b < M; ++b) v[b] = lds[line * F::N + a16 + 16 * b];
      }
      __syncthreads();
      F::template step1<false>(v, H, tw_s, lds);
      __syncthreads();
      float2* X = a.X + S.off + (long long)strip * H * nx;
#pragma unroll
      for (int j = 0; j < F::NI; ++j) {
        float2 d[16];
        int kb, l2;
        if (F::template step2<false>(j, H, tw_s, lds, d, kb, l2)) {
#pragma unroll
          for (int ka = 0; ka < 16; ++ka) X[l2 * F::N + kb + M * ka] = d[ka];
        }
      }
      return;
    }
  } else {
    if (do_fft) fft_lines<false, false, EPT>(lds, P, H, nx, 1, tw_s);
  }
  float4* dst = reinterpret_cast<float4*>((do_fft ? a.X : a.out) + S.off + (long long)strip * H * nx);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * NT;
    if (p < npairs) dst[p] = lds4[p];
  }
}

// ------------------------------------------------------------------ cols
template <int EPT>
__global__ void __launch_bounds__(kThreads) k_cols(KArgs a) {
  extern __shared__ float4 lds4[];
  float2* lds = reinterpret_cast<float2*>(lds4);
  __shared__ float2 tw_s[kMaxN];
  __shared__ float ytab_s[8 * kMaxN];
  __shared__ float red[kThreads / 64][kMaxBands];
  const int2 item = a.work[xcd_item(blockIdx.x, gridDim.x)];
  const int sl = item.x;
  const SliceDev S = a.slices[sl];
  const int ny = S.ny, nx = S.nx, c0 = item.y * kColW, s = a.levels;
  const int tid = threadIdx.x, mode = a.mode;
  const bool first = (mode == CM_VDAMP_FIRST || mode == CM_ZEROFILL || mode == CM_FISTA_FIRST);
  const bool vd = (mode == CM_VDAMP || mode == CM_VDAMP_FIRST);
  const FftPlanDev& P = a.ffts[S.fft_y];
  load_twiddles(tw_s, P, a.twiddles);
  const int ntab = 2 * s;
  if (vd)
    for (int i = tid; i < ntab * ny; i += kThreads) ytab_s[i] = a.tables[S.ytab_off + i];
  constexpr int U = EPT / 2;
  constexpr int PPR = kColW / 2;  // column pairs per row
  const int npairs = ny * PPR;
  const long long base = S.off + c0;
  if (!first) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kThreads;
      v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (p < npairs) {
        const int row = p / PPR, cp = p % PPR;
        v[u] = *reinterpret_cast<const float4*>(a.X + base + (long long)row * nx + 2 * cp);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kThreads;
      if (p < npairs) lds4[p] = v[u];  // LDS index row * 16 + 2 cp = 2 p
    }
  }
  // measurements and weights of this thread's pairs (its column pair is fixed)
  const int cp = tid % PPR;
  float4 yv[U];
  float2 wv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * kThreads;
    yv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    wv[u] = make_float2(0.f, 0.f);
    if (p < npairs) {
      const long long g = base + (long long)(p / PPR) * nx + 2 * cp;
      yv[u] = *reinterpret_cast<const float4*>(a.y + g);
      wv[u] = *reinterpret_cast<const float2*>(a.wgt + g);
    }
  }
  __syncthreads();
  if (!first) fft_lines<false, true, EPT>(lds, P, kColW, 1, kColW, tw_s);
  const float isq = rsqrtf((float)ny * (float)nx);  // unitary scaling, once per direction
  const float sig2 = a.sigma2 ? a.sigma2[sl] : 0.f;
  float Q0[8], Q1[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) { Q0[t] = 0.f; Q1[t] = 0.f; }
  float rsum = 0.f;  // CM_FISTA_OBJ: sum over Omega of |y - X|^2
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * kThreads;
    if (p < npairs) {
      const int row = p / PPR;
      const float4 xr = first ? make_float4(0.f, 0.f, 0.f, 0.f) : lds4[p];
      float2 out[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float2 X = cscale(h ? hi2(xr) : lo2(xr), isq);
        const float2 yy = h ? hi2(yv[u]) : lo2(yv[u]);
        const float w = h ? wv[u].y : wv[u].x;
        float2 o;
        if (vd) {
          o = make_float2(0.f, 0.f);
          if (w > 0.f) {
            const float2 z = csub(yy, X);
            o = cscale(z, w);
            const float cc = w * ((w - 1.0f) * (z.x * z.x + z.y * z.y) + sig2);
#pragma unroll
            for (int t = 0; t < 8; ++t)
              if (t < ntab) {
                if (h) Q1[t] = fmaf(ytab_s[t * ny + row], cc, Q1[t]);
                else Q0[t] = fmaf(ytab_s[t * ny + row], cc, Q0[t]);
              }
          }
        } else if (mode == CM_OUTPUT) {
          o = (w > 0.f) ? yy : X;
        } else if (mode == CM_ZEROFILL) {
          o = yy;
        } else if (mode == CM_FISTA_OBJ) {
          o = make_float2(0.f, 0.f);
          if (w > 0.f) {
            const float2 z = csub(yy, X);
            rsum = fmaf(z.x, z.x, fmaf(z.y, z.y, rsum));
          }
        } else {  // FISTA: m (y - X)
          o = (w > 0.f) ? csub(yy, X) : make_float2(0.f, 0.f);
        }
        out[h] = cscale(o, isq);
      }
      lds4[p] = pack4(out[0], out[1]);
    }
  }
  if (vd) {
    // tau_b partial = sum over this strip's columns of Xtab_b(kx) sum_ky Ytab_b(ky) c
    const float* xtab = a.tables + S.xtab_off;
    const int kx = c0 + 2 * cp;
    const int lane = tid & 63, wid = tid >> 6;
    float vb[16];  // this lane's term of every band (1 + 3 s <= 13 bands)
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      vb[b] = 0.f;
      if (b < a.nbands) {
        int ty, tx;
        if (b == 0) { ty = s - 1; tx = s - 1; }
        else {
          const int l = s - (b - 1) / 3, kind = (b - 1) % 3;
          const int L = l - 1, Hh = s + l - 1;
          ty = (kind == 0) ? L : Hh;
          tx = (kind == 1) ? L : Hh;
        }
        float q0 = 0.f, q1 = 0.f;
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (t == ty) { q0 = Q0[t]; q1 = Q1[t]; }
        vb[b] = q0 * xtab[tx * nx + kx] + q1 * xtab[tx * nx + kx + 1];
      }
    }
    const float part = wave_sum_rs<16>(vb);  // band (lane >> 2) & 15
    const int bl = (lane >> 2) & 15;
    if ((lane & 3) == 0 && bl < a.nbands) red[wid][bl] = part;
  }
  if (mode == CM_FISTA_OBJ) {  // the residual's partial sum is all this mode writes
    const float part = wave_sum(rsum);
    if ((tid & 63) == 0) red[tid >> 6][0] = part;
    __syncthreads();
    if (tid == 0) {
      float acc = 0.f;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) acc += red[w][0];
      a.tau_part[(S.colstrip0 + item.y) * kMaxBands] = acc;
    }
    return;
  }
  __syncthreads();
  if (vd && tid < a.nbands) {
    float acc = 0.f;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) acc += red[w][tid];
    a.tau_part[(S.colstrip0 + item.y) * kMaxBands + tid] = acc;
  }
  fft_lines<true, true, EPT>(lds, P, kColW, 1, kColW, tw_s);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * kThreads;
    if (p < npairs)
      *reinterpret_cast<float4*>(a.X + base + (long long)(p / PPR) * nx + 2 * (p % PPR)) = lds4[p];
  }
}

// ------------------------------------------------------------------ cols, four-step
// Threads of a column workgroup: 256, or one 16-point item each (16 M) for columns
// longer than 256.
constexpr int cols4_threads(int m) { return 16 * m > kThreads ? 16 * m : kThreads; }

// Column strip of 16 columns with ny = 16 M, as two-level FFTs held in registers: the
// forward transform factors ny = 16 x M (thread (a, c) transforms rows a + 16 b,
// b < M, of column c, scales by W_ny^{a kb}, one LDS transpose, then 16-point DFTs give
// k-space rows kb + M ka), the k-space step runs on those registers, and the inverse
// factors ny = M x 16 so that it starts from exactly the rows each thread holds and
// ends, after one more transpose, on the rows the forward transform started from.
// Loads of X, y and m/p are issued at the start (y and m/p after the M-point stage for
// M > 20).
template <int M>
__global__ void __launch_bounds__(cols4_threads(M)) k_cols4(KArgs a) {
  constexpr int N = 16 * M;
  constexpr int NT = cols4_threads(M);
  constexpr int NI = (N + NT - 1) / NT;  // 16-point DFT items per thread
  constexpr int P1 = 256 + 16;                       // LDS pitch of a forward kb block
  constexpr int P2 = N + ((M % 2) ? 0 : 16);         // LDS pitch of an inverse block
  constexpr int TB = (M * P1 > 16 * P2) ? M * P1 : 16 * P2;
  __shared__ float2 tw_s[N];
  __shared__ float2 cs_s[N];  // (cos^2, sin^2)(pi ky / N) per k-space row
  __shared__ float2 tb[TB];
  __shared__ float red[NT / 64][kMaxBands];
  const int2 item = a.work[xcd_item(blockIdx.x, gridDim.x)];
  const int sl = item.x;
  const SliceDev S = a.slices[sl];
  const int nx = S.nx, c0 = item.y * kColW, s = a.levels;
  const int tid = threadIdx.x, mode = a.mode;
  const bool first = (mode == CM_VDAMP_FIRST || mode == CM_ZEROFILL || mode == CM_FISTA_FIRST);
  const bool vd = (mode == CM_VDAMP || mode == CM_VDAMP_FIRST);
  const long long base = S.off + c0;
  const int c = tid & 15, a1 = tid >> 4;
  const bool s1 = a1 < 16;  // threads of the M-point stage (all of them when NT = 256)
  // forward input: rows a1 + 16 b of column c
  float2 xin[M];
#pragma unroll
  for (int b = 0; b < M; ++b)
    xin[b] = (first || !s1) ? make_float2(0.f, 0.f) : a.X[base + (long long)(a1 + 16 * b) * nx + c];
  // y and m/p at the k-space rows kb + M ka of this thread's items: issued with the X
  // loads up to M = 20; for longer columns after the M-point stage, whose inputs then no
  // longer hold registers (two workgroups of 16 M threads fit a CU)
  constexpr bool kEarlyY = M <= 20;
  float2 yv[NI][16];
  float wv[NI][16];
#define COLS4_LOAD_YW()                                                  \
  _Pragma("unroll") for (int j = 0; j < NI; ++j) {                       \
    const int it = tid + j * NT, kb = it >> 4;                           \
    _Pragma("unroll") for (int ka = 0; ka < 16; ++ka) {                  \
      yv[j][ka] = make_float2(0.f, 0.f);                                 \
      wv[j][ka] = 0.f;                                                   \
      if (it < N) {                                                      \
        const long long g = base + (long long)(kb + M * ka) * nx + c;    \
        yv[j][ka] = a.y[g];                                              \
        wv[j][ka] = a.wgt[g];                                            \
      }                                                                  \
    }                                                                    \
  }
  if constexpr (kEarlyY) COLS4_LOAD_YW();
  const FftPlanDev& P = a.ffts[S.fft_y];
  for (int i = tid; i < N; i += NT) tw_s[i] = a.twiddles[P.tw_off + i];
  if (vd) {
    const float* cs = a.tables + S.ytab_off + 2 * s * N;
    for (int i = tid; i < N; i += NT) cs_s[i] = make_float2(cs[2 * i], cs[2 * i + 1]);
  }
  __syncthreads();
  if (!first && s1) {
    RegFft<M, false>::run(xin, tw_s, 16);
#pragma unroll
    for (int kb = 0; kb < M; ++kb) {
      float2 v = xin[kb];
      if (kb) v = cmul(v, tw_s[a1 * kb]);
      tb[kb * P1 + a1 * 16 + c] = v;
    }
  }
  if constexpr (!kEarlyY) COLS4_LOAD_YW();
#undef COLS4_LOAD_YW
  __syncthreads();
  const float isq = rsqrtf((float)N * (float)nx);
  const float sig2 = a.sigma2 ? a.sigma2[sl] : 0.f;
  // QL[j] = sum_ky P_{j+1}(ky) c, QH[j] = sum_ky P_j(ky) s_j(ky) c with c_j, s_j =
  // (cos^2, sin^2)(pi ky 2^j / N) and P_m = prod_{j<m} c_j: the y-axis tau-weight tables
  // L_{j+1} and H_{j+1} up to their factor 2^{j+1} / N, built from the row's (c_0, s_0)
  // by the double-angle identities s_{j+1} = 4 c_j s_j and c_{j+1} = 1 - s_{j+1} =
  // (c_j - s_j)^2 (products in FP32: within 3e-7 of the largest table value, against
  // 6e-8 for tables rounded from FP64)
  float QL[4], QH[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) { QL[t] = 0.f; QH[t] = 0.f; }
  float rsum = 0.f;  // CM_FISTA_OBJ: sum over Omega of |y - X|^2
  float2 d[NI][16];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int it = tid + j * NT, kb = it >> 4;
#pragma unroll
    for (int q = 0; q < 16; ++q) d[j][q] = make_float2(0.f, 0.f);
    if (it < N) {
      if (!first) {
#pragma unroll
        for (int q = 0; q < 16; ++q) d[j][q] = tb[kb * P1 + q * 16 + c];
        RegFft<16, false>::run(d[j], tw_s, M);
      }
#pragma unroll
      for (int ka = 0; ka < 16; ++ka) {
        const int row = kb + M * ka;
        const float2 X = cscale(d[j][ka], isq);
        const float2 yy = yv[j][ka];
        const float w = wv[j][ka];
        float2 o;
        if (vd) {
          o = make_float2(0.f, 0.f);
          if (w > 0.f) {
            const float2 z = csub(yy, X);
            o = cscale(z, w);
            const float cc = w * ((w - 1.0f) * (z.x * z.x + z.y * z.y) + sig2);
            const float2 cs = cs_s[row];
            float cj = cs.x, sj = cs.y, pj = cs.x;
            QH[0] = fmaf(sj, cc, QH[0]);
            QL[0] = fmaf(pj, cc, QL[0]);
#pragma unroll
            for (int t = 1; t < 4; ++t) {
              const float dj = cj - sj;
              sj = 4.0f * cj * sj;
              cj = (sj < 0.5f) ? 1.0f - sj : dj * dj;  // the form without cancellation
              QH[t] = fmaf(pj * sj, cc, QH[t]);
              pj *= cj;
              QL[t] = fmaf(pj, cc, QL[t]);
            }
          }
        } else if (mode == CM_OUTPUT) {
          o = (w > 0.f) ? yy : X;
        } else if (mode == CM_ZEROFILL) {
          o = yy;
        } else if (mode == CM_FISTA_OBJ) {
          o = make_float2(0.f, 0.f);
          if (w > 0.f) {
            const float2 z = csub(yy, X);
            rsum = fmaf(z.x, z.x, fmaf(z.y, z.y, rsum));
          }
        } else {  // FISTA: m (y - X)
          o = (w > 0.f) ? csub(yy, X) : make_float2(0.f, 0.f);
        }
        d[j][ka] = cscale(o, isq);
      }
    }
  }
  if (vd) {
    // tau_b partial = sum over this strip's columns of Xtab_b(kx) sum_ky Ytab_b(ky) c
    const float* xtab = a.tables + S.xtab_off;
    const int kx = c0 + c;
    const int lane = tid & 63, wid = tid >> 6;
    float vb[16];  // this lane's term of every band (1 + 3 s <= 13 bands)
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      vb[b] = 0.f;
      if (b < a.nbands) {
        int ty, tx;
        if (b == 0) { ty = s - 1; tx = s - 1; }
        else {
          const int l = s - (b - 1) / 3, kind = (b - 1) % 3;
          const int L = l - 1, Hh = s + l - 1;
          ty = (kind == 0) ? L : Hh;
          tx = (kind == 1) ? L : Hh;
        }
        const bool hb = ty >= s;
        const int tt = hb ? ty - s : ty;
        float q0 = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t == tt) q0 = hb ? QH[t] : QL[t];
        q0 *= (float)(2 << tt) / (float)N;
        vb[b] = q0 * xtab[tx * nx + kx];
      }
    }
    const float part = wave_sum_rs<16>(vb);  // band (lane >> 2) & 15
    const int bl = (lane >> 2) & 15;
    if ((lane & 3) == 0 && bl < a.nbands) red[wid][bl] = part;
  }
  if (mode == CM_FISTA_OBJ) {  // the residual's partial sum is all this mode writes
    const float part = wave_sum(rsum);
    if ((tid & 63) == 0) red[tid >> 6][0] = part;
    __syncthreads();
    if (tid == 0) {
      float acc = 0.f;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) acc += red[w][0];
      a.tau_part[(S.colstrip0 + item.y) * kMaxBands] = acc;
    }
    return;
  }
  __syncthreads();  // tau partials visible; every forward read of tb done
  if (vd && tid < a.nbands) {
    float acc = 0.f;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) acc += red[w][tid];
    a.tau_part[(S.colstrip0 + item.y) * kMaxBands + tid] = acc;
  }
  // inverse: 16-point DFTs over ka (rows kb + M ka), twiddle, transpose
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int it = tid + j * NT, kb = it >> 4;
    if (it < N) {
      RegFft<16, true>::run(d[j], tw_s, M);
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) {
        float2 v = d[j][k2];
        if (k2 && kb) {
          float2 w = tw_s[kb * k2];
          w.y = -w.y;
          v = cmul(v, w);
        }
        tb[k2 * P2 + kb * 16 + c] = v;
      }
    }
  }
  __syncthreads();
  if (!s1) return;
  float2 f[M];
#pragma unroll
  for (int kb = 0; kb < M; ++kb) f[kb] = tb[a1 * P2 + kb * 16 + c];
  RegFft<M, true>::run(f, tw_s, 16);
#pragma unroll
  for (int b = 0; b < M; ++b) a.X[base + (long long)(a1 + 16 * b) * nx + c] = f[b];
}

// ------------------------------------------------------------------ rows_anal
template <int EPT, int M, int NT = kThreads, int SL = 0>
__global__ void __launch_bounds__(NT) k_rows_anal(KArgs a) {
  extern __shared__ float4 lds4[];
  float2* lds = reinterpret_cast<float2*>(lds4);
  __shared__ float2 tw_s[kMaxN];
  __shared__ float th_s[kMaxBands], t2_s[kMaxBands], al_s[kMaxBands], ia_s[kMaxBands];
  __shared__ int sel_s[kMaxBands];
  __shared__ float l1_s[NT / 64];
  const int2 item = a.work[blockIdx.x];
  const SliceDev S = a.slices[item.x];
  constexpr int NXC = M > 0 ? 16 * M : 0;
  const int strip = item.y, s = SL ? SL : a.levels, H = 1 << s, nx = NXC ? NXC : S.nx, ny = S.ny;
  const int tid = threadIdx.x, mode = a.mode;
  constexpr int U = EPT / 2;
  const int half = nx >> 1, npairs = H * half;
  const float4* src = reinterpret_cast<const float4*>(a.X + S.off + (long long)strip * H * nx);
  constexpr int MV = M > 0 ? M : 1;
  float4 v[M > 0 ? 1 : U];
  float2 v4[MV];  // four-step inputs: samples a + 16 b of row `line`
  if constexpr (M > 0) {
    const int a16 = tid & 15, line = tid >> 4;
    const float2* xs = a.X + S.off + (long long)strip * H * nx;
#pragma unroll
    for (int b = 0; b < MV; ++b)
      v4[b] = (line < H) ? xs[line * nx + a16 + 16 * b] : make_float2(0.f, 0.f);
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * NT;
      v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (p < npairs) v[u] = src[p];
    }
  }
  if (tid < kMaxBands) {
    th_s[tid] = a.theta[item.x * kMaxBands + tid];
    t2_s[tid] = a.thr2[item.x * kMaxBands + tid];
    al_s[tid] = a.alpha[item.x * kMaxBands + tid];
    ia_s[tid] = 1.0f / (1.0f - al_s[tid]);
    if (mode == RA_LEARNED) sel_s[tid] = a.sel[item.x * kMaxBands + tid];
  }
  const FftPlanDev& P = a.ffts[S.fft_x];
  load_twiddles<NT>(tw_s, P, a.twiddles);
  if constexpr (M > 0) {
    using F = RowFft4<M, NT>;
    __syncthreads();  // twiddles
    F::template step1<true>(v4, H, tw_s, lds);
    __syncthreads();
    float2 d[F::NI][16];
    int kbs[F::NI], ls[F::NI];
    bool ok[F::NI];
#pragma unroll
    for (int j = 0; j < F::NI; ++j) ok[j] = F::template step2<true>(j, H, tw_s, lds, d[j], kbs[j], ls[j]);
    __syncthreads();  // every transpose read done before the strip is rewritten
#pragma unroll
    for (int j = 0; j < F::NI; ++j)
      if (ok[j]) {
#pragma unroll
        for (int ka = 0; ka < 16; ++ka) lds[ls[j] * F::N + kbs[j] + M * ka] = d[j][ka];
      }
    __syncthreads();
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * NT;
      if (p < npairs) lds4[p] = v[u];
    }
    __syncthreads();
    fft_lines<true, false, EPT>(lds, P, H, nx, 1, tw_s);
  }
  float2* r = a.r + S.off;
  float2* r2 = a.r2 ? a.r2 + S.off : nullptr;
  const float lam = a.lambda ? a.lambda[item.x] : 0.f;
  const float lam2 = __fmul_rn(lam, lam);
  const bool need_r = (mode == RA_VDAMP || mode == RA_VDAMP_G || mode == RA_FISTA || mode == RA_LEARNED);
  int gi[U];  // offset in the slice
  int bnd[U];
  float4 ro[U], rw[U];
#define RA_LOAD_R()                                                                          \
  _Pragma("unroll") for (int u = 0; u < U; ++u) {                                            \
    const int p = tid + u * NT;                                                        \
    bnd[u] = 0;                                                                              \
    gi[u] = 0;                                                                               \
    ro[u] = make_float4(0.f, 0.f, 0.f, 0.f);                                                 \
    rw[u] = make_float4(0.f, 0.f, 0.f, 0.f);                                                 \
    if (p < npairs) {                                                                        \
      const int lr = p / half, lc = 2 * (p - lr * half);                                     \
      int b;                                                                                 \
      const int gr = strip_to_global_t<SL, NXC>(lr, lc, strip, s, ny, nx, b);               \
      bnd[u] = b;                                                                            \
      gi[u] = gr * nx + lc;                                                                  \
      if (need_r) ro[u] = *reinterpret_cast<const float4*>(r + gi[u]);                       \
    }                                                                                        \
  }
  if (mode == RA_IMAGE) {
    float4* dst = reinterpret_cast<float4*>(a.out + S.off + (long long)strip * H * nx);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * NT;
      if (p < npairs) dst[p] = lds4[p];
    }
    return;
  }
  // With up to 16 elements a thread, r is fetched before the Haar analysis so that the
  // loads are in flight while it runs; with 32 the registers it would hold through it
  // cost more occupancy than the overlap gains.
  if constexpr (EPT <= 16) {
    RA_LOAD_R();
    haar_strip_anal<EPT, NT, SL, NXC>(lds, H, nx, s);
  } else {
    haar_strip_anal<EPT, NT, SL, NXC>(lds, H, nx, s);
    RA_LOAD_R();
  }
#undef RA_LOAD_R
  float l1 = 0.f;
  if (mode == RA_FISTA || mode == RA_LEARNED) {  // the second iterate
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (tid + u * NT < npairs) rw[u] = *reinterpret_cast<const float4*>(r2 + gi[u]);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * NT;
    if (p < npairs) {
      const int b = bnd[u];
      const float4 gv = lds4[p];
      if (mode == RA_VDAMP_G) {  // Onsager-corrected r_tilde of the pair x = 2j, 2j + 1, + coefficients
        float2 x0 = lo2(ro[u]), x1 = hi2(ro[u]);
        rtilde_pair(x0, x1, th_s[b], t2_s[b], al_s[b], ia_s[b]);
        *reinterpret_cast<float4*>(r + gi[u]) = pack4(cadd(x0, lo2(gv)), cadd(x1, hi2(gv)));
        continue;
      }
      float2 o[2], w2[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float2 g = h ? hi2(gv) : lo2(gv);
        switch (mode) {
          case RA_VDAMP_FIRST: o[h] = g; break;
          case RA_VDAMP: {
            const float2 x = h ? hi2(ro[u]) : lo2(ro[u]);
            o[h] = rtilde_ci_add(x, th_s[b], t2_s[b], al_s[b], ia_s[b], g);
          } break;
          case RA_LEARNED: {
            const float2 x = h ? hi2(ro[u]) : lo2(ro[u]);
            const float2 wv = h ? hi2(rw[u]) : lo2(rw[u]);
            if (sel_s[b])
              o[h] = cadd(rtilde_w(wv, x, al_s[b]), g);
            else  // as RA_VDAMP, so that a band left to soft thresholding matches the plain solve
              o[h] = rtilde_ci_add(x, th_s[b], t2_s[b], al_s[b], ia_s[b], g);
          } break;
          case RA_FISTA_FIRST: {
            w2[h] = soft_c(g, lam, lam2);
            o[h] = w2[h];
          } break;
          default: {  // RA_FISTA: w = eta(v + g); v' = w + beta (w - w_prev)
            const float2 x = h ? hi2(ro[u]) : lo2(ro[u]);
            const float2 wp = h ? hi2(rw[u]) : lo2(rw[u]);
            w2[h] = soft_c(cadd(x, g), lam, lam2);
            o[h] = make_float2(w2[h].x + a.beta * (w2[h].x - wp.x), w2[h].y + a.beta * (w2[h].y - wp.y));
          } break;
        }
      }
      *reinterpret_cast<float4*>(r + gi[u]) = pack4(o[0], o[1]);
      if (mode == RA_FISTA || mode == RA_FISTA_FIRST) {
        *reinterpret_cast<float4*>(r2 + gi[u]) = pack4(w2[0], w2[1]);
        if (a.jpart)
          l1 += sqrtf(key_rn(w2[0])) + sqrtf(key_rn(w2[1]));
      }
    }
  }
  if ((mode == RA_FISTA || mode == RA_FISTA_FIRST) && a.jpart) {  // this strip's ||w||_1
    const float part = wave_sum(l1);
    if ((tid & 63) == 0) l1_s[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) {
      float acc = 0.f;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) acc += l1_s[w];
      a.jpart[S.rowstrip0 + strip] = acc;
    }
  }
}


// ------------------------------------------------------------------ wave_anal
// Learned-denoiser support (row strip): Psi of an image strip (no transform), then per
// subband partial sums over the strip.  jmode 0: the image is the denoiser output; write
// its coefficients w to r2 and sum |w - r|^2.  jmode 1: the image is the denoiser's
// Jacobian applied to Psi^H b; sum Re(conj(b) w) with the probe b regenerated.  Partial
// sums go to jpart[jmode][row strip][band], reduced in a fixed order.  jmode 2: only
// write the coefficients to r2 (the plain transform Psi).
template <int EPT>
__global__ void __launch_bounds__(kThreads) k_wave_anal(KArgs a, int jmode) {
  extern __shared__ float4 lds4[];
  float2* lds = reinterpret_cast<float2*>(lds4);
  __shared__ float red[kThreads / 64][kMaxBands];
  const int2 item = a.work[blockIdx.x];
  const SliceDev S = a.slices[item.x];
  const int strip = item.y, s = a.levels, H = 1 << s, nx = S.nx, ny = S.ny;
  const int tid = threadIdx.x;
  constexpr int U = EPT / 2;
  const int half = nx >> 1, npairs = H * half;
  const float4* src = reinterpret_cast<const float4*>(a.X + S.off + (long long)strip * H * nx);
  float4 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * kThreads;
    v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p < npairs) v[u] = src[p];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * kThreads;
    if (p < npairs) lds4[p] = v[u];
  }
  __syncthreads();
  haar_strip_anal<EPT>(lds, H, nx, s);
  float2* r = a.r + S.off;
  float2* wc = a.r2 + S.off;
  long long gi[U];
  int bnd[U];
  float4 ro[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * kThreads;
    bnd[u] = -1;
    gi[u] = 0;
    ro[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p < npairs) {
      const int lr = p / half, lc = 2 * (p - lr * half);
      int b;
      const int gr = strip_to_global(lr, lc, strip, s, ny, nx, b);
      bnd[u] = b;
      gi[u] = (long long)gr * nx + lc;
      if (jmode == 0) ro[u] = *reinterpret_cast<const float4*>(r + gi[u]);
    }
  }
  float cv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int p = tid + u * kThreads;
    cv[u] = 0.f;
    if (p < npairs) {
      const float4 w = lds4[p];
      if (jmode == 2) {
        *reinterpret_cast<float4*>(wc + gi[u]) = w;
      } else if (jmode == 0) {
        *reinterpret_cast<float4*>(wc + gi[u]) = w;
        const float d0 = w.x - ro[u].x, d1 = w.y - ro[u].y, d2 = w.z - ro[u].z, d3 = w.w - ro[u].w;
        cv[u] = (d0 * d0 + d1 * d1) + (d2 * d2 + d3 * d3);
      } else {
        const float2 b0 = probe_c(a.seed, a.iter, item.x, gi[u]);
        const float2 b1 = probe_c(a.seed, a.iter, item.x, gi[u] + 1);
        cv[u] = (b0.x * w.x + b0.y * w.y) + (b1.x * w.z + b1.y * w.w);
      }
    }
  }
  if (jmode == 2) return;
  const int lane = tid & 63, wid = tid >> 6;
  for (int b = 0; b < a.nbands; ++b) {
    float t = 0.f;
#pragma unroll
    for (int u = 0; u < U; ++u) t += (bnd[u] == b) ? cv[u] : 0.f;
    t = wave_sum(t);
    if (lane == 0) red[wid][b] = t;
  }
  __syncthreads();
  if (tid < a.nbands) {
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += red[w][tid];
    a.jpart[((long long)jmode * a.nwork + S.rowstrip0 + strip) * kMaxBands + tid] = t;
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_rows_synth(const KArgs& a, int ept, int do_fft, size_t lds, hipStream_t st) {
  if (ept == 16)
    hipLaunchKernelGGL((k_rows_synth<16, 0>), dim3(a.nwork), dim3(kThreads), lds, st, a, do_fft);
  else
    hipLaunchKernelGGL((k_rows_synth<32, 0>), dim3(a.nwork), dim3(kThreads), lds, st, a, do_fft);
  return hipGetLastError();
}
hipError_t launch_cols(const KArgs& a, int ept, size_t lds, hipStream_t st) {
  if (ept == 16)
    hipLaunchKernelGGL(k_cols<16>, dim3(a.nwork), dim3(kThreads), lds, st, a);
  else
    hipLaunchKernelGGL(k_cols<32>, dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}
#define COLS4_CASE(MM) \
  case MM: hipLaunchKernelGGL(k_cols4<MM>, dim3(a.nwork), dim3(cols4_threads(MM)), 0, st, a); break

hipError_t launch_cols4(const KArgs& a, int m, hipStream_t st) {
  switch (m) {
    COLS4_CASE(1); COLS4_CASE(2); COLS4_CASE(3); COLS4_CASE(4); COLS4_CASE(5);
    COLS4_CASE(6); COLS4_CASE(8); COLS4_CASE(10); COLS4_CASE(12); COLS4_CASE(15);
    COLS4_CASE(16); COLS4_CASE(20); COLS4_CASE(24); COLS4_CASE(30); COLS4_CASE(32);
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool cols4_supported(int ny) {
  if (ny % 16) return false;
  switch (ny / 16) {
    case 1: case 2: case 3: case 4: case 5: case 6: case 8: case 10: case 12: case 15:
    case 16: case 20: case 24: case 30: case 32: return true;
    default: return false;
  }
}

hipError_t launch_rows_anal(const KArgs& a, int ept, size_t lds, hipStream_t st) {
  if (ept == 16)
    hipLaunchKernelGGL((k_rows_anal<16, 0>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  else
    hipLaunchKernelGGL((k_rows_anal<32, 0>), dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

// Four-step row kernels for nx = 16 m; dynamic LDS = the strip or the transpose buffer.
size_t rows4_lds_bytes(int m, int H) {
  const int pr = (m % 2) ? m : m + 1;
  const size_t strip = (size_t)H * 16 * m, tb = (size_t)256 * pr;
  return sizeof(float2) * (strip > tb ? strip : tb);
}

#define ROWS4_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(15) X(16) X(20) X(24) X(30) X(32)
// threads and elements a thread: 256 x 16 up to nx = 256; 256 x nx/16 for nx = 320 and
// 384 (the Haar loops, EPT / 4 blocks a thread, cover the strip exactly); 256 x 32 for
// nx = 480 and 512 (512 x 16 measured no better there: the M-point stage alone holds
// 2 M registers a thread, 166 VGPRs, so only one 8-wave workgroup fits a CU)
#define NT_OF(MM) kThreads
#define EPT_OF(MM) ((MM) <= 16 ? 16 : ((MM) <= 24 ? (MM) : 32))

// Plans of 4 levels (the paper's s) on power-of-two widths, and 192 and 320 wide, run
// kernels with the level count fixed at compile time (measured faster on the mixed
// batch although the 320-wide synthesis then holds 137 VGPRs against 128; for 96, 160,
// 240, 384 and 480 the runtime-level kernels are kept).
template <int MM> constexpr bool fixed_levels() { return (MM & (MM - 1)) == 0 || MM == 12 || MM == 20; }
template <int MM>
static void launch_rs4(const KArgs& a, size_t lds, hipStream_t st) {
  if constexpr (fixed_levels<MM>()) {
    if (a.levels == 4) {
      hipLaunchKernelGGL((k_rows_synth<EPT_OF(MM), MM, NT_OF(MM), 4>), dim3(a.nwork), dim3(NT_OF(MM)), lds, st, a, 1);
      return;
    }
  }
  hipLaunchKernelGGL((k_rows_synth<EPT_OF(MM), MM, NT_OF(MM)>), dim3(a.nwork), dim3(NT_OF(MM)), lds, st, a, 1);
}
template <int MM>
static void launch_ra4(const KArgs& a, size_t lds, hipStream_t st) {
  if constexpr (fixed_levels<MM>()) {
    if (a.levels == 4) {
      hipLaunchKernelGGL((k_rows_anal<EPT_OF(MM), MM, NT_OF(MM), 4>), dim3(a.nwork), dim3(NT_OF(MM)), lds, st, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_rows_anal<EPT_OF(MM), MM, NT_OF(MM)>), dim3(a.nwork), dim3(NT_OF(MM)), lds, st, a);
}
template <int MM>
static hipError_t set_lds_rows4(int bytes) {
  std::vector<const void*> fs = {(const void*)k_rows_synth<EPT_OF(MM), MM, NT_OF(MM)>,
                                 (const void*)k_rows_anal<EPT_OF(MM), MM, NT_OF(MM)>};
  if constexpr (fixed_levels<MM>()) {
    fs.push_back((const void*)k_rows_synth<EPT_OF(MM), MM, NT_OF(MM), 4>);
    fs.push_back((const void*)k_rows_anal<EPT_OF(MM), MM, NT_OF(MM), 4>);
  }
  for (const void* f : fs) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_rows_synth4(const KArgs& a, int m, size_t lds, hipStream_t st) {
  switch (m) {
#define RS4(MM)                                                                                \
  case MM:                                                                                     \
    launch_rs4<MM>(a, lds, st);                                                                \
    break;
    ROWS4_CASES(RS4)
#undef RS4
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rows_anal4(const KArgs& a, int m, size_t lds, hipStream_t st) {
  switch (m) {
#define RA4(MM)                                                                                \
  case MM:                                                                                     \
    launch_ra4<MM>(a, lds, st);                                                                \
    break;
    ROWS4_CASES(RA4)
#undef RA4
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wave_anal(const KArgs& a, int ept, int jmode, size_t lds, hipStream_t st) {
  if (ept == 16)
    hipLaunchKernelGGL(k_wave_anal<16>, dim3(a.nwork), dim3(kThreads), lds, st, a, jmode);
  else
    hipLaunchKernelGGL(k_wave_anal<32>, dim3(a.nwork), dim3(kThreads), lds, st, a, jmode);
  return hipGetLastError();
}

hipError_t set_lds_limits_passes(size_t rows, size_t cols) {
  std::vector<const void*> rk = {(const void*)k_rows_synth<16, 0>, (const void*)k_rows_synth<32, 0>,
                                 (const void*)k_rows_anal<16, 0>, (const void*)k_rows_anal<32, 0>,
                                 (const void*)k_wave_anal<16>, (const void*)k_wave_anal<32>};
  for (const void* f : rk) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rows);
    if (e != hipSuccess) return e;
  }
  const int r4 = (int)rows4_lds_bytes(32, 16);  // the largest four-step row tile
#define LIM4(MM)                                                                                      \
  {                                                                                                   \
    hipError_t e = set_lds_rows4<MM>(r4);                                                             \
    if (e != hipSuccess) return e;                                                                    \
  }
  ROWS4_CASES(LIM4)
#undef LIM4
  const void* ck[] = {(const void*)k_cols<16>, (const void*)k_cols<32>};
  for (const void* f : ck) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cols);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vdamp

// gfx950 kernels of the VDAMP iteration (Algorithm 1) and of the FISTA comparator.
//
// One iteration is four passes over HBM, each one workgroup per work item:
//   rows_synth  (row strip of 2^s image rows): line 8 applied to r_{k-1}, Psi^H on the
//               strip (Haar never couples strips of 2^s rows), then the row FFTs.
//   cols        (column strip of 16 columns): column FFT, k-space residual of line 3,
//               density compensation P^-1 of line 4, the tau partial sums of line 5
//               (S is separable per band for Haar), column IFFT.
//   rows_anal   (row strip): row IFFTs, Psi on the strip, add r_tilde_k (line 4).
//   sure        (one band of one slice): tau reduction, exact SURE threshold search
//               over the sorted band magnitudes (Section 3), alpha of line 7.
// Every transform stays in LDS; the FFT is a mixed-radix (2/3/4/5) Stockham FFT done
// in place with a barrier between the gather and scatter halves of each stage.
#include "vdamp_internal.h"

namespace vdamp {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward sign) or +i (inverse sign)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ------------------------------------------------------------------ small DFTs
template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV> struct Dft<4, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <bool INV> struct Dft<3, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    const float c = -0.5f, s3 = 0.86602540378443864676f;
    float2 sum = cadd(v[1], v[2]);
    float2 dif = cscale(mul_mi<INV>(csub(v[1], v[2])), s3);
    float2 base = make_float2(v[0].x + c * sum.x, v[0].y + c * sum.y);
    v[0] = cadd(v[0], sum);
    v[1] = cadd(base, dif);
    v[2] = csub(base, dif);
  }
};

template <bool INV> struct Dft<5, INV> {
  static __device__ __forceinline__ void run(float2* v) {
    const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
    const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
    const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
    const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
    float2 b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
    float2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    float2 a0 = v[0];
    float2 e1 = make_float2(a0.x + c1 * b1.x + c2 * b2.x, a0.y + c1 * b1.y + c2 * b2.y);
    float2 e2 = make_float2(a0.x + c2 * b1.x + c1 * b2.x, a0.y + c2 * b1.y + c1 * b2.y);
    float2 f1 = mul_mi<INV>(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
    float2 f2 = mul_mi<INV>(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
    v[0] = make_float2(a0.x + b1.x + b2.x, a0.y + b1.y + b2.y);
    v[1] = cadd(e1, f1);
    v[4] = csub(e1, f1);
    v[2] = cadd(e2, f2);
    v[3] = csub(e2, f2);
  }
};

// ------------------------------------------------------------------ LDS Stockham FFT
// Lines of length n live in LDS at buf[line * ls + i * es].  COLS selects the thread
// mapping: consecutive threads take consecutive lines (columns of a column strip) or
// consecutive butterflies of one line (rows), so LDS accesses stay unit-stride.
template <int R, bool INV, bool COLS>
__device__ __forceinline__ void fft_stage(float2* __restrict__ buf, int n, int Ns, int nlines,
                                          int ls, int es, const float2* __restrict__ tw) {
  constexpr int MAXB = (kEpt + R - 1) / R;
  const int nb = n / R;
  const int total = nb * nlines;
  float2 v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int t = threadIdx.x + q * kThreads;
    if (t < total) {
      int line, j;
      if (COLS) { line = t % nlines; j = t / nlines; }
      else { line = t / nb; j = t - line * nb; }
      const float2* src = buf + line * ls;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[(j + r * nb) * es];
    }
  }
  __syncthreads();
  const int twstride = n / (Ns * R);
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int t = threadIdx.x + q * kThreads;
    if (t < total) {
      int line, j;
      if (COLS) { line = t % nlines; j = t / nlines; }
      else { line = t / nb; j = t - line * nb; }
      const int k = j % Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * k * twstride];
        if (INV) w.y = -w.y;
        v[q][r] = cmul(v[q][r], w);
      }
      Dft<R, INV>::run(v[q]);
      const int idx = (j / Ns) * Ns * R + k;
      float2* dst = buf + line * ls;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[(idx + r * Ns) * es] = v[q][r];
    }
  }
  __syncthreads();
}

template <bool INV, bool COLS>
__device__ void fft_lines(float2* buf, const FftPlanDev& P, int nlines, int ls, int es,
                          const float2* __restrict__ twpool) {
  const float2* tw = twpool + P.tw_off;
  int Ns = 1;
  for (int st = 0; st < P.nst; ++st) {
    const int R = P.rad[st];
    switch (R) {
      case 4: fft_stage<4, INV, COLS>(buf, P.n, Ns, nlines, ls, es, tw); break;
      case 2: fft_stage<2, INV, COLS>(buf, P.n, Ns, nlines, ls, es, tw); break;
      case 3: fft_stage<3, INV, COLS>(buf, P.n, Ns, nlines, ls, es, tw); break;
      default: fft_stage<5, INV, COLS>(buf, P.n, Ns, nlines, ls, es, tw); break;
    }
    Ns *= R;
  }
}

// ------------------------------------------------------------------ Haar on a strip
// The strip holds H = 2^s image rows x nx columns.  Its coefficients form the Mallat
// layout of an H x nx image with s levels ("mini-Mallat"); one 2x2 orthonormal Haar
// butterfly per coefficient quadruple (LL, LH, HL, HH):
//   x00 = (a + b + c + d)/2, x01 = (a - b + c - d)/2,
//   x10 = (a + b - c - d)/2, x11 = (a - b - c + d)/2,
// with a = LL, b = LH (low y, high x), c = HL (high y, low x), d = HH.
__device__ void haar_strip_synth(float2* buf, int H, int nx, int s) {
  for (int l = s; l >= 1; --l) {
    const int hp = H >> l, w = nx >> l;
    const int nblk = hp * w;
    constexpr int MAXQ = kEpt / 4;
    float2 o[MAXQ][4];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int t = threadIdx.x + q * kThreads;
      if (t < nblk) {
        const int i = t / w, j = t - (t / w) * w;
        const float2 a = buf[i * nx + j], b = buf[i * nx + w + j];
        const float2 c = buf[(hp + i) * nx + j], d = buf[(hp + i) * nx + w + j];
        const float2 apc = cadd(a, c), amc = csub(a, c), bpd = cadd(b, d), bmd = csub(b, d);
        o[q][0] = cscale(cadd(apc, bpd), 0.5f);
        o[q][1] = cscale(csub(apc, bpd), 0.5f);
        o[q][2] = cscale(cadd(amc, bmd), 0.5f);
        o[q][3] = cscale(csub(amc, bmd), 0.5f);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int t = threadIdx.x + q * kThreads;
      if (t < nblk) {
        const int i = t / w, j = t - (t / w) * w;
        buf[(2 * i) * nx + 2 * j] = o[q][0];
        buf[(2 * i) * nx + 2 * j + 1] = o[q][1];
        buf[(2 * i + 1) * nx + 2 * j] = o[q][2];
        buf[(2 * i + 1) * nx + 2 * j + 1] = o[q][3];
      }
    }
    __syncthreads();
  }
}

__device__ void haar_strip_anal(float2* buf, int H, int nx, int s) {
  for (int l = 1; l <= s; ++l) {
    const int hp = H >> l, w = nx >> l;
    const int nblk = hp * w;
    constexpr int MAXQ = kEpt / 4;
    float2 o[MAXQ][4];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int t = threadIdx.x + q * kThreads;
      if (t < nblk) {
        const int i = t / w, j = t - (t / w) * w;
        const float2 x00 = buf[(2 * i) * nx + 2 * j], x01 = buf[(2 * i) * nx + 2 * j + 1];
        const float2 x10 = buf[(2 * i + 1) * nx + 2 * j], x11 = buf[(2 * i + 1) * nx + 2 * j + 1];
        const float2 s0 = cadd(x00, x01), d0 = csub(x00, x01), s1 = cadd(x10, x11), d1 = csub(x10, x11);
        o[q][0] = cscale(cadd(s0, s1), 0.5f);  // LL
        o[q][1] = cscale(cadd(d0, d1), 0.5f);  // LH: low along y, high along x
        o[q][2] = cscale(csub(s0, s1), 0.5f);  // HL: high along y, low along x
        o[q][3] = cscale(csub(d0, d1), 0.5f);  // HH
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int t = threadIdx.x + q * kThreads;
      if (t < nblk) {
        const int i = t / w, j = t - (t / w) * w;
        buf[i * nx + j] = o[q][0];
        buf[i * nx + w + j] = o[q][1];
        buf[(hp + i) * nx + j] = o[q][2];
        buf[(hp + i) * nx + w + j] = o[q][3];
      }
    }
    __syncthreads();
  }
}

// Position (lr, lc) of a strip's mini-Mallat image -> global Mallat row and band.
// The column is the same in both layouts.
__device__ __forceinline__ int strip_to_global(int lr, int lc, int strip, int s, int ny, int nx,
                                               int& band) {
  const int H = 1 << s;
#pragma unroll 1
  for (int l = 1; l <= s; ++l) {
    const bool hy = lr >= (H >> l);
    const bool hx = lc >= (nx >> l);
    if (hy || hx) {
      const int hp = H >> l;
      band = 1 + 3 * (s - l) + (hy ? (hx ? 2 : 1) : 0);
      return (hy ? (ny >> l) : 0) + strip * hp + (lr - (hy ? hp : 0));
    }
  }
  band = 0;
  return strip;
}

// |r|^2 with each multiply and the add rounded to nearest (no contraction): the key on
// which the threshold search sorts and decides, and on which thresholding tests
// membership, so both see bit-identical values (as does any host computing
// x*x + y*y in IEEE FP32).
__device__ __forceinline__ float key_rn(float2 v) {
  return __fadd_rn(__fmul_rn(v.x, v.x), __fmul_rn(v.y, v.y));
}

// eta(r; theta) = r max(0, 1 - theta/|r|); zero when |r|^2 <= theta^2 (th2 is the
// threshold's own key, so the element that defines theta is zeroed).
__device__ __forceinline__ float2 soft_c(float2 v, float th, float th2) {
  const float key = key_rn(v);
  if (!(key > th2)) return make_float2(0.f, 0.f);
  const float g = 1.0f - th / sqrtf(key);
  return make_float2(v.x * g, v.y * g);
}

// line 8: r_tilde = (eta(r) - alpha r) / (1 - alpha)
__device__ __forceinline__ float2 rtilde_c(float2 v, float th, float th2, float al) {
  const float2 w = soft_c(v, th, th2);
  const float inv = 1.0f / (1.0f - al);
  return make_float2((w.x - al * v.x) * inv, (w.y - al * v.y) * inv);
}

// ------------------------------------------------------------------ pass 1: rows_synth
// do_fft = 0 writes the image rows Psi^H r (FISTA output).
__global__ void __launch_bounds__(kThreads) k_rows_synth(KArgs a, int do_fft) {
  extern __shared__ float2 lds[];
  __shared__ float th_s[kMaxBands], t2_s[kMaxBands], al_s[kMaxBands];
  const int2 item = a.work[blockIdx.x];
  const SliceDev S = a.slices[item.x];
  const int strip = item.y, s = a.levels, H = 1 << s, nx = S.nx, ny = S.ny;
  if (threadIdx.x < kMaxBands) {
    th_s[threadIdx.x] = a.theta[item.x * kMaxBands + threadIdx.x];
    t2_s[threadIdx.x] = a.thr2[item.x * kMaxBands + threadIdx.x];
    al_s[threadIdx.x] = a.alpha[item.x * kMaxBands + threadIdx.x];
  }
  __syncthreads();
  const float2* r = a.r + S.off;
  const int tot = H * nx;
  for (int e = threadIdx.x; e < tot; e += kThreads) {
    const int lr = e / nx, lc = e - (e / nx) * nx;
    int b;
    const int gr = strip_to_global(lr, lc, strip, s, ny, nx, b);
    float2 v = r[(long long)gr * nx + lc];
    if (a.mode == RS_RTILDE) v = rtilde_c(v, th_s[b], t2_s[b], al_s[b]);
    else if (a.mode == RS_WHAT) v = soft_c(v, th_s[b], t2_s[b]);
    lds[e] = v;
  }
  __syncthreads();
  haar_strip_synth(lds, H, nx, s);
  if (do_fft) fft_lines<false, false>(lds, a.ffts[S.fft_x], H, nx, 1, a.twiddles);
  float2* dst = (do_fft ? a.X : a.out) + S.off + (long long)strip * H * nx;
  for (int e = threadIdx.x; e < tot; e += kThreads) dst[e] = lds[e];
}

// ------------------------------------------------------------------ pass 2: cols
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(kThreads) k_cols(KArgs a) {
  extern __shared__ float2 lds[];
  __shared__ float red[kThreads / 64][kMaxBands];
  const int2 item = a.work[blockIdx.x];
  const int sl = item.x;
  const SliceDev S = a.slices[sl];
  const int ny = S.ny, nx = S.nx, c0 = item.y * kColW, s = a.levels;
  const int mode = a.mode;
  const bool first = (mode == CM_VDAMP_FIRST || mode == CM_ZEROFILL || mode == CM_FISTA_FIRST);
  const int tot = ny * kColW;
  const long long base = S.off + c0;
  if (!first) {
    for (int e = threadIdx.x; e < tot; e += kThreads) {
      const int row = e / kColW, c = e - row * kColW;
      lds[e] = a.X[base + (long long)row * nx + c];
    }
    __syncthreads();
    fft_lines<false, true>(lds, a.ffts[S.fft_y], kColW, 1, kColW, a.twiddles);
  }
  const float isq = rsqrtf((float)ny * (float)nx);  // unitary scaling, once per direction
  const bool vd = (mode == CM_VDAMP || mode == CM_VDAMP_FIRST);
  const float sig2 = a.sigma2 ? a.sigma2[sl] : 0.f;
  float Q[2 * 4];
#pragma unroll
  for (int t = 0; t < 8; ++t) Q[t] = 0.f;
  const int ntab = 2 * s;
  const float* ytab = a.tables + S.ytab_off;
  for (int e = threadIdx.x; e < tot; e += kThreads) {
    const int row = e / kColW, c = e - row * kColW;
    const long long g = base + (long long)row * nx + c;
    const float2 X = first ? make_float2(0.f, 0.f) : cscale(lds[e], isq);
    const float wv = a.wgt[g];
    float2 outv;
    if (vd) {
      float2 v = make_float2(0.f, 0.f);
      if (wv > 0.f) {
        const float2 z = csub(a.y[g], X);
        v = cscale(z, wv);
        const float cc = wv * ((wv - 1.0f) * (z.x * z.x + z.y * z.y) + sig2);
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (t < ntab) Q[t] = fmaf(ytab[t * ny + row], cc, Q[t]);
      }
      outv = v;
    } else if (mode == CM_OUTPUT) {
      outv = (wv > 0.f) ? a.y[g] : X;
    } else if (mode == CM_ZEROFILL) {
      outv = a.y[g];
    } else {  // FISTA: m (y - X)
      outv = (wv > 0.f) ? csub(a.y[g], X) : make_float2(0.f, 0.f);
    }
    lds[e] = cscale(outv, isq);
  }
  if (vd) {
    // tau_b partial = sum over this strip's columns of Xtab_b(kx) * sum_ky Ytab_b(ky) c
    const int c = threadIdx.x % kColW;
    const float* xtab = a.tables + S.xtab_off;
    const int kx = c0 + c;
    const int lane = threadIdx.x & 63, wv_id = threadIdx.x >> 6;
    for (int b = 0; b < a.nbands; ++b) {
      int ty, tx;
      if (b == 0) { ty = s - 1; tx = s - 1; }
      else {
        const int l = s - (b - 1) / 3, kind = (b - 1) % 3;
        const int L = l - 1, Hh = s + l - 1;
        ty = (kind == 0) ? L : Hh;
        tx = (kind == 1) ? L : Hh;
      }
      float q = 0.f;
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (t == ty) q = Q[t];
      float part = wave_sum(q * xtab[tx * nx + kx]);
      if (lane == 0) red[wv_id][b] = part;
    }
    __syncthreads();
    if (threadIdx.x < a.nbands) {
      float acc = 0.f;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) acc += red[w][threadIdx.x];
      a.tau_part[(S.colstrip0 + item.y) * kMaxBands + threadIdx.x] = acc;
    }
  }
  __syncthreads();
  fft_lines<true, true>(lds, a.ffts[S.fft_y], kColW, 1, kColW, a.twiddles);
  for (int e = threadIdx.x; e < tot; e += kThreads) {
    const int row = e / kColW, c = e - row * kColW;
    a.X[base + (long long)row * nx + c] = lds[e];
  }
}

// ------------------------------------------------------------------ pass 3: rows_anal
__global__ void __launch_bounds__(kThreads) k_rows_anal(KArgs a) {
  extern __shared__ float2 lds[];
  __shared__ float th_s[kMaxBands], t2_s[kMaxBands], al_s[kMaxBands];
  const int2 item = a.work[blockIdx.x];
  const SliceDev S = a.slices[item.x];
  const int strip = item.y, s = a.levels, H = 1 << s, nx = S.nx, ny = S.ny;
  const int tot = H * nx;
  const float2* src = a.X + S.off + (long long)strip * H * nx;
  for (int e = threadIdx.x; e < tot; e += kThreads) lds[e] = src[e];
  if (threadIdx.x < kMaxBands) {
    th_s[threadIdx.x] = a.theta[item.x * kMaxBands + threadIdx.x];
    t2_s[threadIdx.x] = a.thr2[item.x * kMaxBands + threadIdx.x];
    al_s[threadIdx.x] = a.alpha[item.x * kMaxBands + threadIdx.x];
  }
  __syncthreads();
  fft_lines<true, false>(lds, a.ffts[S.fft_x], H, nx, 1, a.twiddles);
  if (a.mode == RA_IMAGE) {
    float2* dst = a.out + S.off + (long long)strip * H * nx;
    for (int e = threadIdx.x; e < tot; e += kThreads) dst[e] = lds[e];
    return;
  }
  haar_strip_anal(lds, H, nx, s);
  float2* r = a.r + S.off;
  float2* r2 = a.r2 ? a.r2 + S.off : nullptr;
  const float lam = a.lambda ? a.lambda[item.x] : 0.f;
  const float lam2 = __fmul_rn(lam, lam);
  for (int e = threadIdx.x; e < tot; e += kThreads) {
    const int lr = e / nx, lc = e - (e / nx) * nx;
    int b;
    const int gr = strip_to_global(lr, lc, strip, s, ny, nx, b);
    const long long gi = (long long)gr * nx + lc;
    const float2 g = lds[e];
    switch (a.mode) {
      case RA_VDAMP_FIRST: r[gi] = g; break;
      case RA_VDAMP: r[gi] = cadd(rtilde_c(r[gi], th_s[b], t2_s[b], al_s[b]), g); break;
      case RA_FISTA_FIRST: {
        const float2 w = soft_c(g, lam, lam2);
        r[gi] = w;
        r2[gi] = w;
      } break;
      default: {  // RA_FISTA
        const float2 w = soft_c(cadd(r[gi], g), lam, lam2);
        const float2 wp = r2[gi];
        r[gi] = make_float2(w.x + a.beta * (w.x - wp.x), w.y + a.beta * (w.y - wp.y));
        r2[gi] = w;
      } break;
    }
  }
}

// ------------------------------------------------------------------ pass 4: sure
// Band geometry in the global Mallat layout.
__device__ __forceinline__ void band_geom(int b, int s, int ny, int nx, int& r0, int& c0,
                                          int& bh, int& bw) {
  if (b == 0) { r0 = 0; c0 = 0; bh = ny >> s; bw = nx >> s; return; }
  const int l = s - (b - 1) / 3, kind = (b - 1) % 3;
  bh = ny >> l; bw = nx >> l;
  r0 = (kind == 0) ? 0 : bh;
  c0 = (kind == 1) ? 0 : bw;
}

__device__ __forceinline__ double wave_incl_prefix(double v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ double wave_incl_suffix(double v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double t = __shfl_down(v, o, 64);
    if (lane + o < 64) v += t;
  }
  return v;
}

__device__ __forceinline__ int wave_incl_prefix_int(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Bucket of a key for the counting sort, from the FP32 bit pattern of v = key/tau.
// Monotone in key: multiplying by a positive constant with round-to-nearest is
// monotone, and so is the bit pattern of a non-negative float.  The buckets are
// piecewise logarithmic: fine (MB mantissa bits) over v in [2^-4, 2^3), where the
// noise-only keys concentrate (key/tau of a CN(0, tau) coefficient is Exp(1)), and
// coarse (LB bits) over [2^-16, 2^-4) and [2^3, 2^23); keys outside fall into the first
// or last bucket.  NB = 12 * 2^LB + 7 * 2^MB + 20 * 2^LB.  (tau = 0 sends every key to
// the last bucket: the search then takes its full-sort path.)
template <int NB> struct SureBuckets;
template <> struct SureBuckets<4096> { static constexpr int LB = 4, MB = 9; };
template <> struct SureBuckets<1024> { static constexpr int LB = 2, MB = 7; };

template <int NB>
__device__ __forceinline__ int sure_bucket(float key, float inv_tau) {
  constexpr int LB = SureBuckets<NB>::LB, MB = SureBuckets<NB>::MB;
  constexpr unsigned E_LO = 111u << 23, E_MID = 123u << 23, E_HI = 130u << 23;
  constexpr int N_LO = 12 << LB, N_MID = 7 << MB;
  static_assert(N_LO + N_MID + (20 << LB) == NB, "bucket layout");
  const unsigned e = __float_as_uint(key * inv_tau);
  if (e < E_MID) {
    const int v = (e < E_LO) ? 0 : (int)((e - E_LO) >> (23 - LB));
    return v;
  }
  if (e < E_HI) return N_LO + (int)((e - E_MID) >> (23 - MB));
  const unsigned v = (e - E_HI) >> (23 - LB);
  return N_LO + N_MID + (int)min(v, (unsigned)((20 << LB) - 1));
}

// LDS index of sorted position i: one pad word per 16 keys, so that threads walking
// contiguous 16-key chunks hit distinct banks.
__device__ __forceinline__ int skx(int i) { return i + (i >> 4); }

// Exact SURE threshold search for one band (Section 3), one workgroup per band.
//   1. tau_b from the column-strip partials (FP64, fixed order).
//   2. keys = |r|^2 (FP32, see key_rn) held in registers; counting sort by
//      sure_bucket: LDS integer atomics count the buckets and give each key a slot,
//      an exclusive scan gives bucket offsets, the keys are scattered, and each key
//      then takes its final place from its rank inside its bucket (keys smaller than
//      it, plus equal keys in earlier slots).  The result is the sorted key array,
//      identical on every run.  If a bucket holds more than kSureBucketLimit keys the
//      band is sorted with a bitonic network instead.
//   3. Each thread walks a contiguous chunk of the sorted keys: with a = sqrt(key),
//      A_m = sum_{i<=m} a_i^2 and R_m = sum_{i>m} 1/a_i (FP64 accumulation of FP32
//      terms, chunk offsets from FP64 prefix/suffix scans), it evaluates
//      SURE(m) = A_m - m tau + (N_b - m)(a_m^2 + tau) - tau a_m R_m at every candidate
//      (the last index of a run of equal keys, a > 0).
//   4. Workgroup argmin, ties to the smaller index; theta = a_m, theta^2 = key_m and
//      alpha = ((N_b - m) - theta R_m / 2) / N_b (line 7).
constexpr int kSureBucketLimit = 128;

template <int NT, int KPT, int NB>
__global__ void __launch_bounds__(NT) k_sure(KArgs a) {
  extern __shared__ int sure_smem[];
  constexpr int NW = NT / 64;
  constexpr int BPT = NB / NT;
  __shared__ double wsA[NW], wsR[NW], bv[NW], bR[NW];
  __shared__ int bi[NW], wsC[NW], wsM[NW];
  __shared__ float tau_sh;
  __shared__ int maxc_sh;
  int* off = sure_smem;                                      // [NB + 1]
  float* sk = reinterpret_cast<float*>(sure_smem + NB + 1);  // [skx(npad)]
  const int2 item = a.work[blockIdx.x];
  const int sl = item.x, b = item.y, s = a.levels;
  const SliceDev S = a.slices[sl];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int r0, c0, bh, bw;
  band_geom(b, s, S.ny, S.nx, r0, c0, bh, bw);
  const int Nb = bh * bw;
  int npad = 1;
  while (npad < Nb) npad <<= 1;

  for (int i = tid; i <= NB; i += NT) off[i] = 0;
  if (wid == 0) {
    const int ncs = S.nx / kColW;
    double acc = 0.0;
    for (int i = lane; i < ncs; i += 64) acc += (double)a.tau_part[(S.colstrip0 + i) * kMaxBands + b];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) tau_sh = (float)acc;
  }
  // load the band (coalesced along rows) while the counters are cleared
  const float2* r = a.r + S.off + (long long)r0 * S.nx + c0;
  const int lbw = 31 - __clz(bw);  // band widths are powers of two times 1, 3 or 5
  const bool pow2 = (bw & (bw - 1)) == 0;
  float kk[KPT];
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int i = tid + j * NT;
    kk[j] = 0.f;
    if (i < Nb) {
      const int rr = pow2 ? (i >> lbw) : i / bw;
      const int cc = i - rr * bw;
      kk[j] = key_rn(r[(long long)rr * S.nx + cc]);
    }
  }
  __syncthreads();
  const float inv_tau = 1.0f / tau_sh;
  int pos[KPT];
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int i = tid + j * NT;
    if (i < Nb) pos[j] = atomicAdd(&off[sure_bucket<NB>(kk[j], inv_tau)], 1);
  }
  __syncthreads();
  // exclusive scan of the bucket counts, and the largest count
  int cnt[BPT];
  int sum = 0, mx = 0;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    cnt[q] = off[tid * BPT + q];
    sum += cnt[q];
    mx = max(mx, cnt[q]);
  }
  const int incl = wave_incl_prefix_int(sum, lane);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
  if (lane == 63) wsC[wid] = incl;
  if (lane == 0) wsM[wid] = mx;
  __syncthreads();
  int excl = incl - sum;
  for (int w = 0; w < wid; ++w) excl += wsC[w];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    off[tid * BPT + q] = excl;
    excl += cnt[q];
  }
  if (tid == NT - 1) off[NB] = excl;
  if (tid == 0) {
    int m = 0;
    for (int w = 0; w < NW; ++w) m = max(m, wsM[w]);
    maxc_sh = m;
  }
  __syncthreads();
  // scatter into bucket slots
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int i = tid + j * NT;
    if (i < Nb) sk[skx(off[sure_bucket<NB>(kk[j], inv_tau)] + pos[j])] = kk[j];
  }
  __syncthreads();
  if (maxc_sh <= kSureBucketLimit) {
    // final position = bucket offset + rank within the bucket (ties by slot)
    int fin[KPT];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      if (i < Nb) {
        const int bk = sure_bucket<NB>(kk[j], inv_tau);
        const int lo = off[bk], hi = off[bk + 1];
        const float v = kk[j];
        const int me = lo + pos[j];
        int rank = 0;
        for (int x = lo; x < hi; ++x) {
          const float u = sk[skx(x)];
          rank += (u < v) || (u == v && x < me);
        }
        fin[j] = lo + rank;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      if (i < Nb) sk[skx(fin[j])] = kk[j];
    }
    for (int i = Nb + tid; i < npad; i += NT) sk[skx(i)] = __builtin_huge_valf();
    __syncthreads();
  } else {
    for (int i = Nb + tid; i < npad; i += NT) sk[skx(i)] = __builtin_huge_valf();
    __syncthreads();
    for (int k = 2; k <= npad; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = tid; i < (npad >> 1); i += NT) {
          const int lo = 2 * j * (i / j) + (i & (j - 1));
          const int hi = lo + j;
          const bool asc = (lo & k) == 0;
          const float x = sk[skx(lo)], y = sk[skx(hi)];
          if ((x > y) == asc) { sk[skx(lo)] = y; sk[skx(hi)] = x; }
        }
        __syncthreads();
      }
    }
  }
  const double tau = (double)tau_sh;
  const float kmax = sk[skx(Nb - 1)];
  const int E = (npad + NT - 1) / NT;
  const int i0 = tid * E;
  const int i1 = min(i0 + E, Nb);
  double cA = 0.0, cR = 0.0;
  for (int i = i0; i < i1; ++i) {
    const float k2 = sk[skx(i)];
    cA += (double)k2;
    if (k2 > 0.f) cR += (double)__frsqrt_rn(k2);
  }
  const double pA = wave_incl_prefix(cA, lane);
  const double sR = wave_incl_suffix(cR, lane);
  if (lane == 63) wsA[wid] = pA;
  if (lane == 0) wsR[wid] = sR;
  __syncthreads();
  double offA = 0.0, offR = 0.0;
  for (int w = 0; w < wid; ++w) offA += wsA[w];
  for (int w = NW - 1; w > wid; --w) offR += wsR[w];
  double A = offA + pA - cA;          // sum of a^2 over indices < i0
  double Rrun = offR + sR;            // sum of 1/a over indices >= i0
  double best = __builtin_huge_val(), bestR = 0.0;
  int besti = 0x7fffffff;
  const double Nbd = (double)Nb;
  float knext = (i0 < i1) ? sk[skx(i0)] : 0.f;
  for (int i = i0; i < i1; ++i) {
    const float k2 = knext;
    knext = (i + 1 < Nb) ? sk[skx(i + 1)] : __builtin_huge_valf();
    A += (double)k2;
    if (k2 > 0.f) {
      Rrun -= (double)__frsqrt_rn(k2);  // now the sum over indices > i
      if (knext > k2) {                 // last index of a run of equal keys
        const double x = (double)__fsqrt_rn(k2);
        const double m = (double)(i + 1);
        const double sv = A - m * tau + (Nbd - m) * ((double)k2 + tau) - tau * x * Rrun;
        if (sv < best) { best = sv; besti = i; bestR = Rrun; }
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double ov = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(besti, o, 64);
    const double oR = __shfl_xor(bestR, o, 64);
    if (ov < best || (ov == best && oi < besti)) { best = ov; besti = oi; bestR = oR; }
  }
  if (lane == 0) { bv[wid] = best; bi[wid] = besti; bR[wid] = bestR; }
  __syncthreads();
  if (tid == 0) {
    double fb = bv[0], fR = bR[0];
    int fi = bi[0];
    for (int w = 1; w < NW; ++w)
      if (bv[w] < fb || (bv[w] == fb && bi[w] < fi)) { fb = bv[w]; fi = bi[w]; fR = bR[w]; }
    float th, th2, al;
    if (!(kmax > 0.f) || fi == 0x7fffffff) {  // all-zero band: eta = 0, alpha = 0
      th = 0.f;
      th2 = 0.f;
      al = 0.f;
    } else {
      th2 = sk[skx(fi)];
      th = __fsqrt_rn(th2);
      const double m = (double)(fi + 1);
      al = (float)(((Nbd - m) - 0.5 * (double)th * fR) / Nbd);
    }
    a.theta[sl * kMaxBands + b] = th;
    a.thr2[sl * kMaxBands + b] = th2;
    a.alpha[sl * kMaxBands + b] = al;
    a.tau[sl * kMaxBands + b] = tau_sh;
    if (a.trace) {
      float* t = a.trace + (((long long)a.iter * a.batch + sl) * a.nbands + b) * 3;
      t[0] = tau_sh;
      t[1] = th;
      t[2] = al;
    }
  }
}

// ------------------------------------------------------------------ prep
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

}  // namespace vdamp

// ------------------------------------------------------------------ launch wrappers
namespace vdamp {

hipError_t launch_rows_synth(const KArgs& a, int do_fft, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_rows_synth, dim3(a.nwork), dim3(kThreads), lds, st, a, do_fft);
  return hipGetLastError();
}
hipError_t launch_cols(const KArgs& a, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_cols, dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}
hipError_t launch_rows_anal(const KArgs& a, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_rows_anal, dim3(a.nwork), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}
// Bands with more than kSureSmall keys go to the 1024-thread variant (up to 32768 keys,
// 4096 buckets); the rest to the 256-thread one (up to 4096 keys, 1024 buckets).
hipError_t launch_sure(const KArgs& a, bool big, size_t lds, hipStream_t st) {
  if (big)
    hipLaunchKernelGGL((k_sure<1024, 32, 4096>), dim3(a.nwork), dim3(1024), lds, st, a);
  else
    hipLaunchKernelGGL((k_sure<256, 16, 1024>), dim3(a.nwork), dim3(256), lds, st, a);
  return hipGetLastError();
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

// Allow dynamic LDS beyond the default limit where a plan needs it.
hipError_t set_lds_limits(size_t rows, size_t cols, size_t sure_big, size_t sure_small) {
  hipError_t e = hipFuncSetAttribute((const void*)k_rows_synth,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)rows);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_rows_anal, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rows);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_cols, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cols);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_sure<1024, 32, 4096>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sure_big);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_sure<256, 16, 1024>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sure_small);
  return e;
}

}  // namespace vdamp

// Device building blocks shared by the gfx950 kernels: complex helpers, small DFTs,
// the in-LDS mixed-radix Stockham FFT, the strip-local Haar transforms, the Mallat
// mapping of a strip, and complex soft thresholding.
#pragma once

#include <type_traits>

#include "vdamp_internal.h"

namespace vdamp {

// Work item of workgroup b in a launch of n workgroups, arranged so that the workgroups
// the dispatcher sends to one XCD (ids x, x + 8, x + 16, ...: round-robin over the 8
// XCDs) take consecutive items.  Neighbouring column strips share the 128-byte lines of
// the 4-byte weight rows (64 bytes each); on one XCD they share its L2 instead of each
// fetching the line from HBM.  A bijection on [0, n).
__device__ __forceinline__ int xcd_item(int b, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd, x = b % kXcd;
  return x * q + min(x, r) + b / kXcd;
}


__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 lo2(float4 v) { return make_float2(v.x, v.y); }
__device__ __forceinline__ float2 hi2(float4 v) { return make_float2(v.z, v.w); }
__device__ __forceinline__ float4 pack4(float2 a, float2 b) { return make_float4(a.x, a.y, b.x, b.y); }
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
// Lines of length n live in LDS at buf[line * ls + i * es]; tw holds exp(-2 pi i k/n),
// k < n (in LDS).  One stage gathers R inputs per butterfly into registers, waits for
// the workgroup, applies twiddles and the radix-R DFT and scatters to the Stockham
// output positions (in place: every read of the stage precedes every write).  COLS
// selects the thread mapping: consecutive threads take consecutive lines (the columns
// of a column strip) or consecutive butterflies of one line (rows), so LDS accesses
// stay unit-stride.  EPT bounds the elements per thread (n * nlines <= 256 * EPT).
template <int R, bool INV, bool COLS, int EPT>
__device__ __forceinline__ void fft_stage(float2* __restrict__ buf, int n, int Ns, int nlines,
                                          int ls, int es, const float2* __restrict__ tw) {
  constexpr int MAXB = (EPT + R - 1) / R;
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

// Always inlined: a call (the compiler declines to inline some instances) costs the
// row kernels that use it a register save/restore and all constant propagation.
template <bool INV, bool COLS, int EPT>
__device__ __forceinline__ void fft_lines(float2* buf, const FftPlanDev& P, int nlines, int ls, int es,
                                          const float2* __restrict__ tw) {
  int Ns = 1;
  for (int st = 0; st < P.nst; ++st) {
    const int R = P.rad[st];
    switch (R) {
      case 4: fft_stage<4, INV, COLS, EPT>(buf, P.n, Ns, nlines, ls, es, tw); break;
      case 2: fft_stage<2, INV, COLS, EPT>(buf, P.n, Ns, nlines, ls, es, tw); break;
      case 3: fft_stage<3, INV, COLS, EPT>(buf, P.n, Ns, nlines, ls, es, tw); break;
      default: fft_stage<5, INV, COLS, EPT>(buf, P.n, Ns, nlines, ls, es, tw); break;
    }
    Ns *= R;
  }
}

// In-LDS FFTs of the 16 columns of a strip block (element (i, c) at buf[16 i + c]): the
// Stockham stages of fft_lines with the line count fixed at compile time.
template <bool INV, int EPT>
__device__ __forceinline__ void fft_cols16(float2* buf, const FftPlanDev& P, const float2* tw) {
  int Ns = 1;
  for (int st = 0; st < P.nst; ++st) {
    const int R = P.rad[st];
    switch (R) {
      case 4: fft_stage<4, INV, true, EPT>(buf, P.n, Ns, kColW, 1, kColW, tw); break;
      case 2: fft_stage<2, INV, true, EPT>(buf, P.n, Ns, kColW, 1, kColW, tw); break;
      case 3: fft_stage<3, INV, true, EPT>(buf, P.n, Ns, kColW, 1, kColW, tw); break;
      default: fft_stage<5, INV, true, EPT>(buf, P.n, Ns, kColW, 1, kColW, tw); break;
    }
    Ns *= R;
  }
}

// fft_cols16 for a power-of-two length N fixed at compile time: radix-4 stages, one
// radix-2 stage last when log2 N is odd, every stage's constants folded.
template <bool INV, int EPT, int N, int NS = 1>
__device__ __forceinline__ void fft_cols16_n(float2* buf, const float2* tw) {
  static_assert((N & (N - 1)) == 0, "power-of-two length");
  if constexpr (NS < N) {
    constexpr int R = ((N / NS) % 4 == 0) ? 4 : 2;
    fft_stage<R, INV, true, EPT>(buf, N, NS, kColW, 1, kColW, tw);
    fft_cols16_n<INV, EPT, N, NS * R>(buf, tw);
  }
}

// fft_lines (rows: consecutive threads take consecutive butterflies of one line) for a
// power-of-two length N fixed at compile time, lines at buf[line * ls + i].
template <bool INV, int EPT, int N, int NS = 1>
__device__ __forceinline__ void fft_rows_n(float2* buf, int nlines, int ls, const float2* tw) {
  static_assert((N & (N - 1)) == 0, "power-of-two length");
  if constexpr (NS < N) {
    constexpr int R = ((N / NS) % 4 == 0) ? 4 : 2;
    fft_stage<R, INV, false, EPT>(buf, N, NS, nlines, ls, 1, tw);
    fft_rows_n<INV, EPT, N, NS * R>(buf, nlines, ls, tw);
  }
}

// f(std::integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time.
template <int N, int I = 0, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<N, I + 1>(f);
  }
}

// ------------------------------------------------------------------ register FFT
// M-point DFT of v[0..M) held in registers (natural order in and out), decimation in
// time over the radices 4, 2, 3, 5; M = R * M2: the R interleaved sub-sequences
// v[R m + r] are transformed recursively, then combined by R-point DFTs with twiddles
// W_M^{r k}.  Twiddles come from the table tw of exp(-2 pi i j / n) (LDS; every lane
// reads the same entry): W_M^j = tw[j * tstride] with tstride = n / M.
template <int M>
struct FirstRadix {
  static constexpr int value = (M % 4 == 0 && M != 8) ? 4 : (M % 2 == 0 ? 2 : (M % 3 == 0 ? 3 : 5));
};

template <int M, bool INV>
struct RegFft {
  static constexpr int R = FirstRadix<M>::value;
  static constexpr int M2 = M / R;
  static __device__ __forceinline__ void run(float2* v, const float2* __restrict__ tw, int tstride) {
    float2 s[R][M2];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int m = 0; m < M2; ++m) s[r][m] = v[R * m + r];
#pragma unroll
    for (int r = 0; r < R; ++r) RegFft<M2, INV>::run(s[r], tw, tstride * R);
#pragma unroll
    for (int k = 0; k < M2; ++k) {
      float2 t[R];
      t[0] = s[0][k];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        if (k == 0) {
          t[r] = s[r][k];
        } else {
          float2 w = tw[r * k * tstride];
          if (INV) w.y = -w.y;
          t[r] = cmul(s[r][k], w);
        }
      }
      Dft<R, INV>::run(t);
#pragma unroll
      for (int q = 0; q < R; ++q) v[k + M2 * q] = t[q];
    }
  }
};
template <bool INV> struct RegFft<1, INV> {
  static __device__ __forceinline__ void run(float2*, const float2* __restrict__, int) {}
};
template <bool INV> struct RegFft<2, INV> {
  static __device__ __forceinline__ void run(float2* v, const float2* __restrict__, int) { Dft<2, INV>::run(v); }
};
template <bool INV> struct RegFft<3, INV> {
  static __device__ __forceinline__ void run(float2* v, const float2* __restrict__, int) { Dft<3, INV>::run(v); }
};
template <bool INV> struct RegFft<4, INV> {
  static __device__ __forceinline__ void run(float2* v, const float2* __restrict__, int) { Dft<4, INV>::run(v); }
};
template <bool INV> struct RegFft<5, INV> {
  static __device__ __forceinline__ void run(float2* v, const float2* __restrict__, int) { Dft<5, INV>::run(v); }
};

// Copy a plan's twiddle table into LDS (issued alongside the tile loads).
template <int NT = kThreads>
__device__ __forceinline__ void load_twiddles(float2* tw_s, const FftPlanDev& P,
                                              const float2* __restrict__ pool) {
  for (int i = threadIdx.x; i < P.n; i += NT) tw_s[i] = pool[P.tw_off + i];
}

// ------------------------------------------------------------------ four-step row FFTs
// Row FFTs of a strip of H <= 16 rows of length N = 16 M: thread (a, line) transforms
// the M samples a + 16 b of its row (b < M), scales by W_N^{a kb}, and an LDS transpose
// hands the 16 values of each (kb, line) to one thread, whose 16-point DFT gives the
// outputs kb + M ka.  The transpose buffer (pitch PR, odd, so that the lanes of a step
// hit distinct banks) aliases the strip buffer; every thread has read its inputs before
// the first write.
template <int M, int NT = kThreads>
struct RowFft4 {
  static constexpr int N = 16 * M;
  static constexpr int PR = (M % 2) ? M : M + 1;
  static constexpr int NI = (16 * M + NT - 1) / NT;
  static constexpr int LDS_ELEMS = (16 * N > 256 * PR) ? 16 * N : 256 * PR;

  // step 1 (inputs in v, lanes with line >= H idle) and the transpose
  template <bool INV>
  static __device__ __forceinline__ void step1(float2 (&v)[M], int H, const float2* __restrict__ tw,
                                               float2* buf) {
    const int a = threadIdx.x & 15, line = threadIdx.x >> 4;
    if (line < H) {
      RegFft<M, INV>::run(v, tw, 16);
#pragma unroll
      for (int kb = 0; kb < M; ++kb) {
        float2 x = v[kb];
        if (kb && a) {
          float2 w = tw[a * kb];
          if (INV) w.y = -w.y;
          x = cmul(x, w);
        }
        buf[(line * 16 + a) * PR + kb] = x;
      }
    }
  }
  // step 2 for item j of this thread: the 16 outputs kb + M ka of row `line`
  template <bool INV>
  static __device__ __forceinline__ bool step2(int j, int H, const float2* __restrict__ tw,
                                               const float2* buf, float2 (&d)[16], int& kb, int& line) {
    const int it = threadIdx.x + j * NT;
    kb = it % M;
    line = it / M;
    if (line >= H) return false;
#pragma unroll
    for (int q = 0; q < 16; ++q) d[q] = buf[(line * 16 + q) * PR + kb];
    RegFft<16, INV>::run(d, tw, M);
    return true;
  }
};

// ------------------------------------------------------------------ Haar on a strip
// The strip holds H = 2^s image rows x nx columns.  Its coefficients form the Mallat
// layout of an H x nx image with s levels ("mini-Mallat"); one 2x2 orthonormal Haar
// butterfly per coefficient quadruple (LL, LH, HL, HH):
//   x00 = (a + b + c + d)/2, x01 = (a - b + c - d)/2,
//   x10 = (a + b - c - d)/2, x11 = (a - b - c + d)/2,
// with a = LL, b = LH (low y, high x), c = HL (high y, low x), d = HH.
// SL > 0 and NXC > 0 fix the level count and the strip width at compile time (the
// level loop unrolls and every index divides by a constant); 0 reads them at run time.
template <int EPT, int NT = kThreads, int SL = 0, int NXC = 0>
__device__ __forceinline__ void haar_strip_synth(float2* buf, int H, int nx_, int s_) {
  constexpr int MAXQ = EPT / 4;
  const int s = SL ? SL : s_, nx = NXC ? NXC : nx_;
#pragma unroll
  for (int l = s; l >= 1; --l) {
    const int hp = H >> l, w = nx >> l;
    const int nblk = hp * w;
    float2 o[MAXQ][4];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int t = threadIdx.x + q * NT;
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
      const int t = threadIdx.x + q * NT;
      if (t < nblk) {
        const int i = t / w, j = t - (t / w) * w;
        float4* row0 = reinterpret_cast<float4*>(buf + (2 * i) * nx + 2 * j);
        float4* row1 = reinterpret_cast<float4*>(buf + (2 * i + 1) * nx + 2 * j);
        *row0 = pack4(o[q][0], o[q][1]);
        *row1 = pack4(o[q][2], o[q][3]);
      }
    }
    __syncthreads();
  }
}

template <int EPT, int NT = kThreads, int SL = 0, int NXC = 0>
__device__ __forceinline__ void haar_strip_anal(float2* buf, int H, int nx_, int s_) {
  constexpr int MAXQ = EPT / 4;
  const int s = SL ? SL : s_, nx = NXC ? NXC : nx_;
#pragma unroll
  for (int l = 1; l <= s; ++l) {
    const int hp = H >> l, w = nx >> l;
    const int nblk = hp * w;
    float2 o[MAXQ][4];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < nblk) {
        const int i = t / w, j = t - (t / w) * w;
        const float4 r0 = *reinterpret_cast<const float4*>(buf + (2 * i) * nx + 2 * j);
        const float4 r1 = *reinterpret_cast<const float4*>(buf + (2 * i + 1) * nx + 2 * j);
        const float2 x00 = lo2(r0), x01 = hi2(r0), x10 = lo2(r1), x11 = hi2(r1);
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
      const int t = threadIdx.x + q * NT;
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
// The column is the same in both layouts.  Band boundaries along x sit at multiples
// of nx >> s (even), so an even-aligned pair (lc, lc + 1) shares row and band.
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

// strip_to_global with the level count SL and the width NXC known at compile time: the
// level is the first l whose high half along y (lr >= 2^(SL-l)) or along x
// (lc >= NXC >> l) holds the position, found without a loop.
template <int SL, int NXC>
__device__ __forceinline__ int strip_to_global_c(int lr, int lc, int strip, int ny, int& band) {
  int l = SL + 1;
#pragma unroll
  for (int k = SL; k >= 1; --k)
    if (lr >= (1 << (SL - k)) || lc >= (NXC >> k)) l = k;
  if (l > SL) {
    band = 0;
    return strip;
  }
  const int hp = (1 << SL) >> l;
  const bool hy = lr >= hp, hx = lc >= (NXC >> l);
  band = 1 + 3 * (SL - l) + (hy ? (hx ? 2 : 1) : 0);
  return (hy ? (ny >> l) : 0) + strip * hp + (lr - (hy ? hp : 0));
}
template <int SL, int NXC>
__device__ __forceinline__ int strip_to_global_t(int lr, int lc, int strip, int s, int ny, int nx, int& band) {
  if constexpr (SL > 0 && NXC > 0)
    return strip_to_global_c<SL, NXC>(lr, lc, strip, ny, band);
  else
    return strip_to_global(lr, lc, strip, s, ny, nx, band);
}

// |r|^2 with each multiply and the add rounded to nearest (no contraction): the key on
// which the threshold search sorts and decides, and on which thresholding tests
// membership, so both see bit-identical values (as does any host computing
// x*x + y*y in IEEE FP32).
__device__ __forceinline__ float key_rn(float2 v) {
#pragma clang fp contract(off)
  // (without the pragma the compiler fuses the add into the second multiply, an FMA
  // with a single rounding, and the key differs from x*x + y*y by an ulp)
  const float xx = v.x * v.x;
  const float yy = v.y * v.y;
  return xx + yy;
}

// eta(r; theta) = r max(0, 1 - theta/|r|); zero when |r|^2 <= theta^2 (th2 is the
// threshold's own key, so the element that defines theta is zeroed).
// The shrink factor takes theta times the hardware reciprocal square root of the key
// (within an ulp or two of 1/|r|), not an IEEE square root and division.
__device__ __forceinline__ float2 soft_c(float2 v, float th, float th2) {
  const float key = key_rn(v);
  if (!(key > th2)) return make_float2(0.f, 0.f);
  const float g = 1.0f - th * rsqrtf(key);
  return make_float2(v.x * g, v.y * g);
}

// the Onsager correction: r_tilde = (eta(r) - alpha r) / (1 - alpha) = r (g - alpha) / (1 - alpha) with
// g = max(0, 1 - theta/|r|) the shrink factor of eta (0 at or below the threshold's key),
// inv = 1 / (1 - alpha) of the band computed once (the same IEEE quotient rtilde_c forms
// per coefficient): one factor a coefficient, then two multiplies
__device__ __forceinline__ float2 rtilde_ci(float2 v, float th, float th2, float al, float inv) {
  const float key = key_rn(v);
  const float g = (key > th2) ? 1.0f - th * rsqrtf(key) : 0.f;
  const float f = (g - al) * inv;
  return make_float2(v.x * f, v.y * f);
}
__device__ __forceinline__ float2 rtilde_c(float2 v, float th, float th2, float al) {
  return rtilde_ci(v, th, th2, al, 1.0f / (1.0f - al));
}
// r_tilde + c with the factor form and one rounding per component (an explicit fused
// multiply-add, so that every pass that adds the back-projected coefficients c to the
// corrected iterate rounds alike, whatever the compiler contracts elsewhere)
__device__ __forceinline__ float2 rtilde_ci_add(float2 v, float th, float th2, float al, float inv, float2 c) {
  const float key = key_rn(v);
  const float g = (key > th2) ? 1.0f - th * rsqrtf(key) : 0.f;
  const float f = (g - al) * inv;
  return make_float2(__fmaf_rn(v.x, f, c.x), __fmaf_rn(v.y, f, c.y));
}

// Group soft thresholding of a horizontal pair g = (u, v) of one subband row (the
// structured-sparsity denoiser): both shrink by max(0, 1 - theta/||g||), and the pair is
// zeroed when its key |u|^2 + |v|^2 (key_rn of each, the sum rounded to nearest) is at
// most th2, the threshold's own key.
__device__ __forceinline__ float key_pair_rn(float2 u, float2 v) { return key_rn(u) + key_rn(v); }
__device__ __forceinline__ void soft_pair(float2& u, float2& v, float th, float th2) {
  const float key = key_pair_rn(u, v);
  if (!(key > th2)) {
    u = make_float2(0.f, 0.f);
    v = make_float2(0.f, 0.f);
    return;
  }
  const float g = 1.0f - th * rsqrtf(key);
  u = make_float2(u.x * g, u.y * g);
  v = make_float2(v.x * g, v.y * g);
}
// the Onsager correction for the pair: (eta(g) - alpha g) / (1 - alpha) = g (s - alpha) / (1 - alpha)
// with s the pair's shrink factor, inv = 1 / (1 - alpha)
__device__ __forceinline__ void rtilde_pair(float2& u, float2& v, float th, float th2, float al, float inv) {
  const float key = key_pair_rn(u, v);
  const float g = (key > th2) ? 1.0f - th * rsqrtf(key) : 0.f;
  const float f = (g - al) * inv;
  u = make_float2(u.x * f, u.y * f);
  v = make_float2(v.x * f, v.y * f);
}

// the Onsager correction for a general denoiser output w: (w - alpha r) / (1 - alpha)
__device__ __forceinline__ float2 rtilde_w(float2 w, float2 v, float al) {
  const float inv = 1.0f / (1.0f - al);
  return make_float2((w.x - al * v.x) * inv, (w.y - al * v.y) * inv);
}

// Probe of the Monte-Carlo divergence: a complex Rademacher value (+-1 +- i)/sqrt(2)
// per wavelet coefficient, drawn by SplitMix64 (Steele, Lea and Flood, 2014) used as a
// counter-based generator: the value at counter c of the stream with seed k is
// mix(k + (c + 1) * 0x9E3779B97F4A7C15), with c = iteration << 48 | slice << 32 | index
// (index = row * nx + column of the coefficient in its slice).  Bit 0 gives the sign of
// the real part, bit 1 that of the imaginary part (set = negative).
__device__ __forceinline__ unsigned long long splitmix64_mix(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ float2 probe_c(unsigned long long seed, int iter, int slice,
                                          long long index) {
  const unsigned long long c = ((unsigned long long)iter << 48) |
                               ((unsigned long long)slice << 32) | (unsigned long long)index;
  const unsigned long long z = splitmix64_mix(seed + (c + 1ull) * 0x9E3779B97F4A7C15ull);
  const float h = 0.70710678118654752f;
  return make_float2((z & 1ull) ? -h : h, (z & 2ull) ? -h : h);
}

// Band geometry in the global Mallat layout.
__device__ __forceinline__ void band_geom(int b, int s, int ny, int nx, int& r0, int& c0,
                                          int& bh, int& bw) {
  if (b == 0) { r0 = 0; c0 = 0; bh = ny >> s; bw = nx >> s; return; }
  const int l = s - (b - 1) / 3, kind = (b - 1) % 3;
  bh = ny >> l; bw = nx >> l;
  r0 = (kind == 0) ? 0 : bh;
  c0 = (kind == 1) ? 0 : bw;
}

// Band b of a slice (nd == 1: the 2D layout above, 1 + 3 s bands) or of a volume (nd > 1:
// 3D Mallat layout, 1 + 7 s bands: b = 0 is LLL_s, then for l = s .. 1 the octants of
// kind k = 1 .. 7, bit 0 of k high along x, bit 1 along y, bit 2 along z): origin
// (d0, r0, c0) and extent (bd, bh, bw) of its block.
__device__ __forceinline__ void band_geom3(int b, int s, int nd, int ny, int nx, int& d0, int& r0,
                                           int& c0, int& bd, int& bh, int& bw) {
  if (nd <= 1) {
    d0 = 0;
    bd = 1;
    band_geom(b, s, ny, nx, r0, c0, bh, bw);
    return;
  }
  if (b == 0) { d0 = 0; r0 = 0; c0 = 0; bd = nd >> s; bh = ny >> s; bw = nx >> s; return; }
  const int l = s - (b - 1) / 7, k = (b - 1) % 7 + 1;
  bd = nd >> l; bh = ny >> l; bw = nx >> l;
  d0 = (k & 4) ? bd : 0;
  r0 = (k & 2) ? bh : 0;
  c0 = (k & 1) ? bw : 0;
}

// Offset of element i (row-major within the block) of a band block from the block's
// first element, in a slice or volume of ny x nx planes.
struct BandWalk {
  int bd, bh, bw, lbw, plane;
  bool pow2;
  long long zs, nx;
  __device__ __forceinline__ long long at(int i) const {
    if (bd == 1) {
      const int rr = pow2 ? (i >> lbw) : i / bw;
      return (long long)rr * nx + (i - rr * bw);
    }
    const int dd = i / plane, rem = i - dd * plane;
    const int rr = pow2 ? (rem >> lbw) : rem / bw;
    return (long long)dd * zs + (long long)rr * nx + (rem - rr * bw);
  }
};
__device__ __forceinline__ BandWalk band_walk(int bd, int bh, int bw, int ny, int nx) {
  BandWalk w;
  w.bd = bd; w.bh = bh; w.bw = bw;
  w.lbw = 31 - __clz(bw);
  w.pow2 = (bw & (bw - 1)) == 0;
  w.plane = bh * bw;
  w.zs = (long long)ny * nx;
  w.nx = nx;
  return w;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums over the wave of NV values a lane at once (reduce-scatter, NV = 2^k <= 64): at
// each step xor 32, 16, ... a lane keeps the half of its values its lane bit selects
// and adds the partner's copy of it; once one value is left, the remaining xor steps
// finish its sum.  Lane l returns the sum of v[(l >> (6 - k)) & (NV - 1)] over the 64
// lanes: NV + 6 - k shuffles where NV wave_sum calls take 6 NV.
template <int NV, int O = 32>
__device__ __forceinline__ float wave_sum_rs(const float (&v)[NV]) {
  if constexpr (NV == 1) {
    float w = v[0];
#pragma unroll
    for (int o = O; o >= 1; o >>= 1) w += __shfl_xor(w, o, 64);
    return w;
  } else {
    const bool hi = threadIdx.x & O;
    float h[NV / 2];
#pragma unroll
    for (int i = 0; i < NV / 2; ++i)
      h[i] = (hi ? v[i + NV / 2] : v[i]) + __shfl_xor(hi ? v[i] : v[i + NV / 2], O, 64);
    return wave_sum_rs<NV / 2, O / 2>(h);
  }
}

}  // namespace vdamp

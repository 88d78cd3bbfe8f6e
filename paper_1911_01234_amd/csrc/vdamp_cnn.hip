// gfx950 kernels of the learned denoiser: a 6-layer circular 3x3 CNN (2 -> 48 -> ... ->
// 48 -> 2, ReLU, residual output) conditioned on the per-band noise levels tau_b, with
// BF16 weights and activations and FP32 accumulation on MFMA (v_mfma_f32_16x16x32_bf16).
//
// Convolution as an implicit GEMM per 16x16 pixel tile: M = output channels (16 per
// MFMA tile), N = 16 pixels of one tile row, K = (tap, input channel) with the tap
// outermost, so every operand fragment (8 consecutive K values) is 8 channels of one
// pixel: one 16-byte LDS read.  The input halo (18x18 pixels, circular wrap) and the
// whole weight matrix sit in LDS; workgroups are persistent over tiles so weights are
// loaded once per workgroup.  Operand layout of the MFMA (lane l, g = l / 16):
// A[m = l % 16][k = 8 g + i], B[k = 8 g + i][n = l % 16], D[m = 4 g + i][n = l % 16].
//
// Activations are [pixel][channels] BF16 (raw bits in uint16); channel counts are 48
// or 8 (the 2-channel input and output padded with zeros).
#include "vdamp_cnn_args.h"

namespace vdamp {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kCh = 48;
constexpr int kThr = 256;

// round-to-nearest-even FP32 -> BF16 bits (finite inputs)
__device__ __forceinline__ u16 f2bf(float f) {
  const unsigned u = __float_as_uint(f);
  return (u16)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(u16 b) { return __uint_as_float(((unsigned)b) << 16); }

// noise-level feature t_b = log(tau_b / s0^2), the ratio clamped below at 1e-12 so that
// a noiseless band (tau = 0) gives a finite value
__device__ __forceinline__ float tau_feature(float tau, float s0) {
  return logf(fmaxf(tau / (s0 * s0), 1e-12f));
}

// Waves a SIMD the register budget is sized for (the k-loop is fully unrolled so that
// fragment loads run ahead of the MFMAs; at 3 waves the 1-tile output layer spills).
constexpr int conv_waves(int) { return 2; }

template <int CIN, int KSTEPS, int MT, int MODE>
__global__ void __launch_bounds__(kThr) __attribute__((amdgpu_waves_per_eu(conv_waves(MT)))) k_conv(ConvArgs a) {
  constexpr int KPAD = KSTEPS * 32;
  // LDS pitches chosen for the 128-bank LDS, which serves a 16-byte read as two 8-byte
  // halves for 32 lanes at a time: 16 lanes read rows c of a fragment 16 bytes apart per
  // lane group, and these pitches map their 64 dwords to distinct banks (measured: the
  // former pitches of CIN + 8 and KPAD + 8 halves cost four conflict cycles a read)
  constexpr int PS = CIN;        // LDS halves per halo pixel
  constexpr int WS = KPAD + 16;  // LDS halves per weight row
  constexpr int CH8 = CIN / 8;
  __shared__ __align__(16) u16 s_in[18 * 18 * PS];
  __shared__ __align__(16) u16 s_w[MT * 16 * WS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, c = lane & 15;
  for (int i = tid; i < MT * 16 * (KPAD / 8); i += kThr) {
    const int row = i / (KPAD / 8), c8 = i - row * (KPAD / 8);
    *reinterpret_cast<uint4*>(&s_w[row * WS + c8 * 8]) =
        *reinterpret_cast<const uint4*>(&a.w[row * KPAD + c8 * 8]);
  }
  // the halo of the next tile is fetched into registers while the current one is
  // computed (software pipelining across the persistent tile loop)
  constexpr int HV = 18 * 18 * CH8;                 // 16-byte vectors of a halo
  constexpr int HPT = (HV + kThr - 1) / kThr;       // ... per thread
  uint4 pre[HPT];
#define CONV_FETCH(TI)                                                                   \
  {                                                                                      \
    const int2 tf = a.tiles[TI];                                                         \
    const SliceDev Sf = a.slices[tf.x];                                                  \
    const int fnx = Sf.nx, fny = Sf.ny, ftpr = fnx >> 4;                                 \
    const int fty0 = (tf.y / ftpr) * 16, ftx0 = (tf.y - (tf.y / ftpr) * ftpr) * 16;      \
    _Pragma("unroll") for (int q = 0; q < HPT; ++q) {                                    \
      const int i = tid + q * kThr;                                                      \
      pre[q] = make_uint4(0u, 0u, 0u, 0u);                                               \
      if (i < HV) {                                                                      \
        const int hp = i / CH8, c8 = i - hp * CH8;                                       \
        const int hy = hp / 18, hx = hp - hy * 18;                                       \
        int gy = fty0 + hy - 1, gx = ftx0 + hx - 1;                                      \
        gy += (gy < 0) ? fny : 0; gy -= (gy >= fny) ? fny : 0;                           \
        gx += (gx < 0) ? fnx : 0; gx -= (gx >= fnx) ? fnx : 0;                           \
        const long long pix = Sf.off + (long long)gy * fnx + gx;                         \
        pre[q] = *reinterpret_cast<const uint4*>(&a.in[pix * CIN + c8 * 8]);             \
      }                                                                                  \
    }                                                                                    \
  }
  if (blockIdx.x < a.ntiles) CONV_FETCH(blockIdx.x);
  // bias of this lane's output channels (mt * 16 + 4 g + i), loaded once
  float bias_r[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = mt * 16 + 4 * g + i;
      bias_r[mt][i] = (a.bias && (MODE == CV_RELU || co < 2)) ? a.bias[co] : 0.f;
    }
  for (int ti = blockIdx.x; ti < a.ntiles; ti += gridDim.x) {
    const int2 t = a.tiles[ti];
    const SliceDev S = a.slices[t.x];
    const int nx = S.nx, tpr = nx >> 4;
    const int ty0 = (t.y / tpr) * 16, tx0 = (t.y - (t.y / tpr) * tpr) * 16;
    __syncthreads();  // weights staged / previous tile done with s_in
#pragma unroll
    for (int q = 0; q < HPT; ++q) {
      const int i = tid + q * kThr;
      if (i < HV) {
        const int hp = i / CH8, c8 = i - hp * CH8;
        *reinterpret_cast<uint4*>(&s_in[hp * PS + c8 * 8]) = pre[q];
      }
    }
    __syncthreads();
    if (ti + (int)gridDim.x < a.ntiles) CONV_FETCH(ti + gridDim.x);
    float sb[MT][4];  // per-slice bias of the first layer
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        sb[mt][i] = (MODE == CV_RELU && a.sbias) ? a.sbias[t.x * kCh + mt * 16 + 4 * g + i] : 0.f;
    f32x4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
      const int k = ks * 32 + g * 8;
      const int tap = k / CIN, ci0 = k - tap * CIN;
      const bool valid = tap < 9;
      const int dy = tap / 3, dx = tap - dy * 3;
      bf16x8 A[MT], B[4];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        A[mt] = *reinterpret_cast<const bf16x8*>(&s_w[(mt * 16 + c) * WS + k]);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int r = wv * 4 + nt;
        if (valid)
          B[nt] = *reinterpret_cast<const bf16x8*>(&s_in[((r + dy) * 18 + c + dx) * PS + ci0]);
        else
          B[nt] = (bf16x8){};
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B[nt], acc[mt][nt], 0, 0, 0);
    }
    // epilogue: lane holds channels mt*16 + 4g + i of pixel (row wv*4 + nt, column c)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const long long gp = S.off + (long long)(ty0 + wv * 4 + nt) * nx + tx0 + c;
      if (MODE == CV_RELU || MODE == CV_MASK) {
        uint2 bw = make_uint2(0u, 0u);  // this pixel's ReLU pattern (read, or built)
        if (MODE == CV_MASK && a.bits) bw = a.bits[gp];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int co0 = mt * 16 + 4 * g;
          float z[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) z[i] = acc[mt][nt][i];
          if (MODE == CV_RELU) {
#pragma unroll
            for (int i = 0; i < 4; ++i) z[i] = fmaxf(z[i] + bias_r[mt][i] + sb[mt][i], 0.f);
          } else if (a.bits) {
            const unsigned word = (mt < 2 ? bw.x >> (16 * mt) : bw.y) >> (4 * g);
#pragma unroll
            for (int i = 0; i < 4; ++i) z[i] = ((word >> i) & 1u) ? z[i] : 0.f;
          } else {
            const uint2 mk = *reinterpret_cast<const uint2*>(&a.mask[gp * kCh + co0]);
            const u16 m4[4] = {(u16)(mk.x & 0xFFFF), (u16)(mk.x >> 16), (u16)(mk.y & 0xFFFF), (u16)(mk.y >> 16)};
#pragma unroll
            for (int i = 0; i < 4; ++i) z[i] = (bf2f(m4[i]) > 0.f) ? z[i] : 0.f;
          }
          uint2 o;
          o.x = (unsigned)f2bf(z[0]) | ((unsigned)f2bf(z[1]) << 16);
          o.y = (unsigned)f2bf(z[2]) | ((unsigned)f2bf(z[3]) << 16);
          *reinterpret_cast<uint2*>(&a.out[gp * kCh + co0]) = o;
          if (MODE == CV_RELU) {  // bit set where the stored BF16 activation is > 0
            const unsigned b4 = ((o.x & 0xFFFFu) ? 1u : 0u) | ((o.x >> 16) ? 2u : 0u) |
                                ((o.y & 0xFFFFu) ? 4u : 0u) | ((o.y >> 16) ? 8u : 0u);
            if (mt < 2) bw.x |= b4 << (16 * mt + 4 * g);
            else bw.y |= b4 << (4 * g);
          }
        }
        if (MODE == CV_RELU && a.bits_out) {  // uniform branch: every lane shuffles
          // the four lanes c + 16 g of a pixel hold its channel groups g
          bw.x |= __shfl_xor(bw.x, 16, 64);
          bw.y |= __shfl_xor(bw.y, 16, 64);
          bw.x |= __shfl_xor(bw.x, 32, 64);
          bw.y |= __shfl_xor(bw.y, 32, 64);
          if (g == 0) a.bits_out[gp] = bw;
        }
      } else if (g == 0) {  // channels 0 (real) and 1 (imaginary) of the output
        const float2 rin = a.resid[gp];
        float o0 = acc[0][nt][0], o1 = acc[0][nt][1];
        if (MODE == CV_LAST) {
          const float s = a.s0[t.x];
          o0 = s * (o0 + bias_r[0][0]);
          o1 = s * (o1 + bias_r[0][1]);
        }
        a.img_out[gp] = make_float2(rin.x - o0, rin.y - o1);
      }
    }
  }
#undef CONV_FETCH
}

// ------------------------------------------------------------------ weight gradient
// dW[co][k] = sum_p dz[p][co] h[p + off(tap(k))][ci(k)], k = tap * CIN + ci, as a GEMM
// with the pixels as reduction dimension: per tile the gradient tile dz is staged as
// [co][pixel] and the halo of h as [ci][halo pixel], so A fragments are 8 consecutive
// pixels of one channel (one 16-byte read) and B fragments 8 consecutive pixels of one
// shifted input channel.  Each workgroup accumulates over its tiles in registers and
// writes one partial matrix; a second kernel sums the partials in a fixed order.
// Also: partial bias gradients (sum over pixels of dz) and, for the first layer, the
// per-tile channel sums of dz that the per-slice bias gradient needs.

template <int CIN, int MT, int NT>
__global__ void __launch_bounds__(kThr) k_wgrad(WgradArgs a) {
  constexpr int DP = 256 + 8;      // LDS halves per gradient channel row
  constexpr int HP = 18 * 18 + 4;  // LDS halves per input channel (halo)
  constexpr int NACC = (MT * NT + 3) / 4;
  __shared__ __align__(16) u16 s_dz[MT * 16 * DP];
  __shared__ __align__(16) u16 s_h[CIN * HP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, c = lane & 15;
  f32x4 acc[NACC];
#pragma unroll
  for (int j = 0; j < NACC; ++j) acc[j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;  // thread 4 co (co < MT * 16): bias gradient of channel co
  for (int ti = blockIdx.x; ti < a.ntiles; ti += gridDim.x) {
    const int2 t = a.tiles[ti];
    const SliceDev S = a.slices[t.x];
    const int nx = S.nx, ny = S.ny, tpr = nx >> 4;
    const int ty0 = (t.y / tpr) * 16, tx0 = (t.y - (t.y / tpr) * tpr) * 16;
    __syncthreads();
    // gradient tile, transposed: s_dz[co][p] (channels >= cout are zero); each pixel's
    // channels arrive as 16-byte vectors of 8 (a pixel's dzc channels are 16-byte aligned)
    {
      const int p = tid;  // one pixel per thread
      const long long gp = S.off + (long long)(ty0 + (p >> 4)) * nx + tx0 + (p & 15);
      const uint4* src = reinterpret_cast<const uint4*>(a.dz + gp * a.dzc);
#pragma unroll
      for (int q = 0; q < MT * 2; ++q) {
        const uint4 v = (8 * q < a.dzc) ? src[q] : make_uint4(0u, 0u, 0u, 0u);
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int co = 8 * q + e;
          s_dz[co * DP + p] = (co < a.cout) ? (u16)(w[e >> 1] >> (16 * (e & 1))) : (u16)0;
        }
      }
    }
    // input halo, transposed: s_h[ci][hp], read as 16-byte vectors of 8 channels
    constexpr int CH8 = CIN / 8;
    for (int i = tid; i < 18 * 18 * CH8; i += kThr) {
      const int hp = i / CH8, c8 = i - hp * CH8;
      const int hy = hp / 18, hx = hp - hy * 18;
      int gy = ty0 + hy - 1, gx = tx0 + hx - 1;
      gy += (gy < 0) ? ny : 0; gy -= (gy >= ny) ? ny : 0;
      gx += (gx < 0) ? nx : 0; gx -= (gx >= nx) ? nx : 0;
      const uint4 v = *reinterpret_cast<const uint4*>(a.h + (S.off + (long long)gy * nx + gx) * CIN + 8 * c8);
      const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) s_h[(8 * c8 + e) * HP + hp] = (u16)(w[e >> 1] >> (16 * (e & 1)));
    }
    __syncthreads();
    // bias gradient and the tile's channel sums: four threads a channel, 64 pixels each
    // in order, the four partial sums combined in a fixed order ((q0 + q1) + (q2 + q3));
    // the threads of a channel are neighbouring lanes of one wave and whole waves take
    // part or not
    if (tid < 4 * MT * 16) {
      const int co = tid >> 2, qq = tid & 3;
      const uint4* row = reinterpret_cast<const uint4*>(&s_dz[co * DP + qq * 64]);
      float sacc = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint4 v = row[q];
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) sacc += bf2f((u16)(w[e >> 1] >> (16 * (e & 1))));
      }
      sacc += __shfl_xor(sacc, 1, 64);
      sacc += __shfl_xor(sacc, 2, 64);
      if (qq == 0) {
        bsum += sacc;
        if (a.tile_sums && co < kCh) a.tile_sums[(long long)ti * kCh + co] = sacc;
      }
    }
    // the k-loop stays rolled: unrolled, the hoisted fragment reads of its eight steps hold
    // about 370 registers (one wave a SIMD); rolled, about 200 (two workgroups a CU)
#pragma unroll 1
    for (int ks = 0; ks < 8; ++ks) {  // 256 pixels = 8 steps of 32
      const int p0 = ks * 32 + g * 8;   // 8 consecutive pixels of one tile row
      const int py = p0 >> 4, px = p0 & 15;
#pragma unroll
      for (int j = 0; j < NACC; ++j) {
        const int tile = wv + 4 * j;
        if (tile < MT * NT) {
          const int mt = tile / NT, nt = tile - mt * NT;
          const bf16x8 A = *reinterpret_cast<const bf16x8*>(&s_dz[(mt * 16 + c) * DP + p0]);
          const int n = nt * 16 + c;
          const int tap = n / CIN, ci = n - tap * CIN;
          bf16x8 B = (bf16x8){};
          if (tap < 9) {
            const int dy = tap / 3, dx = tap - dy * 3;
            const u16* hrow = &s_h[ci * HP + (py + dy) * 18 + px + dx];
            // with CIN a multiple of 16 the 16 columns of an n-tile share one tap, so dx
            // is the same on every lane; HP, the row pitch and px are even, so for even dx
            // the 8 values are 4-byte aligned and arrive as four 32-bit reads
            if (CIN % 16 == 0 && (dx & 1) == 0) {
              const unsigned* h32 = reinterpret_cast<const unsigned*>(hrow);
              const uint4 q = make_uint4(h32[0], h32[1], h32[2], h32[3]);
              B = *reinterpret_cast<const bf16x8*>(&q);
            } else {
              u16 tmp[8];
#pragma unroll
              for (int e = 0; e < 8; ++e) tmp[e] = hrow[e];
              B = *reinterpret_cast<const bf16x8*>(tmp);
            }
          }
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[j], 0, 0, 0);
        }
      }
    }
  }
  // partials: D[m = 4g + i][n = c] of each accumulator tile
  float* P = a.part + (long long)blockIdx.x * (MT * 16) * (NT * 16);
#pragma unroll
  for (int j = 0; j < NACC; ++j) {
    const int tile = wv + 4 * j;
    if (tile < MT * NT) {
      const int mt = tile / NT, nt = tile - mt * NT;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        P[(mt * 16 + 4 * g + i) * (NT * 16) + nt * 16 + c] = acc[j][i];
    }
  }
  if (tid < 4 * MT * 16 && (tid & 3) == 0) a.part_bias[(long long)blockIdx.x * (MT * 16) + (tid >> 2)] = bsum;
}

// Sum per-workgroup partials in a fixed order: out[i] = sum_w part[w][i].
__global__ void __launch_bounds__(kThr) k_sum_partials(const float* __restrict__ part, int nwg,
                                                       long long n, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * kThr + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int w = 0; w < nwg; ++w) s += part[(long long)w * n + i];
  out[i] = s;
}


// Reduce the weight-gradient partials of one layer into the flat FP32 gradient in the
// parameter layout W[co][ci][3][3], b[co]: gW[(co * cin + ci) * 9 + tap] = sum over
// workgroups of part[w][co][tap * cinp + ci]; gb[co] = sum of part_bias.  Two stages in a
// fixed order: up to kWgradReduceGroups contiguous groups of workgroups are summed in order,
// then the group sums in group order.
// Stage 1: column c of the partial matrices (or bias row c - rows * cols), summed over the
// workgroups of group blockIdx.y (a contiguous range of them, in order).  Neighbouring
// threads read neighbouring columns of one partial matrix.
__global__ void __launch_bounds__(kThr) k_reduce_wgrad1(const float* __restrict__ part,
                                                        const float* __restrict__ part_bias,
                                                        int nwg, int rows, int cols,
                                                        float* __restrict__ stage) {
  const int c = blockIdx.x * kThr + threadIdx.x;
  const int nm = rows * cols, n1 = nm + rows, G = gridDim.y, g = blockIdx.y;
  const int w0 = (int)((long long)g * nwg / G), w1 = (int)((long long)(g + 1) * nwg / G);
  if (c < nm) {
    float s = 0.f;
    for (int w = w0; w < w1; ++w) s += part[(long long)w * nm + c];
    stage[(long long)g * n1 + c] = s;
  } else if (c < n1) {
    float s = 0.f;
    for (int w = w0; w < w1; ++w) s += part_bias[(long long)w * rows + (c - nm)];
    stage[(long long)g * n1 + c] = s;
  }
}
// Stage 2: the group sums of each weight (co, ci, tap) and bias, in group order.
__global__ void __launch_bounds__(kThr) k_reduce_wgrad2(const float* __restrict__ stage, int G,
                                                        int rows, int cols, int cinp, int cout,
                                                        int cin, float* __restrict__ gW,
                                                        float* __restrict__ gb) {
  const int i = blockIdx.x * kThr + threadIdx.x;
  const int nw = cout * cin * 9, n1 = rows * cols + rows;
  int col = -1;
  if (i < nw) {
    const int co = i / (cin * 9), rem = i - co * cin * 9, ci = rem / 9, tap = rem - ci * 9;
    col = co * cols + tap * cinp + ci;
  } else if (i < nw + cout) {
    col = rows * cols + (i - nw);
  }
  if (col < 0) return;
  float s = 0.f;
  for (int g = 0; g < G; ++g) s += stage[(long long)g * n1 + col];
  if (i < nw)
    gW[i] = s;
  else
    gb[i - nw] = s;
}

// ------------------------------------------------------------------ small kernels
// u = (Re x, Im x) / s (s = s0 of the slice, or 1 for tangents) as BF16 [pixel][8].
__global__ void __launch_bounds__(kThr) k_pack_input(const SliceDev* slices, int batch,
                                                     const float2* __restrict__ x,
                                                     const float* __restrict__ s0,
                                                     long long npx, u16* __restrict__ out) {
  const long long p = (long long)blockIdx.x * kThr + threadIdx.x;
  if (p >= npx) return;
  float inv = 1.f;
  if (s0) {
    int lo = 0, hi = batch - 1;  // slice of pixel p
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (slices[mid].off <= p) lo = mid; else hi = mid - 1;
    }
    inv = 1.0f / s0[lo];
  }
  const float2 v = x[p];
  uint4 o;
  o.x = (unsigned)f2bf(v.x * inv) | ((unsigned)f2bf(v.y * inv) << 16);
  o.y = 0u; o.z = 0u; o.w = 0u;
  *reinterpret_cast<uint4*>(&out[p * 8]) = o;
}

// Per-slice first-layer bias: b1 + Wt log(tau / s0^2); tau[slice * tau_stride + band].
__global__ void k_slice_bias(const float* __restrict__ b1, const float* __restrict__ wt,
                             const float* __restrict__ tau, const float* __restrict__ s0,
                             int nb, int batch, int tau_stride, float* __restrict__ sb) {
  const int sl = blockIdx.x, co = threadIdx.x;
  if (sl >= batch || co >= kCh) return;
  float z = b1[co];
  for (int b = 0; b < nb; ++b) z += wt[co * nb + b] * tau_feature(tau[sl * tau_stride + b], s0[sl]);
  sb[sl * kCh + co] = z;
}

// Loss sum |x_out - x0|^2 / (s0^2 N_slice nsl) (per-block partials) and its gradient
// with respect to the last layer's output o: -2 s0 (x_out - x0) / (s0^2 N nsl), BF16 [p][8].
__global__ void __launch_bounds__(kThr) k_loss_grad(const SliceDev* slices, int batch,
                                                    const float2* __restrict__ xo,
                                                    const float2* __restrict__ x0,
                                                    const float* __restrict__ s0,
                                                    long long npx, u16* __restrict__ go,
                                                    float* __restrict__ part) {
  __shared__ float red[kThr / 64];
  const long long p = (long long)blockIdx.x * kThr + threadIdx.x;
  float l = 0.f;
  if (p < npx) {
    int lo = 0, hi = batch - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (slices[mid].off <= p) lo = mid; else hi = mid - 1;
    }
    const float s = s0[lo];
    const float nn = (float)slices[lo].ny * (float)slices[lo].nx * (float)batch;
    const float2 d = make_float2(xo[p].x - x0[p].x, xo[p].y - x0[p].y);
    l = (d.x * d.x + d.y * d.y) / (s * s * nn);
    const float k = -2.0f / (s * nn);
    uint4 o;
    o.x = (unsigned)f2bf(k * d.x) | ((unsigned)f2bf(k * d.y) << 16);
    o.y = 0u; o.z = 0u; o.w = 0u;
    *reinterpret_cast<uint4*>(&go[p * 8]) = o;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Fixed-order sum of n values into *out (one block).
__global__ void __launch_bounds__(kThr) k_sum_all(const float* __restrict__ v, long long n,
                                                  float* __restrict__ out) {
  __shared__ double red[kThr];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += kThr) s += (double)v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThr / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (float)red[0];
}

// Gradient of the per-slice bias weights: dWt[co][b] = sum_slices S[slice][co] t[slice][b],
// with S the per-slice sums of the first layer's pre-activation gradient (the slice's
// per-tile sums, added in a fixed order: lane-strided, then a wave tree).
__global__ void __launch_bounds__(256) k_wt_grad(const float* __restrict__ tile_sums,
                                                 const int* __restrict__ tile_off,
                                                 const float* __restrict__ tau,
                                                 const float* __restrict__ s0, int nb, int batch,
                                                 int tau_stride, float* __restrict__ dwt) {
  // one workgroup per output channel; wave w takes slices w, w + 4, ...: its lanes sum
  // the slice's tile partials, and lane b < nb accumulates the band-b term
  __shared__ float red[4][kMaxBands];
  const int co = blockIdx.x, lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (co >= kCh) return;
  float acc = 0.f;
  for (int sl = wid; sl < batch; sl += 4) {
    float ssum = 0.f;
    for (int ti = tile_off[sl] + lane; ti < tile_off[sl + 1]; ti += 64) ssum += tile_sums[(long long)ti * kCh + co];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) ssum += __shfl_xor(ssum, o, 64);
    if (lane < nb) acc += ssum * tau_feature(tau[sl * tau_stride + lane], s0[sl]);
  }
  if (lane < kMaxBands) red[wid][lane] = acc;
  __syncthreads();
  if (threadIdx.x < nb) dwt[co * nb + threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// Adam on the flat FP32 parameters.
__global__ void __launch_bounds__(kThr) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                               float* __restrict__ m, float* __restrict__ v,
                                               int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * kThr + threadIdx.x;
  if (i >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Pack FP32 weights W[co][ci][3][3] into the BF16 forward layout [co][tap * CINP + ci]
// (rows up to coutp, K padded with zeros to kpad), and into the input-gradient layout
// [ci][tap' * COUTP' + co] with the flipped tap (tap' = 8 - tap).
__global__ void k_pack_w(const float* __restrict__ W, int cout, int cin, int cinp, int coutp,
                         int kpad, u16* __restrict__ wf, int dgrad_coutp, int dgrad_kpad,
                         u16* __restrict__ wd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < coutp * kpad) {
    const int co = i / kpad, k = i - co * kpad;
    const int tap = k / cinp, ci = k - tap * cinp;
    float v = 0.f;
    if (co < cout && tap < 9 && ci < cin) v = W[(co * cin + ci) * 9 + tap];
    wf[i] = f2bf(v);
  }
  if (wd && i < cin * dgrad_kpad) {
    const int ci = i / dgrad_kpad, k = i - ci * dgrad_kpad;
    const int tapf = k / dgrad_coutp, co = k - tapf * dgrad_coutp;
    float v = 0.f;
    if (tapf < 9 && co < cout) v = W[(co * cin + ci) * 9 + (8 - tapf)];
    wd[i] = f2bf(v);
  }
}

// ------------------------------------------------------------------ launchers
#define CONV_CASE(CIN, KS, MT, MODE)                                                       \
  hipLaunchKernelGGL((k_conv<CIN, KS, MT, MODE>), dim3(grid), dim3(kThr), 0, st, a)

hipError_t launch_conv(const ConvArgs& a, int cin, int mt, int mode, int grid, hipStream_t st) {
  if (cin == 8 && mt == 3 && mode == CV_RELU) CONV_CASE(8, 3, 3, CV_RELU);
  else if (cin == 8 && mt == 3 && mode == CV_MASK) CONV_CASE(8, 3, 3, CV_MASK);
  else if (cin == 48 && mt == 3 && mode == CV_RELU) CONV_CASE(48, 14, 3, CV_RELU);
  else if (cin == 48 && mt == 3 && mode == CV_MASK) CONV_CASE(48, 14, 3, CV_MASK);
  else if (cin == 48 && mt == 1 && mode == CV_LAST) CONV_CASE(48, 14, 1, CV_LAST);
  else if (cin == 48 && mt == 1 && mode == CV_LAST_TAN) CONV_CASE(48, 14, 1, CV_LAST_TAN);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs& a, int layer, int grid, hipStream_t st) {
  if (layer == 1)
    hipLaunchKernelGGL((k_wgrad<8, 3, 5>), dim3(grid), dim3(kThr), 0, st, a);
  else if (layer == 6)
    hipLaunchKernelGGL((k_wgrad<48, 1, 27>), dim3(grid), dim3(kThr), 0, st, a);
  else
    hipLaunchKernelGGL((k_wgrad<48, 3, 27>), dim3(grid), dim3(kThr), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_reduce_wgrad(const float* part, const float* part_bias, int nwg, int rows,
                               int cols, int cinp, int cout, int cin, float* stage, float* gW,
                               float* gb, hipStream_t st) {
  const int n1 = rows * cols + rows, n = cout * cin * 9 + cout;
  const int G = nwg < kWgradReduceGroups ? nwg : kWgradReduceGroups;
  hipLaunchKernelGGL(k_reduce_wgrad1, dim3((n1 + kThr - 1) / kThr, G), dim3(kThr), 0, st, part,
                     part_bias, nwg, rows, cols, stage);
  hipLaunchKernelGGL(k_reduce_wgrad2, dim3((n + kThr - 1) / kThr), dim3(kThr), 0, st, stage, G,
                     rows, cols, cinp, cout, cin, gW, gb);
  return hipGetLastError();
}
hipError_t launch_sum_partials(const float* part, int nwg, long long n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)((n + kThr - 1) / kThr)), dim3(kThr), 0, st,
                     part, nwg, n, out);
  return hipGetLastError();
}
hipError_t launch_pack_input(const SliceDev* slices, int batch, const float2* x, const float* s0,
                             long long npx, u16* out, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((npx + kThr - 1) / kThr)), dim3(kThr), 0, st,
                     slices, batch, x, s0, npx, out);
  return hipGetLastError();
}
hipError_t launch_slice_bias(const float* b1, const float* wt, const float* tau, const float* s0,
                             int nb, int batch, int tau_stride, float* sb, hipStream_t st) {
  hipLaunchKernelGGL(k_slice_bias, dim3(batch), dim3(64), 0, st, b1, wt, tau, s0, nb, batch, tau_stride, sb);
  return hipGetLastError();
}
hipError_t launch_loss_grad(const SliceDev* slices, int batch, const float2* xo, const float2* x0,
                            const float* s0, long long npx, u16* go, float* part, float* loss,
                            hipStream_t st) {
  const unsigned blocks = (unsigned)((npx + kThr - 1) / kThr);
  hipLaunchKernelGGL(k_loss_grad, dim3(blocks), dim3(kThr), 0, st, slices, batch, xo, x0, s0, npx,
                     go, part);
  hipLaunchKernelGGL(k_sum_all, dim3(1), dim3(kThr), 0, st, part, (long long)blocks, loss);
  return hipGetLastError();
}
hipError_t launch_wt_grad(const float* tile_sums, const int* tile_off, const float* tau,
                          const float* s0, int nb, int batch, int tau_stride, float* dwt, hipStream_t st) {
  hipLaunchKernelGGL(k_wt_grad, dim3(kCh), dim3(256), 0, st, tile_sums, tile_off, tau, s0, nb,
                     batch, tau_stride, dwt);
  return hipGetLastError();
}
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float c1,
                       float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((n + kThr - 1) / kThr), dim3(kThr), 0, st, p, g, m, v, n, lr, c1, c2);
  return hipGetLastError();
}
hipError_t launch_pack_w(const float* W, int cout, int cin, int cinp, int coutp, int kpad, u16* wf,
                         int dcoutp, int dkpad, u16* wd, hipStream_t st) {
  const int n = (coutp * kpad > cin * dkpad) ? coutp * kpad : cin * dkpad;
  hipLaunchKernelGGL(k_pack_w, dim3((n + kThr - 1) / kThr), dim3(kThr), 0, st, W, cout, cin, cinp,
                     coutp, kpad, wf, dcoutp, dkpad, wd);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace vdamp

// gfx950 kernel of the per-band threshold search (Section 3: complex soft thresholding
// with a SURE-optimal threshold per subband; Algorithm 1, lines 6-7).
#include "vdamp_device.hpp"

namespace vdamp {

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
// piecewise logarithmic: fine (2^MB per binade) over v in [2^-6, 2^3), where the
// noise-only keys concentrate (key/tau of a CN(0, tau) coefficient is Exp(1)), coarse
// (2^LB per binade) over [2^-16, 2^-6) and [2^3, 2^23); keys outside fall into the first
// or the last used bucket.  (tau = 0 sends every key to the last bucket: the search
// then takes its full-sort path.)
template <int NB> struct SureBuckets;
template <> struct SureBuckets<10240> { static constexpr int LB = 5, MB = 10; };
template <> struct SureBuckets<2560> { static constexpr int LB = 3, MB = 8; };

template <int NB>
__device__ __forceinline__ int sure_bucket(float key, float inv_tau) {
  constexpr int LB = SureBuckets<NB>::LB, MB = SureBuckets<NB>::MB;
  constexpr unsigned E_LO = 111u << 23, E_MID = 121u << 23, E_HI = 130u << 23;
  constexpr int N_LO = 10 << LB, N_MID = 9 << MB, N_HI = 20 << LB;
  static_assert(N_LO + N_MID + N_HI <= NB, "bucket layout");
  const unsigned e = __float_as_uint(key * inv_tau);
  if (e < E_MID) return (e < E_LO) ? 0 : (int)((e - E_LO) >> (23 - LB));
  if (e < E_HI) return N_LO + (int)((e - E_MID) >> (23 - MB));
  const unsigned v = (e - E_HI) >> (23 - LB);
  return N_LO + N_MID + (int)min(v, (unsigned)(N_HI - 1));
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
constexpr int kSureBucketLimit = 64;

// LDS words of a size class: the bucket table and the sorted keys with one pad word per
// 16 keys.  With up to 16 keys a thread the keys overlay the table (each thread keeps
// its keys' bucket bounds in registers before the table is overwritten), which halves
// the LDS of the 16384-key class; with 32 keys a thread those registers would spill.
constexpr bool sure_overlay(int KPT) { return KPT <= 16; }
// Waves per SIMD the compiler is asked to fit (register budget): 8 for the classes with
// up to 16 keys a thread (two 1024-thread workgroups per CU; a few registers spill,
// measured faster than one workgroup), no constraint for the 32-key class.
constexpr int sure_waves(int NT, int KPT) { return KPT <= 16 ? 8 : 1; }
constexpr int sure_smem_words(int NB, int MAXK, int KPT) {
  return sure_overlay(KPT) ? ((NB + 1 > MAXK + MAXK / 16 + 1) ? NB + 1 : MAXK + MAXK / 16 + 1)
                           : NB + 1 + MAXK + MAXK / 16 + 1;
}

template <int NT, int KPT, int NB, int MAXK>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sure_waves(NT, KPT))))
k_sure(KArgs a) {
  static_assert(NT * KPT >= MAXK, "keys per thread");
  constexpr bool OV = sure_overlay(KPT);
  __shared__ __align__(16) int sure_smem[sure_smem_words(NB, MAXK, KPT)];
  constexpr int NW = NT / 64;
  constexpr int BPT = NB / NT;
  __shared__ double wsA[NW], wsR[NW], bv[NW], bR[NW];
  __shared__ int bi[NW], wsC[NW], wsM[NW];
  __shared__ float tau_sh;
  __shared__ int maxc_sh;
  int* off = sure_smem;                                                 // [NB + 1]
  float* const sk = reinterpret_cast<float*>(sure_smem + (OV ? 0 : NB + 1));  // sorted keys
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
  if (maxc_sh <= kSureBucketLimit) {
    // bucket bounds and slot into registers, packed as offset | count << 15 | slot << 22
    // (offsets < 2^15, counts and slots <= kSureBucketLimit < 2^7); the table is then
    // overwritten by the keys
    static_assert(MAXK < (1 << 15) && kSureBucketLimit < (1 << 7), "packed bucket bounds");
    int bpk[OV ? KPT : 1];
    if constexpr (OV) {
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const int i = tid + j * NT;
        bpk[j] = 0;
        if (i < Nb) {
          const int bk = sure_bucket<NB>(kk[j], inv_tau);
          const int lo = off[bk];
          bpk[j] = lo | ((off[bk + 1] - lo) << 15) | (pos[j] << 22);
        }
      }
      __syncthreads();
    }
#define SURE_BOUNDS(j, lo, hi, slot)                 \
  if constexpr (OV) {                                \
    lo = bpk[j] & 0x7FFF;                            \
    hi = lo + ((bpk[j] >> 15) & 0x7F);               \
    slot = bpk[j] >> 22;                             \
  } else {                                           \
    const int bk_ = sure_bucket<NB>(kk[j], inv_tau); \
    lo = off[bk_];                                   \
    hi = off[bk_ + 1];                               \
    slot = pos[j];                                   \
  }
    // scatter into bucket slots
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      if (i < Nb) {
        int lo, hi, slot;
        SURE_BOUNDS(j, lo, hi, slot);
        (void)hi;
        sk[skx(lo + slot)] = kk[j];
      }
    }
    __syncthreads();
    // final position = bucket offset + rank within the bucket (ties by slot)
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      if (i < Nb) {
        int lo, hi, slot;
        SURE_BOUNDS(j, lo, hi, slot);
        const float v = kk[j];
        const int me = lo + slot;
        int rank = 0;
        for (int x = lo; x < hi; ++x) {
          const float u = sk[skx(x)];
          rank += (u < v) || (u == v && x < me);
        }
        if constexpr (OV) bpk[j] = lo + rank;  // final position
        else pos[j] = lo + rank;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      if (i < Nb) sk[skx(OV ? bpk[j] : pos[j])] = kk[j];
    }
    __syncthreads();
#undef SURE_BOUNDS
  } else {
    // Full sort: a bitonic network whose compare-exchanges all put the smaller key
    // first (each merge starts by comparing mirrored positions), so +inf padding up to
    // the next power of two never moves and needs no storage: only pairs with both
    // indices < Nb are compared.
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      if (i < Nb) sk[skx(i)] = kk[j];
    }
    __syncthreads();
    for (int k = 2; k <= npad; k <<= 1) {
      for (int i = tid; i < (npad >> 1); i += NT) {
        const int half = k >> 1;
        const int blk = i / half, ofs = i - blk * half;
        const int lo = blk * k + ofs, hi = blk * k + k - 1 - ofs;
        if (hi < Nb) {
          const float x = sk[skx(lo)], y = sk[skx(hi)];
          if (x > y) { sk[skx(lo)] = y; sk[skx(hi)] = x; }
        }
      }
      __syncthreads();
      for (int j = k >> 2; j > 0; j >>= 1) {
        for (int i = tid; i < (npad >> 1); i += NT) {
          const int lo = 2 * j * (i / j) + (i & (j - 1));
          const int hi = lo + j;
          if (hi < Nb) {
            const float x = sk[skx(lo)], y = sk[skx(hi)];
            if (x > y) { sk[skx(lo)] = y; sk[skx(hi)] = x; }
          }
        }
        __syncthreads();
      }
    }
  }
  const double tau = (double)tau_sh;
  const float kmax = sk[skx(Nb - 1)];
  const int E = (Nb + NT - 1) / NT;
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
    if (a.smin)  // all-zero band: eta = 0 gives SURE = -N_b tau
      a.smin[sl * kMaxBands + b] = (!(kmax > 0.f) || fi == 0x7fffffff) ? (float)(-Nbd * tau) : (float)fb;
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

// Size classes: up to 4096 keys (256 threads, 2560 buckets), up to 16384 keys
// (1024 threads, 16 keys each) and up to kSureMaxKeys keys (1024 threads, 32 keys each),
// the last two with 10240 buckets.  All LDS is static: the largest class uses about
// 158 KB of the 160 KB a gfx950 workgroup may hold.
hipError_t launch_sure(const KArgs& a, int cls, hipStream_t st) {
  if (cls == 2)
    hipLaunchKernelGGL((k_sure<1024, 32, 10240, kSureMaxKeys>), dim3(a.nwork), dim3(1024), 0, st, a);
  else if (cls == 1)
    hipLaunchKernelGGL((k_sure<1024, 16, 10240, 4 * kSureSmall>), dim3(a.nwork), dim3(1024), 0, st, a);
  else
    hipLaunchKernelGGL((k_sure<256, 16, 2560, kSureSmall>), dim3(a.nwork), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace vdamp

// gfx950 kernel of the per-band threshold search (Section 3: complex soft thresholding
// with a SURE-optimal threshold per subband; the denoising and alpha steps of Algorithm 1).
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

// The wave index of a thread, as a scalar (it is the same for every lane of a wave;
// held in a scalar register, the values derived from it need no vector registers).
__device__ __forceinline__ int wave_id(int tid) { return __builtin_amdgcn_readfirstlane(tid >> 6); }

// Value of lane src (the same for every lane of the wave, e.g. derived from the wave
// index) broadcast to the wave: a scalar read of the lane, no LDS permute and no
// per-lane address register.
__device__ __forceinline__ int wave_bcast(int v, int src) {
  return __builtin_amdgcn_readlane(v, __builtin_amdgcn_readfirstlane(src));
}
__device__ __forceinline__ double wave_bcast(double v, int src) {
  const int s = __builtin_amdgcn_readfirstlane(src);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), s),
                          __builtin_amdgcn_readlane(__double2loint(v), s));
}

// Exclusive prefix (and suffix) over the NW per-wave totals tot[0..NW) at wave wid, for
// every lane of the wave: lanes load one total each and scan with shuffles (no per-thread
// loop over the waves, which would hold the totals in registers).
template <int NW>
__device__ __forceinline__ int wave_offset_int(const int* tot, int wid, int lane) {
  const int v = wave_incl_prefix_int(lane < NW ? tot[lane] : 0, lane);
  const int o = wave_bcast(v, wid > 0 ? wid - 1 : 0);
  return wid > 0 ? o : 0;
}
template <int NW>
__device__ __forceinline__ double wave_offset_prefix(const double* tot, int wid, int lane) {
  const double v = wave_incl_prefix(lane < NW ? tot[lane] : 0.0, lane);
  const double o = wave_bcast(v, wid > 0 ? wid - 1 : 0);
  return wid > 0 ? o : 0.0;
}
template <int NW>
__device__ __forceinline__ double wave_offset_suffix(const double* tot, int wid, int lane) {
  const double v = wave_incl_suffix(lane < NW ? tot[lane] : 0.0, lane);
  const double o = wave_bcast(v, wid + 1 < NW ? wid + 1 : 0);
  return wid + 1 < NW ? o : 0.0;
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
template <> struct SureBuckets<5120> { static constexpr int LB = 3, MB = 9; };
template <> struct SureBuckets<19456> { static constexpr int LB = 5, MB = 11; };
template <> struct SureBuckets<3072> { static constexpr int LB = 4, MB = 8; };

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

// The best threshold found so far by a thread: SURE value v; m keys at or below the
// threshold; R = sum of 1/a over the keys above it; key = the FP32 key thresholding
// compares |r|^2 against; for a threshold strictly between two keys (continuous search)
// inner = 1 and th its value, else theta = sqrt(key).  Order: smaller v, then smaller m,
// then a key before a threshold just above it (ties go to the smaller theta).
struct SureBest {
  double v, R, th;
  int m, inner;
  float key;
};
__device__ __forceinline__ bool sure_better(double v, int m, int inner, const SureBest& b) {
  return v < b.v || (v == b.v && (m < b.m || (m == b.m && inner < b.inner)));
}
__device__ __forceinline__ SureBest sure_none() {
  SureBest b;
  b.v = __builtin_huge_val();
  b.R = 0.0;
  b.th = 0.0;
  b.m = 0x7fffffff;
  b.inner = 0;
  b.key = 0.f;
  return b;
}

// Continuous search inside an open interval between keys klo < khi holding m keys at or
// below it, with A = sum of those keys and R = sum of 1/a above: SURE is the convex
// quadratic A - m tl + (N_b - m)(theta^2 + tl) - td theta R, minimised at
// theta* = td R / (2 (N_b - m)); it counts when sqrt(klo) < theta* < sqrt(khi).  Its key
// is fl(theta*)^2 kept inside [klo, khi) so that thresholding keeps exactly the keys
// above the interval.  For single coefficients tl = td = tau; for groups of d
// coefficients (keys = squared group norms, N_b = the number of groups) tl = d tau and
// td = (2d - 1) tau: Stein's estimate over the group's 2d real dimensions.
__device__ __forceinline__ void sure_inner(float klo, float khi, double A, int m, double R, double tl,
                                           double td, double Nbd, SureBest& best) {
  const double nm = Nbd - (double)m;
  if (!(nm > 0.0) || !(R > 0.0)) return;
  const double t = td * R / (2.0 * nm);
  if (!(t > sqrt((double)klo)) || !(t < sqrt((double)khi))) return;
  const double v = A - (double)m * tl + nm * (t * t + tl) - td * t * R;
  if (!sure_better(v, m, 1, best)) return;
  const float tf = (float)t;
  float key = __fmul_rn(tf, tf);
  if (!(key < khi)) key = __uint_as_float(__float_as_uint(khi) - 1u);  // largest float below khi
  if (key < klo) key = klo;
  best.v = v;
  best.m = m;
  best.inner = 1;
  best.R = R;
  best.key = key;
  best.th = t;
}

// SURE at every candidate of the sorted keys: each thread walks a contiguous chunk with
// a = sqrt(key), A_m = sum_{i<=m} a_i^2 and R_m = sum_{i>m} 1/a_i (FP64 accumulation of
// FP32 terms, chunk offsets from FP64 prefix/suffix scans) and evaluates
// SURE(m) = A_m - m tl + (N_b - m)(a_m^2 + tl) - td a_m R_m at the last index of each
// run of equal keys with a > 0 (tl, td as in sure_inner); with cont, also the
// quadratic's minimum inside every interval between distinct keys (sure_inner), from 0
// up to the smallest positive key onwards.  Per thread the best (SureBest).
// One key of the walk: key k2 at sorted index i, the next key knext (+inf after the
// last), the previous key kprev (continuous mode); A (sum of a^2 below i) and Rrun (sum
// of 1/a from i on) advance past the key.
template <bool CONT>
__device__ __forceinline__ void walk_step(float k2, float knext, float kprev, int i, int Nb, double& A,
                                          double& Rrun, double tl, double td, double Nbd, SureBest& best) {
  if (CONT && k2 > 0.f && !(kprev > 0.f))  // the interval (0, a_i) below the first positive key
    sure_inner(0.f, k2, A, i, Rrun, tl, td, Nbd, best);
  A += (double)k2;
  if (k2 > 0.f) {
    Rrun -= (double)__frsqrt_rn(k2);  // now the sum over indices > i
    if (knext > k2) {                 // last index of a run of equal keys
      const double x = (double)__fsqrt_rn(k2);
      const double m = (double)(i + 1);
      const double sv = A - m * tl + (Nbd - m) * ((double)k2 + tl) - td * x * Rrun;
      // a thread's candidates come in increasing m, so without inner thresholds a
      // strictly smaller value is the only way to win
      if (CONT ? sure_better(sv, i + 1, 0, best) : sv < best.v) {
        best.v = sv;
        best.m = i + 1;
        best.inner = 0;
        best.R = Rrun;
        best.key = k2;
      }
      if (CONT && i + 1 < Nb) sure_inner(k2, knext, A, i + 1, Rrun, tl, td, Nbd, best);
    }
  }
}

// SURE at every candidate of the sorted keys: each thread walks a contiguous chunk with
// a = sqrt(key), A_m = sum_{i<=m} a_i^2 and R_m = sum_{i>m} 1/a_i (FP64 accumulation of
// FP32 terms, chunk offsets from FP64 prefix/suffix scans) and evaluates
// SURE(m) = A_m - m tl + (N_b - m)(a_m^2 + tl) - td a_m R_m at the last index of each
// run of equal keys with a > 0 (tl, td as in sure_inner); with cont, also the
// quadratic's minimum inside every interval between distinct keys (sure_inner), from 0
// up to the smallest positive key onwards.  Per thread the best (SureBest).
// CH = 16: a thread whose chunk holds exactly 16 keys starting at a multiple of 16 reads
// them once into registers (contiguous in the padded layout) and walks them unrolled;
// the sums and the order of every operation are those of the general loop.
template <int NT, bool CONT, int CH>
__device__ void sure_walk_t(const float* sk, int Nb, double tl, double td, double* wsA, double* wsR,
                            SureBest& best) {
  static_assert(CH == 0 || CH == 16, "chunk of 16 keys or none");
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = wave_id(tid);
  const int E = (Nb + NT - 1) / NT;
  const int i0 = tid * E;
  const int i1 = min(i0 + E, Nb);
  const bool full = CH > 0 && E == CH && i1 - i0 == CH;
  double cA = 0.0, cR = 0.0;
  float kc[CH > 0 ? CH : 1];
  if (full) {
    const float* base = sk + skx(i0);
#pragma unroll
    for (int k = 0; k < CH; ++k) kc[k] = base[k];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      cA += (double)kc[k];
      if (kc[k] > 0.f) cR += (double)__frsqrt_rn(kc[k]);
    }
  } else {
    for (int i = i0; i < i1; ++i) {
      const float k2 = sk[skx(i)];
      cA += (double)k2;
      if (k2 > 0.f) cR += (double)__frsqrt_rn(k2);
    }
  }
  const double pA = wave_incl_prefix(cA, lane);
  const double sR = wave_incl_suffix(cR, lane);
  if (lane == 63) wsA[wid] = pA;
  if (lane == 0) wsR[wid] = sR;
  __syncthreads();
  const double offA = wave_offset_prefix<NW>(wsA, wid, lane);
  const double offR = wave_offset_suffix<NW>(wsR, wid, lane);
  double A = offA + pA - cA;          // sum of a^2 over indices < i0
  double Rrun = offR + sR;            // sum of 1/a over indices >= i0
  best = sure_none();
  const double Nbd = (double)Nb;
  if (full) {
    const float after = (i1 < Nb) ? sk[skx(i1)] : __builtin_huge_valf();
    float kprev = (CONT && i0 > 0) ? sk[skx(i0 - 1)] : 0.f;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      walk_step<CONT>(kc[k], k + 1 < CH ? kc[k + 1] : after, kprev, i0 + k, Nb, A, Rrun, tl, td, Nbd, best);
      if (CONT) kprev = kc[k];
    }
    return;
  }
  float knext = (i0 < i1) ? sk[skx(i0)] : 0.f;
  float kprev = (CONT && i0 > 0 && i0 < i1) ? sk[skx(i0 - 1)] : 0.f;
  for (int i = i0; i < i1; ++i) {
    const float k2 = knext;
    knext = (i + 1 < Nb) ? sk[skx(i + 1)] : __builtin_huge_valf();
    walk_step<CONT>(k2, knext, kprev, i, Nb, A, Rrun, tl, td, Nbd, best);
    if (CONT) kprev = k2;
  }
}
template <int NT, int CH = 0>
__device__ void sure_walk(const float* sk, int Nb, double tl, double td, bool cont, double* wsA, double* wsR,
                          SureBest& best) {
  if (cont)  // the continuous mode's inner-interval checks keep the general loop
    sure_walk_t<NT, true, 0>(sk, Nb, tl, td, wsA, wsR, best);
  else
    sure_walk_t<NT, false, CH>(sk, Nb, tl, td, wsA, wsR, best);
}

// Workgroup argmin of the per-thread bests (sure_better), then theta (sqrt(key) for a
// key, the continuous minimiser otherwise), its key and alpha = ((N_b - m) - theta R /
// 2) / N_b (alpha step) for the band, and the band's outputs.  No candidate (every key
// zero): eta = 0, alpha = 0.  With groups of GD coefficients (Nb groups) alpha is half
// the real divergence per coefficient, (GD (N_b - m) - (2 GD - 1) theta R / 2) / (GD N_b).
template <int NT, int GD = 1>
__device__ void sure_finish(const KArgs& a, int sl, int b, int Nb, float tau_f, SureBest best,
                            SureBest* fin) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = wave_id(tid);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    SureBest ob;
    ob.v = __shfl_xor(best.v, o, 64);
    ob.m = __shfl_xor(best.m, o, 64);
    ob.inner = __shfl_xor(best.inner, o, 64);
    ob.R = __shfl_xor(best.R, o, 64);
    ob.th = __shfl_xor(best.th, o, 64);
    ob.key = __shfl_xor(best.key, o, 64);
    if (sure_better(ob.v, ob.m, ob.inner, best)) best = ob;
  }
  if (lane == 0) fin[wid] = best;
  __syncthreads();
  if (tid == 0) {
    SureBest f = fin[0];
    for (int w = 1; w < NW; ++w)
      if (sure_better(fin[w].v, fin[w].m, fin[w].inner, f)) f = fin[w];
    const double Nbd = (double)Nb, tau = (double)tau_f, dd = (double)GD;
    const bool none = f.m == 0x7fffffff;
    float th, th2, al;
    if (none) {
      th = 0.f;
      th2 = 0.f;
      al = 0.f;
    } else {
      th2 = f.key;
      th = f.inner ? (float)f.th : __fsqrt_rn(th2);
      const double m = (double)f.m;
      al = (float)(((Nbd - m) * dd - 0.5 * (2.0 * dd - 1.0) * (double)th * f.R) / (dd * Nbd));
    }
    if (a.smin)  // every key zero: eta = 0 gives SURE = -N_b tau per coefficient
      a.smin[sl * kMaxBands + b] = none ? (float)(-Nbd * (dd * tau)) : (float)f.v;
    a.theta[sl * kMaxBands + b] = th;
    a.thr2[sl * kMaxBands + b] = th2;
    a.alpha[sl * kMaxBands + b] = al;
    a.tau[sl * kMaxBands + b] = tau_f;
    if (a.trace) {
      float* t = a.trace + (((long long)a.iter * a.batch + sl) * a.nbands + b) * 3;
      t[0] = tau_f;
      t[1] = th;
      t[2] = al;
    }
  }
}

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
//      alpha = ((N_b - m) - theta R_m / 2) / N_b (alpha step).
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

// GD = 2: keys are the squared norms of horizontal pairs (VDAMP_FLAG_GROUP_PAIRS, slices
// only), N_b the number of pairs.
template <int NT, int KPT, int NB, int MAXK, int GD>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sure_waves(NT, KPT))))
k_sure(KArgs a) {
  static_assert(NT * KPT >= MAXK, "keys per thread");
  constexpr bool OV = sure_overlay(KPT);
  __shared__ __align__(16) int sure_smem[sure_smem_words(NB, MAXK, KPT)];
  constexpr int NW = NT / 64;
  constexpr int BPT = NB / NT;
  __shared__ double wsA[NW], wsR[NW];
  __shared__ int wsC[NW], wsM[NW];
  __shared__ SureBest fin[NW];
  __shared__ float tau_sh;
  __shared__ int maxc_sh;
  int* off = sure_smem;                                                 // [NB + 1]
  float* const sk = reinterpret_cast<float*>(sure_smem + (OV ? 0 : NB + 1));  // sorted keys
  const int2 item = a.work[blockIdx.x];
  const int sl = item.x, b = item.y, s = a.levels;
  const SliceDev S = a.slices[sl];
  const int tid = threadIdx.x, lane = tid & 63, wid = wave_id(tid);
  int d0, r0, c0, bd, bh, bw;
  band_geom3(b, s, S.nd, S.ny, S.nx, d0, r0, c0, bd, bh, bw);
  const int Nb = bd * bh * bw / GD;
  int npad = 1;
  while (npad < Nb) npad <<= 1;

  for (int i = tid; i <= NB; i += NT) off[i] = 0;
  if (wid == 0) {
    const int ncs = S.ncs;
    double acc = 0.0;
    for (int i = lane; i < ncs; i += 64) acc += (double)a.tau_part[(S.colstrip0 + i) * kMaxBands + b];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) tau_sh = (float)acc;
  }
  // load the band (coalesced along rows) while the counters are cleared
  const float2* r = a.r + S.off + ((long long)d0 * S.ny + r0) * S.nx + c0;
  const int lbw = 31 - __clz(bw);  // band widths are powers of two times 1, 3 or 5
  const bool pow2 = (bw & (bw - 1)) == 0;
  float kk[KPT];
  if constexpr (GD == 2) {  // pairs x = 2j, 2j + 1 of a slice's band rows (bw is even)
    const int lbp = lbw - 1, bwp = bw >> 1;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      kk[j] = 0.f;
      if (i < Nb) {
        const int rr = pow2 ? (i >> lbp) : i / bwp;
        const float4 v = *reinterpret_cast<const float4*>(r + (long long)rr * S.nx + 2 * (i - rr * bwp));
        kk[j] = key_pair_rn(lo2(v), hi2(v));
      }
    }
  } else if (bd == 1) {  // a slice's band (the branch stays outside the unrolled loads)
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      kk[j] = 0.f;
      if (i < Nb) {
        const int rr = pow2 ? (i >> lbw) : i / bw;
        kk[j] = key_rn(r[(long long)rr * S.nx + (i - rr * bw)]);
      }
    }
  } else {  // a volume's band
    const BandWalk bwk = band_walk(bd, bh, bw, S.ny, S.nx);
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      kk[j] = 0.f;
      if (i < Nb) kk[j] = key_rn(r[bwk.at(i)]);
    }
  }
  __syncthreads();
  const float inv_tau = 1.0f / tau_sh;
  // slot of each key in its bucket (slots above 255 saturate: such a bucket exceeds
  // kSureBucketLimit and takes the bitonic path).  Overlay classes on single keys keep
  // the bucket and the slot of each key packed in one register, bucket | slot << 15, so
  // the bounds step below needs no second bucket computation; the others (pair keys
  // would spill with those registers live through the bucket scan) keep the slots one
  // byte per key, four to a register, and recompute the bucket where they need it.
  static_assert(NB < (1 << 15), "bucket index in 15 bits");
  constexpr bool KEEPB = OV && GD == 1;
  constexpr int KP = KEEPB ? 1 : (KPT + 3) / 4;
  unsigned pk[KP];
  int pos[KPT];
#pragma unroll
  for (int q = 0; q < KP; ++q) pk[q] = 0u;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int i = tid + j * NT;
    pos[j] = 0;
    if (i < Nb) {
      const int bk = sure_bucket<NB>(kk[j], inv_tau);
      const unsigned sl = min((unsigned)atomicAdd(&off[bk], 1), 255u);
      if constexpr (KEEPB)
        pos[j] = bk | (int)(sl << 15);
      else
        pk[j >> 2] |= sl << (8 * (j & 3));
    }
  }
  __syncthreads();
  // exclusive scan of the bucket counts, and the largest count (the counts are read
  // from LDS twice rather than held in registers)
  int sum = 0, mx = 0;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int c = off[tid * BPT + q];
    sum += c;
    mx = max(mx, c);
  }
  const int incl = wave_incl_prefix_int(sum, lane);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
  if (lane == 63) wsC[wid] = incl;
  if (lane == 0) wsM[wid] = mx;
  __syncthreads();
  int excl = incl - sum + wave_offset_int<NW>(wsC, wid, lane);
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int c = off[tid * BPT + q];
    off[tid * BPT + q] = excl;
    excl += c;
  }
  if (tid == NT - 1) off[NB] = excl;
  if (tid == 0) {
    int m = 0;
    for (int w = 0; w < NW; ++w) m = max(m, wsM[w]);
    maxc_sh = m;
  }
  __syncthreads();
  if (maxc_sh <= kSureBucketLimit) {
#define SURE_SLOT(j) ((int)((pk[(j) >> 2] >> (8 * ((j) & 3))) & 0xFFu))
    // per key: bucket bounds and slot, packed as offset | count << 15 | slot << 22
    // (offsets < 2^15, counts and slots <= kSureBucketLimit < 2^7); with the overlay
    // they are taken into registers before the keys overwrite the table, later the
    // same registers hold the final positions
    static_assert(MAXK < (1 << 15) && kSureBucketLimit < (1 << 7), "packed bucket bounds");
    if constexpr (OV) {
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const int i = tid + j * NT;
        if (i < Nb) {
          int bk, slot;
          if constexpr (KEEPB) {
            bk = pos[j] & 0x7FFF;
            slot = pos[j] >> 15;
          } else {
            bk = sure_bucket<NB>(kk[j], inv_tau);
            slot = SURE_SLOT(j);
          }
          const int lo = off[bk];
          pos[j] = lo | ((off[bk + 1] - lo) << 15) | (slot << 22);
        }
      }
      __syncthreads();
    }
#define SURE_BOUNDS(j, lo, hi, slot)                 \
  if constexpr (OV) {                                \
    lo = pos[j] & 0x7FFF;                            \
    hi = lo + ((pos[j] >> 15) & 0x7F);               \
    slot = pos[j] >> 22;                             \
  } else {                                           \
    const int bk_ = sure_bucket<NB>(kk[j], inv_tau); \
    lo = off[bk_];                                   \
    hi = off[bk_ + 1];                               \
    slot = SURE_SLOT(j);                             \
  }
    // scatter into bucket slots, unpadded (the rank loop then walks plain addresses; the
    // padded sorted layout is written only after every rank read)
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      if (i < Nb) {
        int lo, hi, slot;
        SURE_BOUNDS(j, lo, hi, slot);
        (void)hi;
        sk[lo + slot] = kk[j];
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
        const float* me = sk + lo + slot;
        int rank = 0;
        for (const float* x = sk + lo; x < sk + hi; ++x) {
          const float u = *x;
          rank += (u < v) || (u == v && x < me);
        }
        pos[j] = lo + rank;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = tid + j * NT;
      if (i < Nb) sk[skx(pos[j])] = kk[j];
    }
    __syncthreads();
#undef SURE_BOUNDS
#undef SURE_SLOT
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
  SureBest best;
  // (the unrolled walk of 16-key chunks on single keys: with pair keys it would spill)
  sure_walk<NT, (KPT == 16 && GD == 1 ? 16 : 0)>(sk, Nb, GD * (double)tau_sh, (2 * GD - 1) * (double)tau_sh,
                                                 a.sure_cont != 0, wsA, wsR, best);
  sure_finish<NT, GD>(a, sl, b, Nb, tau_sh, best, fin);
}

// In-place ascending sort of the keys sk[skx(0 .. Nb)) by a bitonic network whose
// compare-exchanges all put the smaller key first (each merge starts by comparing
// mirrored positions), so +inf padding up to npad (the next power of two) never moves
// and needs no storage: only pairs with both indices < Nb are compared.
template <int NT>
__device__ void sure_bitonic(float* sk, int Nb, int npad) {
  const int tid = threadIdx.x;
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

// ------------------------------------------------------------------ large bands
// Bands of more than kSureMaxKeys keys (up to 65536: the finest band of a 512 x 512
// slice) do not fit LDS, so the argmin is found without sorting the band.  Keys are
// re-read from r for each pass (the band stays in L2).  Per bucket of the key/tau
// bucket map: count, smallest positive and largest key (integer atomics on the bit
// patterns), and the sums of the keys and of their reciprocal square roots in 64-bit
// fixed point with a power-of-two scale per bucket (integer additions commute, so the
// sums do not depend on the order the atomics land in).  Bucket prefix/suffix scans
// (FP64, fixed order) give for every bucket its first index P, the key sum A before it
// and the 1/a sum R after it.  Then
//   - the last key of each bucket is a candidate whose SURE is known from the sums;
//     U = the smallest of these;
//   - a candidate inside bucket b (t of its c keys at or below it, 1 <= t < c) has
//     SURE >= A + t kmin - m tau + (N_b - m)(kmin + tau) - tau sqrt(kmax)(R + (c - t)/sqrt(kmin+))
//     with m = P + t, linear in t, so its smallest value is at t = 1 or t = c - 1;
//   - only buckets whose bound or end value is within a rounding margin of U can hold
//     the argmin: their keys are gathered, ranked inside their bucket (one wave per
//     bucket) and walked exactly, A and R carried in FP64 from the bucket boundaries.
// A band with too many surviving keys or buckets (tau = 0 puts every key in one bucket)
// is sorted in full in its global scratch region and walked there instead.
constexpr int kSureBigBucketLimit = 256;  // keys of one surviving bucket
constexpr int kSureBigMaxSeg = 256;       // surviving buckets
constexpr int kSureBigCap = 6144;         // surviving keys
constexpr int kSureBigNB = 3072;

template <int NT, int NB, int CAP, int GD>
__global__ void __launch_bounds__(NT) k_sure_big(KArgs a, float* __restrict__ scratch, int stride) {
  constexpr int NW = NT / 64, BPT = NB / NT;
  static_assert(NB % NT == 0, "buckets per thread");
  __shared__ __align__(16) int smem[8 * NB + CAP];
  int* cnt = smem;                   // [NB] counts, later fill counters
  int* kmn = smem + NB;              // [NB] smallest positive key (bits), +inf if none
  int* kmx = smem + 2 * NB;          // [NB] largest key (bits)
  int* coff = smem + 3 * NB;         // [NB] offset of a surviving bucket in comp, else -1
  unsigned long long* sA = reinterpret_cast<unsigned long long*>(smem + 4 * NB);  // [NB]
  unsigned long long* sRq = sA + NB;                                              // [NB]
  float* comp = reinterpret_cast<float*>(smem + 8 * NB);  // [CAP] surviving keys
  __shared__ double wsA[NW], wsR[NW], wsU[NW];
  __shared__ int wsC[NW], wsS[NW], wsM[NW];
  __shared__ SureBest fin[NW];
  __shared__ float tau_sh;
  __shared__ double ustar_sh, mag_sh;
  __shared__ int tot_sh, bigc_sh, nseg_sh;
  __shared__ int seg_off[kSureBigMaxSeg], seg_n[kSureBigMaxSeg], seg_p[kSureBigMaxSeg];
  __shared__ double seg_a[kSureBigMaxSeg], seg_r[kSureBigMaxSeg];
  const int2 item = a.work[blockIdx.x];
  const int sl = item.x, b = item.y, s = a.levels;
  const SliceDev S = a.slices[sl];
  const int tid = threadIdx.x, lane = tid & 63, wid = wave_id(tid);
  int d0, r0, c0, bd, bh, bw;
  band_geom3(b, s, S.nd, S.ny, S.nx, d0, r0, c0, bd, bh, bw);
  const int Nb = bd * bh * bw / GD;  // keys: coefficients, or pairs x = 2j, 2j + 1
  const float2* r = a.r + S.off + ((long long)d0 * S.ny + r0) * S.nx + c0;
  const BandWalk bwk = band_walk(bd, bh, bw, S.ny, S.nx);
#define KEY_AT(i) (GD == 2 ? key_pair_rn(r[bwk.at(2 * (i))], r[bwk.at(2 * (i)) + 1]) : key_rn(r[bwk.at(i)]))
  for (int i = tid; i < NB; i += NT) {
    cnt[i] = 0;
    kmn[i] = 0x7f800000;
    kmx[i] = 0;
    sA[i] = 0ull;
    sRq[i] = 0ull;
  }
  if (wid == 0) {
    const int ncs = S.ncs;
    double acc = 0.0;
    for (int i = lane; i < ncs; i += 64) acc += (double)a.tau_part[(S.colstrip0 + i) * kMaxBands + b];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) tau_sh = (float)acc;
  }
  __syncthreads();
  const float inv_tau = 1.0f / tau_sh;
  const double tau = (double)tau_sh;
  const double tl = GD * tau, td = (2 * GD - 1) * tau;  // sure_inner
  for (int i = tid; i < Nb; i += NT) {
    const float k = KEY_AT(i);
    const int bk = sure_bucket<NB>(k, inv_tau);
    atomicAdd(&cnt[bk], 1);
    const int bits = (int)__float_as_uint(k);
    atomicMax(&kmx[bk], bits);
    if (k > 0.f) atomicMin(&kmn[bk], bits);
  }
  __syncthreads();
  // fixed-point sums: scale 2^(40 - e) with 2^e >= the bucket's largest term
  for (int i = tid; i < Nb; i += NT) {
    const float k = KEY_AT(i);
    if (k > 0.f) {
      const int bk = sure_bucket<NB>(k, inv_tau);
      int e;
      frexp((double)__uint_as_float((unsigned)kmx[bk]), &e);
      atomicAdd(&sA[bk], (unsigned long long)ldexp((double)k, 40 - e));
      frexp((double)__frsqrt_rn(__uint_as_float((unsigned)kmn[bk])), &e);
      atomicAdd(&sRq[bk], (unsigned long long)ldexp((double)__frsqrt_rn(k), 40 - e));
    }
  }
  __syncthreads();
  // this thread's buckets tid*BPT .. +BPT: counts and sums, then block scans
  int c[BPT];
  double dA[BPT], dR[BPT];
  int csum = 0;
  double asum = 0.0, rsum = 0.0;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int bk = tid * BPT + q;
    c[q] = cnt[bk];
    dA[q] = 0.0;
    dR[q] = 0.0;
    const float kx = __uint_as_float((unsigned)kmx[bk]);
    if (c[q] && kx > 0.f) {
      int e;
      frexp((double)kx, &e);
      dA[q] = ldexp((double)sA[bk], e - 40);
      frexp((double)__frsqrt_rn(__uint_as_float((unsigned)kmn[bk])), &e);
      dR[q] = ldexp((double)sRq[bk], e - 40);
    }
    csum += c[q];
    asum += dA[q];
    rsum += dR[q];
  }
  const int cinc = wave_incl_prefix_int(csum, lane);
  const double ainc = wave_incl_prefix(asum, lane);
  const double rinc = wave_incl_suffix(rsum, lane);
  if (lane == 63) { wsC[wid] = cinc; wsA[wid] = ainc; }
  if (lane == 0) wsR[wid] = rinc;
  __syncthreads();
  int P = cinc - csum;
  double Ab = ainc - asum, Ra = rinc - rsum;
  for (int w = 0; w < wid; ++w) { P += wsC[w]; Ab += wsA[w]; }
  for (int w = NW - 1; w > wid; --w) Ra += wsR[w];
  double Atot = 0.0;
  for (int w = 0; w < NW; ++w) Atot += wsA[w];
  int Pq[BPT];
  double Abq[BPT], Raq[BPT];
  {
    int pp = P;
    double aa = Ab, rr = Ra + rsum;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      Pq[q] = pp;
      Abq[q] = aa;
      rr -= dR[q];
      Raq[q] = rr;
      pp += c[q];
      aa += dA[q];
    }
  }
  const double Nbd = (double)Nb;
  double endv[BPT];
  double umin = __builtin_huge_val();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    endv[q] = __builtin_huge_val();
    const float kx = __uint_as_float((unsigned)kmx[tid * BPT + q]);
    if (c[q] && kx > 0.f) {
      const double m = (double)(Pq[q] + c[q]);
      const double x = (double)__fsqrt_rn(kx);
      endv[q] = (Abq[q] + dA[q]) - m * tl + (Nbd - m) * ((double)kx + tl) - td * x * Raq[q];
      umin = fmin(umin, endv[q]);
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) umin = fmin(umin, __shfl_xor(umin, o, 64));
  if (lane == 0) wsU[wid] = umin;
  __syncthreads();
  if (tid == 0) {
    double u = wsU[0];
    for (int w = 1; w < NW; ++w) u = fmin(u, wsU[w]);
    ustar_sh = u;
    mag_sh = Atot;
  }
  __syncthreads();
  const double ustar = ustar_sh;
  const double margin = 1e-9 * (fabs(ustar) + Nbd * tl + mag_sh) + 1e-300;
  bool surv[BPT];
  int ssum = 0, nseg = 0, big = 0;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    surv[q] = false;
    const int bk = tid * BPT + q;
    const float kx = __uint_as_float((unsigned)kmx[bk]);
    if (!c[q] || !(kx > 0.f)) continue;  // empty, or every key zero: no candidate
    bool sv = endv[q] <= ustar + margin;
    if (c[q] >= 2) {
      const float kn = __uint_as_float((unsigned)kmn[bk]);
      const double kminA = (bk == 0) ? 0.0 : (double)kn;  // zero keys only in bucket 0
      const double rmax = (double)__frsqrt_rn(kn);
      const double sx = (double)__fsqrt_rn(kx);
      double lb = __builtin_huge_val();
      for (int e2 = 0; e2 < 2; ++e2) {
        const int t = e2 ? c[q] - 1 : 1;
        const double m = (double)(Pq[q] + t);
        lb = fmin(lb, Abq[q] + t * kminA - m * tl + (Nbd - m) * (kminA + tl) -
                          td * sx * (Raq[q] + (c[q] - t) * rmax));
      }
      sv = sv || lb <= ustar + margin;
    }
    surv[q] = sv;
    if (sv) {
      ssum += c[q];
      nseg += 1;
      big = max(big, c[q]);
    }
  }
  const int sinc = wave_incl_prefix_int(ssum, lane);
  const int ginc = wave_incl_prefix_int(nseg, lane);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) big = max(big, __shfl_xor(big, o, 64));
  if (lane == 63) { wsS[wid] = sinc; wsC[wid] = ginc; }
  if (lane == 0) wsM[wid] = big;
  __syncthreads();
  int soff = sinc - ssum, goff = ginc - nseg, gtot = 0;
  for (int w = 0; w < wid; ++w) { soff += wsS[w]; goff += wsC[w]; }
  for (int w = 0; w < NW; ++w) gtot += wsC[w];
  const bool fits = gtot <= kSureBigMaxSeg;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int bk = tid * BPT + q;
    coff[bk] = surv[q] ? soff : -1;
    cnt[bk] = 0;  // fill counter of the gather
    if (surv[q]) {
      if (fits) {
        seg_off[goff] = soff;
        seg_n[goff] = c[q];
        seg_p[goff] = Pq[q];
        seg_a[goff] = Abq[q];
        seg_r[goff] = Raq[q];
      }
      soff += c[q];
      goff += 1;
    }
  }
  if (tid == NT - 1) tot_sh = soff;
  if (tid == 0) {
    int m = 0;
    for (int w = 0; w < NW; ++w) m = max(m, wsM[w]);
    bigc_sh = m;
    nseg_sh = gtot;
  }
  __syncthreads();
  SureBest best = sure_none();
  // the pruning bounds hold for thresholds at keys; the continuous search walks the
  // whole band
  if (!a.sure_cont && tot_sh <= CAP && bigc_sh <= kSureBigBucketLimit && nseg_sh <= kSureBigMaxSeg) {
    for (int i = tid; i < Nb; i += NT) {
      const float k = KEY_AT(i);
      const int bk = sure_bucket<NB>(k, inv_tau);
      const int o = coff[bk];
      if (o >= 0) comp[o + atomicAdd(&cnt[bk], 1)] = k;
    }
    __syncthreads();
    // one wave per surviving bucket: rank its keys (every lane reads the same key in
    // turn), put them in order, then walk them with wave prefix sums
    for (int g = wid; g < nseg_sh; g += NW) {
      const int off0 = seg_off[g], n = seg_n[g];
      constexpr int MAXL = kSureBigBucketLimit / 64;
      float v[MAXL];
      int rk[MAXL];
#pragma unroll
      for (int h = 0; h < MAXL; ++h) {
        const int l = lane + 64 * h;
        v[h] = (l < n) ? comp[off0 + l] : __builtin_huge_valf();
        rk[h] = 0;
      }
      for (int x = 0; x < n; ++x) {
        const float u = comp[off0 + x];
#pragma unroll
        for (int h = 0; h < MAXL; ++h) rk[h] += (u < v[h]) || (u == v[h] && x < lane + 64 * h);
      }
#pragma unroll
      for (int h = 0; h < MAXL; ++h)
        if (lane + 64 * h < n) comp[off0 + rk[h]] = v[h];
      __builtin_amdgcn_wave_barrier();
      double A = seg_a[g], R = seg_r[g], rtot = 0.0;
#pragma unroll
      for (int h = 0; h < MAXL; ++h) {
        const int l = lane + 64 * h;
        v[h] = (l < n) ? comp[off0 + l] : 0.f;
        rtot += (l < n && v[h] > 0.f) ? (double)__frsqrt_rn(v[h]) : 0.0;
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) rtot += __shfl_xor(rtot, o, 64);
      R += rtot;  // 1/a over this bucket and above
      const int P0 = seg_p[g];
#pragma unroll
      for (int h = 0; h < MAXL; ++h) {
        if (64 * h >= n) break;
        const int l = lane + 64 * h;
        const float k2 = v[h];
        const double ka = (l < n) ? (double)k2 : 0.0;
        const double ra = (l < n && k2 > 0.f) ? (double)__frsqrt_rn(k2) : 0.0;
        const double pa = wave_incl_prefix(ka, lane);
        const double pr = wave_incl_prefix(ra, lane);
        const double chA = __shfl(pa, 63, 64), chR = __shfl(pr, 63, 64);
        if (l < n && k2 > 0.f) {
          const float kn = (l + 1 < n) ? comp[off0 + l + 1] : __builtin_huge_valf();
          if (kn > k2) {  // last index of a run of equal keys
            const double Am = A + pa, Rm = R - pr;
            const double xx = (double)__fsqrt_rn(k2);
            const double m = (double)(P0 + l + 1);
            const double sv = Am - m * tl + (Nbd - m) * ((double)k2 + tl) - td * xx * Rm;
            if (sure_better(sv, P0 + l + 1, 0, best)) {
              best.v = sv;
              best.m = P0 + l + 1;
              best.inner = 0;
              best.R = Rm;
              best.key = k2;
            }
          }
        }
        A += chA;
        R -= chR;
      }
    }
  } else {
    // sort the whole band in its scratch region and walk it there
    float* sk = scratch + (long long)blockIdx.x * stride;
    int npad = 1;
    while (npad < Nb) npad <<= 1;
    for (int i = tid; i < Nb; i += NT) sk[skx(i)] = KEY_AT(i);
    __syncthreads();
    sure_bitonic<NT>(sk, Nb, npad);
    sure_walk<NT>(sk, Nb, tl, td, a.sure_cont != 0, wsA, wsR, best);
  }
#undef KEY_AT
  sure_finish<NT, GD>(a, sl, b, Nb, tau_sh, best, fin);
}

// Size classes: up to 4096 keys (0: 256 threads x 16 keys, 2560 buckets; 1: 512 x 8,
// 5120 buckets), up to 16384 keys (2: 1024 x 16, 19456 buckets, the most whose table
// still lets two workgroups share a CU) and up to kSureMaxKeys keys (3: 1024 x 32,
// 10240 buckets).  By default bands of up to 2048 keys take
// class 0 and bands of 2049-16384 keys class 2 (measured faster than classes 0 and 1 on
// 4096-key bands of VDAMP iterates; class 1 is left to the plan-time tuner).  All LDS is static: the largest class uses about
// 158 KB of the 160 KB a gfx950 workgroup may hold.
template <int GD>
static void launch_sure_t(const KArgs& a, int cls, float* scratch, hipStream_t st) {
  if (cls == kSureBigClass)
    hipLaunchKernelGGL((k_sure_big<1024, kSureBigNB, kSureBigCap, GD>), dim3(a.nwork), dim3(1024), 0, st, a,
                       scratch, kSureBigStride);
  else if (cls == 3)
    hipLaunchKernelGGL((k_sure<1024, 32, 10240, kSureMaxKeys, GD>), dim3(a.nwork), dim3(1024), 0, st, a);
  else if (cls == 2)
    hipLaunchKernelGGL((k_sure<1024, 16, 19456, 4 * kSureSmall, GD>), dim3(a.nwork), dim3(1024), 0, st, a);
  else if (cls == 1)
    hipLaunchKernelGGL((k_sure<512, 8, 5120, kSureSmall, GD>), dim3(a.nwork), dim3(512), 0, st, a);
  else
    hipLaunchKernelGGL((k_sure<256, 16, 2560, kSureSmall, GD>), dim3(a.nwork), dim3(256), 0, st, a);
}
hipError_t launch_sure(const KArgs& a, int cls, float* scratch, hipStream_t st) {
  if (a.grp == 2)
    launch_sure_t<2>(a, cls, scratch, st);
  else
    launch_sure_t<1>(a, cls, scratch, st);
  return hipGetLastError();
}

}  // namespace vdamp

/*
 * vdamp.h -- C ABI of libvdamp: VDAMP (variable density approximate message passing)
 * and its FISTA comparator for variable-density partial-Fourier sensing, on gfx950.
 *
 * Problem (Section 1, eq. 1): y = Phi x0 + eps with Phi = M_Omega F, F the unitary 2D
 * DFT, M_Omega the selector of the sampled set Omega, Prob(j in Omega) = p_j, and
 * eps ~ CN(0, sigma^2 I) (E|eps_j|^2 = sigma^2).  The solver runs Algorithm 1
 * (Section 2) with an s-level orthonormal periodic Haar wavelet Psi and, as denoiser,
 * complex soft thresholding with one threshold per subband chosen by minimising the
 * complex colored SURE (Section 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - A plan covers a batch of B independent slices ("ragged": each slice has its own
 *   ny x nx).  Every per-pixel array is packed slice after slice in plan order, slice b
 *   starting at pixel offset off_b = sum_{b' < b} ny[b'] * nx[b'], row-major [ny][nx].
 * - complex64 arrays are interleaved (re, im) float pairs ("float *" of 2*N floats).
 * - k-space arrays are in natural FFT order (DC at [0][0]) under the unitary DFT.
 * - Wavelet coefficients use the Mallat layout with band order b = 0 for LL_s, then for
 *   l = s .. 1 the triple (LH_l, HL_l, HH_l); LH = low along y / high along x (top-right
 *   block of level l), HL = high along y / low along x (bottom-left), HH bottom-right.
 *   A slice has nb = 1 + 3 s bands (eqs. 6-7).
 * - Every data pointer is a DEVICE pointer unless marked "host".  The caller owns all
 *   data buffers and the workspace; the plan owns only small device constants.
 * - Calls are asynchronous on the given stream: they return after enqueueing and the
 *   results are valid once the stream has synchronised.  A plan must not be used on
 *   two streams at the same time.
 * - Argument checks (shapes, pointers, sizes) run on the host before anything is
 *   enqueued; on failure nothing is written and a status != VDAMP_OK is returned, with
 *   a detail string in vdamp_last_error().  HIP failures map to VDAMP_ERR_HIP.  Nothing
 *   throws across this boundary.
 */
#ifndef VDAMP_H
#define VDAMP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vdamp_plan_t* vdamp_plan_h;

typedef enum {
  VDAMP_OK = 0,
  VDAMP_ERR_ARG = 1,          /* null pointer, negative count, bad enum value        */
  VDAMP_ERR_SHAPE = 2,        /* ny, nx not divisible by 2^levels, or out of range   */
  VDAMP_ERR_UNSUPPORTED = 3,  /* size or option this build does not implement        */
  VDAMP_ERR_WORKSPACE = 4,    /* workspace missing, too small or misaligned          */
  VDAMP_ERR_HIP = 5,          /* a HIP runtime call failed                           */
  VDAMP_ERR_NONFINITE = 6,    /* VDAMP_FLAG_CHECK_FINITE found bad data              */
  VDAMP_ERR_STATE = 7         /* no solve has produced the requested state yet       */
} vdamp_status;

enum { VDAMP_WAVELET_HAAR = 0 };

enum {
  /* Capture the whole solve (all iterations) in one hipGraph on first use and replay
     it while pointers and iteration count stay the same; re-captured otherwise.  The
     stream must not be the legacy null stream. */
  VDAMP_FLAG_USE_GRAPH = 1u << 3,
  /* Validate data before solving: p in (0, 1] wherever mask = 1, and y finite.  The
     solve then synchronises the stream and returns VDAMP_ERR_NONFINITE on failure. */
  VDAMP_FLAG_CHECK_FINITE = 1u << 2,
  /* Record HIP events around every kernel launch (eager launches only; overrides
     VDAMP_FLAG_USE_GRAPH) so that vdamp_pass_times() can report per-pass times. */
  VDAMP_FLAG_TIMING = 1u << 5
};

/* Kernel classes reported by vdamp_pass_times(). */
enum {
  VDAMP_PASS_PREP = 0,      /* mask/p -> m/p weights, data checks                   */
  VDAMP_PASS_ROWS_SYNTH = 1,/* line 8 + Psi^H on row strips, then row FFT            */
  VDAMP_PASS_COLS = 2,      /* column FFT, k-space residual, tau partials, col IFFT  */
  VDAMP_PASS_ROWS_ANAL = 3, /* row IFFT, Psi on row strips, + r_tilde (line 4)       */
  VDAMP_PASS_SURE = 4,      /* tau reduction, SURE threshold search, alpha           */
  VDAMP_PASS_COUNT = 5
};

/*
 * vdamp_plan -- plan a batch of slices.
 *   plan            out: opaque handle (release with vdamp_plan_destroy)
 *   batch           B >= 1 slices
 *   ny, nx          host int32[B]: slice sizes; each divisible by 2^levels, each in
 *                   [2^levels, 512] and of the form 2^a 3^b 5^c (mixed-radix FFT)
 *   levels          s, Haar decomposition scales, 1..4 (Section 3 uses s = 4)
 *   wavelet         VDAMP_WAVELET_HAAR
 *   flags           VDAMP_FLAG_* bits
 *   workspace_bytes out: size of the device workspace every solve call needs
 * Builds, on the host in FP64 then rounded to FP32, the separable tau weights
 * S_b = |Phi Psi^H|^2 of line 1 (Section 2: S has 1 + 3s unique columns), the FFT
 * twiddles and the work lists, and uploads them (synchronous, once per plan).
 */
vdamp_status vdamp_plan(vdamp_plan_h* plan, int32_t batch, const int32_t* ny, const int32_t* nx,
                        int32_t levels, int32_t wavelet, uint32_t flags, size_t* workspace_bytes);

vdamp_status vdamp_plan_destroy(vdamp_plan_h plan);

/*
 * vdamp_solve -- run `iters` iterations of Algorithm 1 on every slice, then line 10.
 *   stream          HIP stream to enqueue on
 *   workspace       device buffer of at least workspace_bytes, 256-byte aligned; holds
 *                   the iterate r_k and the per-band state between calls
 *   y               complex64[sum N]: zero-filled measurements (0 where mask = 0)
 *   mask            uint8[sum N]: 1 where j in Omega, else 0
 *   p               float32[sum N]: Prob(j in Omega); must be in (0, 1] where mask = 1,
 *                   ignored elsewhere
 *   sigma2          float32[B]: measurement noise variance E|eps_j|^2 per slice
 *   iters           K >= 0; K = 0 returns the zero-filled F^H y
 *   x_hat           complex64[sum N] out: Psi^H w + Phi^H (y - Phi Psi^H w), with
 *                   w = w_hat_{K-1} (line 10)
 *   trace           nullable float32[iters][B][nb][3] out: (tau_k, theta_k, alpha_k) per
 *                   band (lines 5-7); theta_k = lambda_k tau_k in eq. 7's terms
 * FP32 arithmetic with FP64 threshold search; results are bitwise reproducible for a
 * given plan (fixed-order reductions, no floating-point atomics).
 */
vdamp_status vdamp_solve(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                         size_t workspace_bytes, const float* y, const uint8_t* mask,
                         const float* p, const float* sigma2, int32_t iters, float* x_hat,
                         float* trace);

/*
 * fista_solve -- FISTA on 1/2 ||y - M_Omega F Psi^H w||^2 + lambda ||w||_1 (eq. 2 with
 * f = lambda ||Psi x||_1, in synthesis form), step size 1, zero start, every band
 * thresholded (Section 3's comparator).
 *   lambda          float32[B]: sparse weighting per slice
 *   x_hat           complex64[sum N] out: Psi^H w_K (K = 0 gives zeros)
 * Other arguments as in vdamp_solve (p and sigma2 are not used).
 */
vdamp_status fista_solve(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                         size_t workspace_bytes, const float* y, const uint8_t* mask,
                         const float* lambda, int32_t iters, float* x_hat);

/*
 * vdamp_state_export -- copy the state left by the last vdamp_solve on this workspace:
 *   r               nullable complex64[sum N] out: r_{K-1} (Mallat layout per slice)
 *   theta, alpha, tau  nullable float32[B][nb] out: the last iteration's values
 * Returns VDAMP_ERR_STATE if no vdamp_solve with iters >= 1 ran on this plan.
 */
vdamp_status vdamp_state_export(vdamp_plan_h plan, hipStream_t stream, const void* workspace,
                                float* r, float* theta, float* alpha, float* tau);

/*
 * vdamp_pass_times -- with VDAMP_FLAG_TIMING: synchronise the recorded events and return,
 * per kernel class (VDAMP_PASS_*), the summed kernel time in milliseconds and the
 * number of launches since the previous call (which resets the counters).
 *   ms, launches    host arrays of npass entries
 */
vdamp_status vdamp_pass_times(vdamp_plan_h plan, double* ms, int64_t* launches, int32_t npass);

/* Static description of a status code. */
const char* vdamp_status_string(vdamp_status s);

/* Detail string of the last failure on the calling thread ("" if none). */
const char* vdamp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VDAMP_H */

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
  VDAMP_ERR_STATE = 7,        /* no solve has produced the requested state yet       */
  VDAMP_STATUS_MAX_ENUM = 0x7FFFFFFF  /* not a status: makes every int32 value a valid
                                         vdamp_status, so vdamp_status_string may be
                                         handed any code */
} vdamp_status;

enum { VDAMP_WAVELET_HAAR = 0 };

enum {
  /* Bitwise reproducible results.  Every path of this library already is (fixed-order
     reductions, no floating-point atomics, plan-time kernel choices fixed for the plan),
     so the flag is accepted and changes nothing. */
  VDAMP_FLAG_DETERMINISTIC = 1u << 0,
  /* Capture the whole solve (all iterations) in one hipGraph on first use and replay
     it while pointers and iteration count stay the same; re-captured otherwise.  The
     stream must not be the legacy null stream. */
  VDAMP_FLAG_USE_GRAPH = 1u << 3,
  /* Validate data before solving: p in (0, 1] wherever mask = 1, and y finite.  The
     solve then synchronises the stream and returns VDAMP_ERR_NONFINITE on failure. */
  VDAMP_FLAG_CHECK_FINITE = 1u << 2,
  /* Record HIP events around every kernel launch (eager launches only; overrides
     VDAMP_FLAG_USE_GRAPH) so that vdamp_pass_times() can report per-pass times. */
  VDAMP_FLAG_TIMING = 1u << 5,
  /* Tune the launch configuration when the plan is built: for every size group, time
     the four-step register FFT against the in-LDS Stockham FFT in the row and column
     passes, and every threshold-search size class that holds the band size, on synthetic
     data in temporary device buffers (allocated and freed inside vdamp_plan, which
     synchronises), and keep the fastest (3 % margin in favour of the default).  The FFT
     choice changes results at FP32 rounding level; the choice is fixed for the plan.
     vdamp_plan_describe() reports the measurements. */
  VDAMP_FLAG_AUTOTUNE = 1u << 6,
  /* Threshold search over every theta > 0 instead of the candidates theta in {|r_i|}
     (Section 3 solves the SURE problem "approximately"; this is its exact minimiser):
     between consecutive distinct magnitudes SURE is a convex quadratic in theta, whose
     minimum tau R_m / (2 (N_b - m)) competes with the candidates when it lies inside its
     interval.  The alpha step's alpha and the denoising step's eta use the threshold found. */
  VDAMP_FLAG_SURE_CONTINUOUS = 1u << 7,
  /* Structured sparsity (Section 4 names it among the richer models SURE can tune):
     the two horizontally adjacent coefficients x = 2j, 2j+1 of every subband row form a
     group, shrunk jointly by group soft thresholding g max(0, 1 - theta/||g||).  theta
     minimises the group's SURE (Stein's estimate over the 4 real dimensions of a pair
     under CN(0, tau) noise per coefficient) over the candidates ||g|| (or over every
     theta > 0 with VDAMP_FLAG_SURE_CONTINUOUS); the alpha step's alpha is half the real
     divergence per coefficient.  theta's key is the FP32 squared norm of the pair
     (|g_0|^2 + |g_1|^2, each term as for one coefficient, their sum rounded to nearest).
     2D Haar plans of vdamp_plan only (VDAMP_ERR_UNSUPPORTED elsewhere); fista_solve and
     the learned denoiser refuse such plans. */
  VDAMP_FLAG_GROUP_PAIRS = 1u << 8
};

/* Kernel classes reported by vdamp_pass_times(). */
enum {
  VDAMP_PASS_PREP = 0,      /* mask/p -> m/p weights, data checks                   */
  VDAMP_PASS_ROWS_SYNTH = 1,/* the Onsager correction + Psi^H on row strips, then row FFT            */
  VDAMP_PASS_COLS = 2,      /* column FFT, k-space residual, tau partials, col IFFT  */
  VDAMP_PASS_ROWS_ANAL = 3, /* row IFFT, Psi on row strips, + r_tilde (back-projection)       */
  VDAMP_PASS_SURE = 4,      /* tau reduction, SURE threshold search, alpha           */
  VDAMP_PASS_DENOISER = 5,  /* learned denoiser: Psi / Psi^H, probe, partial sums, judge */
  VDAMP_PASS_CNN = 6,       /* learned denoiser: the network's forward pass and JVP    */
  VDAMP_PASS_COUNT = 7
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
 * S_b = |Phi Psi^H|^2 of the initialisation (Section 2: S has 1 + 3s unique columns), the FFT
 * twiddles and the work lists, and uploads them (synchronous, once per plan).
 */
vdamp_status vdamp_plan(vdamp_plan_h* plan, int32_t batch, const int32_t* ny, const int32_t* nx,
                        int32_t levels, int32_t wavelet, uint32_t flags, size_t* workspace_bytes);

/*
 * vdamp_plan_ortho -- plan a batch with a general orthonormal wavelet Psi (Algorithm 1
 * asks only for an orthogonal wavelet transform; Section 2).
 *   lowpass         host float64[filter_len]: the lowpass filter h of a two-channel
 *                   orthonormal filter bank (sum h = sqrt 2, sum_t h[t] h[t + 2j] =
 *                   delta_j, checked to 1e-9); the highpass is g[t] = (-1)^t h[L-1-t].
 *                   Read during the call only.  h = (1, 1)/sqrt 2 is Haar.
 *   filter_len      L, even, 2..64
 *   other arguments as vdamp_plan (levels 1..4; VDAMP_FLAG_AUTOTUNE is not accepted).
 * Psi is the s-level periodic Mallat transform: one level filters the top-left block
 * along x, a[j] = sum_t h[t] x[(2j + t) mod M] to the left half and d[j] with g to the
 * right, then the same along y; band order and layout as for Haar.  Any filter length
 * works: the filters wrap periodically at the coarse levels.  The tau weights of the initialisation
 * are |DFT of each band's basis function|^2, separable, computed on the host in FP64.
 * The plan serves vdamp_solve, vdamp_solve_resume, vdamp_solve_noalloc,
 * vdamp_state_export and vdamp_wavelet_ws; fista_solve, vdamp_wavelet and the learned
 * denoiser return VDAMP_ERR_UNSUPPORTED for it.  Its workspace also holds the group rows
 * of the Fourier-domain wavelet passes: 15 bytes a pixel more at s = 4.
 * Errors: VDAMP_ERR_ARG for a null or non-orthonormal filter or a bad length.
 */
vdamp_status vdamp_plan_ortho(vdamp_plan_h* plan, int32_t batch, const int32_t* ny, const int32_t* nx,
                              int32_t levels, const double* lowpass, int32_t filter_len,
                              uint32_t flags, size_t* workspace_bytes);

/*
 * vdamp_plan_3d -- plan a batch of volumes: Phi = M_Omega F with F the unitary 3D DFT
 * (Section 1 allows a 2D or 3D DFT) and Psi the s-level periodic orthonormal 3D Haar
 * transform.
 *   nz, ny, nx      host int32[B]: volume sizes ([nz][ny][nx] row-major, packed volume
 *                   after volume); each divisible by 2^levels, in [2^levels, 512], of the
 *                   form 2^a 3^b 5^c; nx a multiple of 16; the finest band (nz ny nx / 8
 *                   coefficients) at most 65536
 *   levels          s, 1..4; 1 + 7 s bands: b = 0 is LLL_s, then for l = s .. 1 the
 *                   octants of kind k = 1 .. 7 (bit 0: high along x, bit 1: along y,
 *                   bit 2: along z), each block at (k&4 ? nz>>l : 0, k&2 ? ny>>l : 0,
 *                   k&1 ? nx>>l : 0) of size (nz>>l, ny>>l, nx>>l)
 *   flags           as vdamp_plan (VDAMP_FLAG_AUTOTUNE is not accepted)
 * The tau weights of the initialisation are separable: S_b = Z_b(kz) Y_b(ky) X_b(kx).  The plan
 * serves vdamp_solve, vdamp_solve_resume, vdamp_solve_noalloc, vdamp_state_export and
 * vdamp_wavelet_ws, with y, mask, p, x_hat, r as packed volumes and theta, alpha, tau
 * with 1 + 7 s entries per volume; fista_solve, vdamp_wavelet and the learned
 * denoiser return VDAMP_ERR_UNSUPPORTED.
 */
vdamp_status vdamp_plan_3d(vdamp_plan_h* plan, int32_t batch, const int32_t* nz, const int32_t* ny,
                           const int32_t* nx, int32_t levels, uint32_t flags, size_t* workspace_bytes);

vdamp_status vdamp_plan_destroy(vdamp_plan_h plan);

/*
 * vdamp_plan_describe -- the plan's launch configuration as text: per run of equal slice
 * size the row/column kernel (four-step M or Stockham) and its work items, the
 * threshold-search size classes and their band counts, the workspace size, and with
 * VDAMP_FLAG_AUTOTUNE what the tuner measured.
 *   buf, len        host buffer receiving at most len - 1 characters and a NUL
 *                   (nothing is written when buf is null or len is 0)
 *   needed          nullable out: characters of the full text plus the NUL
 */
vdamp_status vdamp_plan_describe(vdamp_plan_h plan, char* buf, size_t len, size_t* needed);

/*
 * vdamp_solve -- run `iters` iterations of Algorithm 1 on every slice, then the output step.
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
 *                   w = w_hat_{K-1} (output step)
 *   trace           nullable float32[iters][B][nb][3] out: (tau_k, theta_k, alpha_k) per
 *                   band (tau estimate, denoising and alpha steps); theta_k = lambda_k tau_k
 *                   in eq. 7's terms
 * FP32 arithmetic with FP64 threshold search; results are bitwise reproducible for a
 * given plan (fixed-order reductions, no floating-point atomics).
 */
vdamp_status vdamp_solve(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                         size_t workspace_bytes, const float* y, const uint8_t* mask,
                         const float* p, const float* sigma2, int32_t iters, float* x_hat,
                         float* trace);

/*
 * vdamp_solve_resume -- vdamp_solve from a given state, with an optional per-iteration
 * output.  The state of Algorithm 1 between iterations is (r_k, theta_k, alpha_k): the
 * denoising, alpha and Onsager-correction steps rebuild r_tilde_{k+1} from it, and the
 * k-space step needs nothing else.
 *   r_init          nullable complex64[sum N]: r_k (Mallat layout per slice).  Null: a
 *                   fresh start (r_tilde_0 = 0), exactly vdamp_solve; theta_init,
 *                   theta2_init and alpha_init must then be null too.
 *   theta_init      float32[B][nb] (required with r_init): theta_k per band, >= 0
 *   theta2_init     nullable float32[B][nb]: the FP32 key of each threshold, the squared
 *                   magnitude thresholding compares |r|^2 (rounded FP32 x*x + y*y)
 *                   against; vdamp_state_export returns it.  Null: fl(theta * theta).
 *                   With it, a solve split into two calls is bitwise equal to one call.
 *   alpha_init      float32[B][nb] (required with r_init): alpha_k per band, in [0, 1)
 *   iters           K >= 0 further iterations; each starts with the Onsager correction applied to the
 *                   previous state.  K = 0 with r_init gives the output step with w = eta(r_k; theta_k).
 *   x_hat, trace    as in vdamp_solve (trace rows count this call's iterations)
 *   x_monitor       nullable complex64[iters][sum N] out: the output step evaluated after every
 *                   iteration (the estimate x_hat_k a solve stopped there would return);
 *                   costs one more transform pass per iteration
 * Under VDAMP_FLAG_CHECK_FINITE the imported theta and alpha are validated too.
 * The input arrays are read on the stream; the caller may reuse them once it has synchronised.
 */
vdamp_status vdamp_solve_resume(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                                size_t workspace_bytes, const float* y, const uint8_t* mask,
                                const float* p, const float* sigma2, const float* r_init,
                                const float* theta_init, const float* theta2_init,
                                const float* alpha_init, int32_t iters, float* x_hat, float* trace,
                                float* x_monitor);

/*
 * vdamp_solve_noalloc -- vdamp_solve for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid allocation).
 * The workspace is a device array inside the library, VDAMP_NOALLOC_MAX_WORKSPACE bytes
 * per GPU, held from the first call on that GPU until the process ends; the call itself
 * allocates nothing (no hipMalloc, hipFree, graph instantiation or event creation: launches are
 * always eager, VDAMP_FLAG_USE_GRAPH and VDAMP_FLAG_TIMING of the plan are ignored).
 *   plan            as for vdamp_solve; its workspace_bytes must not exceed
 *                   VDAMP_NOALLOC_MAX_WORKSPACE, else VDAMP_ERR_WORKSPACE (nothing enqueued)
 *   other arguments as in vdamp_solve (caller-owned inputs and outputs)
 * Every call on one GPU shares that GPU's array, whose contents persist between calls:
 * nothing the solve reads is taken from an earlier call (every byte is written by the
 * solve before it is read), but two calls that overlap in time on one GPU (different
 * streams, or host threads) race on it and give undefined results.
 * vdamp_state_export is not available after this call (the workspace is not the caller's).
 */
#define VDAMP_NOALLOC_MAX_WORKSPACE ((size_t)64 << 20)
vdamp_status vdamp_solve_noalloc(vdamp_plan_h plan, hipStream_t stream, const float* y,
                                 const uint8_t* mask, const float* p, const float* sigma2,
                                 int32_t iters, float* x_hat, float* trace);

/*
 * fista_solve -- FISTA on 1/2 ||y - M_Omega F Psi^H w||^2 + lambda ||w||_1 (eq. 2 with
 * f = lambda ||Psi x||_1, in synthesis form), step size 1, zero start, every band
 * thresholded (Section 3's comparator).
 *   lambda          float32[B]: sparse weighting per slice
 *   x_hat           complex64[sum N] out: Psi^H w_K (K = 0 gives zeros)
 *   objective       nullable float32[iters][B] out: eq. 2's objective at each iterate
 *                   w_k, 1/2 ||y - M_Omega F Psi^H w_k||^2 + lambda ||w_k||_1 (costs one
 *                   more forward transform per iteration)
 * Other arguments as in vdamp_solve (p and sigma2 are not used).
 */
vdamp_status fista_solve(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                         size_t workspace_bytes, const float* y, const uint8_t* mask,
                         const float* lambda, int32_t iters, float* x_hat, float* objective);

/*
 * vdamp_state_export -- copy the state left by the last vdamp_solve (or
 * vdamp_solve_resume, or vdamp_solve_learned) on this workspace:
 *   r               nullable complex64[sum N] out: r_{K-1} (Mallat layout per slice)
 *   theta, theta2, alpha, tau  nullable float32[B][nb] out: the last iteration's
 *                   threshold, its FP32 key (see vdamp_solve_resume), alpha and tau
 * (r, theta, theta2, alpha) passed to vdamp_solve_resume continue the solve exactly.
 * Returns VDAMP_ERR_STATE if no solve with iters >= 1 (or a resume) ran on this workspace.
 */
vdamp_status vdamp_state_export(vdamp_plan_h plan, hipStream_t stream, const void* workspace,
                                float* r, float* theta, float* theta2, float* alpha, float* tau);

/*
 * vdamp_pass_times -- with VDAMP_FLAG_TIMING: synchronise the recorded events and return,
 * per kernel class (VDAMP_PASS_*), the summed kernel time in milliseconds and the
 * number of launches since the previous call (which resets the counters).
 *   ms, launches    host arrays of npass entries
 */
vdamp_status vdamp_pass_times(vdamp_plan_h plan, double* ms, int64_t* launches, int32_t npass);

/* ------------------------------------------------------------------------------------
 * Learned denoiser.  Algorithm 1 accepts any denoiser g(r; tau) together with its mean
 * derivative (alpha step); the conclusion proposes denoisers trained for wavelet
 * coefficients under the known colored Gaussian noise of VDAMP.  This one is a CNN in
 * the image domain, g(r) = Psi f(Psi^H r; tau), with
 *   u = (Re x, Im x) / s0,  t_b = log(max(tau_b / s0^2, 1e-12)),
 *   a1 = relu(conv(u; W1) + b1 + Wt t),  a_l = relu(conv(a_{l-1}; W_l) + b_l), l = 2..5,
 *   o = conv(a5; W6) + b6,  f(x) = s0 (u - o),
 * six circular 3x3 convolutions (2 -> 48 -> 48 -> 48 -> 48 -> 48 -> 2 channels).  BF16
 * weights and activations, FP32 accumulation (MFMA).  Parameters are FP32 masters,
 * flat, in the order W1[48][2][3][3], b1[48], Wt[48][nb], W2[48][48][3][3], b2[48], ...,
 * W5, b5, W6[2][48][3][3], b6[2].  Every slice's ny and nx must be multiples of 16.
 * A denoiser object is not shared by concurrently running streams.
 * ---------------------------------------------------------------------------------- */
typedef struct vdamp_cnn_t* vdamp_cnn_h;

/* How vdamp_solve_learned picks the denoiser of each subband. */
enum {
  VDAMP_JUDGE_SURE = 0, /* learned where its SURE is below soft thresholding's minimum */
  VDAMP_JUDGE_NONE = 1  /* learned in every subband (subject to the bound on alpha)   */
};

enum {
  VDAMP_CNN_WS_FORWARD = 0, /* vdamp_cnn_forward (with or without the JVP) */
  VDAMP_CNN_WS_TRAIN = 1,   /* vdamp_cnn_train_step */
  VDAMP_CNN_WS_SOLVE = 2    /* vdamp_solve_learned */
};

/* Create a denoiser for nbands = 1 + 3 levels noise levels; parameters start at zero. */
vdamp_status vdamp_cnn_create(vdamp_cnn_h* cnn, int32_t nbands);
vdamp_status vdamp_cnn_destroy(vdamp_cnn_h cnn);
/* Number of FP32 parameters. */
vdamp_status vdamp_cnn_param_count(vdamp_cnn_h cnn, int64_t* count);
/* Copy count parameters from device memory (layout above) and reset the Adam state. */
vdamp_status vdamp_cnn_set_params(vdamp_cnn_h cnn, hipStream_t stream, const float* params);
/* Copy the parameters (and, if grad is non-null, the last training step's gradient) to
 * device memory. */
vdamp_status vdamp_cnn_get_params(vdamp_cnn_h cnn, hipStream_t stream, float* params, float* grad);
/* Workspace bytes for one of the VDAMP_CNN_WS_* uses on this plan's batch. */
vdamp_status vdamp_cnn_workspace(vdamp_cnn_h cnn, vdamp_plan_h plan, int32_t kind, size_t* bytes);

/*
 * vdamp_cnn_forward -- x_out = f(x; tau) for every slice of the plan and, if tangent is
 * non-null, jvp_out = J_f(x) tangent (the Jacobian-vector product the divergence
 * estimate of the alpha step needs).
 *   x, tangent       complex64[sum N] images (device)
 *   tau              float32[B][16] noise levels per band (first nbands used)
 *   s0               float32[B] input scales (> 0)
 *   x_out, jvp_out   complex64[sum N] out
 */
vdamp_status vdamp_cnn_forward(vdamp_cnn_h cnn, vdamp_plan_h plan, hipStream_t stream,
                               void* workspace, size_t workspace_bytes, const float* x,
                               const float* tau, const float* s0, float* x_out,
                               const float* tangent, float* jvp_out);

/*
 * vdamp_cnn_train_step -- one Adam step (beta = 0.9, 0.999, eps = 1e-8, learning rate
 * lr) on the loss (1/B) sum_slices ||f(x; tau) - x0||^2 / (s0^2 N), with the gradient
 * by backpropagation; loss (device float32[1]) receives the loss before the step.
 */
vdamp_status vdamp_cnn_train_step(vdamp_cnn_h cnn, vdamp_plan_h plan, hipStream_t stream,
                                  void* workspace, size_t workspace_bytes, const float* x,
                                  const float* tau, const float* s0, const float* x0, float lr,
                                  float* loss);

/*
 * vdamp_solve_learned -- Algorithm 1 with the learned denoiser judged against SURE soft
 * thresholding per subband: each iteration computes soft thresholding's SURE minimum
 * (denoising and alpha steps as in vdamp_solve), then w_cnn = Psi f(Psi^H r; tau) and
 * its mean derivative alpha from one complex Rademacher probe b (Psi J_f Psi^H b, drawn
 * from seed by SplitMix64 as a counter-based generator), and uses w_cnn with that alpha
 * in the Onsager correction and the output step in the subbands where its SURE,
 * ||w_cnn - r||^2 + (2 alpha - 1) N_b tau,
 * is below soft thresholding's (judge = VDAMP_JUDGE_SURE; with VDAMP_JUDGE_NONE in
 * every subband) and alpha <= 1 - 1/N_b.  Iterations k < learned_from use soft
 * thresholding alone (the network is not evaluated), so a solve can spend the network's
 * cost on its last iterations only; learned_from >= iters gives vdamp_solve's result.
 * s0 per slice is sqrt(mean over pixels of (m / p) |y|^2) (1 if that is zero).
 * Arguments as in vdamp_solve plus the denoiser, its VDAMP_CNN_WS_SOLVE workspace,
 * learned_from, the judge and the seed; trace holds soft thresholding's (tau, theta,
 * alpha).
 */
vdamp_status vdamp_solve_learned(vdamp_plan_h plan, vdamp_cnn_h cnn, hipStream_t stream,
                                 void* workspace, size_t workspace_bytes, void* cnn_workspace,
                                 size_t cnn_workspace_bytes, const float* y, const uint8_t* mask,
                                 const float* p, const float* sigma2, int32_t iters,
                                 int32_t learned_from, int32_t judge, uint64_t seed, float* x_hat,
                                 float* trace);

/*
 * vdamp_learned_export -- after vdamp_solve_learned whose last iteration evaluated the
 * network (iters > learned_from), that iteration's judge: per
 * band the choice (int32[B][nb], 1 = learned denoiser), the learned denoiser's SURE, its
 * alpha estimate and soft thresholding's SURE minimum (float32[B][nb] each), and the
 * input scales s0 (float32[B]); any output may be null.  vdamp_state_export gives r, theta and tau of that iteration and
 * the alpha that the Onsager correction used (the learned one where chosen).
 */
vdamp_status vdamp_learned_export(vdamp_cnn_h cnn, vdamp_plan_h plan, hipStream_t stream,
                                  const void* cnn_workspace, int32_t* sel, float* s0,
                                  float* sure_cnn, float* alpha_cnn, float* sure_soft);

/*
 * vdamp_wavelet -- Psi (inverse = 0) or Psi^H (inverse = 1) of every slice: s-level
 * periodic orthonormal Haar, Mallat layout.  in and out are complex64[sum N] and must
 * not overlap.
 */
vdamp_status vdamp_wavelet(vdamp_plan_h plan, hipStream_t stream, int32_t inverse,
                           const float* in, float* out);

/*
 * vdamp_wavelet_ws -- Psi (inverse = 0) or Psi^H (inverse = 1) of every slice for any
 * plan (Haar or vdamp_plan_ortho's wavelet; Section 2's orthogonal Psi), on the plan's
 * workspace (workspace_bytes >= the plan's size; its contents are overwritten, so a
 * solve's state on it is lost).  in and out are complex64[sum N] and must not overlap.
 */
vdamp_status vdamp_wavelet_ws(vdamp_plan_h plan, hipStream_t stream, void* workspace,
                              size_t workspace_bytes, int32_t inverse, const float* in, float* out);

/* Static description of a status code. */
const char* vdamp_status_string(vdamp_status s);

/* Detail string of the last failure on the calling thread ("" if none). */
const char* vdamp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VDAMP_H */

"""FP64 oracle of VDAMP with the learned denoiser judged against SURE soft thresholding.

TEST INFRASTRUCTURE ONLY: used by tests/ (and nothing in the product path).

Algorithm 1 leaves the denoiser g(r; tau) open, with its mean derivative in the alpha step (the
same reading as for soft thresholding: the mean Wirtinger derivative dg/dr of the
band).  For the learned denoiser g(r) = Psi f(Psi^H r; tau) (oracle/cnn_ref.py), per
iteration and subband b:
  w_cnn = Psi f(Psi^H r)
  alpha_cnn = (1/N_b) sum_{i in b} Re(conj(q_i) (Psi J_f Psi^H q)_i)
for one complex Rademacher probe q in {+-1 +- i}/sqrt2 (its expectation is the mean
Wirtinger derivative: E[q q^H] = I and E[q q^T] = 0), and the Stein estimate of its
error, with tau the complex variance of the band's noise (real components tau/2):
  SURE_cnn = ||w_cnn - r||^2 + tau div_R2 g - N_b tau,   div_R2 g = 2 N_b alpha_cnn,
which for soft thresholding reduces to the scan form of the threshold search.  The
learned output replaces soft thresholding in the band when SURE_cnn is below the SURE
minimum of soft thresholding and alpha_cnn <= 1 - 1/N_b (soft thresholding's range of
alpha, which keeps the Onsager correction's 1/(1 - alpha) bounded); otherwise the band keeps soft
thresholding with its own theta and alpha.

The probe comes from SplitMix64 (Steele, Lea and Flood, 2014) used as a counter-based
generator: value(c) = mix(seed + (c + 1) * 0x9E3779B97F4A7C15 mod 2^64), with the
counter c = iteration << 48 | slice << 32 | (row * nx + column); bit 0 set makes the
real part negative, bit 1 the imaginary part.

The input scale is s0 = sqrt((1/N) sum_j (m_j / p_j) |y_j|^2) (1 if that is zero).
"""
from __future__ import annotations

import numpy as np

from . import cnn_ref, vdamp_ref

GOLDEN = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


def splitmix64_mix(z):
    """The SplitMix64 output function on uint64 values (numpy arrays wrap mod 2^64)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def splitmix64_stream(seed, n, start=0):
    """Outputs start+1 .. start+n of a SplitMix64 generator started from state seed."""
    c = np.uint64(start) + np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return splitmix64_mix(np.uint64(seed) + c * np.uint64(GOLDEN))


def probe(seed, it, slice_id, ny, nx):
    """Complex Rademacher probe of one slice at one iteration (wavelet layout)."""
    idx = np.arange(ny * nx, dtype=np.uint64)
    c = (np.uint64(it) << np.uint64(48)) | (np.uint64(slice_id) << np.uint64(32)) | idx
    with np.errstate(over="ignore"):
        z = splitmix64_mix(np.uint64(seed) + (c + np.uint64(1)) * np.uint64(GOLDEN))
    h = 1.0 / np.sqrt(2.0)
    re = np.where((z & np.uint64(1)) != 0, -h, h)
    im = np.where((z & np.uint64(2)) != 0, -h, h)
    return (re + 1j * im).reshape(ny, nx)


def input_scale(y, mask, p):
    om = np.asarray(mask).astype(bool)
    w = np.zeros(y.shape)
    w[om] = 1.0 / np.asarray(p, dtype=np.float64)[om]
    m = float(np.sum(w * np.abs(y) ** 2) / y.size)
    return np.sqrt(m) if m > 0 else 1.0


def mc_alpha(jvp_band_fn, q, bands_list):
    """Per-band probe estimate of the mean Wirtinger derivative: jvp_band_fn(q) is the
    denoiser's Jacobian applied to q (wavelet layout)."""
    jq = jvp_band_fn(q)
    out = []
    for (rs, cs, _, _) in bands_list:
        qb, jb = q[rs, cs], jq[rs, cs]
        out.append(float(np.mean((np.conj(qb) * jb).real)))
    return np.array(out)


def sure_general(r_band, w_band, alpha, tau):
    """Stein estimate of ||w - w0||^2 for a denoiser with output w and mean Wirtinger
    derivative alpha on a band with complex noise variance tau."""
    nb = r_band.size
    return float(np.sum(np.abs(w_band - r_band) ** 2) + (2.0 * alpha - 1.0) * nb * tau)


def cnn_candidate(params, r, tau, s, s0, seed, it, slice_id, bf16=True):
    """w_cnn, alpha_cnn and SURE_cnn per band for the learned denoiser at r."""
    ny, nx = r.shape
    x = vdamp_ref.haar_synthesis(r, s)
    xo = cnn_ref.forward(params, x, tau, s0, bf16=bf16)
    w = vdamp_ref.haar_analysis(xo, s)
    q = probe(seed, it, slice_id, ny, nx)
    bl = vdamp_ref.bands(ny, nx, s)

    def jvp_fn(v):
        return vdamp_ref.haar_analysis(
            cnn_ref.jvp(params, x, tau, s0, vdamp_ref.haar_synthesis(v, s), bf16=bf16), s)

    al = mc_alpha(jvp_fn, q, bl)
    sure = np.array([sure_general(r[rs, cs], w[rs, cs], al[b], tau[b])
                     for b, (rs, cs, _, _) in enumerate(bl)])
    return w, al, sure


def judged_denoise(params, r, tau, s, s0, seed, it, slice_id, bf16=True, always=False):
    """The denoising, alpha and Onsager-correction steps with the per-band choice
    between soft thresholding and the learned denoiser (always=True: the learned one wherever alpha_cnn <= 1 - 1/N_b, without the
    SURE comparison).  Returns w_hat, r_tilde_next and a record of the decision."""
    ny, nx = r.shape
    w_cnn, al_c, sure_c = cnn_candidate(params, r, tau, s, s0, seed, it, slice_id, bf16)
    w_hat = np.zeros_like(r)
    rt = np.zeros_like(r)
    rec = dict(sel=[], theta=[], alpha=[], alpha_soft=[], alpha_cnn=al_c, sure_cnn=sure_c,
               sure_soft=[])
    for b, (rs, cs, _, _) in enumerate(vdamp_ref.bands(ny, nx, s)):
        rb = r[rs, cs]
        nb = rb.size
        th, al, _, smin = vdamp_ref.sure_threshold(np.abs(rb), tau[b])
        use = bool((always or sure_c[b] < smin) and al_c[b] <= 1.0 - 1.0 / nb)
        if use:
            wb, a = w_cnn[rs, cs], al_c[b]
        else:
            wb, a = vdamp_ref.soft(rb, th), al
        w_hat[rs, cs] = wb
        rt[rs, cs] = (wb - a * rb) / (1.0 - a)
        rec["sel"].append(int(use))
        rec["theta"].append(th)
        rec["alpha"].append(a)
        rec["alpha_soft"].append(al)
        rec["sure_soft"].append(smin)
    return w_hat, rt, {k: np.asarray(v) for k, v in rec.items()}


def vdamp_learned(y, mask, p, sigma2, s, iters, params, seed, slice_id=0, bf16=True, always=False,
                  learned_from=0):
    """Algorithm 1 with the judged learned denoiser, in FP64 (BF16 rounding of the
    network's weights and activations where the kernels store BF16 when bf16=True).
    Iterations before learned_from use soft thresholding alone."""
    y = np.asarray(y, dtype=np.complex128)
    p = np.asarray(p, dtype=np.float64)
    ny, nx = y.shape
    vdamp_ref.check_shape(ny, nx, s)
    S = vdamp_ref.tau_weights(ny, nx, s)
    s0 = input_scale(y, mask, p)
    rt = np.zeros((ny, nx), dtype=np.complex128)
    w_hat = np.zeros_like(rt)
    recs = []
    for it in range(iters):
        r, tau = vdamp_ref.vdamp_step(rt, y, mask, p, sigma2, s, S)
        if it < learned_from:
            w_hat, rt, th, al = vdamp_ref.denoise(r, tau, s)
            rec = dict(sel=np.zeros(len(th), dtype=int), theta=th, alpha=al)
        else:
            w_hat, rt, rec = judged_denoise(params, r, tau, s, s0, seed, it, slice_id, bf16, always)
        rec["tau"] = tau
        rec["r"] = r
        recs.append(rec)
    x_hat = vdamp_ref.output_step(w_hat, y, mask, s)
    return dict(x_hat=x_hat, records=recs, s0=s0)

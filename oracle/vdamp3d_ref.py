"""FP64 CPU oracle for VDAMP on 3D k-space (Section 1 allows Phi = M_Omega F with a 3D
DFT; Algorithm 1 is unchanged with a 3D orthogonal wavelet).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute
this module: it is used by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  It shares no code with the HIP library; it reuses
the 2D oracle's SURE search, soft threshold and tau estimate, which do not depend on
the dimension.

Conventions (the 2D ones extended; each pinned by a test):
* F is the unitary 3D DFT in natural order (numpy ``fftn``, ``norm="ortho"``).
* Psi is the s-level periodic orthonormal 3D Haar transform, Mallat layout: one level
  acts on the front-top-left block, along x ((even + odd)/sqrt2 to the left half,
  (even - odd)/sqrt2 to the right), then along y (top / bottom), then along z (front /
  back).  Bands: b = 0 is LLL_s, then for l = s .. 1 the seven detail octants of kind
  k = 1 .. 7, where bit 0 of k means high along x, bit 1 high along y, bit 2 high along
  z (k = 1, 2, 3 with z low are the 2D LH, HL, HH).  1 + 7 s bands.
* S_b(kz, ky, kx) = Z_b(kz) Y_b(ky) X_b(kx): products of the 1D Haar scaling/wavelet
  powers (separable basis functions).
"""
from __future__ import annotations

import numpy as np

from oracle import vdamp_ref as o

SQRT2 = np.sqrt(2.0)


def fft3u(x):
    return np.fft.fftn(x, norm="ortho")


def ifft3u(X):
    return np.fft.ifftn(X, norm="ortho")


def _anal_axis(blk, axis):
    e = np.take(blk, np.arange(0, blk.shape[axis], 2), axis=axis)
    d = np.take(blk, np.arange(1, blk.shape[axis], 2), axis=axis)
    return np.concatenate([(e + d) / SQRT2, (e - d) / SQRT2], axis=axis)


def _synth_axis(blk, axis):
    n = blk.shape[axis]
    lo = np.take(blk, np.arange(0, n // 2), axis=axis)
    hi = np.take(blk, np.arange(n // 2, n), axis=axis)
    out = np.empty_like(blk)
    idx_e = [slice(None)] * blk.ndim
    idx_o = [slice(None)] * blk.ndim
    idx_e[axis] = slice(0, n, 2)
    idx_o[axis] = slice(1, n, 2)
    out[tuple(idx_e)] = (lo + hi) / SQRT2
    out[tuple(idx_o)] = (lo - hi) / SQRT2
    return out


def haar3_analysis(x, s):
    """w = Psi x: s-level periodic orthonormal 3D Haar, Mallat layout."""
    w = np.array(x, dtype=np.complex128, copy=True)
    d, h, wd = w.shape
    for _ in range(s):
        blk = w[:d, :h, :wd]
        for axis in (2, 1, 0):
            blk = _anal_axis(blk, axis)
        w[:d, :h, :wd] = blk
        d, h, wd = d // 2, h // 2, wd // 2
    return w


def haar3_synthesis(w, s):
    """x = Psi^H w, the inverse of haar3_analysis."""
    x = np.array(w, dtype=np.complex128, copy=True)
    nz, ny, nx = x.shape
    for l in range(s, 0, -1):
        d, h, wd = nz >> (l - 1), ny >> (l - 1), nx >> (l - 1)
        blk = x[:d, :h, :wd]
        for axis in (0, 1, 2):
            blk = _synth_axis(blk, axis)
        x[:d, :h, :wd] = blk
    return x


def bands3(nz, ny, nx, s):
    """Band blocks in band order: (z slice, y slice, x slice, level, kind)."""
    out = [(slice(0, nz >> s), slice(0, ny >> s), slice(0, nx >> s), s, 0)]
    for l in range(s, 0, -1):
        d, h, w = nz >> l, ny >> l, nx >> l
        for k in range(1, 8):
            z0 = d if k & 4 else 0
            y0 = h if k & 2 else 0
            x0 = w if k & 1 else 0
            out.append((slice(z0, z0 + d), slice(y0, y0 + h), slice(x0, x0 + w), l, k))
    return out


def check_shape3(nz, ny, nx, s):
    if s < 1 or nz % (1 << s) or ny % (1 << s) or nx % (1 << s):
        raise ValueError(f"volume {nz}x{ny}x{nx} is not divisible by 2^{s}")


def tau_weights3(nz, ny, nx, s):
    """S_b for every band: float64 [nz][ny][nx] arrays, separable per band."""
    out = []
    for (_, _, _, l, k) in bands3(nz, ny, nx, s):
        f = []
        for n, hi in ((nz, k & 4), (ny, k & 2), (nx, k & 1)):
            f.append(o.haar_wavelet_power(n, l) if hi else o.haar_scaling_power(n, l))
        out.append(f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :])
    return out


def vdamp3_step(rt, y, mask, p, sigma2, s, S):
    """The k-space step: from r_tilde_k to (r_k, tau_k)."""
    om = mask.astype(bool)
    z = np.where(om, y - fft3u(haar3_synthesis(rt, s)), 0.0)   # residual step
    v = np.zeros_like(z)
    v[om] = z[om] / p[om]
    r = rt + haar3_analysis(ifft3u(v), s)                       # back-projection
    return r, o.tau_estimate(z, mask, p, sigma2, S)            # tau estimate


def denoise3(r, tau, s, theta_override=None, alpha_override=None):
    """The denoising, alpha and Onsager-correction steps per band (SURE threshold, eta,
    alpha, r_tilde_{k+1})."""
    nz, ny, nx = r.shape
    w_hat = np.zeros_like(r)
    rt_next = np.zeros_like(r)
    thetas, alphas = [], []
    for b, (zs, ys, xs, _, _) in enumerate(bands3(nz, ny, nx, s)):
        rb = r[zs, ys, xs]
        if theta_override is None:
            th, al, _, _ = o.sure_threshold(np.abs(rb), tau[b])
        else:
            th = float(theta_override[b])
            al = (o.wirtinger_mean_soft(rb, th) if alpha_override is None else float(alpha_override[b]))
        wb = o.soft(rb, th)
        w_hat[zs, ys, xs] = wb
        rt_next[zs, ys, xs] = (wb - al * rb) / (1.0 - al)
        thetas.append(th)
        alphas.append(al)
    return w_hat, rt_next, np.array(thetas), np.array(alphas)


def output_step3(w_hat, y, mask, s):
    """The output step: x_hat = Psi^H w + Phi^H (y - Phi Psi^H w)."""
    x = haar3_synthesis(w_hat, s)
    om = mask.astype(bool)
    return x + ifft3u(np.where(om, y - fft3u(x), 0.0))


def _run(rt, w_hat, y, mask, p, sigma2, s, S, iters, record):
    taus, thetas, alphas, rs = [], [], [], []
    for _ in range(iters):
        r, tau = vdamp3_step(rt, y, mask, p, sigma2, s, S)
        w_hat, rt, th, al = denoise3(r, tau, s)
        taus.append(tau)
        thetas.append(th)
        alphas.append(al)
        if record:
            rs.append(r)
    out = dict(x_hat=output_step3(w_hat, y, mask, s), tau=np.array(taus), theta=np.array(thetas),
               alpha=np.array(alphas))
    if record:
        out["r"] = rs
    return out


def vdamp3(y, mask, p, sigma2, s, iters, record=False):
    """Algorithm 1 in FP64 on a volume [nz][ny][nx] (3D Haar, 3D unitary DFT)."""
    y = np.asarray(y, dtype=np.complex128)
    p = np.asarray(p, dtype=np.float64)
    check_shape3(*y.shape, s)
    S = tau_weights3(*y.shape, s)
    rt = np.zeros(y.shape, dtype=np.complex128)            # initialisation: r_tilde_0 = 0
    return _run(rt, np.zeros_like(rt), y, mask, p, sigma2, s, S, iters, record)


def vdamp3_resume(y, mask, p, sigma2, s, r, theta, alpha, iters, record=False):
    """Algorithm 1 continued from the state (r_k, theta_k, alpha_k): each further
    iteration starts with the denoising, alpha and Onsager-correction steps on the
    previous state.  iters = 0 gives the output step with w = eta(r_k; theta_k)."""
    y = np.asarray(y, dtype=np.complex128)
    p = np.asarray(p, dtype=np.float64)
    check_shape3(*y.shape, s)
    S = tau_weights3(*y.shape, s)
    w_hat, rt, _, _ = denoise3(np.asarray(r, dtype=np.complex128), None, s, theta_override=theta,
                               alpha_override=alpha)
    return _run(rt, w_hat, y, mask, p, sigma2, s, S, iters, record)

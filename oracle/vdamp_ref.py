"""FP64 CPU oracle for VDAMP (Algorithm 1) with SURE-tuned complex soft thresholding,
and for the FISTA comparator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute
this module: it is used by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  It shares no code with the HIP library.

It is written to be checked by eye against the paper: plain NumPy in complex128, the
steps in the order of Algorithm 1, library primitives only for the FFT and the sort.

Conventions (readings of the paper where it is silent; each is pinned by a test):
* F is the unitary 2D DFT in natural order (numpy ``norm="ortho"``); exact consistency
  of the output step (Section 2, final line of Algorithm 1) needs F^H F = I.
* Psi is an s-level periodic orthonormal 2D wavelet transform, Mallat layout: Haar by
  default, or the transform of any orthonormal lowpass filter h (``wavelet=h``; see
  dwt2).  For Haar, one level
  acts on the top-left block: along x, a = (x[2i] + x[2i+1]) / sqrt2 goes left and
  d = (x[2i] - x[2i+1]) / sqrt2 goes right; then the same along y (top / bottom).
  Band order b = 0 is LL_s, then for l = s .. 1 the triple (LH_l, HL_l, HH_l), where
  LH = low along y / high along x (top-right block), HL = high along y / low along x
  (bottom-left), HH = bottom-right.  Scale 1 is the finest (Section 3).
* The denoiser is complex soft thresholding eta(r; theta) = r max(0, 1 - theta/|r|),
  with one threshold per subband (eq. 7).  The threshold minimises the complex,
  colored SURE over the candidate set theta in {|r_i|} of the band (Section 3).
* g' of the alpha step is the Wirtinger derivative (half the R^2 divergence), averaged within
  each subband, so alpha has 1+3s entries.
* The output step's w is the last denoised estimate w_hat_{K-1}; with K = 0 the output is the
  zero-filled F^H y.
* Structured sparsity (group=2; Section 4 names structured sparsity as a richer model
  that SURE can tune): the two horizontally adjacent coefficients (x = 2j, 2j+1) of each
  band row form a group, shrunk jointly by group soft thresholding
  r_g max(0, 1 - theta/||r_g||), with theta minimising the group SURE (2d real
  dimensions per group of d complex coefficients) and alpha the mean Wirtinger
  derivative, i.e. half the real divergence per complex coefficient.
"""
from __future__ import annotations

import numpy as np

SQRT2 = np.sqrt(2.0)


# ----------------------------------------------------------------------------------
# Linear operators (Section 1: Phi = M_Omega F; Section 2: orthogonal wavelet Psi)

def fft2u(x):
    """Unitary 2D DFT, natural order."""
    return np.fft.fft2(x, norm="ortho")


def ifft2u(X):
    """Inverse unitary 2D DFT (F^H)."""
    return np.fft.ifft2(X, norm="ortho")


def haar_analysis(x, s):
    """w = Psi x: s-level periodic orthonormal 2D Haar, Mallat layout."""
    w = np.array(x, dtype=np.complex128, copy=True)
    h, wd = w.shape
    for _ in range(s):
        blk = w[:h, :wd]
        t = np.concatenate([(blk[:, 0::2] + blk[:, 1::2]) / SQRT2,
                            (blk[:, 0::2] - blk[:, 1::2]) / SQRT2], axis=1)
        w[:h, :wd] = np.concatenate([(t[0::2, :] + t[1::2, :]) / SQRT2,
                                     (t[0::2, :] - t[1::2, :]) / SQRT2], axis=0)
        h //= 2
        wd //= 2
    return w


def haar_synthesis(w, s):
    """x = Psi^H w, the inverse of haar_analysis."""
    x = np.array(w, dtype=np.complex128, copy=True)
    ny, nx = x.shape
    for l in range(s, 0, -1):
        h, wd = ny >> l, nx >> l
        blk = x[:2 * h, :2 * wd]
        t = np.empty_like(blk)
        lo, hi = blk[:h, :], blk[h:, :]
        t[0::2, :] = (lo + hi) / SQRT2
        t[1::2, :] = (lo - hi) / SQRT2
        out = np.empty_like(blk)
        lo, hi = t[:, :wd], t[:, wd:]
        out[:, 0::2] = (lo + hi) / SQRT2
        out[:, 1::2] = (lo - hi) / SQRT2
        x[:2 * h, :2 * wd] = out
    return x


# General orthonormal wavelets (Algorithm 1 asks only for an orthogonal Psi).  The
# textbook periodic Mallat algorithm: one level filters the top-left block along x,
#   a[j] = sum_t h[t] x[(2j + t) mod M]  (left half),
#   d[j] = sum_t g[t] x[(2j + t) mod M]  (right half),  g[t] = (-1)^t h[L-1-t],
# then the same along y (top / bottom); the next level repeats on the top-left quarter.
# With h = (1, 1)/sqrt2 this is haar_analysis.

def highpass(h):
    h = np.asarray(h, dtype=np.float64)
    L = len(h)
    return np.array([(-1.0) ** t * h[L - 1 - t] for t in range(L)])


def _analysis_1d(x, h, g, axis):
    M = x.shape[axis]
    j2 = 2 * np.arange(M // 2)
    lo = sum(h[t] * np.take(x, (j2 + t) % M, axis=axis) for t in range(len(h)))
    hi = sum(g[t] * np.take(x, (j2 + t) % M, axis=axis) for t in range(len(g)))
    return np.concatenate([lo, hi], axis=axis)


def _synthesis_1d(c, h, g, axis):
    """Adjoint of _analysis_1d: x[(2j + t) mod M] += h[t] a[j] + g[t] d[j]."""
    c = np.moveaxis(c, axis, 0)
    M = c.shape[0]
    a, d = c[: M // 2], c[M // 2:]
    x = np.zeros_like(c)
    j2 = 2 * np.arange(M // 2)
    for t in range(len(h)):
        np.add.at(x, (j2 + t) % M, h[t] * a + g[t] * d)
    return np.moveaxis(x, 0, axis)


def dwt2(x, h, s):
    """w = Psi x for the orthonormal lowpass h: s levels, periodic, Mallat layout."""
    h = np.asarray(h, dtype=np.float64)
    g = highpass(h)
    w = np.array(x, dtype=np.complex128, copy=True)
    hh, wd = w.shape
    for _ in range(s):
        blk = _analysis_1d(w[:hh, :wd], h, g, axis=1)
        w[:hh, :wd] = _analysis_1d(blk, h, g, axis=0)
        hh //= 2
        wd //= 2
    return w


def idwt2(w, h, s):
    """x = Psi^H w, the inverse (and adjoint) of dwt2."""
    h = np.asarray(h, dtype=np.float64)
    g = highpass(h)
    x = np.array(w, dtype=np.complex128, copy=True)
    ny, nx = x.shape
    for l in range(s, 0, -1):
        hh, wd = ny >> (l - 1), nx >> (l - 1)
        blk = _synthesis_1d(x[:hh, :wd], h, g, axis=0)
        x[:hh, :wd] = _synthesis_1d(blk, h, g, axis=1)
    return x


def analysis(x, s, wavelet=None):
    """Psi x: Haar when wavelet is None, else dwt2 with lowpass filter `wavelet`."""
    return haar_analysis(x, s) if wavelet is None else dwt2(x, wavelet, s)


def synthesis(w, s, wavelet=None):
    """Psi^H w: Haar when wavelet is None, else idwt2."""
    return haar_synthesis(w, s) if wavelet is None else idwt2(w, wavelet, s)


def bands(ny, nx, s):
    """Subband blocks in band order: LL_s, then (LH_l, HL_l, HH_l) for l = s..1.
    Returns a list of (row slice, column slice, level, kind)."""
    out = [(slice(0, ny >> s), slice(0, nx >> s), s, "LL")]
    for l in range(s, 0, -1):
        h, w = ny >> l, nx >> l
        out.append((slice(0, h), slice(w, 2 * w), l, "LH"))
        out.append((slice(h, 2 * h), slice(0, w), l, "HL"))
        out.append((slice(h, 2 * h), slice(w, 2 * w), l, "HH"))
    return out


def check_shape(ny, nx, s):
    if s < 1 or ny % (1 << s) or nx % (1 << s):
        raise ValueError(f"image {ny}x{nx} is not divisible by 2^{s}")


# ----------------------------------------------------------------------------------
# initialisation: S = |Phi Psi^H|^2.  For Haar it is separable per band, S_b(ky,kx) =
# Y_b(ky) X_b(kx), with 1D factors the squared DFT magnitudes of the 1D scaling
# function (length 2^m, height 2^(-m/2)) and wavelet (+- 2^(-l/2) on two halves).

def _dirichlet(k, M, n):
    """D_M(k) = sum_{t<M} exp(-2 pi i k t / n) in magnitude: sin(pi k M/n)/sin(pi k/n)."""
    k = np.asarray(k, dtype=np.float64)
    num = np.sin(np.pi * k * M / n)
    den = np.sin(np.pi * k / n)
    out = np.empty_like(k)
    z = np.isclose(np.mod(k, n), 0.0)
    out[~z] = num[~z] / den[~z]
    out[z] = M
    return out


def haar_scaling_power(n, m):
    """|DFT of the level-m scaling function|^2 over k = 0..n-1 (unitary DFT)."""
    k = np.arange(n)
    return _dirichlet(k, 2 ** m, n) ** 2 / (n * 2.0 ** m)


def haar_wavelet_power(n, l):
    """|DFT of the level-l wavelet|^2 over k = 0..n-1 (unitary DFT)."""
    k = np.arange(n)
    h = 2 ** (l - 1)
    return 4.0 * _dirichlet(k, h, n) ** 2 * np.sin(np.pi * k * h / n) ** 2 / (n * 2.0 ** l)


def tau_weights_filter(ny, nx, s, h):
    """The initialisation for a general orthonormal Psi, from the definition S = |Phi Psi^H|^2: the
    squared unitary DFT of the basis function of the first coefficient of each band
    (periodic filtering makes every coefficient of a band a shift of it, so the column
    of S is the same for the whole band).  A list of float64 [ny][nx] arrays."""
    out = []
    for (rs, cs, _, _) in bands(ny, nx, s):
        e = np.zeros((ny, nx), dtype=np.complex128)
        e[rs.start, cs.start] = 1.0
        out.append(np.abs(fft2u(idwt2(e, h, s))) ** 2)
    return out


def tau_weights(ny, nx, s, wavelet=None):
    """S_b(ky, kx) for every band b, as a list of float64 [ny][nx] arrays."""
    if wavelet is not None:
        return tau_weights_filter(ny, nx, s, wavelet)
    out = []
    for (_, _, l, kind) in bands(ny, nx, s):
        Ly, Lx = haar_scaling_power(ny, l), haar_scaling_power(nx, l)
        Hy, Hx = haar_wavelet_power(ny, l), haar_wavelet_power(nx, l)
        fy, fx = {"LL": (Ly, Lx), "LH": (Ly, Hx), "HL": (Hy, Lx), "HH": (Hy, Hx)}[kind]
        out.append(np.outer(fy, fx))
    return out


# ----------------------------------------------------------------------------------
# denoising step: complex soft thresholding, and its SURE-optimal threshold (Section 3).

def soft(r, theta):
    """eta(r; theta) = r * max(0, 1 - theta/|r|); zero when |r| <= theta."""
    a = np.abs(r)
    out = np.zeros_like(r)
    keep = a > theta
    out[keep] = r[keep] * (1.0 - theta / a[keep])
    return out


def sure_value(a, theta, tau, d=1):
    """Complex colored SURE of soft thresholding one band at threshold theta, summed
    over the band: Stein's estimate with n ~ CN(0, tau) (2 real dimensions per
    coefficient), written directly from its definition, O(N_b).

    With d > 1, a holds the norms of groups of d coefficients thresholded jointly
    (D = 2d real dimensions, noise variance tau/2 in each): a group at or below theta
    contributes ||r_g||^2 - D tau/2, one above it D tau/2 + theta^2 - (D - 1) tau theta/||r_g||
    (Stein: E||eta - mu||^2 = D sigma^2 + E||eta - r||^2 + 2 sigma^2 E div(eta - r))."""
    a = np.asarray(a, dtype=np.float64)
    below = a <= theta
    above = ~below
    return (np.sum(a[below] ** 2 - d * tau)
            + np.sum(theta ** 2 + d * tau - (2 * d - 1) * tau * theta / a[above]))


def sure_threshold(a, tau, d=1):
    """SURE-minimising threshold for one band.

    a: magnitudes |r_i| of the band (float64), tau: effective noise variance of the band.
    Candidates theta = a_(m) (m = number of magnitudes <= theta), theta > 0, taking only
    the last index of a run of equal values; ties of the SURE value go to the smallest
    theta.  With sorted a, A_m = sum_{i<=m} a_(i)^2 and R_m = sum_{i>m} 1/a_(i):
        SURE(m) = A_m - m tau + (N_b - m)(theta^2 + tau) - tau theta R_m.
    alpha (alpha step) = mean over the band of the Wirtinger derivative of eta, which is
    1 - theta/(2|r|) above the threshold and 0 below:
        alpha = ((N_b - m) - (theta/2) R_m) / N_b.
    Returns (theta, alpha, m, sure_min).  All-zero band: theta = 0, alpha = 0.

    Groups (d > 1): a are the n group norms and, with tl = d tau and td = (2d - 1) tau
    (sure_value),
        SURE(m) = A_m - m tl + (n - m)(theta^2 + tl) - td theta R_m,
        alpha = (d (n - m) - (td / tau)(theta/2) R_m) / (d n);
    with d = 1 both reduce to the formulas above.
    """
    a = np.sort(np.asarray(a, dtype=np.float64).ravel())
    n = a.size
    tl, td = d * tau, (2 * d - 1) * tau
    if n == 0:
        raise ValueError("empty band")
    if a[-1] == 0.0:
        return 0.0, 0.0, n, float(n * (0.0 - tl))
    A = np.cumsum(a ** 2)                                  # A[m-1] = A_m
    inv = np.zeros(n)
    pos = a > 0
    inv[pos] = 1.0 / a[pos]
    Rsuf = np.concatenate([np.cumsum(inv[::-1])[::-1][1:], [0.0]])  # Rsuf[m-1] = R_m
    m = np.arange(1, n + 1, dtype=np.float64)
    sure = A - m * tl + (n - m) * (a ** 2 + tl) - td * a * Rsuf
    last_of_run = np.concatenate([a[:-1] < a[1:], [True]])
    valid = last_of_run & (a > 0)
    sure_v = np.where(valid, sure, np.inf)
    i = int(np.argmin(sure_v))                             # first minimum = smallest theta
    theta = float(a[i])
    mm = i + 1
    alpha = float((d * (n - mm) - 0.5 * (2 * d - 1) * theta * Rsuf[i]) / (d * n))
    return theta, alpha, mm, float(sure_v[i])


def sure_threshold_continuous(a, tau, d=1):
    """SURE-minimising threshold over every theta > 0, not only the candidates |r_i|
    (the paper's SURE step is solved "approximately"; this is the exact minimiser).

    Between consecutive distinct sorted magnitudes, theta in (a_(m), a_(m+1)) with m
    magnitudes at or below theta, SURE(theta) = A_m - m tau + (N_b - m)(theta^2 + tau)
    - tau theta R_m is a convex quadratic, minimised at theta* = tau R_m / (2 (N_b - m));
    theta* counts where it lies strictly inside its interval (the interval below the
    smallest positive magnitude starts at 0).  The candidates a_(m) themselves are those
    of sure_threshold.  The smallest value wins, ties to the smaller theta.
    Returns (theta, alpha, m, sure_min), alpha = ((N_b - m) - (theta/2) R_m) / N_b.
    Groups (d > 1, a = group norms): tau becomes tl = d tau in the first two terms and
    td = (2d - 1) tau in the last, so the vertex is td R_m / (2 (n - m)) (sure_threshold)."""
    a = np.sort(np.asarray(a, dtype=np.float64).ravel())
    n = a.size
    tl, td = d * tau, (2 * d - 1) * tau
    th_d, al_d, m_d, v_d = sure_threshold(a, tau, d)
    if a[-1] == 0.0:
        return th_d, al_d, m_d, v_d
    best = (v_d, th_d, m_d)
    A = np.concatenate([[0.0], np.cumsum(a ** 2)])          # A[m] = sum of the m smallest
    inv = np.where(a > 0, 1.0 / np.where(a > 0, a, 1.0), 0.0)
    Rs = np.concatenate([np.cumsum(inv[::-1])[::-1], [0.0]])  # Rs[m] = sum over indices >= m
    for m in range(n):
        if m > 0 and not a[m - 1] < a[m]:
            continue                                          # m must end a run
        lo = a[m - 1] if m > 0 else 0.0
        hi = a[m]
        if hi == 0.0:
            continue
        R = Rs[m]
        t = td * R / (2.0 * (n - m))
        if lo < t < hi:
            v = A[m] - m * tl + (n - m) * (t * t + tl) - td * t * R
            if v < best[0] or (v == best[0] and t < best[1]):
                best = (v, t, m)
    v, t, m = best
    R = Rs[m]
    return float(t), float((d * (n - m) - 0.5 * (2 * d - 1) * t * R) / (d * n)), int(m), float(v)


def sure_threshold_brute(a, tau, d=1):
    """O(N_b^2) reference for sure_threshold: evaluate sure_value at every candidate."""
    a = np.asarray(a, dtype=np.float64).ravel()
    cands = np.unique(a[a > 0])
    if cands.size == 0:
        return 0.0, float(a.size * (0.0 - d * tau))
    vals = np.array([sure_value(a, t, tau, d) for t in cands])
    i = int(np.argmin(vals))
    return float(cands[i]), float(vals[i])


def wirtinger_mean_soft(r, theta, d=1):
    """alpha for one band straight from its definition: the mean over the band of
    1 - theta/(2|r_i|) for |r_i| > theta, 0 otherwise.  With groups of d coefficients
    (d > 1, r a band block): half the real divergence of group soft thresholding per
    complex coefficient; the Jacobian of g (1 - theta/||g||) on R^D (D = 2d) has trace
    D - (D - 1) theta/||g|| above the threshold and 0 below."""
    if d == 1:
        a = np.abs(r)
        keep = a > theta
        return float(np.sum(1.0 - theta / (2.0 * a[keep])) / a.size)
    a, _ = group_norms(r, d)
    keep = a > theta
    D = 2 * d
    return float(np.sum(D - (D - 1) * theta / a[keep]) / (2.0 * r.size))


def group_norms(rb, d):
    """Norms of the groups of d horizontally adjacent coefficients (x = d j .. d j + d - 1)
    of a band block rb, and the groups themselves ([rows][nx/d][d])."""
    h, w = rb.shape
    g = np.asarray(rb).reshape(h, w // d, d)
    return np.sqrt(np.sum(np.abs(g) ** 2, axis=2)), g


def soft_group(rb, theta, d):
    """Group soft thresholding of a band block: each group g -> g max(0, 1 - theta/||g||);
    d = 1 is soft()."""
    if d == 1:
        return soft(rb, theta)
    a, g = group_norms(rb, d)
    out = np.zeros_like(g)
    keep = a > theta
    out[keep] = g[keep] * (1.0 - theta / a[keep])[:, None]
    return out.reshape(rb.shape)


# ----------------------------------------------------------------------------------
# Algorithm 1

def tau_estimate(z, mask, p, sigma2, S):
    """The tau estimate: tau_b = sum_{j in Omega} S_b(j) p_j^-1 [(p_j^-1 - 1)|z_j|^2 + sigma^2]."""
    w = np.zeros(z.shape)
    om = mask.astype(bool)
    w[om] = 1.0 / p[om]
    c = w * ((w - 1.0) * np.abs(z) ** 2 + sigma2)
    return np.array([np.sum(Sb * c) for Sb in S])


def vdamp_step(rt, y, mask, p, sigma2, s, S, wavelet=None):
    """The k-space step for one iteration: from r_tilde_k to (r_k, tau_k)."""
    om = mask.astype(bool)
    x_t = synthesis(rt, s, wavelet)
    z = np.where(om, y - fft2u(x_t), 0.0)                  # residual step (zero off Omega)
    v = np.zeros_like(z)
    v[om] = z[om] / p[om]                                  # P^-1 z, zero-filled
    r = rt + analysis(ifft2u(v), s, wavelet)              # back-projection
    tau = tau_estimate(z, mask, p, sigma2, S)              # tau estimate
    return r, tau


def denoise(r, tau, s, theta_override=None, alpha_override=None, continuous=False, group=1):
    """The denoising, alpha and Onsager-correction steps: per band SURE threshold, eta,
    alpha, and the corrected r_tilde_{k+1}.
    theta_override (optional, per band) replaces the SURE search; alpha then follows
    from its definition at that threshold unless alpha_override gives it too (a test
    that replays another implementation's decisions supplies both).  continuous=True
    minimises SURE over every theta > 0 (sure_threshold_continuous); group = 2
    thresholds horizontal pairs jointly (structured sparsity, module docstring)."""
    ny, nx = r.shape
    w_hat = np.zeros_like(r)
    rt_next = np.zeros_like(r)
    thetas, alphas = [], []
    for b, (rs, cs, _, _) in enumerate(bands(ny, nx, s)):
        rb = r[rs, cs]
        if theta_override is None:
            search = sure_threshold_continuous if continuous else sure_threshold
            if group == 1:
                th, al, _, _ = search(np.abs(rb), tau[b])
            else:
                th, al, _, _ = search(group_norms(rb, group)[0], tau[b], group)
        else:
            th = float(theta_override[b])
            al = (wirtinger_mean_soft(rb, th, group) if alpha_override is None
                  else float(alpha_override[b]))
        wb = soft_group(rb, th, group)
        w_hat[rs, cs] = wb
        rt_next[rs, cs] = (wb - al * rb) / (1.0 - al)      # Onsager correction
        thetas.append(th)
        alphas.append(al)
    return w_hat, rt_next, np.array(thetas), np.array(alphas)


def output_step(w_hat, y, mask, s, wavelet=None):
    """The output step: x_hat = Psi^H w + Phi^H (y - Phi Psi^H w)."""
    x = synthesis(w_hat, s, wavelet)
    om = mask.astype(bool)
    resid = np.where(om, y - fft2u(x), 0.0)
    return x + ifft2u(resid)


def vdamp(y, mask, p, sigma2, s, iters, record=False, continuous=False, wavelet=None, group=1):
    """Algorithm 1 in FP64.  y: zero-filled measurements (natural order), mask: 0/1,
    p: sampling probabilities (used on Omega), sigma2: E|eps_j|^2, s: wavelet levels.
    continuous=True takes each threshold as SURE's minimiser over every theta > 0;
    wavelet: None for Haar, else an orthonormal lowpass filter (dwt2); group = 2 for
    joint thresholding of horizontal pairs (structured sparsity).
    Returns dict with x_hat and, per iteration, tau, theta, alpha (and r if record)."""
    y = np.asarray(y, dtype=np.complex128)
    p = np.asarray(p, dtype=np.float64)
    ny, nx = y.shape
    check_shape(ny, nx, s)
    S = tau_weights(ny, nx, s, wavelet)
    rt = np.zeros((ny, nx), dtype=np.complex128)           # initialisation: r_tilde_0 = 0
    w_hat = np.zeros_like(rt)
    taus, thetas, alphas, rs = [], [], [], []
    for _ in range(iters):
        r, tau = vdamp_step(rt, y, mask, p, sigma2, s, S, wavelet)
        w_hat, rt, th, al = denoise(r, tau, s, continuous=continuous, group=group)
        taus.append(tau)
        thetas.append(th)
        alphas.append(al)
        if record:
            rs.append(r)
    x_hat = output_step(w_hat, y, mask, s, wavelet)
    out = dict(x_hat=x_hat, tau=np.array(taus), theta=np.array(thetas),
               alpha=np.array(alphas))
    if record:
        out["r"] = rs
    return out


def vdamp_resume(y, mask, p, sigma2, s, r, theta, alpha, iters, record=False, continuous=False,
                 wavelet=None, group=1):
    """Algorithm 1 continued from the state (r_k, theta_k, alpha_k) of an earlier
    iteration: every further iteration starts with the denoising, alpha and
    Onsager-correction steps applied to the previous state (eta with the given thresholds,
    the Onsager correction with the given alpha), then the k-space, denoising and alpha
    steps.  With iters = 0 the output is the output step with w = eta(r_k; theta_k).
    Returns the same
    dict as vdamp(); the per-iteration entries count the iterations of this call."""
    y = np.asarray(y, dtype=np.complex128)
    p = np.asarray(p, dtype=np.float64)
    r = np.asarray(r, dtype=np.complex128)
    ny, nx = y.shape
    check_shape(ny, nx, s)
    S = tau_weights(ny, nx, s, wavelet)
    w_hat, rt, _, _ = denoise(r, None, s, theta_override=theta, alpha_override=alpha, group=group)
    taus, thetas, alphas, rs = [], [], [], []
    for _ in range(iters):
        r, tau = vdamp_step(rt, y, mask, p, sigma2, s, S, wavelet)
        w_hat, rt, th, al = denoise(r, tau, s, continuous=continuous, group=group)
        taus.append(tau)
        thetas.append(th)
        alphas.append(al)
        if record:
            rs.append(r)
    out = dict(x_hat=output_step(w_hat, y, mask, s, wavelet), tau=np.array(taus), theta=np.array(thetas),
               alpha=np.array(alphas))
    if record:
        out["r"] = rs
    return out


# ----------------------------------------------------------------------------------
# FISTA comparator (Section 1, eq. 2 with f = lambda ||Psi x||_1; Section 3 setup):
# synthesis form over w = Psi x (equal to the analysis form since Psi is orthogonal),
# step 1 because ||M F Psi^H|| <= 1, zero initialisation, every band thresholded.

def fista(y, mask, lam, s, iters):
    y = np.asarray(y, dtype=np.complex128)
    om = mask.astype(bool)
    ny, nx = y.shape
    check_shape(ny, nx, s)
    v = np.zeros((ny, nx), dtype=np.complex128)
    w_prev = np.zeros_like(v)
    t = 1.0
    objective = []
    for _ in range(iters):
        resid = np.where(om, y - fft2u(haar_synthesis(v, s)), 0.0)
        w = soft(v + haar_analysis(ifft2u(resid), s), lam)
        t_next = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        v = w + ((t - 1.0) / t_next) * (w - w_prev)
        w_prev, t = w, t_next
        objective.append(fista_objective(w, y, mask, lam, s))
    return dict(x_hat=haar_synthesis(w_prev, s), w=w_prev, objective=np.array(objective))


def fista_objective(w, y, mask, lam, s):
    om = mask.astype(bool)
    resid = np.where(om, y - fft2u(haar_synthesis(w, s)), 0.0)
    return float(0.5 * np.sum(np.abs(resid) ** 2) + lam * np.sum(np.abs(w)))


def nmse_db(x_hat, x0):
    return float(10.0 * np.log10(np.sum(np.abs(x_hat - x0) ** 2) / np.sum(np.abs(x0) ** 2)))

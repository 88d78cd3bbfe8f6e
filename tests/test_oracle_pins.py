"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics, not by
the oracle itself: brute-force DFT and Haar bases built from their textbook
definitions, closed forms, invariants, special cases and brute force on tiny inputs.
All CPU-only."""
import numpy as np
import pytest

from oracle import vdamp_ref as o
from paper_1911_01234_amd import synth

RNG = np.random.default_rng(12345)


def crandn(*shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def dft_matrix(n):
    """Unitary DFT matrix from its definition F[k, t] = n^-1/2 exp(-2 pi i k t / n)."""
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


# ---------------------------------------------------------------------- F (Section 1)

@pytest.mark.parametrize("n", [8, 12, 20, 24, 40, 64])
def test_fft_matches_bruteforce_dft(n):
    x = crandn(n, n + 4 if n < 64 else n)
    ny, nx = x.shape
    ref = dft_matrix(ny) @ x @ dft_matrix(nx).T
    assert np.abs(o.fft2u(x) - ref).max() <= 1e-13 * np.abs(ref).max() * 10
    assert np.allclose(o.ifft2u(o.fft2u(x)), x, atol=1e-13)
    assert np.isclose(np.linalg.norm(o.fft2u(x)), np.linalg.norm(x), rtol=1e-13)  # Parseval


# ---------------------------------------------------------------------- Psi (eq. 6)

def haar_1d_basis(n, l):
    """Level-l scaling functions phi_{l,k} and wavelets psi_{l,k} of length n from the
    textbook definition: phi = 2^-l/2 on [k 2^l, (k+1) 2^l); psi = +2^-l/2 on the first
    half of that support and -2^-l/2 on the second half."""
    L = 2 ** l
    phi = np.zeros((n // L, n))
    psi = np.zeros((n // L, n))
    for k in range(n // L):
        phi[k, k * L:(k + 1) * L] = 2.0 ** (-l / 2)
        psi[k, k * L:k * L + L // 2] = 2.0 ** (-l / 2)
        psi[k, k * L + L // 2:(k + 1) * L] = -(2.0 ** (-l / 2))
    return phi, psi


@pytest.mark.parametrize("shape,s", [((16, 16), 2), ((32, 16), 3), ((24, 40), 3)])
def test_haar_coefficients_are_inner_products_with_textbook_basis(shape, s):
    """Every Mallat-layout coefficient equals <x, basis function> for the separable
    Haar basis: LH = low along y / high along x (top right), HL = high along y / low
    along x (bottom left), HH bottom right, LL_s top left."""
    ny, nx = shape
    x = crandn(ny, nx)
    w = o.haar_analysis(x, s)
    for (rs, cs, l, kind) in o.bands(ny, nx, s):
        phy, psy = haar_1d_basis(ny, l)
        phx, psx = haar_1d_basis(nx, l)
        By = phy if kind in ("LL", "LH") else psy
        Bx = phx if kind in ("LL", "HL") else psx
        ref = By @ x @ Bx.T
        assert np.abs(w[rs, cs] - ref).max() < 1e-12, kind


def test_haar_orthonormal_and_perfect_reconstruction():
    for ny, nx, s in [(8, 8, 3), (16, 16, 2), (16, 8, 3)]:
        N = ny * nx
        B = np.zeros((N, N), dtype=complex)
        for i in range(N):
            e = np.zeros(N, dtype=complex)
            e[i] = 1.0
            B[:, i] = o.haar_analysis(e.reshape(ny, nx), s).ravel()
        assert np.abs(B @ B.conj().T - np.eye(N)).max() < 1e-13
        x = crandn(ny, nx)
        assert np.abs(o.haar_synthesis(o.haar_analysis(x, s), s) - x).max() < 1e-13


def test_haar_constant_image_lands_in_ll_only():
    c = 0.7 - 0.2j
    s = 3
    w = o.haar_analysis(np.full((32, 48), c), s)
    ll = w[:32 >> s, :48 >> s]
    assert np.allclose(ll, c * 2 ** s)
    w[:32 >> s, :48 >> s] = 0
    assert np.abs(w).max() < 1e-13


def test_band_sizes_and_partition():
    ny, nx, s = 64, 96, 4
    seen = np.zeros((ny, nx), int)
    for (rs, cs, l, kind) in o.bands(ny, nx, s):
        seen[rs, cs] += 1
        assert seen[rs, cs].size == (ny * nx) // 4 ** l
    assert (seen == 1).all()
    assert len(o.bands(ny, nx, s)) == 1 + 3 * s


# ---------------------------------------------------------------------- S, the initialisation

@pytest.mark.parametrize("ny,nx,s", [(32, 32, 3), (48, 80, 4), (24, 40, 3)])
def test_tau_weights_closed_form_vs_bruteforce(ny, nx, s):
    """S_b(k) = |(F Psi^H e_i)(k)|^2 for a coefficient i of band b, with F the brute
    DFT matrix; and the same for a second coefficient of the band (shift invariance)."""
    S = o.tau_weights(ny, nx, s)
    Fy, Fx = dft_matrix(ny), dft_matrix(nx)
    for b, (rs, cs, _, _) in enumerate(o.bands(ny, nx, s)):
        for (di, dj) in [(0, 0), (rs.stop - rs.start - 1, cs.stop - cs.start - 1)]:
            e = np.zeros((ny, nx), dtype=complex)
            e[rs.start + di, cs.start + dj] = 1.0
            brute = np.abs(Fy @ o.haar_synthesis(e, s) @ Fx.T) ** 2
            assert np.abs(brute - S[b]).max() < 1e-12


@pytest.mark.parametrize("ny,nx,s", [(64, 64, 3), (192, 320, 4), (40, 24, 3)])
def test_tau_weights_invariants(ny, nx, s):
    S = o.tau_weights(ny, nx, s)
    Nb = [(rs.stop - rs.start) * (cs.stop - cs.start) for (rs, cs, _, _) in o.bands(ny, nx, s)]
    for Sb in S:
        assert abs(Sb.sum() - 1.0) < 1e-12           # unit-norm basis functions, unitary F
        assert (Sb >= 0).all()
    tot = sum(n * Sb for n, Sb in zip(Nb, S))        # completeness of an orthonormal basis
    assert np.abs(tot - 1.0).max() < 1e-12


# ---------------------------------------------------------------------- eta and SURE

def test_soft_threshold_closed_form_and_phase_equivariance():
    r = np.array([0.0, 0.5, 1.0, 2.0 + 0j, 3j, -4.0, 1 + 1j])
    th = 1.0
    ref = np.array([0.0, 0.0, 0.0, 1.0, 2j, -3.0, (1 + 1j) * (1 - 1 / np.sqrt(2))])
    assert np.allclose(o.soft(r, th), ref, atol=1e-15)
    z = crandn(1000)
    for phi in (0.3, 2.0, -1.1):
        assert np.allclose(o.soft(np.exp(1j * phi) * z, 0.8), np.exp(1j * phi) * o.soft(z, 0.8))


def test_sure_scan_matches_bruteforce():
    rng = np.random.default_rng(7)
    for trial in range(20):
        n = int(rng.integers(1, 300))
        w = np.where(rng.random(n) < 0.2, 5 * crandn(n, rng=rng), 0)
        r = w + crandn(n, rng=rng) * np.sqrt(0.5)
        a = np.abs(r)
        if trial % 4 == 0:                      # force ties and exact zeros
            a = np.round(a, 1)
        tau = 1.0
        th, al, m, sv = o.sure_threshold(a, tau)
        thb, svb = o.sure_threshold_brute(a, tau)
        if a.max() == 0:
            continue
        assert th == thb
        assert abs(sv - svb) <= 1e-12 * (abs(svb) + n * tau)
        assert m == int(np.sum(a <= th))
        assert abs(al - o.wirtinger_mean_soft(a.astype(complex), th)) < 1e-12


def test_sure_golden_hand_example():
    """Hand-computed (tests/golden/sure_hand_example.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "sure_hand_example.txt")
    vals = {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = np.array([float(t) for t in v.split()])
    a, tau = vals["a"], float(vals["tau"][0])
    for th, sref in zip(vals["theta_candidates"], vals["sure_at_candidates"]):
        assert abs(o.sure_value(a, th, tau) - sref) < 1e-12
    th, al, m, sv = o.sure_threshold(a, tau)
    assert th == float(vals["theta_star"][0])
    assert abs(al - float(vals["alpha_star"][0])) < 1e-12
    assert m == int(vals["m_star"][0])


def test_sure_all_zero_band():
    th, al, m, _ = o.sure_threshold(np.zeros(16), 0.3)
    assert th == 0.0 and al == 0.0 and m == 16


def test_sure_is_unbiased_mse_estimate():
    """E[SURE(theta)] = E||eta(r;theta) - w||^2 for r = w + CN(0, tau), at fixed theta."""
    rng = np.random.default_rng(3)
    n, tau, trials = 512, 0.8, 2000
    w = np.where(rng.random(n) < 0.15, 3 * crandn(n, rng=rng), 0)
    for theta in (0.4, 1.0, 1.8):
        d_sure, d_mse = [], []
        for _ in range(trials):
            r = w + crandn(n, rng=rng) * np.sqrt(tau / 2)
            d_sure.append(o.sure_value(np.abs(r), theta, tau))
            d_mse.append(np.sum(np.abs(o.soft(r, theta) - w) ** 2))
        diff = np.array(d_sure) - np.array(d_mse)
        assert abs(diff.mean()) < 4 * diff.std() / np.sqrt(trials)


def test_alpha_is_mean_wirtinger_derivative_finite_difference():
    """g'(r) = 1/2 (du/dx + dv/dy) for g = u + i v, r = x + i y, by central differences."""
    rng = np.random.default_rng(5)
    r = 2 * crandn(200, rng=rng)
    th = 1.1
    h = 1e-6
    dudx = (o.soft(r + h, th).real - o.soft(r - h, th).real) / (2 * h)
    dvdy = (o.soft(r + 1j * h, th).imag - o.soft(r - 1j * h, th).imag) / (2 * h)
    fd = np.mean(0.5 * (dudx + dvdy))
    assert abs(fd - o.wirtinger_mean_soft(r, th)) < 1e-8
    # identity map (theta = 0) has derivative 1
    assert abs(o.wirtinger_mean_soft(r, 0.0) - 1.0) < 1e-15


# ---------------------------------------------------------------------- the k-space and output steps

def tiny_problem(ny=32, nx=32, R=3.0, seed=0, full=False):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[:ny, :nx]
    x0 = ((((yy - ny / 2) / (0.35 * ny)) ** 2 + ((xx - nx / 2) / (0.3 * nx)) ** 2) < 1) * (1.0 + 0.3j)
    x0 = x0 + 0.5 * ((np.abs(yy - 10) < 4) & (np.abs(xx - 12) < 5))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    rad = np.sqrt(ky ** 2 + kx ** 2) / np.sqrt(0.5)
    p = np.clip((1 - rad) ** 3 + 0.15, 0.05, 1.0) if not full else np.ones((ny, nx))
    return x0, p, rng


def test_tau_full_sampling_is_sigma2():
    ny = nx = 32
    S = o.tau_weights(ny, nx, 3)
    sigma2 = 0.37
    z = crandn(ny, nx)
    tau = o.tau_estimate(z, np.ones((ny, nx)), np.ones((ny, nx)), sigma2, S)
    assert np.allclose(tau, sigma2, rtol=1e-13)


@pytest.mark.slow
def test_tau_unbiased_monte_carlo():
    """The tau estimate is an unbiased estimate of E|r_k - w0|^2 per band, for r_tilde fixed
    (independent of Omega and eps): Section 2."""
    ny = nx = 32
    s = 3
    x0, p, rng = tiny_problem(ny, nx)
    w0 = o.haar_analysis(x0, s)
    S = o.tau_weights(ny, nx, s)
    rt = w0 + 0.2 * crandn(ny, nx, rng=rng)          # fixed r_tilde, with its own error
    sigma2 = 0.01
    draws = 2000
    taus, errs = [], []
    Fx0 = o.fft2u(x0)
    for _ in range(draws):
        mask = (rng.random((ny, nx)) < p).astype(np.uint8)
        eps = crandn(ny, nx, rng=rng) * np.sqrt(sigma2 / 2)
        y = mask * (Fx0 + eps)
        r, tau = o.vdamp_step(rt, y, mask, p, sigma2, s, S)
        taus.append(tau)
        errs.append([np.mean(np.abs(r[rs, cs] - w0[rs, cs]) ** 2) for (rs, cs, _, _) in o.bands(ny, nx, s)])
    taus, errs = np.array(taus), np.array(errs)
    d = taus - errs
    z = d.mean(0) / (d.std(0) / np.sqrt(draws))
    assert np.all(np.abs(z) < 4), z


@pytest.mark.slow
def test_r0_unbiased_monte_carlo():
    """k = 0: r_0 = Psi Phi^H P^-1 y has E r_0 = w0 (Section 2, density compensation)."""
    ny = nx = 16
    s = 2
    x0, p, rng = tiny_problem(ny, nx)
    w0 = o.haar_analysis(x0, s)
    S = o.tau_weights(ny, nx, s)
    Fx0 = o.fft2u(x0)
    acc = np.zeros((ny, nx), complex)
    acc2 = np.zeros((ny, nx))
    draws = 3000
    for _ in range(draws):
        mask = (rng.random((ny, nx)) < p).astype(np.uint8)
        r, _ = o.vdamp_step(np.zeros((ny, nx), complex), mask * Fx0, mask, p, 0.0, s, S)
        acc += r
        acc2 += np.abs(r - w0) ** 2
    mean = acc / draws
    se = np.sqrt(acc2 / draws / draws)
    assert np.all(np.abs(mean - w0) < 5 * se + 1e-12)


def test_output_step_is_exactly_consistent():
    """The output step: M F x_hat = y on Omega for any w."""
    ny = nx = 32
    x0, p, rng = tiny_problem(ny, nx)
    mask = (rng.random((ny, nx)) < p).astype(np.uint8)
    y = mask * (o.fft2u(x0) + 0.05 * crandn(ny, nx, rng=rng))
    w = crandn(ny, nx, rng=rng)
    xh = o.output_step(w, y, mask, 3)
    assert np.abs(mask * o.fft2u(xh) - y).max() < 1e-12


def test_full_sampling_special_cases():
    """p = 1 everywhere: r_0 = Psi F^H y, tau = sigma^2 in every band, and the output
    of any number of iterations is F^H y (exact consistency with all of k-space)."""
    ny = nx = 32
    s = 3
    x0, p, rng = tiny_problem(ny, nx, full=True)
    mask = np.ones((ny, nx), np.uint8)
    sigma2 = 0.02
    y = o.fft2u(x0) + crandn(ny, nx, rng=rng) * np.sqrt(sigma2 / 2)
    S = o.tau_weights(ny, nx, s)
    r0, tau0 = o.vdamp_step(np.zeros((ny, nx), complex), y, mask, p, sigma2, s, S)
    assert np.abs(r0 - o.haar_analysis(o.ifft2u(y), s)).max() < 1e-13
    assert np.allclose(tau0, sigma2, rtol=1e-12)
    out = o.vdamp(y, mask, p, sigma2, s, 5)
    assert np.abs(out["x_hat"] - o.ifft2u(y)).max() < 1e-12


def test_zero_iterations_is_zero_filled():
    ny = nx = 32
    x0, p, rng = tiny_problem(ny, nx)
    mask = (rng.random((ny, nx)) < p).astype(np.uint8)
    y = mask * o.fft2u(x0)
    out = o.vdamp(y, mask, p, 0.0, 3, 0)
    assert np.abs(out["x_hat"] - o.ifft2u(y)).max() < 1e-13


def test_onsager_correction_needs_no_guard():
    """alpha in [0, 1 - 1/N_b] for every band and iteration."""
    ny = nx = 32
    x0, p, rng = tiny_problem(ny, nx)
    mask = (rng.random((ny, nx)) < p).astype(np.uint8)
    y = mask * (o.fft2u(x0) + 0.01 * crandn(ny, nx, rng=rng))
    out = o.vdamp(y, mask, p, 1e-4, 3, 10)
    Nb = np.array([(rs.stop - rs.start) * (cs.stop - cs.start) for (rs, cs, _, _) in o.bands(ny, nx, 3)])
    assert (out["alpha"] >= 0).all()
    assert (out["alpha"] <= 1 - 1 / Nb + 1e-15).all()


@pytest.mark.slow
def test_onsager_correction_decorrelates():
    """With the Wirtinger alpha, r_tilde_{k+1} - w0 is uncorrelated with the input noise
    n = r - w0: E Re<r_tilde - w0, n> = 0 for r = w0 + CN(0, tau) (Onsager correction).  The
    real-derivative reading 1[|r| > theta] fails this check."""
    rng = np.random.default_rng(11)
    n, tau, trials = 4096, 1.0, 300
    w0 = np.where(rng.random(n) < 0.1, 4 * crandn(n, rng=rng), 0)
    th = 1.2
    good, bad = [], []
    for _ in range(trials):
        nz = crandn(n, rng=rng) * np.sqrt(tau / 2)
        r = w0 + nz
        wh = o.soft(r, th)
        al = o.wirtinger_mean_soft(r, th)
        good.append(np.real(np.vdot(nz, (wh - al * r) / (1 - al) - w0)) / n)
        al_bad = np.mean(np.abs(r) > th)
        bad.append(np.real(np.vdot(nz, (wh - al_bad * r) / (1 - al_bad) - w0)) / n)
    good, bad = np.array(good), np.array(bad)
    assert abs(good.mean()) < 4 * good.std() / np.sqrt(trials)
    assert abs(bad.mean()) > 10 * bad.std() / np.sqrt(trials)


# ---------------------------------------------------------------------- FISTA (eq. 2)

def test_fista_full_sampling_one_step_is_exact_prox():
    """With M = I the minimiser of 1/2||y - F Psi^H w||^2 + lam ||w||_1 is
    eta(Psi F^H y; lam), reached after one step from zero and kept afterwards."""
    ny = nx = 32
    s = 3
    x0, p, rng = tiny_problem(ny, nx, full=True)
    y = o.fft2u(x0) + 0.05 * crandn(ny, nx, rng=rng)
    lam = 0.08
    ref = o.soft(o.haar_analysis(o.ifft2u(y), s), lam)
    for K in (1, 7):
        out = o.fista(y, np.ones((ny, nx), np.uint8), lam, s, K)
        assert np.abs(out["w"] - ref).max() < 1e-12


def test_fista_reaches_fixed_point_and_lowers_objective():
    ny = nx = 32
    s = 3
    x0, p, rng = tiny_problem(ny, nx)
    mask = (rng.random((ny, nx)) < p).astype(np.uint8)
    y = mask * (o.fft2u(x0) + 0.01 * crandn(ny, nx, rng=rng))
    lam = 0.01
    out = o.fista(y, mask, lam, s, 3000)
    w = out["w"]
    resid = mask * (y - o.fft2u(o.haar_synthesis(w, s)))
    w_next = o.soft(w + o.haar_analysis(o.ifft2u(resid), s), lam)
    assert np.abs(w_next - w).max() < 1e-9
    obj = out["objective"]
    assert obj[-1] < obj[0]
    # the minimiser is optimal: random perturbations do not lower the objective
    f0 = o.fista_objective(w, y, mask, lam, s)
    for _ in range(5):
        dw = 1e-4 * crandn(ny, nx, rng=rng)
        assert o.fista_objective(w + dw, y, mask, lam, s) >= f0 - 1e-12


def test_resume_continues_the_iteration_exactly():
    """The state between iterations of Algorithm 1 is (r_k, theta_k, alpha_k): the
    denoising, alpha and Onsager-correction steps rebuild r_tilde_{k+1} from it and the
    k-space step needs nothing else.  Resuming the oracle from a recorded state therefore reproduces the rest of the uninterrupted run bit for
    bit, and a resume with no further iteration returns the output step at that state."""
    sl = synth.workload_single64()[0][0]
    K, k = 9, 4
    full = o.vdamp(sl.y, sl.mask, sl.p, sl.sigma2, 3, K, record=True)
    rest = o.vdamp_resume(sl.y, sl.mask, sl.p, sl.sigma2, 3, full["r"][k], full["theta"][k],
                          full["alpha"][k], K - k - 1, record=True)
    assert np.array_equal(rest["x_hat"], full["x_hat"])
    for j in range(K - k - 1):
        assert np.array_equal(rest["r"][j], full["r"][k + 1 + j])
        assert np.array_equal(rest["theta"][j], full["theta"][k + 1 + j])
        assert np.array_equal(rest["alpha"][j], full["alpha"][k + 1 + j])
    last = o.vdamp_resume(sl.y, sl.mask, sl.p, sl.sigma2, 3, full["r"][-1], full["theta"][-1],
                          full["alpha"][-1], 0)
    assert np.array_equal(last["x_hat"], full["x_hat"])


# ------------------------------------------------------- continuous-theta SURE variant

def test_continuous_sure_hand_example():
    """a = (2, 3), tau = 1, worked by hand: below a_(1) = 2 no magnitude is at or below
    theta, R = 1/2 + 1/3 = 5/6, and SURE = 2 (theta^2 + 1) - (5/6) theta has its minimum
    at theta* = (5/6) / 4 = 5/24 inside (0, 2), value 2 (25/576 + 1) - 25/144 = 551/288;
    the candidates give SURE(2) = 3 + 5 - 2/3 = 22/3 and SURE(3) = 3 + 8 = 11.  So theta =
    5/24 and alpha = (2 - (5/24)(5/6)/2) / 2 = 551/576."""
    th, al, m, v = o.sure_threshold_continuous(np.array([2.0, 3.0]), 1.0)
    assert abs(th - 5 / 24) < 1e-15 and m == 0
    assert abs(v - 551 / 288) < 1e-14
    assert abs(al - 551 / 576) < 1e-15
    thd, _, md, vd = o.sure_threshold(np.array([2.0, 3.0]), 1.0)
    assert thd == 2.0 and md == 1 and abs(vd - 22 / 3) < 1e-14


@pytest.mark.parametrize("seed", range(6))
def test_continuous_sure_matches_dense_grid(seed):
    """The continuous minimiser against SURE evaluated from its definition (sure_value) on
    a dense grid of thresholds plus every magnitude: no grid point is lower, the grid
    comes within its resolution, the returned value is the definition's at the returned
    theta, it is at most the candidate search's, and alpha is the Wirtinger mean there."""
    rng = np.random.default_rng(seed)
    n = 60
    r = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * np.where(rng.random(n) < 0.2, 4.0, 1.0)
    if seed == 0:
        r[:5] = 0.0                       # zero magnitudes below every threshold
    a = np.abs(r)
    tau = float(rng.uniform(0.5, 2.0))
    th, al, m, v = o.sure_threshold_continuous(a, tau)
    grid = np.concatenate([np.linspace(1e-9, a.max() * 1.01, 60001), a[a > 0]])
    dense = np.array([o.sure_value(a, t, tau) for t in grid])
    assert dense.min() >= v - 1e-9 * (abs(v) + n * tau)
    assert dense.min() <= v + 1e-5 * (abs(v) + n * tau)
    assert abs(o.sure_value(a, th, tau) - v) < 1e-10 * (abs(v) + n * tau)
    assert v <= o.sure_threshold(a, tau)[3] + 1e-12
    assert m == int(np.sum(a <= th))
    assert abs(al - o.wirtinger_mean_soft(r, th)) < 1e-12

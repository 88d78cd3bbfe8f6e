"""Pins of the oracle's structured-sparsity denoiser (group soft thresholding of
horizontal pairs, tuned by SURE; Section 4 names structured sparsity as a richer model
for SURE to tune) against mathematics: a hand-worked example, the proximal property of
group soft thresholding, the sorted scan against brute force, Stein unbiasedness by
Monte Carlo, alpha against a finite-difference divergence, the continuous minimiser
against a dense grid, the decorrelation of the Onsager correction, the colored state evolution of a
whole run, and exact resumption.  CPU only."""
import os

import numpy as np
import pytest
from scipy import optimize

from oracle import vdamp_ref as o
from paper_1911_01234_amd import synth

RNG = np.random.default_rng(29)


def crandn(*shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "group_sure_hand_example.txt")
    vals = {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = np.array([float(t) for t in v.split()])
    return vals


def test_group_sure_golden_hand_example():
    v = _golden()
    a, tau, d = v["a"], float(v["tau"][0]), int(v["d"][0])
    for th, sref in zip(v["theta_candidates"], v["sure_at_candidates"]):
        assert abs(o.sure_value(a, th, tau, d) - sref) < 1e-12
    th, al, m, sv = o.sure_threshold(a, tau, d)
    assert th == float(v["theta_star"][0]) and m == int(v["m_star"][0])
    assert abs(al - float(v["alpha_star"][0])) < 1e-12
    assert abs(o.sure_value(a, float(v["inner_vertex"][0]), tau, d) - float(v["sure_at_inner_vertex"][0])) < 1e-12
    thc, alc, mc, svc = o.sure_threshold_continuous(a, tau, d)
    assert thc == th and mc == m and abs(svc - sv) < 1e-12 and abs(alc - al) < 1e-12
    # the same example through the band-level functions: groups with these norms
    rb = np.array([[1.0, 0.0, 0.0, 2.0j, 4.0 * np.cos(0.3), 4.0j * np.sin(0.3)]])
    assert np.allclose(o.group_norms(rb, 2)[0].ravel(), a, rtol=0, atol=1e-15)
    assert abs(o.wirtinger_mean_soft(rb, th, 2) - float(v["alpha_star"][0])) < 1e-12


def test_group_soft_is_the_prox_of_the_group_norm():
    """eta(y) = argmin_x 1/2 ||x - y||^2 + theta ||x|| over C^2 = R^4 (numerical
    minimisation, independent of the closed form)."""
    for _ in range(20):
        y = crandn(1, 2) * RNG.uniform(0.2, 2.0)
        th = float(RNG.uniform(0.1, 1.5))

        def f(v):
            x = v[:2] + 1j * v[2:]
            return 0.5 * np.sum(np.abs(x - y.ravel()) ** 2) + th * np.sqrt(np.sum(np.abs(x) ** 2) + 1e-30)
        yv = np.concatenate([y.real.ravel(), y.imag.ravel()])
        res = optimize.minimize(f, yv, method="Nelder-Mead",
                                options={"xatol": 1e-10, "fatol": 1e-15, "maxiter": 20000})
        x = res.x[:2] + 1j * res.x[2:]
        eta = o.soft_group(y, th, 2).ravel()
        assert np.allclose(eta, x, atol=1e-4), (y, th)
        # convex objective: no perturbation of eta does better
        ev = np.concatenate([eta.real, eta.imag])
        for scale in (1e-2, 1e-4):
            for _ in range(50):
                assert f(ev) <= f(ev + scale * RNG.standard_normal(4)) + 1e-15


def test_group_soft_with_one_nonzero_coefficient_is_scalar_soft():
    r = crandn(8, 16)
    r[:, 1::2] = 0.0
    th = 0.9
    assert np.allclose(o.soft_group(r, th, 2), o.soft(r, th), rtol=0, atol=1e-15)


@pytest.mark.parametrize("d", [2, 4])
def test_group_sure_scan_matches_brute_force(d):
    for trial in range(20):
        n = int(RNG.integers(1, 60))
        a = np.abs(RNG.standard_normal(n)) * 2
        if trial % 3 == 0:
            a[: n // 3] = a[0]          # ties
        if trial % 5 == 0:
            a[: n // 4] = 0.0           # zero groups
        tau = float(RNG.uniform(0.1, 2.0))
        th, al, m, sv = o.sure_threshold(a, tau, d)
        thb, svb = o.sure_threshold_brute(a, tau, d)
        if thb == 0.0:
            assert th == 0.0
            continue
        assert th == thb
        assert abs(sv - svb) <= 1e-12 * (abs(svb) + n * d * tau)
        assert m == int(np.sum(a <= th))


def test_group_sure_is_unbiased_for_the_mse():
    """E SURE(theta) = E ||eta(r) - w0||^2 for r = w0 + CN(0, tau) per coefficient, at
    fixed thresholds (Monte Carlo over 4000 draws of 256 pairs)."""
    rng = np.random.default_rng(5)
    G, tau, draws = 256, 0.7, 4000
    w0 = np.where(rng.random((1, 2 * G)) < 0.2, 2.0 * crandn(1, 2 * G, rng=rng), 0.0)
    for th in (0.5, 1.2, 2.0):
        diff = []
        for _ in range(draws):
            r = w0 + crandn(1, 2 * G, rng=rng) * np.sqrt(tau / 2)
            a = o.group_norms(r, 2)[0].ravel()
            diff.append(o.sure_value(a, th, tau, 2) - np.sum(np.abs(o.soft_group(r, th, 2) - w0) ** 2))
        diff = np.array(diff)
        z = diff.mean() / (diff.std() / np.sqrt(draws))
        assert abs(z) < 4, (th, z)


def test_group_alpha_is_half_the_divergence():
    """wirtinger_mean_soft(d = 2) against a central finite-difference trace of the
    Jacobian of soft_group over the 4 real coordinates of every pair."""
    r = crandn(4, 8)
    th = 1.1
    a = o.group_norms(r, 2)[0]
    assert np.all(np.abs(a - th) > 1e-3)
    h = 1e-6
    div = 0.0
    for idx in np.ndindex(r.shape):
        for unit in (1.0, 1j):
            rp, rm = r.copy(), r.copy()
            rp[idx] += h * unit
            rm[idx] -= h * unit
            dv = (o.soft_group(rp, th, 2)[idx] - o.soft_group(rm, th, 2)[idx]) / (2 * h)
            div += (dv / unit).real
    assert abs(o.wirtinger_mean_soft(r, th, 2) - div / (2 * r.size)) < 1e-7


def test_group_continuous_minimiser_against_dense_grid():
    for _ in range(10):
        a = np.abs(RNG.standard_normal(40)) * 1.5
        tau = float(RNG.uniform(0.2, 1.5))
        th, al, m, sv = o.sure_threshold_continuous(a, tau, 2)
        grid = np.linspace(1e-4, a.max() * 1.01, 20001)
        vals = np.array([o.sure_value(a, t, tau, 2) for t in grid])
        assert sv <= vals.min() + 1e-9
        assert abs(o.sure_value(a, th, tau, 2) - sv) < 1e-9 * (1 + abs(sv))
        assert sv <= o.sure_threshold(a, tau, 2)[3] + 1e-12


def test_group_onsager_correction_decorrelates():
    """With alpha = half the divergence per coefficient, r_tilde - w0 is uncorrelated
    with the noise n = r - w0 (Onsager correction), for group soft thresholding too."""
    rng = np.random.default_rng(12)
    n, tau, trials = 4096, 1.0, 300
    w0 = np.where(rng.random((1, n)) < 0.1, 4 * crandn(1, n, rng=rng), 0)
    th = 1.6
    good = []
    for _ in range(trials):
        nz = crandn(1, n, rng=rng) * np.sqrt(tau / 2)
        r = w0 + nz
        wh = o.soft_group(r, th, 2)
        al = o.wirtinger_mean_soft(r, th, 2)
        good.append(np.real(np.vdot(nz, (wh - al * r) / (1 - al) - w0)) / n)
    good = np.array(good)
    assert abs(good.mean()) < 4 * good.std() / np.sqrt(trials)


def test_group_vdamp_colored_state_evolution_and_resume():
    """A whole run with pair groups on the 256x256 recipe (R = 6): tau_k tracks the
    per-subband error of r_k in the bands of N_b >= 4096 coefficients within four
    standard deviations of the model's sampling spread, (10/ln 10)/sqrt(N_b) dB each; a
    run split in two equals the uninterrupted one; and it ends well below zero filling."""
    sl, s, _ = synth.workload_single256(6.0)
    sl = sl[0]
    K = 16
    out = o.vdamp(sl.y, sl.mask, sl.p, sl.sigma2, s, K, record=True, group=2)
    w0 = o.haar_analysis(sl.x0, s)
    bl = o.bands(256, 256, s)
    Nb = np.array([(rs.stop - rs.start) * (cs.stop - cs.start) for (rs, cs, _, _) in bl])
    for k, r in enumerate(out["r"]):
        err = np.array([np.sum(np.abs(r[rs, cs] - w0[rs, cs]) ** 2) for (rs, cs, _, _) in bl])
        dev = np.abs(10 * np.log10(Nb * out["tau"][k]) - 10 * np.log10(err))
        big = Nb >= 4096
        assert (dev[big] <= 4.0 * (10.0 / np.log(10.0)) / np.sqrt(Nb[big])).all(), (k, dev[big])
    k = 6
    rest = o.vdamp_resume(sl.y, sl.mask, sl.p, sl.sigma2, s, out["r"][k - 1], out["theta"][k - 1],
                          out["alpha"][k - 1], K - k, group=2)
    assert np.allclose(rest["x_hat"], out["x_hat"], rtol=0, atol=1e-12)
    n_grp = o.nmse_db(out["x_hat"], sl.x0)
    assert n_grp < o.nmse_db(o.ifft2u(sl.y), sl.x0) - 10.0

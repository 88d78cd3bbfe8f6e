"""Pins of the oracle of VDAMP with the learned denoiser (oracle/learned_ref.py): the
probe generator against SplitMix64's published outputs and the probe's moments, the
divergence estimator against closed forms (exact for linear maps, unbiased for soft
thresholding, Section 2.2's Wirtinger reading), the general SURE against its closed
expectation for a linear shrinkage and against the soft-threshold scan form, a
hand-built network whose map is known, and the reduction to plain VDAMP when the
network is the identity."""
import os

import numpy as np
import pytest

from oracle import cnn_ref as cr
from oracle import learned_ref as lr
from oracle import vdamp_ref as o
from paper_1911_01234_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")


def test_splitmix64_matches_published_outputs():
    want = [int(l) for l in open(GOLD) if l.strip() and not l.startswith("#")]
    got = [int(v) for v in lr.splitmix64_stream(1234567, len(want))]
    assert got == want


def test_probe_values_and_moments():
    q = lr.probe(7, 3, 2, 256, 256)
    assert np.allclose(np.abs(q.real), 1 / np.sqrt(2)) and np.allclose(np.abs(q.imag), 1 / np.sqrt(2))
    n = q.size
    assert abs(q.mean()) < 5 / np.sqrt(n)                 # E q = 0
    assert abs((q * q).mean()) < 5 / np.sqrt(n)           # E q^2 = 0 (pseudo-covariance)
    assert np.allclose(np.abs(q) ** 2, 1.0)               # E |q|^2 = 1
    # different iterations / slices / seeds give different probes
    assert np.mean(lr.probe(7, 4, 2, 256, 256) == q) < 0.3
    assert np.mean(lr.probe(7, 3, 3, 256, 256) == q) < 0.3
    assert np.mean(lr.probe(8, 3, 2, 256, 256) == q) < 0.3


def test_probe_counter_layout():
    # value at (it, slice, index) is the SplitMix64 stream of the seed at position c + 1
    seed, it, sl = 99, 5, 3
    q = lr.probe(seed, it, sl, 4, 8).ravel()
    c0 = (it << 48) | (sl << 32)
    z = lr.splitmix64_stream(seed, 32, start=c0)          # positions c0+1 .. c0+32
    h = 1 / np.sqrt(2)
    want = np.where(z & 1, -h, h) + 1j * np.where(z & 2, -h, h)
    assert np.array_equal(q, want)


def test_mc_alpha_exact_for_holomorphic_linear_maps():
    rng = np.random.default_rng(1)
    ny, nx, s = 16, 16, 2
    c = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    q = lr.probe(1, 0, 0, ny, nx)
    al = lr.mc_alpha(lambda v: c * v, q, o.bands(ny, nx, s))
    want = [float(np.mean(c[rs, cs].real)) for (rs, cs, _, _) in o.bands(ny, nx, s)]
    assert np.allclose(al, want, atol=1e-14)


def test_mc_alpha_ignores_antiholomorphic_part_on_average():
    # g(r) = B conj(r): dg/dr = 0, so the estimate has zero mean
    rng = np.random.default_rng(2)
    ny = nx = 64
    B = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    bl = [(slice(0, ny), slice(0, nx), 0, 0)]
    est = [lr.mc_alpha(lambda v: B * np.conj(v), lr.probe(k, 0, 0, ny, nx), bl)[0] for k in range(40)]
    sd = np.sqrt(np.mean(np.abs(B) ** 2) / (ny * nx))
    assert abs(np.mean(est)) < 5 * sd / np.sqrt(40)


def test_mc_alpha_unbiased_for_soft_thresholding():
    # probe estimate with the Jacobian of eta taken by central differences -> the mean
    # Wirtinger derivative 1 - theta/(2|r|) above threshold (Section 2.2 reading)
    rng = np.random.default_rng(3)
    ny = nx = 64
    r = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))) * 0.7
    th = 0.6
    eps = 1e-7
    bl = [(slice(0, ny), slice(0, nx), 0, 0)]

    def jac(v):
        return (o.soft(r + eps * v, th) - o.soft(r - eps * v, th)) / (2 * eps)

    est = np.array([lr.mc_alpha(jac, lr.probe(k, 1, 0, ny, nx), bl)[0] for k in range(64)])
    want = o.wirtinger_mean_soft(r, th)
    assert abs(est.mean() - want) < 5 * est.std(ddof=1) / np.sqrt(len(est)) + 1e-9


def test_sure_general_expectation_for_linear_shrinkage():
    # w = c r, r = w0 + n, n ~ CN(0, tau): E||w - w0||^2 = (1-c)^2 ||w0||^2 + c^2 N tau, and
    # SURE has the same expectation
    rng = np.random.default_rng(4)
    n, tau, c = 4096, 0.3, 0.6
    w0 = rng.standard_normal(n) * 0.8 + 1j * rng.standard_normal(n) * 0.5
    vals = []
    for _ in range(400):
        noise = np.sqrt(tau / 2) * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
        r = w0 + noise
        vals.append(lr.sure_general(r, c * r, c, tau))
    want = (1 - c) ** 2 * np.sum(np.abs(w0) ** 2) + c ** 2 * n * tau
    assert abs(np.mean(vals) - want) < 4 * np.std(vals) / np.sqrt(len(vals))


def test_sure_general_equals_soft_threshold_scan_form():
    rng = np.random.default_rng(5)
    r = rng.standard_normal(2000) + 1j * rng.standard_normal(2000)
    tau = 0.7
    for th in (0.3, 1.0, 2.5):
        al = o.wirtinger_mean_soft(r, th)
        got = lr.sure_general(r, o.soft(r, th), al, tau)
        assert abs(got - o.sure_value(np.abs(r), th, tau)) < 1e-9 * r.size


def shrink_params(nb, c, channels=48):
    """A network whose map is exactly f(x) = (1 - c) x: layer 1 splits (Re, Im) into
    their positive and negative parts, layers 2-5 pass them on, layer 6 recombines them
    scaled by c, so o = c u and f = s0 (u - o)."""
    p = {k: np.zeros_like(v) for k, v in cr.init_params(nb, 0, channels).items()}
    for ch, (src, sgn) in enumerate([(0, 1), (0, -1), (1, 1), (1, -1)]):
        p["W1"][ch, src, 1, 1] = sgn
        for l in range(2, 6):
            p[f"W{l}"][ch, ch, 1, 1] = 1.0
        p["W6"][src, ch, 1, 1] = sgn * c
    return p


def half_shrink_params(nb, c, channels=48):
    """A network whose map is f(x) = x - c (max(Re x, 0) + i max(Im x, 0)): layer 1 keeps
    the positive parts of (Re, Im), layers 2-5 pass them on, layer 6 scales them by c."""
    p = {k: np.zeros_like(v) for k, v in cr.init_params(nb, 0, channels).items()}
    for ch in range(2):
        p["W1"][ch, ch, 1, 1] = 1.0
        for l in range(2, 6):
            p[f"W{l}"][ch, ch, 1, 1] = 1.0
        p["W6"][ch, ch, 1, 1] = c
    return p


def test_hand_built_network_shrinks_positive_parts():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    p = half_shrink_params(7, 0.125)
    tau = np.full(7, 0.1)
    want = x - 0.125 * (np.maximum(x.real, 0) + 1j * np.maximum(x.imag, 0))
    assert np.allclose(cr.forward(p, x, tau, 0.9), want, atol=1e-14)
    v = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    jw = v - 0.125 * (v.real * (x.real > 0) + 1j * v.imag * (x.imag > 0))
    assert np.allclose(cr.jvp(p, x, tau, 0.9, v), jw, atol=1e-14)


def test_hand_built_network_is_a_linear_shrinkage():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    p = shrink_params(7, 0.25)
    tau = np.full(7, 0.1)
    assert np.allclose(cr.forward(p, x, tau, 1.7), 0.75 * x, atol=1e-14)
    r = o.haar_analysis(x, 2)
    w, al, sure = lr.cnn_candidate(p, r, tau, 2, 1.7, seed=3, it=0, slice_id=0, bf16=False)
    assert np.allclose(w, 0.75 * r, atol=1e-13)
    assert np.allclose(al, 0.75, atol=1e-13)
    for b, (rs, cs, _, _) in enumerate(o.bands(16, 16, 2)):
        nb = r[rs, cs].size
        assert abs(sure[b] - (0.0625 * np.sum(np.abs(r[rs, cs]) ** 2) + 0.5 * nb * 0.1)) < 1e-10


def test_identity_network_reduces_to_plain_vdamp():
    sl = synth.workload_single64()[0][0]
    s = 3
    p = {k: np.zeros_like(v) for k, v in cr.init_params(1 + 3 * s, 0).items()}
    got = lr.vdamp_learned(sl.y, sl.mask, sl.p, sl.sigma2, s, 4, p, seed=11)
    ref = o.vdamp(sl.y, sl.mask, sl.p, sl.sigma2, s, 4)
    assert all(rec["sel"].sum() == 0 for rec in got["records"])
    assert np.abs(got["x_hat"] - ref["x_hat"]).max() < 1e-12


def test_input_scale_hand_example():
    """s0^2 = (1/N) sum_j (m_j / p_j) |y_j|^2, worked by hand on a 2 x 2 case: the three
    sampled entries give (1/0.5) 2 + (1/0.25) 4 + (1/1) 9 = 29, the unsampled y = 5 is
    ignored, so s0 = sqrt(29/4); an all-zero y gives s0 = 1."""
    y = np.array([[1 + 1j, 5.0], [2.0, 3j]])
    mask = np.array([[1, 0], [1, 1]], dtype=np.uint8)
    p = np.array([[0.5, 0.3], [0.25, 1.0]])
    assert abs(lr.input_scale(y, mask, p) - np.sqrt(29.0 / 4.0)) < 1e-15
    assert lr.input_scale(np.zeros_like(y), mask, p) == 1.0


def test_input_scale_is_unbiased_for_energy_plus_noise():
    """E over (Omega, eps) of s0^2 = mean |x0|^2 + sigma^2 (E[m/p] = 1 and the unitary F
    keeps the energy), by Monte Carlo over fresh masks and noise for a fixed image."""
    rng = np.random.default_rng(21)
    n = 32
    x0 = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    p = synth.density(n, n, 3.0, 4.0, 4)
    X = o.fft2u(x0)
    sigma2 = 0.3
    vals = []
    for _ in range(3000):
        mask = (rng.random((n, n)) < p).astype(np.uint8)
        eps = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * np.sqrt(sigma2 / 2)
        vals.append(lr.input_scale(mask * (X + eps), mask, p) ** 2)
    vals = np.array(vals)
    truth = np.mean(np.abs(x0) ** 2) + sigma2
    assert abs(vals.mean() - truth) < 4 * vals.std() / np.sqrt(vals.size)


def test_input_scale_estimates_image_energy():
    sl = synth.workload_single64()[0][0]
    s0 = lr.input_scale(sl.y, sl.mask, sl.p)
    e = np.sqrt(np.mean(np.abs(sl.x0) ** 2))
    assert 0.5 * e < s0 < 2.0 * e


def test_learned_from_beyond_iterations_is_plain_vdamp():
    sl = synth.workload_single64()[0][0]
    p = half_shrink_params(10, 0.125)
    got = lr.vdamp_learned(sl.y, sl.mask, sl.p, sl.sigma2, 3, 3, p, seed=1, always=True, learned_from=3)
    ref = o.vdamp(sl.y, sl.mask, sl.p, sl.sigma2, 3, 3)
    assert np.array_equal(got["x_hat"], ref["x_hat"])

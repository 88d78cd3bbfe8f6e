"""Pins of the FP64 oracle of the learned denoiser: brute-force convolution, adjointness,
JVP and gradients against central finite differences, scale equivariance, the Adam
step's closed form, and the Monte-Carlo divergence estimator against a brute-force
Jacobian."""
import numpy as np
import pytest

from oracle import cnn_ref as cr

RNG = np.random.default_rng(99)


def small_params(nb=4, channels=4, seed=0):
    p = cr.init_params(nb, seed, channels=channels)
    rng = np.random.default_rng(seed + 1)
    for k in p:
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)  # nonzero biases and Wt
    return p


def test_conv_matches_bruteforce_loops():
    x = RNG.standard_normal((3, 5, 6))
    W = RNG.standard_normal((2, 3, 3, 3))
    ref = np.zeros((2, 5, 6))
    for co in range(2):
        for y in range(5):
            for xx in range(6):
                s = 0.0
                for ci in range(3):
                    for dy in range(3):
                        for dx in range(3):
                            s += W[co, ci, dy, dx] * x[ci, (y + dy - 1) % 5, (xx + dx - 1) % 6]
                ref[co, y, xx] = s
    assert np.abs(cr.conv(x, W) - ref).max() < 1e-12


def test_conv_t_is_adjoint():
    x = RNG.standard_normal((3, 7, 4))
    g = RNG.standard_normal((5, 7, 4))
    W = RNG.standard_normal((5, 3, 3, 3))
    assert abs(np.sum(cr.conv(x, W) * g) - np.sum(x * cr.conv_t(g, W))) < 1e-10


def _img(h, w, rng):
    return rng.standard_normal((h, w)) + 1j * rng.standard_normal((h, w))


def test_jvp_matches_finite_differences():
    rng = np.random.default_rng(5)
    p = small_params()
    x, v = _img(6, 8, rng), _img(6, 8, rng)
    tau, s0 = np.array([0.5, 1.0, 2.0, 0.1]), 1.3
    eps = 1e-6
    fd = (cr.forward(p, x + eps * v, tau, s0) - cr.forward(p, x - eps * v, tau, s0)) / (2 * eps)
    assert np.abs(cr.jvp(p, x, tau, s0, v) - fd).max() < 1e-6


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(6)
    p = small_params()
    batch = []
    for _ in range(2):
        x = _img(5, 6, rng)
        batch.append((x, np.array([0.3, 0.7, 1.1, 0.2]), 0.9, x + 0.2 * _img(5, 6, rng)))
    L, g = cr.loss_and_grad(p, batch)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp, _ = cr.loss_and_grad(p, batch)
            flat[idx] = old - eps
            lm, _ = cr.loss_and_grad(p, batch)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[k].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_scale_equivariance():
    rng = np.random.default_rng(7)
    p = small_params()
    x = _img(6, 6, rng)
    tau, s0, c = np.array([0.2, 0.4, 0.8, 1.6]), 0.7, 3.5
    a = cr.forward(p, c * x, c * c * tau, c * s0)
    b = c * cr.forward(p, x, tau, s0)
    assert np.abs(a - b).max() < 1e-11 * np.abs(b).max()


def test_adam_first_step_closed_form():
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -0.01, 2.0])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    cr.adam_step(p, g, m, v, 1, lr=0.1, eps=0.0)
    assert np.allclose(p["w"], np.array([1.0, -2.0, 0.5]) - 0.1 * np.sign(g["w"]))


def test_adam_second_step_hand_worked():
    """Two Adam steps on one parameter (p = 1, gradients 0.3 then -0.1, lr 0.1,
    beta1 = 0.9, beta2 = 0.999, eps = 0), worked by hand in exact fractions:
      step 1: m = 3/100, v = 9/100000; m_hat = 3/10, v_hat = 9/100 -> p = 1 - 0.1 = 9/10
      step 2: m = 0.9 (3/100) - 1/100 = 17/1000, v = 0.999 (9/100000) + 1/100000
              = 9991/100000000; m_hat = (17/1000) / (19/100) = 17/190,
              v_hat = (9991/100000000) / (1999/1000000) = 9991/199900
              -> p = 9/10 - 0.1 (17/190) / sqrt(9991/199900) = 0.8599781428045573.
    At step 1 bias correction makes the update lr sign(g) whatever the betas are; step 2
    separates them (swapping the roles of beta1 and beta2 gives 0.85435...)."""
    p = {"w": np.array([1.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    cr.adam_step(p, {"w": np.array([0.3])}, m, v, 1, lr=0.1, eps=0.0)
    assert abs(p["w"][0] - 0.9) < 1e-15
    cr.adam_step(p, {"w": np.array([-0.1])}, m, v, 2, lr=0.1, eps=0.0)
    assert abs(m["w"][0] - 17 / 1000) < 1e-16
    assert abs(v["w"][0] - 9991 / 100000000) < 1e-18
    assert abs(p["w"][0] - 0.8599781428045573) < 1e-14


def test_rademacher_divergence_estimates_wirtinger_mean():
    """E Re(conj(b) (J b)) over b in {+-1 +- i}/sqrt2 equals the mean Wirtinger derivative
    1/2 (du/dx + dv/dy) of the map, computed here from the brute-force Jacobian."""
    rng = np.random.default_rng(8)
    p = small_params(channels=3)
    h, w = 4, 4
    x = _img(h, w, rng)
    tau, s0 = np.array([0.5, 0.5, 0.5, 0.5]), 1.0
    N = h * w
    diag = 0.0
    for i in range(N):
        e = np.zeros(N, complex)
        e[i] = 1.0
        col_re = cr.jvp(p, x, tau, s0, e.reshape(h, w)).ravel()
        e[i] = 1j
        col_im = cr.jvp(p, x, tau, s0, e.reshape(h, w)).ravel()
        diag += 0.5 * (col_re[i].real + col_im[i].imag)
    exact = diag / N
    est = []
    for _ in range(3000):
        b = (rng.choice([-1.0, 1.0], size=(h, w)) + 1j * rng.choice([-1.0, 1.0], size=(h, w))) / np.sqrt(2)
        est.append(np.mean(np.real(np.conj(b) * cr.jvp(p, x, tau, s0, b))))
    est = np.array(est)
    assert abs(est.mean() - exact) < 4 * est.std() / np.sqrt(est.size) + 1e-12


def test_bf16_rounding_is_round_to_nearest_even():
    vals = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, -3.0e-3, 65504.0])
    got = cr.bf16_round(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to even (1.0)
    assert got[0] == 1.0 and got[1] == 1.0
    assert got[2] == 1.0078125 and got[3] == 1.0078125
    for g, v in zip(got, vals):
        assert abs(g - v) <= abs(v) * 2.0 ** -8

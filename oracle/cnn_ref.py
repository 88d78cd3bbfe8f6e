"""FP64 oracle of the learned colored-noise denoiser that can replace soft thresholding in
VDAMP (the paper's conclusion suggests a denoiser built for wavelet coefficients under
known colored Gaussian noise; Algorithm 1 admits any denoiser g(r; tau) with its
divergence in the alpha step).

TEST INFRASTRUCTURE ONLY: used by tests/ (and nothing in the product path).

Network (image domain, circular padding to match the periodic model):
  u  = (Re x, Im x) / s0                                   2 channels
  t  = log(max(tau_b / s0^2, 1e-12)), b = 0..nb-1         per-slice noise levels
  a1 = relu(conv(u; W1) + b1 + Wt t)                       48 channels
  a_l = relu(conv(a_{l-1}; W_l) + b_l), l = 2..5           48 channels
  o  = conv(a5; W6) + b6                                   2 channels
  f  = u - o;   x_out = s0 (f_0 + i f_1)
conv(in; W)[co, y, x] = sum_{ci, dy, dx} W[co, ci, dy, dx] in[ci, y + dy - 1, x + dx - 1]
(indices modulo the image size).  The wavelet-domain denoiser is
  g(r) = Psi x_out(Psi^H r),  so  J_g = Psi J_f Psi^H  (s0 cancels),
and its divergence enters the alpha step through alpha_b = mean_{i in b} Re(conj(b_i) (J_g b)_i)
for a complex Rademacher probe b in {+-1 +- i}/sqrt2, whose expectation is the mean
Wirtinger derivative (the same reading as for soft thresholding).

`bf16=True` rounds the weights and every conv input to bfloat16 (round to nearest
even) at the points where the GPU kernels store BF16, and keeps FP64 elsewhere.
"""
from __future__ import annotations

import numpy as np

C = 48
LAYERS = 6


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(a32)
    if nan.any():
        out[nan] = np.nan
    return out


def init_params(nb, seed, channels=C):
    """He-normal weights (seeded), zero biases; Wt starts at zero."""
    rng = np.random.default_rng(seed)
    p = {}
    cin = [2] + [channels] * 4 + [channels]
    cout = [channels] * 5 + [2]
    for l in range(LAYERS):
        fan_in = cin[l] * 9
        std = np.sqrt(2.0 / fan_in) if l < LAYERS - 1 else 0.1 * np.sqrt(1.0 / fan_in)
        p[f"W{l + 1}"] = rng.standard_normal((cout[l], cin[l], 3, 3)) * std
        p[f"b{l + 1}"] = np.zeros(cout[l])
    p["Wt"] = np.zeros((channels, nb))
    return p


def conv(x, W):
    """Circular 3x3 correlation: x [ci][H][W], W [co][ci][3][3] -> [co][H][W]."""
    co = W.shape[0]
    out = np.zeros((co,) + x.shape[1:])
    for dy in range(3):
        for dx in range(3):
            sh = np.roll(np.roll(x, -(dy - 1), axis=1), -(dx - 1), axis=2)  # x[., y+dy-1, x+dx-1]
            out += np.einsum("oc,chw->ohw", W[:, :, dy, dx], sh)
    return out


def conv_t(g, W):
    """Adjoint of conv: g [co][H][W] -> [ci][H][W]."""
    ci = W.shape[1]
    out = np.zeros((ci,) + g.shape[1:])
    for dy in range(3):
        for dx in range(3):
            t = np.einsum("oc,ohw->chw", W[:, :, dy, dx], g)
            out += np.roll(np.roll(t, dy - 1, axis=1), dx - 1, axis=2)
    return out


def _maybe(a, bf16):
    return bf16_round(a) if bf16 else a


def forward(p, x, tau, s0, bf16=False, keep=False):
    """x: complex image [H][W]; tau: [nb]; returns x_out (complex) and, with keep, the
    cached layer inputs/activations."""
    u = np.stack([x.real, x.imag]) / s0
    t = np.log(np.maximum(np.asarray(tau, dtype=np.float64) / s0 ** 2, 1e-12))
    acts = [_maybe(u, bf16)]
    h = acts[0]
    for l in range(1, LAYERS + 1):
        W = _maybe(p[f"W{l}"], bf16)
        z = conv(h, W) + p[f"b{l}"][:, None, None]
        if l == 1:
            z = z + (p["Wt"] @ t)[:, None, None]
        if l < LAYERS:
            h = _maybe(np.maximum(z, 0.0), bf16)
            acts.append(h)
        else:
            o = z
    f = u - o
    out = s0 * (f[0] + 1j * f[1])
    if keep:
        return out, dict(acts=acts, u=u, t=t, o=o)
    return out


def jvp(p, x, tau, s0, v, bf16=False):
    """J_f v for the image-domain map x -> x_out at x (v complex image)."""
    _, cache = forward(p, x, tau, s0, bf16=bf16, keep=True)
    acts = cache["acts"]
    tv = np.stack([v.real, v.imag])
    h = _maybe(tv, bf16)
    for l in range(1, LAYERS + 1):
        W = _maybe(p[f"W{l}"], bf16)
        z = conv(h, W)
        if l < LAYERS:
            h = _maybe(z * (acts[l] > 0), bf16)
        else:
            o = z
    f = tv - o
    return f[0] + 1j * f[1]


def loss_and_grad(p, batch, bf16=False):
    """Mean over slices of ||x_out - x0||^2 / (s0^2 N); batch = list of (x, tau, s0, x0).
    Returns (loss, grads) with grads keyed like p."""
    g = {k: np.zeros_like(v) for k, v in p.items()}
    L = 0.0
    nsl = len(batch)
    for (x, tau, s0, x0) in batch:
        out, cache = forward(p, x, tau, s0, bf16=bf16, keep=True)
        N = x.size
        d = out - x0
        L += np.sum(np.abs(d) ** 2) / (s0 ** 2 * N) / nsl
        # dL/do: x_out = s0 (u - o) => dL/do = -(2/(s0^2 N nsl)) s0 (Re d, Im d)
        go = -2.0 / (s0 * N * nsl) * np.stack([d.real, d.imag])
        acts = cache["acts"]
        gh = _maybe(go, bf16)
        for l in range(LAYERS, 0, -1):
            W = _maybe(p[f"W{l}"], bf16)
            hin = acts[l - 1]
            # weights and biases of layer l
            for dy in range(3):
                for dx in range(3):
                    sh = np.roll(np.roll(hin, -(dy - 1), axis=1), -(dx - 1), axis=2)
                    g[f"W{l}"][:, :, dy, dx] += np.einsum("ohw,chw->oc", gh, sh)
            g[f"b{l}"] += gh.sum(axis=(1, 2))
            if l == 1:
                g["Wt"] += np.outer(gh.sum(axis=(1, 2)), cache["t"])
                break
            gin = conv_t(gh, W)
            gh = _maybe(gin * (acts[l - 1] > 0), bf16)
    return L, g


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place; step counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v

"""Training of the learned denoiser on states of plain VDAMP (argument marshalling and
loop control only: every solve, transform and training step runs in libvdamp).

Training pairs follow the denoiser's use in Algorithm 1: for an iteration count k the
plain solve's last iterate r_{k-1} and its noise levels tau_{k-1} give the network input
x = Psi^H r_{k-1} with tau, and the target is the ground-truth image x0; s0 is the
solve's input scale.  One training step uses every slice of the plan at one k, cycling
through the given k.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import vdamp as V


def input_scales(plan: "V.Plan", cnn: "V.Cnn", ws, y, mask, p, sigma2, stream=None):
    """Per-slice input scales s0, from a zero-iteration learned solve."""
    import torch
    cws = cnn.workspace(plan, V.VDAMP_CNN_WS_SOLVE)
    x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, 0, 0, x, stream=stream)
    s0 = torch.empty(plan.batch, dtype=torch.float32, device="cuda")
    cnn.learned_export(plan, cws, s0=s0, stream=stream)
    return s0


def make_pairs(plan: "V.Plan", ws, y, mask, p, sigma2, ks: Sequence[int], stream=None):
    """Network inputs (Psi^H r_{k-1}) and noise levels [B][16] of plain VDAMP after k
    iterations, for each k in ks."""
    import torch
    pairs = []
    xh = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    r = torch.empty_like(xh)
    for k in ks:
        if k < 1:
            raise ValueError("iteration counts must be >= 1")
        plan.vdamp_solve(ws, y, mask, p, sigma2, int(k), xh, stream=stream)
        tau = torch.empty(plan.batch * plan.nbands, dtype=torch.float32, device="cuda")
        plan.vdamp_state_export(ws, r=r, tau=tau, stream=stream)
        x = torch.empty_like(xh)
        plan.vdamp_wavelet(r, x, inverse=True, stream=stream)
        t16 = torch.zeros(plan.batch, 16, dtype=torch.float32, device="cuda")
        t16[:, :plan.nbands] = tau.view(plan.batch, plan.nbands)
        pairs.append((x, t16.contiguous()))
    return pairs


def train(cnn: "V.Cnn", plan: "V.Plan", pairs, s0, x0, steps: int, lr: float, stream=None,
          lr_final: float | None = None):
    """Adam steps over the pairs in turn; returns the loss before each step (host array).
    With lr_final the learning rate decays geometrically from lr to lr_final."""
    import torch
    ws = cnn.workspace(plan, V.VDAMP_CNN_WS_TRAIN)
    losses = torch.zeros(steps, dtype=torch.float32, device="cuda")
    for i in range(steps):
        x, tau = pairs[i % len(pairs)]
        rate = lr if lr_final is None or steps < 2 else lr * (lr_final / lr) ** (i / (steps - 1))
        cnn.train_step(plan, ws, x, tau, s0, x0, rate, losses[i:i + 1], stream=stream)
    return losses.cpu().numpy()


def init_flat(nbands: int, seed: int, channels: int = 48) -> np.ndarray:
    """Seeded He-normal initial parameters in the library's flat order (zero biases,
    zero noise-level weights, a small last layer so the network starts near f(x) = x)."""
    rng = np.random.default_rng(seed)
    cin = [2] + [channels] * 5
    cout = [channels] * 5 + [2]
    p = {}
    for l in range(6):
        fan_in = cin[l] * 9
        std = np.sqrt(2.0 / fan_in) if l < 5 else 0.1 * np.sqrt(1.0 / fan_in)
        p[f"W{l + 1}"] = rng.standard_normal((cout[l], cin[l], 3, 3)) * std
        p[f"b{l + 1}"] = np.zeros(cout[l])
    p["Wt"] = np.zeros((channels, nbands))
    return V.cnn_flatten(p).astype(np.float32)

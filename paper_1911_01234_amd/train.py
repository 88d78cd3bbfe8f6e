"""Training of the learned denoiser on states of plain VDAMP (argument marshalling and
loop control only: every solve, transform and training step runs in libvdamp).

Training pairs follow the denoiser's use in Algorithm 1: for an iteration count k the
plain solve's last iterate r_{k-1} and its noise levels tau_{k-1} give the network input
x = Psi^H r_{k-1} with tau, and the target is the ground-truth image x0; s0 is the
solve's input scale.  `train` uses every slice of one plan at one k per step, cycling
through the given k; `TripleStore` holds (x, tau, s0, x0) for many slices and iteration
counts in device memory and `train_store` draws seeded random batches from it.
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


class TripleStore:
    """Training triples (Psi^H r_{k-1}, tau_{k-1}, x0) with each slice's s0, resident in
    device memory: x [n][N] complex64, tau [n][16], and per slice s0 and x0.  Triple t
    belongs to slice t // len(ks) and iteration count ks[t % len(ks)]."""

    def __init__(self, n_slices: int, npx: int, ks: Sequence[int]):
        import torch
        self.ks = tuple(int(k) for k in ks)
        self.npx = npx
        n = n_slices * len(self.ks)
        self.x = torch.empty((n, npx), dtype=torch.complex64, device="cuda")
        self.tau = torch.zeros((n, 16), dtype=torch.float32, device="cuda")
        self.s0 = torch.empty(n_slices, dtype=torch.float32, device="cuda")
        self.x0 = torch.empty((n_slices, npx), dtype=torch.complex64, device="cuda")
        self.filled = 0

    def __len__(self):
        return self.filled * len(self.ks)

    def add(self, plan: "V.Plan", cnn: "V.Cnn", slices, stream=None):
        """Solve `slices` (all of the plan's size) with plain VDAMP and store their
        triples for every iteration count."""
        import torch
        ws = plan.workspace()
        y, mask, p, sigma2 = V.to_device(plan, slices)
        s0 = input_scales(plan, cnn, ws, y, mask, p, sigma2, stream=stream)
        pairs = make_pairs(plan, ws, y, mask, p, sigma2, self.ks, stream=stream)
        b0, nb, nk = self.filled, plan.batch, len(self.ks)
        rows = torch.arange(b0, b0 + nb, device="cuda") * nk
        for j, (x, t16) in enumerate(pairs):
            self.x[rows + j] = x.view(nb, self.npx)
            self.tau[rows + j] = t16
        self.s0[b0:b0 + nb] = s0
        self.x0[b0:b0 + nb] = torch.from_numpy(plan.pack([sl.x0 for sl in slices], np.complex64)).cuda().view(nb, -1)
        self.filled += nb
        return self


def train_store(cnn: "V.Cnn", plan: "V.Plan", store: TripleStore, steps: int, lr: float, seed: int = 0,
                stream=None, lr_final: float | None = None):
    """Adam steps on batches of plan.batch triples drawn without replacement from the
    store (a fresh seeded permutation each pass over it); returns the loss before each
    step (host array).  With lr_final the learning rate decays geometrically."""
    import torch
    ws = cnn.workspace(plan, V.VDAMP_CNN_WS_TRAIN)
    losses = torch.zeros(steps, dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    nb, nk = plan.batch, len(store.ks)
    perm = torch.randperm(len(store), generator=g)
    pos = 0
    for i in range(steps):
        if pos + nb > len(perm):
            perm, pos = torch.randperm(len(store), generator=g), 0
        idx = perm[pos:pos + nb].cuda()
        pos += nb
        sl = torch.div(idx, nk, rounding_mode="floor")
        x = store.x[idx].reshape(-1)
        tau = store.tau[idx].contiguous()
        s0 = store.s0[sl].contiguous()
        x0 = store.x0[sl].reshape(-1)
        rate = lr if lr_final is None or steps < 2 else lr * (lr_final / lr) ** (i / (steps - 1))
        cnn.train_step(plan, ws, x, tau, s0, x0, rate, losses[i:i + 1], stream=stream)
    return losses.cpu().numpy()


def paired_gain(nmse_plain_db, nmse_learned_db):
    """Per-slice paired NMSE gain of the learned form (plain minus learned, dB; positive
    = learned better): mean, standard deviation and the two-sided 95 % confidence
    interval of the mean (Student t with n - 1 degrees of freedom)."""
    from scipy import stats
    d = np.asarray(nmse_plain_db, dtype=np.float64) - np.asarray(nmse_learned_db, dtype=np.float64)
    n = d.size
    m, sd = float(d.mean()), float(d.std(ddof=1)) if n > 1 else 0.0
    h = float(stats.t.ppf(0.975, n - 1) * sd / np.sqrt(n)) if n > 1 else float("inf")
    return {"slices": n, "mean_db": m, "sd_db": sd, "ci95_db": [m - h, m + h]}

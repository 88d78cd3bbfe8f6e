"""Helpers shared by the GPU tests: run the library through its C ABI on seeded inputs
and bring results back as numpy arrays."""
from __future__ import annotations

import numpy as np

from oracle import vdamp_ref as o  # band geometry only (o.bands)


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def fp32_inputs(sl):
    """The measurements exactly as the library reads them (y as complex64, p and sigma^2
    as float32), upcast to FP64 for the oracle: rounding of the inputs is then not
    booked as an error of the kernels."""
    y = np.asarray(sl.y).astype(np.complex64).astype(np.complex128)
    p = np.asarray(sl.p).astype(np.float32).astype(np.float64)
    return y, sl.mask, p, float(np.float32(sl.sigma2))


def fp32_state(r, theta, alpha):
    """An oracle state (r_k, theta_k, alpha_k) rounded to the FP32 values the library
    takes, upcast again for the oracle."""
    return (np.asarray(r).astype(np.complex64).astype(np.complex128),
            np.asarray(theta).astype(np.float32).astype(np.float64),
            np.asarray(alpha).astype(np.float32).astype(np.float64))


def oracle_states_batch256(task):
    """Worker (no GPU): slice b of the 256x256 benchmark batch regenerated from its seeds,
    the oracle run on its FP32-rounded inputs, and its state at each iteration k of ks
    rounded to FP32: (b, {k: (r_k, theta_k, alpha_k)})."""
    b, ks = task
    from paper_1911_01234_amd import synth
    sl = synth.workload_batch256(1, first_slice=b)[0][0]
    traj = o.vdamp(*fp32_inputs(sl), 4, max(ks) + 1, record=True)
    return b, {k: (traj["r"][k].astype(np.complex64), traj["theta"][k].astype(np.float32),
                   traj["alpha"][k].astype(np.float32)) for k in ks}


def oracle_states_of(task):
    """Worker (no GPU): the oracle on one slice's FP32 inputs (y complex64, mask, p and
    sigma^2 float32, upcast here; wavelet: None for Haar or a lowpass filter; group 1 or
    2), its state at each iteration k of ks rounded to FP32:
    (b, {k: (r_k, theta_k, alpha_k)})."""
    b, y, mask, p, s2, s, ks, wavelet, group = task
    traj = o.vdamp(y.astype(np.complex128), mask, p.astype(np.float64), float(s2), s, max(ks) + 1, record=True,
                   wavelet=wavelet, group=group)
    return b, {k: (traj["r"][k].astype(np.complex64), traj["theta"][k].astype(np.float32),
                   traj["alpha"][k].astype(np.float32)) for k in ks}


def oracle3_states_of(task):
    """Worker (no GPU): the 3D oracle on one volume's FP32 inputs (upcast here), its state
    at each iteration k of ks rounded to FP32: (b, {k: (r_k, theta_k, alpha_k)})."""
    b, y, mask, p, s2, s, ks = task
    from oracle import vdamp3d_ref as o3
    traj = o3.vdamp3(y.astype(np.complex128), mask, p.astype(np.float64), float(s2), s, max(ks) + 1, record=True)
    return b, {k: (traj["r"][k].astype(np.complex64), np.asarray(traj["theta"][k], np.float32),
                   np.asarray(traj["alpha"][k], np.float32)) for k in ks}


def run_resume(plan, slices, states, iters, want_state=True, x_monitor=False, stream=None):
    """vdamp_solve_resume on every slice of the plan: states maps slice index b to an
    FP32 state (r_k [ny][nx], theta_k [nb], alpha_k [nb]); slices not in states start
    from r = 0, theta = 0, alpha = 0 (Onsager correction then gives r_tilde = 0)."""
    import torch
    from paper_1911_01234_amd import vdamp as V
    ws = plan.workspace()
    y, mask, p, sigma2 = V.to_device(plan, slices)
    r0 = [np.zeros((plan.ny[b], plan.nx[b]), np.complex64) for b in range(plan.batch)]
    th0 = np.zeros((plan.batch, plan.nbands), np.float32)
    al0 = np.zeros((plan.batch, plan.nbands), np.float32)
    for b, (r, th, al) in states.items():
        r0[b] = np.asarray(r).astype(np.complex64)
        th0[b] = np.asarray(th, dtype=np.float32)
        al0[b] = np.asarray(al, dtype=np.float32)
    r_in = torch.from_numpy(plan.pack(r0, np.complex64)).cuda()
    th_in = torch.from_numpy(th0.ravel()).cuda()
    al_in = torch.from_numpy(al0.ravel()).cuda()
    x_hat = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    trace = torch.empty(max(iters, 1) * plan.batch * plan.nbands * 3, dtype=torch.float32, device="cuda")
    mon = (torch.empty(max(iters, 1) * plan.ntot, dtype=torch.complex64, device="cuda")
           if x_monitor else None)
    plan.vdamp_solve_resume(ws, y, mask, p, sigma2, r_in, th_in, None, al_in, iters, x_hat, trace,
                            mon, stream=stream)
    out = {}
    if want_state:
        r = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
        th = torch.empty(plan.batch * plan.nbands, dtype=torch.float32, device="cuda")
        al = torch.empty_like(th)
        ta = torch.empty_like(th)
        t2 = torch.empty_like(th)
        plan.vdamp_state_export(ws, r, th, al, ta, theta2=t2, stream=stream)
        torch.cuda.synchronize()
        out["r"] = plan.unpack(r.cpu().numpy())
        out["theta"] = th.cpu().numpy().reshape(plan.batch, plan.nbands)
        out["theta2"] = t2.cpu().numpy().reshape(plan.batch, plan.nbands)
        out["alpha"] = al.cpu().numpy().reshape(plan.batch, plan.nbands)
        out["tau"] = ta.cpu().numpy().reshape(plan.batch, plan.nbands)
    torch.cuda.synchronize()
    out["x_hat"] = plan.unpack(x_hat.cpu().numpy())
    out["trace"] = trace.cpu().numpy()[: iters * plan.batch * plan.nbands * 3].reshape(
        iters, plan.batch, plan.nbands, 3)
    if x_monitor:
        m = mon.cpu().numpy()
        out["monitor"] = [plan.unpack(m[k * plan.ntot:(k + 1) * plan.ntot]) for k in range(iters)]
    return out


def run_vdamp(slices, s, iters, flags=0, want_state=False, plan=None, stream=None, lowpass=None):
    import torch
    from paper_1911_01234_amd import vdamp as V
    own = plan is None
    if own:
        plan = V.Plan([sl.y.shape[0] for sl in slices], [sl.y.shape[1] for sl in slices], s, flags,
                      lowpass=lowpass)
    ws = plan.workspace()
    y, mask, p, sigma2 = V.to_device(plan, slices)
    x_hat = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    trace = torch.empty(max(iters, 1) * plan.batch * plan.nbands * 3, dtype=torch.float32, device="cuda")
    plan.vdamp_solve(ws, y, mask, p, sigma2, iters, x_hat, trace, stream=stream)
    out = {}
    if want_state and iters > 0:
        r = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
        th = torch.empty(plan.batch * plan.nbands, dtype=torch.float32, device="cuda")
        al = torch.empty_like(th)
        ta = torch.empty_like(th)
        t2 = torch.empty_like(th)
        plan.vdamp_state_export(ws, r, th, al, ta, theta2=t2, stream=stream)
        torch.cuda.synchronize()
        out["r"] = plan.unpack(r.cpu().numpy())
        out["theta"] = th.cpu().numpy().reshape(plan.batch, plan.nbands)
        out["theta2"] = t2.cpu().numpy().reshape(plan.batch, plan.nbands)
        out["alpha"] = al.cpu().numpy().reshape(plan.batch, plan.nbands)
        out["tau"] = ta.cpu().numpy().reshape(plan.batch, plan.nbands)
    torch.cuda.synchronize()
    out["x_hat"] = plan.unpack(x_hat.cpu().numpy())
    out["trace"] = trace.cpu().numpy()[: iters * plan.batch * plan.nbands * 3].reshape(
        iters, plan.batch, plan.nbands, 3)
    out["plan"] = plan
    return out


def run_fista(slices, s, lams, iters, objective=False):
    import torch
    from paper_1911_01234_amd import vdamp as V
    plan = V.Plan([sl.y.shape[0] for sl in slices], [sl.y.shape[1] for sl in slices], s)
    ws = plan.workspace()
    y, mask, _, _ = V.to_device(plan, slices)
    lam = torch.tensor(lams, dtype=torch.float32, device="cuda")
    x_hat = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    obj = torch.empty(max(iters, 1) * plan.batch, dtype=torch.float32, device="cuda") if objective else None
    plan.fista_solve(ws, y, mask, lam, iters, x_hat, objective=obj)
    torch.cuda.synchronize()
    xs = plan.unpack(x_hat.cpu().numpy())
    if objective:
        return xs, obj.cpu().numpy()[: iters * plan.batch].reshape(iters, plan.batch)
    return xs


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def band_list(ny, nx, s):
    return o.bands(ny, nx, s)


def key32(r):
    """|r|^2 as the kernels compute it: IEEE FP32 x*x + y*y, each step rounded.  The
    threshold search sorts and decides on these keys, and thresholding tests membership
    |r|^2 > theta^2 on them."""
    r = np.asarray(r).astype(np.complex64)
    x, y = r.real.astype(np.float32), r.imag.astype(np.float32)
    return (x * x + y * y).astype(np.float32)


def group_keys32(r_band, d=1):
    """The kernels' keys of a band block: key32 per coefficient (d = 1), or per
    horizontal pair x = 2j, 2j+1 (d = 2) the FP32 sum of the two coefficients' keys."""
    k = key32(r_band)
    if d == 1:
        return k
    return (k[:, 0::2] + k[:, 1::2]).astype(np.float32)


def group_mags(r_band, d=1):
    """FP64 magnitudes of a band block's thresholding units: |r| per coefficient, or the
    norm of each horizontal pair."""
    r = np.asarray(r_band, dtype=np.complex128)
    if d == 1:
        return np.abs(r)
    return np.sqrt(np.abs(r[:, 0::2]) ** 2 + np.abs(r[:, 1::2]) ** 2)


def snap_theta(r_band, theta_gpu, d=1):
    """The FP64 candidate magnitude nearest to a threshold the GPU took on its FP32
    keys (used only to tell whether two trajectories chose the same element)."""
    a = np.unique(group_mags(r_band, d).ravel())
    if float(theta_gpu) == 0.0:
        return 0.0
    i = int(np.argmin(np.abs(a - float(theta_gpu))))
    return float(a[i])


def theta_keys(r_band, theta_gpu, d=1):
    """Keys (FP32 squared magnitudes) the GPU's theta may stand for.  The kernel decides
    on keys and reports theta = sqrt(key) in FP32, which its sqrt can leave one ulp off
    the correctly rounded value, so the candidates are the keys whose FP32 square root
    is within one ulp of theta (two keys one ulp apart can both qualify); the nearest
    key if none does."""
    k = np.unique(group_keys32(r_band, d).ravel())
    if float(theta_gpu) == 0.0:
        return [0.0]
    t = np.float32(theta_gpu)
    lo = np.nextafter(t, np.float32(0))
    hi = np.nextafter(t, np.float32(np.inf))
    sq = np.sqrt(k)
    hit = k[(sq >= lo) & (sq <= hi)]
    if hit.size:
        return [float(v) for v in hit]
    k64 = k.astype(np.float64)
    return [float(k64[int(np.argmin(np.abs(np.sqrt(k64) - float(theta_gpu))))])]


def theta_key(r_band, theta_gpu):
    return theta_keys(r_band, theta_gpu)[0]


def sure_scan(a, tau, d=1):
    """SURE of complex soft thresholding at every candidate threshold, evaluated
    directly from its definition (Stein's estimate for noise CN(0, tau)):
        SURE(theta) = sum_{a_i <= theta} (a_i^2 - tau)
                      + sum_{a_i > theta} (theta^2 + tau - tau theta / a_i),
    for the candidates theta = the distinct positive magnitudes.  Written here for the
    validity check of a GPU result on the GPU's own data, independently of the oracle.
    With groups of d coefficients (a = group norms, 2d real dimensions each, noise
    variance tau/2 in each) Stein's estimate reads
        sum_{a <= theta} (a^2 - d tau) + sum_{a > theta} (theta^2 + d tau - (2d - 1) tau theta / a).
    Returns (candidates, values)."""
    a = np.sort(np.asarray(a, dtype=np.float64).ravel())
    n = a.size
    cand = np.unique(a[a > 0])
    if cand.size == 0:
        return np.array([0.0]), np.array([-n * tau])
    below = np.searchsorted(a, cand, side="right")          # count of a <= theta
    c2 = np.concatenate([[0.0], np.cumsum(a ** 2)])
    inv = np.where(a > 0, 1.0 / np.where(a > 0, a, 1.0), 0.0)
    cinv = np.concatenate([[0.0], np.cumsum(inv)])
    s_below = c2[below] - below * (d * tau)
    n_above = n - below
    r_above = cinv[n] - cinv[below]
    vals = s_below + n_above * (cand ** 2 + d * tau) - (2 * d - 1) * tau * cand * r_above
    return cand, vals


def theta_accepted(r, tau_b, rs, cs, theta_gpu, alpha_gpu=None, return_key=False, d=1):
    """Validity of the GPU's threshold on the GPU's own iterate: the SURE argmin is an
    index decided in floating point, so it is taken on the kernel's FP32 keys of that r
    (magnitudes sqrt(key32) in FP64).  The GPU's threshold is accepted when its SURE is
    the minimum over all candidates up to 1e-6 (|SURE_min| + N_b tau) (a near tie).
    Among keys theta may stand for, the one whose alpha (alpha step) matches the GPU's
    alpha is the GPU's choice.  d = 2: the keys are those of horizontal pairs (group
    soft thresholding)."""
    band = np.asarray(r)[rs, cs]
    a = np.sqrt(group_keys32(band, d).astype(np.float64)).ravel()
    cand, vals = sure_scan(a, float(tau_b), d)
    s_min = float(vals.min())
    cands = theta_keys(band, theta_gpu, d)
    if alpha_gpu is not None and len(cands) > 1:
        cands.sort(key=lambda kth: abs(alpha_at_key(band, kth, d) - float(alpha_gpu)))
    ok_key = None
    for kth in cands:
        th = float(np.sqrt(kth))
        if th == 0.0:
            ok = cand.size == 1 and cand[0] == 0.0
        else:
            i = int(np.argmin(np.abs(cand - th)))
            ok = cand[i] == th and vals[i] <= s_min + 1e-6 * (abs(s_min) + a.size * d * tau_b)
        if ok:
            ok_key = kth
            break
    return (ok_key is not None, ok_key) if return_key else ok_key is not None


def alpha_at_key(r_band, kth, d=1):
    """alpha (alpha step) at the threshold with key kth, membership on the FP32 keys.  For
    pairs (d = 2): half the real divergence of group soft thresholding per coefficient,
    4 - 3 theta/||g|| per pair above the threshold, over 2 N_b."""
    k = group_keys32(r_band, d).astype(np.float64).ravel()
    keep = k > kth
    th = np.sqrt(kth)
    if d == 1:
        return float(np.sum(1.0 - th / (2.0 * np.sqrt(k[keep]))) / k.size)
    return float(np.sum(2 * d - (2 * d - 1) * th / np.sqrt(k[keep])) / (2.0 * d * k.size))


def sure_min_continuous(a, tau, d=1):
    """The minimum over every theta > 0 of complex soft thresholding's SURE on magnitudes
    a (test code written from the definition, independently of the oracle): SURE is a
    quadratic in theta between consecutive distinct magnitudes, n_above (theta^2 + tau)
    - tau theta R_above + const, so its infimum on each interval is at the clipped vertex
    or the interval's left end (a magnitude, counted below).  Groups of d coefficients
    (a = group norms): tau becomes d tau in the first two terms and (2d - 1) tau in the
    last (sure_scan).  Returns the minimum."""
    a = np.sort(np.asarray(a, dtype=np.float64).ravel())
    n = a.size
    tl, td = d * tau, (2 * d - 1) * tau
    u = np.unique(a[a > 0])
    if u.size == 0:
        return -n * tl
    ends = np.concatenate([[0.0], u])
    best = np.inf
    for j in range(u.size):
        lo, hi = ends[j], ends[j + 1]
        below = a <= lo
        nb = int(np.sum(~below))
        A = float(np.sum(a[below] ** 2))
        R = float(np.sum(1.0 / a[~below]))
        c = A - (n - nb) * tl
        if lo > 0:   # theta = lo itself (a candidate)
            best = min(best, c + nb * (lo * lo + tl) - td * lo * R)
        t = td * R / (2.0 * nb)
        if lo < t < hi:
            best = min(best, c + nb * (t * t + tl) - td * t * R)
    return best


def theta_accepted_continuous(r, tau_b, rs, cs, theta_gpu, thr2_gpu, d=1):
    """The continuous search's threshold on the library's own iterate: the SURE of what
    the kernels apply (coefficients whose FP32 key is at most the threshold's key
    thr2_gpu are zeroed, the others shrunk by theta_gpu), from the definition on the FP32
    keys, is the continuous minimum up to the near-tie margin 1e-6 (|SURE_min| + N_b tau)."""
    band = np.asarray(r)[rs, cs]
    k = group_keys32(band, d).astype(np.float64).ravel()
    a = np.sqrt(k)
    th = float(theta_gpu)
    below = k <= float(np.float32(thr2_gpu))
    v = float(np.sum(a[below] ** 2 - d * tau_b)
              + np.sum(th * th + d * tau_b - (2 * d - 1) * tau_b * th / a[~below]))
    m = sure_min_continuous(a, float(tau_b), d)
    return v <= m + 1e-6 * (abs(m) + a.size * d * tau_b)

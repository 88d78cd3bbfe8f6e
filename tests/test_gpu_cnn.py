"""GPU parity of the learned denoiser (BF16 MFMA kernels through the C ABI) against the
FP64 oracle with BF16 rounding at the same storage points (oracle/cnn_ref.py,
oracle/learned_ref.py), on seeded synthetic inputs.

Tolerances.  Both sides round weights and activations to BF16 (8-bit significand); they
differ where an FP32 accumulation and its FP64 counterpart fall on different sides of a
BF16 rounding boundary, which flips that activation by one BF16 ulp (2^-8 relative).
The network's residual output o (x - f(x)) is compared in relative L2 with 5e-3
(measured 5e-4; one flip moves an element by 2^-8 relative).  The JVP (v - J_f v) also
carries the ReLU decisions z > 0, which FP32 and FP64 take differently where z is
within rounding of 0 (about one of the 10^6 pre-activations of a 64x64 slice): such a
flip switches one tangent element on or off, and the layers after it spread that to
the 11x11 pixel neighbourhood of the output.  The JVP is judged by the fraction of
output pixels off by more than 1% of its RMS (at most the area of three such 11x11
neighbourhoods, 3 * 121 / (ny nx); measured up to 2.1e-2 of a 64x64 slice, under one
neighbourhood) and by relative L2 (at most 3e-2; measured 4e-7 to 8.3e-3).  The gradient
per parameter tensor with 1e-2 (measured at most 4.4e-3, in W1, whose gradient has
passed through five BF16-rounded backward layers), the loss with 1e-4.  Plain-transform and bookkeeping
results that involve no BF16 rounding are compared at FP32 level."""
import numpy as np
import pytest

from oracle import cnn_ref as cr
from oracle import learned_ref as lr
from oracle import vdamp_ref as o
from paper_1911_01234_amd import synth

from gpu_helpers import fp32_inputs, rel_l2

pytestmark = pytest.mark.gpu

TOL_OUT = 5e-3
TOL_GRAD = 1e-2
TOL_LOSS = 1e-4


def rand_params(nb, seed, scale_last=3.0):
    """He-initialised weights with nonzero biases and noise-level weights."""
    p = cr.init_params(nb, seed)
    rng = np.random.default_rng(seed + 100)
    for k in p:
        if k.startswith("b") or k == "Wt":
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    p["W6"] = p["W6"] * scale_last
    return p


def images(shapes, seed):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal(sh) + 1j * rng.standard_normal(sh)) * (0.5 + i) for i, sh in enumerate(shapes)]


def setup(shapes, s, params, seed=0):
    import torch
    from paper_1911_01234_amd import vdamp as V
    plan = V.Plan([a for a, _ in shapes], [b for _, b in shapes], s)
    cnn = V.Cnn(plan.nbands)
    flat = torch.from_numpy(V.cnn_flatten(params).astype(np.float32)).cuda()
    cnn.set_params(flat)
    return plan, cnn


def dev_c64(plan, arrs):
    import torch
    return torch.from_numpy(plan.pack(arrs, np.complex64)).cuda()


def taus_for(plan, seed):
    rng = np.random.default_rng(seed)
    t = np.zeros((plan.batch, 16), dtype=np.float32)
    t[:, :plan.nbands] = rng.uniform(1e-4, 1e-1, size=(plan.batch, plan.nbands))
    return t


SHAPES = [(64, 64), (48, 80), (32, 32)]


def jvp_far_limit(shape):
    """Pixels a JVP may miss by more than 1% of its RMS: three 11x11 neighbourhoods, the
    reach of a tangent element switched by a ReLU decision z > 0 that FP32 and FP64
    take differently (z within rounding of 0) through the five layers after it."""
    return 3 * 121 / (shape[0] * shape[1])


def test_forward_and_jvp_match_oracle():
    import torch
    from paper_1911_01234_amd import vdamp as V
    s = 2
    params = rand_params(1 + 3 * s, 1)
    plan, cnn = setup(SHAPES, s, params)
    xs = images(SHAPES, 2)
    vs = images(SHAPES, 3)
    tau = taus_for(plan, 4)
    s0 = np.array([0.7, 1.3, 2.1], dtype=np.float32)
    ws = cnn.workspace(plan, V.VDAMP_CNN_WS_FORWARD)
    x, v = dev_c64(plan, xs), dev_c64(plan, vs)
    xo = torch.empty_like(x)
    jo = torch.empty_like(x)
    tau_d, s0_d = torch.from_numpy(tau).cuda(), torch.from_numpy(s0).cuda()
    cnn.forward(plan, ws, x, tau_d, s0_d, xo, v, jo)
    # forward alone gives the same output bit for bit
    xo2 = torch.empty_like(x)
    cnn.forward(plan, ws, x, tau_d, s0_d, xo2)
    torch.cuda.synchronize()
    assert torch.equal(xo, xo2)
    g_out = plan.unpack(xo.cpu().numpy())
    g_jvp = plan.unpack(jo.cpu().numpy())
    errs = []
    for b in range(plan.batch):
        xq = xs[b].astype(np.complex64).astype(np.complex128)
        vq = vs[b].astype(np.complex64).astype(np.complex128)
        ref = cr.forward(params, xq, tau[b, :plan.nbands].astype(np.float64), float(s0[b]), bf16=True)
        e = rel_l2(xq - g_out[b], xq - ref)
        refj = cr.jvp(params, xq, tau[b, :plan.nbands].astype(np.float64), float(s0[b]), vq, bf16=True)
        dj, wj = vq - g_jvp[b], vq - refj
        ej = rel_l2(dj, wj)
        far = np.mean(np.abs(dj - wj) > 1e-2 * np.sqrt(np.mean(np.abs(wj) ** 2)))
        print(f"slice {b} {SHAPES[b]}: residual rel {e:.2e}, jvp rel {ej:.2e}, jvp far fraction {far:.1e}")
        errs.append((e, ej, far))
    assert max(e for e, _, _ in errs) < TOL_OUT
    assert max(ej for _, ej, _ in errs) < 3e-2
    for (_, _, f), sh in zip(errs, SHAPES):
        assert f <= jvp_far_limit(sh)


def test_training_gradient_and_loss_match_oracle():
    import torch
    from paper_1911_01234_amd import vdamp as V
    s = 2
    params = rand_params(1 + 3 * s, 5)
    plan, cnn = setup(SHAPES, s, params)
    xs = images(SHAPES, 6)
    x0s = [x + 0.3 * im for x, im in zip(xs, images(SHAPES, 7))]
    tau = taus_for(plan, 8)
    s0 = np.array([0.9, 1.1, 1.7], dtype=np.float32)
    ws = cnn.workspace(plan, V.VDAMP_CNN_WS_TRAIN)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    cnn.train_step(plan, ws, dev_c64(plan, xs), torch.from_numpy(tau).cuda(), torch.from_numpy(s0).cuda(),
                   dev_c64(plan, x0s), 0.0, loss)
    grad = torch.empty(cnn.param_count, dtype=torch.float32, device="cuda")
    after = torch.empty_like(grad)
    cnn.get_params(after, grad)
    torch.cuda.synchronize()
    batch = [(xs[b].astype(np.complex64).astype(np.complex128), tau[b, :plan.nbands].astype(np.float64),
              float(s0[b]), x0s[b].astype(np.complex64).astype(np.complex128)) for b in range(plan.batch)]
    L, g = cr.loss_and_grad(params, batch, bf16=True)
    el = abs(float(loss.item()) - L) / L
    print(f"loss gpu {loss.item():.6e} oracle {L:.6e} rel {el:.2e}")
    assert el < TOL_LOSS
    gg = V.cnn_unflatten(grad.cpu().numpy(), plan.nbands)
    for k in V.CNN_PARAM_ORDER:
        e = rel_l2(gg[k], g[k])
        print(f"grad {k}: rel {e:.2e}")
        assert e < TOL_GRAD, k
    # lr = 0 leaves the parameters unchanged
    assert np.array_equal(after.cpu().numpy(), V.cnn_flatten(params).astype(np.float32))


def test_adam_step_matches_oracle():
    import torch
    from paper_1911_01234_amd import vdamp as V
    s = 2
    params = rand_params(1 + 3 * s, 9)
    plan, cnn = setup(SHAPES[:2], s, params)
    xs = images(SHAPES[:2], 10)
    x0s = [0.8 * x for x in xs]
    tau = taus_for(plan, 11)
    s0 = np.array([1.0, 1.5], dtype=np.float32)
    ws = cnn.workspace(plan, V.VDAMP_CNN_WS_TRAIN)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    lr_ = 1e-3
    args = (dev_c64(plan, xs), torch.from_numpy(tau).cuda(), torch.from_numpy(s0).cuda(), dev_c64(plan, x0s))
    cnn.train_step(plan, ws, *args, lr_, loss)
    cnn.train_step(plan, ws, *args, lr_, loss)
    after = torch.empty(cnn.param_count, dtype=torch.float32, device="cuda")
    cnn.get_params(after)
    torch.cuda.synchronize()
    batch = [(xs[b].astype(np.complex64).astype(np.complex128), tau[b, :plan.nbands].astype(np.float64),
              float(s0[b]), x0s[b].astype(np.complex64).astype(np.complex128)) for b in range(plan.batch)]
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v2 = {k: np.zeros_like(v) for k, v in p.items()}
    for step in (1, 2):
        _, g = cr.loss_and_grad(p, batch, bf16=True)
        p, m, v2 = cr.adam_step(p, g, m, v2, step, lr_)
    got = V.cnn_unflatten(after.cpu().numpy(), plan.nbands)
    for k in V.CNN_PARAM_ORDER:
        d = got[k] - p[k]
        # Adam's early steps move each parameter by about lr; allow a full step of
        # disagreement only where the gradient is tiny (its sign is not determined)
        frac_far = np.mean(np.abs(d) > 0.05 * lr_)
        print(f"adam {k}: max |d| {np.abs(d).max():.2e}, fraction beyond 5% of lr {frac_far:.3f}")
        assert np.abs(d).max() <= 2.05 * lr_ * 2 and frac_far < 0.05, k


def test_wavelet_transform_matches_oracle_and_inverts():
    import torch
    from paper_1911_01234_amd import vdamp as V
    shapes = [(64, 64), (48, 80), (256, 256)]
    s = 3
    plan = V.Plan([a for a, _ in shapes], [b for _, b in shapes], s)
    xs = images(shapes, 12)
    x = dev_c64(plan, xs)
    w = torch.empty_like(x)
    back = torch.empty_like(x)
    plan.vdamp_wavelet(x, w, inverse=False)
    plan.vdamp_wavelet(w, back, inverse=True)
    torch.cuda.synchronize()
    gw = plan.unpack(w.cpu().numpy())
    for b in range(plan.batch):
        ref = o.haar_analysis(xs[b].astype(np.complex64).astype(np.complex128), s)
        assert rel_l2(gw[b], ref) < 1e-6
    assert rel_l2(back.cpu().numpy(), x.cpu().numpy()) < 1e-6


def _learned_inputs(slices, s, params):
    import torch
    from paper_1911_01234_amd import vdamp as V
    plan = V.Plan([sl.y.shape[0] for sl in slices], [sl.y.shape[1] for sl in slices], s)
    cnn = V.Cnn(plan.nbands)
    cnn.set_params(torch.from_numpy(V.cnn_flatten(params).astype(np.float32)).cuda())
    ws = plan.workspace()
    cws = cnn.workspace(plan, V.VDAMP_CNN_WS_SOLVE)
    y, mask, p, sigma2 = V.to_device(plan, slices)
    return plan, cnn, ws, cws, (y, mask, p, sigma2)


def _export(plan, cnn, cws):
    import torch
    n = plan.batch * plan.nbands
    sel = torch.empty(n, dtype=torch.int32, device="cuda")
    sc = torch.empty(n, dtype=torch.float32, device="cuda")
    ac, ss = torch.empty_like(sc), torch.empty_like(sc)
    s0 = torch.empty(plan.batch, dtype=torch.float32, device="cuda")
    cnn.learned_export(plan, cws, sel, s0, sc, ac, ss)
    torch.cuda.synchronize()
    sh = (plan.batch, plan.nbands)
    return dict(sel=sel.cpu().numpy().reshape(sh), s0=s0.cpu().numpy(), sure_cnn=sc.cpu().numpy().reshape(sh),
                alpha_cnn=ac.cpu().numpy().reshape(sh), sure_soft=ss.cpu().numpy().reshape(sh))


def test_identity_network_gives_plain_vdamp_bit_for_bit():
    import torch
    from paper_1911_01234_amd import vdamp as V
    slices, s, _ = synth.workload_single64()
    slices = slices + [synth.workload_single256(4)[0][0]]
    s = 3
    zero = {k: np.zeros_like(v) for k, v in cr.init_params(1 + 3 * s, 0).items()}
    plan, cnn, ws, cws, (y, mask, p, sigma2) = _learned_inputs(slices, s, zero)
    iters = 6
    xl = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    xp = torch.empty_like(xl)
    plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, iters, 17, xl, judge=V.VDAMP_JUDGE_SURE)
    ex = _export(plan, cnn, cws)
    plan.vdamp_solve(ws, y, mask, p, sigma2, iters, xp)
    torch.cuda.synchronize()
    assert ex["sel"].sum() == 0
    assert np.allclose(ex["alpha_cnn"], 1.0, atol=1e-5)
    assert torch.equal(xl, xp)
    for b, sl in enumerate(slices):
        assert abs(ex["s0"][b] - lr.input_scale(sl.y, sl.mask, sl.p)) < 1e-5 * ex["s0"][b]


def test_half_shrink_network_in_every_band_matches_oracle():
    """A nonlinear network with a known map (test_oracle_learned.half_shrink_params; a
    linear one would make the Onsager correction cancel to the BF16 rounding residue alone), used in
    every band for two iterations (the second applies the Onsager correction to the learned output and
    its alpha): x_hat to the FP32 gate 1e-5 (the network's weights are exact in BF16 and
    its activations are rounded at the same points on both sides)."""
    import torch
    from paper_1911_01234_amd import vdamp as V
    from test_oracle_learned import half_shrink_params
    slices, s, _ = synth.workload_single64()
    c, iters = 0.125, 2
    params = half_shrink_params(1 + 3 * s, c)
    plan, cnn, ws, cws, (y, mask, p, sigma2) = _learned_inputs(slices, s, params)
    x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, iters, 23, x, judge=V.VDAMP_JUDGE_NONE)
    ex = _export(plan, cnn, cws)
    torch.cuda.synchronize()
    sl = slices[0]
    ref = lr.vdamp_learned(*fp32_inputs(sl), s, iters, params, seed=23, always=True)
    last = ref["records"][-1]
    assert ex["sel"].sum() == plan.nbands and last["sel"].sum() == plan.nbands
    da = np.abs(ex["alpha_cnn"][0] - last["alpha_cnn"]).max()
    e = rel_l2(plan.unpack(x.cpu().numpy())[0], ref["x_hat"])
    print(f"half-shrink network, {iters} iterations: x_hat rel {e:.2e}, alpha max diff {da:.2e}")
    assert da < 1e-5
    assert e < 1e-5


def test_learned_from_schedule():
    """learned_from >= iters gives vdamp_solve bit for bit; learned_from = 2 of 3 matches
    the oracle's schedule (two iterations of soft thresholding, then the half-shrink
    network in every band) at the FP32 gate 1e-5.  (This network's map is expansive: two
    learned iterations in a row grow the few BF16 roundings that FP32 and FP64 take
    differently to 2e-4; the half-shrink test checks the Onsager correction after a
    learned iteration.)"""
    import torch
    from paper_1911_01234_amd import vdamp as V
    from test_oracle_learned import half_shrink_params
    slices, s, _ = synth.workload_single64()
    params = half_shrink_params(1 + 3 * s, 0.125)
    plan, cnn, ws, cws, (y, mask, p, sigma2) = _learned_inputs(slices, s, params)
    xl = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    xp = torch.empty_like(xl)
    plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, 5, 3, xl, judge=V.VDAMP_JUDGE_NONE, learned_from=5)
    plan.vdamp_solve(ws, y, mask, p, sigma2, 5, xp)
    torch.cuda.synchronize()
    assert torch.equal(xl, xp)
    iters, lf = 3, 2
    plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, iters, 3, xl, judge=V.VDAMP_JUDGE_NONE,
                             learned_from=lf)
    torch.cuda.synchronize()
    sl = slices[0]
    ref = lr.vdamp_learned(*fp32_inputs(sl), s, iters, params, seed=3, always=True, learned_from=lf)
    e = rel_l2(plan.unpack(xl.cpu().numpy())[0], ref["x_hat"])
    print(f"learned_from {lf} of {iters}: x_hat rel {e:.2e}")
    assert e < 1e-5


def test_random_network_judge_values_match_oracle():
    import torch
    from paper_1911_01234_amd import vdamp as V
    slices, s, _ = synth.workload_single64()
    params = rand_params(1 + 3 * s, 31, scale_last=0.3)
    plan, cnn, ws, cws, (y, mask, p, sigma2) = _learned_inputs(slices, s, params)
    x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, 1, 41, x, judge=V.VDAMP_JUDGE_SURE)
    ex = _export(plan, cnn, cws)
    sl = slices[0]
    ref = lr.vdamp_learned(sl.y, sl.mask, sl.p, sl.sigma2, s, 1, params, seed=41)
    rec = ref["records"][0]
    nbs = np.array([(rs.stop - rs.start) * (cs.stop - cs.start) for (rs, cs, _, _) in o.bands(64, 64, s)])
    scale = np.abs(rec["sure_cnn"]) + nbs * rec["tau"]
    d_sc = np.abs(ex["sure_cnn"][0] - rec["sure_cnn"]) / scale
    d_ac = np.abs(ex["alpha_cnn"][0] - rec["alpha_cnn"])
    d_ss = np.abs(ex["sure_soft"][0] - rec["sure_soft"]) / (np.abs(rec["sure_soft"]) + nbs * rec["tau"])
    print(f"judge: sure_cnn {d_sc.max():.2e}, alpha_cnn {d_ac.max():.2e}, sure_soft {d_ss.max():.2e} "
          f"(relative); sel gpu {ex['sel'][0]} oracle {rec['sel']}")
    assert d_sc.max() < 5e-3 and d_ac.max() < 5e-3 and d_ss.max() < 1e-4
    # the choice follows the rule on the exported values
    want = (ex["sure_cnn"][0] < ex["sure_soft"][0]) & (ex["alpha_cnn"][0] <= 1 - 1 / nbs)
    assert np.array_equal(ex["sel"][0].astype(bool), want)


def test_learned_solve_rejects_bad_arguments():
    import torch
    from paper_1911_01234_amd import vdamp as V
    slices, s, _ = synth.workload_single64()
    zero = {k: np.zeros_like(v) for k, v in cr.init_params(1 + 3 * s, 0).items()}
    plan, cnn, ws, cws, (y, mask, p, sigma2) = _learned_inputs(slices, s, zero)
    x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    with pytest.raises(V.VdampError) as e:
        plan.vdamp_solve_learned(cnn, ws, cws[:-256], y, mask, p, sigma2, 2, 1, x)
    assert e.value.status == 4
    with pytest.raises(V.VdampError) as e:
        plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, 2, 1, x, judge=7)
    assert e.value.status == 1
    other = V.Cnn(7)
    with pytest.raises(V.VdampError) as e:
        plan.vdamp_solve_learned(other, ws, cws, y, mask, p, sigma2, 2, 1, x)
    assert e.value.status == 1
    with pytest.raises(V.VdampError) as e:
        plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, 2, 1, x, learned_from=-1)
    assert e.value.status == 1


def test_training_on_vdamp_states_and_learned_solve():
    """Train on plain-VDAMP states of 16 slices (64x64), then solve 8 held-out slices:
    the loss must fall, and the judged learned solve must not lose to plain VDAMP by more
    than 0.1 dB of mean NMSE (the judge keeps soft thresholding wherever the network's
    SURE is not lower)."""
    import torch
    from paper_1911_01234_amd import train as T
    from paper_1911_01234_amd import vdamp as V
    s, K = 3, 30
    tr = [synth.workload_single64(slice_id=i)[0][0] for i in range(1, 17)]
    te = [synth.workload_single64(slice_id=i)[0][0] for i in range(100, 108)]
    plan = V.Plan([64] * len(tr), [64] * len(tr), s)
    ws = plan.workspace()
    y, mask, p, sigma2 = V.to_device(plan, tr)
    cnn = V.Cnn(plan.nbands)
    cnn.set_params(torch.from_numpy(T.init_flat(plan.nbands, 0)).cuda())
    s0 = T.input_scales(plan, cnn, ws, y, mask, p, sigma2)
    pairs = T.make_pairs(plan, ws, y, mask, p, sigma2, (1, 2, 3, 5, 8, 12, 20))
    x0 = torch.from_numpy(plan.pack([sl.x0 for sl in tr], np.complex64)).cuda()
    losses = T.train(cnn, plan, pairs, s0, x0, 420, 1e-3, lr_final=1e-4)
    first, last = losses[:7].mean(), losses[-7:].mean()
    print(f"training loss {first:.4e} -> {last:.4e}")
    assert np.all(np.isfinite(losses)) and last < 0.7 * first

    plan2 = V.Plan([64] * len(te), [64] * len(te), s)
    ws2 = plan2.workspace()
    cws2 = cnn.workspace(plan2, V.VDAMP_CNN_WS_SOLVE)
    y2, m2, p2, s2 = V.to_device(plan2, te)
    xp = torch.empty(plan2.ntot, dtype=torch.complex64, device="cuda")
    xl = torch.empty_like(xp)
    plan2.vdamp_solve(ws2, y2, m2, p2, s2, K, xp)
    plan2.vdamp_solve_learned(cnn, ws2, cws2, y2, m2, p2, s2, K, 5, xl)
    ex = _export(plan2, cnn, cws2)
    torch.cuda.synchronize()
    gp, gl = plan2.unpack(xp.cpu().numpy()), plan2.unpack(xl.cpu().numpy())
    np_ = np.mean([o.nmse_db(gp[b], te[b].x0) for b in range(len(te))])
    nl = np.mean([o.nmse_db(gl[b], te[b].x0) for b in range(len(te))])
    print(f"held-out mean NMSE: plain {np_:.3f} dB, learned {nl:.3f} dB; "
          f"learned bands at the last iteration: {ex['sel'].sum(axis=0)}")
    assert np.isfinite(nl) and nl <= np_ + 0.1


def test_forward_and_jvp_persistent_tile_loop():
    """33 slices of 64x64 give 528 tiles, more than the 512 persistent convolution
    workgroups: workgroups 0..15 run a second tile after prefetching its halo during the
    first.  The slices holding the first and the last tiles are compared with the oracle
    at the tolerances of test_forward_and_jvp_match_oracle."""
    import torch
    from paper_1911_01234_amd import vdamp as V
    s = 3
    shapes = [(64, 64)] * 33
    params = rand_params(1 + 3 * s, 41)
    plan, cnn = setup(shapes, s, params)
    xs = images(shapes, 42)
    vs = images(shapes, 43)
    tau = taus_for(plan, 44)
    s0 = np.linspace(0.5, 2.0, plan.batch).astype(np.float32)
    ws = cnn.workspace(plan, V.VDAMP_CNN_WS_FORWARD)
    x, v = dev_c64(plan, xs), dev_c64(plan, vs)
    xo, jo = torch.empty_like(x), torch.empty_like(x)
    cnn.forward(plan, ws, x, torch.from_numpy(tau).cuda(), torch.from_numpy(s0).cuda(), xo, v, jo)
    torch.cuda.synchronize()
    g_out, g_jvp = plan.unpack(xo.cpu().numpy()), plan.unpack(jo.cpu().numpy())
    for b in (0, 16, 32):
        xq = xs[b].astype(np.complex64).astype(np.complex128)
        vq = vs[b].astype(np.complex64).astype(np.complex128)
        t = tau[b, :plan.nbands].astype(np.float64)
        ref = cr.forward(params, xq, t, float(s0[b]), bf16=True)
        refj = cr.jvp(params, xq, t, float(s0[b]), vq, bf16=True)
        e = rel_l2(xq - g_out[b], xq - ref)
        dj, wj = vq - g_jvp[b], vq - refj
        ej = rel_l2(dj, wj)
        far = np.mean(np.abs(dj - wj) > 1e-2 * np.sqrt(np.mean(np.abs(wj) ** 2)))
        print(f"slice {b} (tiles {16 * b}..{16 * b + 15}): residual rel {e:.2e}, jvp rel {ej:.2e}, "
              f"far fraction {far:.1e}")
        assert e < TOL_OUT and ej < 3e-2 and far <= jvp_far_limit(shapes[b]), b


MANY_TILES = [(64, 64)] * 35 + [(64, 128), (128, 64)]  # 624 tiles: 512 workgroups, 1-2 tiles each


def test_gradient_over_many_tiles_matches_oracle():
    """624 tiles against 512 weight-gradient workgroups: workgroups 0..111 accumulate two
    tiles' partial products before the fixed-order reduction.  Loss and gradient against
    the oracle over the whole batch."""
    import torch
    from paper_1911_01234_amd import vdamp as V
    s = 3
    params = rand_params(1 + 3 * s, 51)
    plan, cnn = setup(MANY_TILES, s, params)
    xs = images(MANY_TILES, 52)
    x0s = [x + 0.3 * im for x, im in zip(xs, images(MANY_TILES, 53))]
    tau = taus_for(plan, 54)
    s0 = np.linspace(0.6, 1.8, plan.batch).astype(np.float32)
    ws = cnn.workspace(plan, V.VDAMP_CNN_WS_TRAIN)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    cnn.train_step(plan, ws, dev_c64(plan, xs), torch.from_numpy(tau).cuda(), torch.from_numpy(s0).cuda(),
                   dev_c64(plan, x0s), 0.0, loss)
    grad = torch.empty(cnn.param_count, dtype=torch.float32, device="cuda")
    cnn.get_params(None, grad)
    torch.cuda.synchronize()
    batch = [(xs[b].astype(np.complex64).astype(np.complex128), tau[b, :plan.nbands].astype(np.float64),
              float(s0[b]), x0s[b].astype(np.complex64).astype(np.complex128)) for b in range(plan.batch)]
    L, g = cr.loss_and_grad(params, batch, bf16=True)
    el = abs(float(loss.item()) - L) / L
    print(f"{plan.batch} slices, {sum(h * w for h, w in MANY_TILES) // 256} tiles: loss rel {el:.2e}")
    assert el < TOL_LOSS
    gg = V.cnn_unflatten(grad.cpu().numpy(), plan.nbands)
    for k in V.CNN_PARAM_ORDER:
        e = rel_l2(gg[k], g[k])
        print(f"grad {k}: rel {e:.2e}")
        assert e < TOL_GRAD, k


def test_adam_over_many_tiles_matches_oracle():
    """Two Adam steps over the 624-tile batch (multi-tile gradient partials) against the
    oracle's two steps, at the tolerances of test_adam_step_matches_oracle."""
    import torch
    from paper_1911_01234_amd import vdamp as V
    s = 3
    params = rand_params(1 + 3 * s, 61)
    plan, cnn = setup(MANY_TILES, s, params)
    xs = images(MANY_TILES, 62)
    x0s = [0.8 * x for x in xs]
    tau = taus_for(plan, 63)
    s0 = np.linspace(0.8, 1.4, plan.batch).astype(np.float32)
    ws = cnn.workspace(plan, V.VDAMP_CNN_WS_TRAIN)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    lr_ = 1e-3
    args = (dev_c64(plan, xs), torch.from_numpy(tau).cuda(), torch.from_numpy(s0).cuda(), dev_c64(plan, x0s))
    cnn.train_step(plan, ws, *args, lr_, loss)
    cnn.train_step(plan, ws, *args, lr_, loss)
    after = torch.empty(cnn.param_count, dtype=torch.float32, device="cuda")
    cnn.get_params(after)
    torch.cuda.synchronize()
    batch = [(xs[b].astype(np.complex64).astype(np.complex128), tau[b, :plan.nbands].astype(np.float64),
              float(s0[b]), x0s[b].astype(np.complex64).astype(np.complex128)) for b in range(plan.batch)]
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v2 = {k: np.zeros_like(v) for k, v in p.items()}
    for step in (1, 2):
        _, g = cr.loss_and_grad(p, batch, bf16=True)
        p, m, v2 = cr.adam_step(p, g, m, v2, step, lr_)
    got = V.cnn_unflatten(after.cpu().numpy(), plan.nbands)
    for k in V.CNN_PARAM_ORDER:
        d = got[k] - p[k]
        frac_far = np.mean(np.abs(d) > 0.05 * lr_)
        print(f"adam {k}: max |d| {np.abs(d).max():.2e}, fraction beyond 5% of lr {frac_far:.3f}")
        assert np.abs(d).max() <= 2.05 * lr_ * 2 and frac_far < 0.05, k


def _learned_against_oracle(slices, s, params, iters, seed, judge, what):
    import torch
    from paper_1911_01234_amd import vdamp as V
    plan, cnn, ws, cws, (y, mask, p, sigma2) = _learned_inputs(slices, s, params)
    x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    trace = torch.empty(iters * plan.batch * plan.nbands * 3, dtype=torch.float32, device="cuda")
    plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, iters, seed, x, trace, judge=judge)
    ex = _export(plan, cnn, cws)
    torch.cuda.synchronize()
    gx = plan.unpack(x.cpu().numpy())
    nbs = np.array([(rs.stop - rs.start) * (cs.stop - cs.start)
                    for (rs, cs, _, _) in o.bands(slices[0].y.shape[0], slices[0].y.shape[1], s)])
    for b, sl in enumerate(slices):
        ref = lr.vdamp_learned(*fp32_inputs(sl), s, iters, params, seed=seed, slice_id=b,
                               always=(judge == V.VDAMP_JUDGE_NONE))
        rec = ref["records"][-1]
        scale = np.abs(rec["sure_cnn"]) + nbs * rec["tau"]
        d_sc = (np.abs(ex["sure_cnn"][b] - rec["sure_cnn"]) / scale).max()
        d_ac = np.abs(ex["alpha_cnn"][b] - rec["alpha_cnn"]).max()
        d_ss = (np.abs(ex["sure_soft"][b] - rec["sure_soft"]) / (np.abs(rec["sure_soft"]) + nbs * rec["tau"])).max()
        e = rel_l2(gx[b], ref["x_hat"])
        print(f"{what} slice {b}: sure_cnn {d_sc:.2e}, alpha_cnn {d_ac:.2e}, sure_soft {d_ss:.2e}, "
              f"x_hat rel {e:.2e}; sel gpu {ex['sel'][b]} oracle {rec['sel']}")
        assert d_sc < 5e-3 and d_ac < 5e-3 and d_ss < 1e-4, b
        assert np.array_equal(ex["sel"][b], rec["sel"]), b
        assert e < TOL_OUT, b


def test_learned_iteration_at_256():
    """One learned iteration (the network in every band where alpha allows it) on two
    256x256 slices of the benchmark's recipe (256 tiles each, 512 in the batch), with a
    random network: the judge's values, the choice per band and x_hat against the
    oracle; x_hat holds the network's BF16 output, so its tolerance is the network's
    (5e-3).  (A second learned iteration starts from the first one's BF16 output, which
    both sides round differently at a few elements: its comparison would measure that
    difference grown through the Onsager correction; the 64x64 half-shrink test covers
    the Onsager correction with the learned output at the FP32 gate.)"""
    from paper_1911_01234_amd import vdamp as V
    slices = synth.workload_batch256(2, cfg_id=41)[0]
    s = 4
    params = rand_params(1 + 3 * s, 71, scale_last=0.3)
    _learned_against_oracle(slices, s, params, 1, 77, V.VDAMP_JUDGE_NONE, "256x256")


def test_learned_iteration_at_512_textured():
    """One judged learned iteration on a 512x512 textured slice at R = 8 (1024 tiles,
    two per convolution workgroup) against the oracle."""
    from paper_1911_01234_amd import vdamp as V
    slices = synth.workload_batch512(1)[0]
    s = 4
    params = rand_params(1 + 3 * s, 81, scale_last=0.3)
    _learned_against_oracle(slices, s, params, 1, 88, V.VDAMP_JUDGE_SURE, "512x512")

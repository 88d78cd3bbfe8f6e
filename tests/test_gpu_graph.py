"""hipGraph replays (VDAMP_FLAG_USE_GRAPH) of the learned solve and of FISTA against the
same calls launched eagerly: every replay, with eager work of the program and
synchronisations between replays, must reproduce the eager result bit for bit (the
plain solve has the same test in test_gpu_parity.py)."""
import numpy as np
import pytest

from paper_1911_01234_amd import synth

from test_gpu_cnn import rand_params

pytestmark = pytest.mark.gpu


def _slices():
    return [synth.make_slice(9, i, 64, 64, 8, 4.0, 4.0, 8, 30.0) for i in range(2)], 3


def test_learned_solve_graph_replays_match_eager_bitwise():
    import torch
    from paper_1911_01234_amd import vdamp as V
    slices, s = _slices()
    params = rand_params(1 + 3 * s, 12, scale_last=0.3)
    flat = torch.from_numpy(V.cnn_flatten(params).astype(np.float32)).cuda()
    stream = torch.cuda.Stream()
    out = {}
    for name, flags in (("eager", 0), ("graph", V.VDAMP_FLAG_USE_GRAPH)):
        plan = V.Plan([64, 64], [64, 64], s, flags)
        cnn = V.Cnn(plan.nbands)
        cnn.set_params(flat)
        ws = plan.workspace()
        cws = cnn.workspace(plan, V.VDAMP_CNN_WS_SOLVE)
        y, mask, p, sigma2 = V.to_device(plan, slices)
        x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
        reps = []
        for rep in range(3 if flags else 1):
            x.fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, 4, 7, x, learned_from=1,
                                         judge=V.VDAMP_JUDGE_SURE, stream=stream)
            stream.synchronize()
            reps.append(x.cpu().numpy().copy())
        out[name] = reps
        plan.close()
    assert np.all(np.isfinite(out["eager"][0]))
    for rep, got in enumerate(out["graph"]):
        assert np.array_equal(got, out["eager"][0]), rep


def test_fista_graph_replays_match_eager_bitwise():
    import torch
    from paper_1911_01234_amd import vdamp as V
    slices, s = _slices()
    stream = torch.cuda.Stream()
    out = {}
    for name, flags in (("eager", 0), ("graph", V.VDAMP_FLAG_USE_GRAPH)):
        plan = V.Plan([64, 64], [64, 64], s, flags)
        ws = plan.workspace()
        y, mask, _, _ = V.to_device(plan, slices)
        lam = torch.tensor([0.01, 0.02], dtype=torch.float32, device="cuda")
        x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
        reps = []
        for rep in range(3 if flags else 1):
            x.fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                plan.fista_solve(ws, y, mask, lam, 6, x, stream=stream)
            stream.synchronize()
            reps.append(x.cpu().numpy().copy())
        out[name] = reps
        plan.close()
    assert np.all(np.isfinite(out["eager"][0]))
    for rep, got in enumerate(out["graph"]):
        assert np.array_equal(got, out["eager"][0]), rep


def _learned_eager(slices, s, flat, seed, judge):
    import torch
    from paper_1911_01234_amd import vdamp as V
    plan = V.Plan([64, 64], [64, 64], s)
    cnn = V.Cnn(plan.nbands)
    cnn.set_params(flat)
    ws = plan.workspace()
    cws = cnn.workspace(plan, V.VDAMP_CNN_WS_SOLVE)
    y, mask, p, sigma2 = V.to_device(plan, slices)
    x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, 3, seed, x, judge=judge)
    torch.cuda.synchronize()
    out = x.cpu().numpy().copy()
    cnn.close()
    plan.close()
    return out


def test_learned_graph_rekeyed_when_denoiser_recreated_or_seed_judge_change():
    """The captured learned solve holds the denoiser's device buffers: destroying the
    denoiser and creating another one (which may reuse the handle's host address)
    between two graph solves must re-capture, as must a change of seed or judge (also
    the pair seed ^ 2^63 with the other judge).  Every graph result equals the eager one."""
    import torch
    from paper_1911_01234_amd import vdamp as V
    slices, s = _slices()
    flats = [torch.from_numpy(V.cnn_flatten(rand_params(1 + 3 * s, seed, scale_last=0.3)).astype(np.float32)).cuda()
             for seed in (21, 22)]
    plan = V.Plan([64, 64], [64, 64], s, V.VDAMP_FLAG_USE_GRAPH)
    ws = plan.workspace()
    y, mask, p, sigma2 = V.to_device(plan, slices)
    x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    stream = torch.cuda.Stream()
    cws = None
    cases = [(0, 5, V.VDAMP_JUDGE_SURE), (1, 5, V.VDAMP_JUDGE_SURE), (1, 5 ^ (1 << 63), V.VDAMP_JUDGE_NONE),
             (1, 5, V.VDAMP_JUDGE_NONE)]
    for net, seed, judge in cases:
        cnn = V.Cnn(plan.nbands)  # a fresh denoiser for every case, the previous one destroyed
        cnn.set_params(flats[net])
        if cws is None:
            cws = cnn.workspace(plan, V.VDAMP_CNN_WS_SOLVE)
        x.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            plan.vdamp_solve_learned(cnn, ws, cws, y, mask, p, sigma2, 3, seed, x, judge=judge, stream=stream)
        stream.synchronize()
        got = x.cpu().numpy().copy()
        cnn.close()
        want = _learned_eager(slices, s, flats[net], seed, judge)
        assert np.all(np.isfinite(want))
        assert np.array_equal(got, want), (net, seed, judge)


def test_resume_and_fista_objective_graph_replays_match_eager_bitwise():
    """vdamp_solve_resume with a monitor output and fista_solve with its objective output,
    captured and replayed three times, against eager calls."""
    import torch
    from paper_1911_01234_amd import vdamp as V
    slices, s = _slices()
    stream = torch.cuda.Stream()
    out = {}
    for name, flags in (("eager", 0), ("graph", V.VDAMP_FLAG_USE_GRAPH)):
        plan = V.Plan([64, 64], [64, 64], s, flags)
        planf = V.Plan([64, 64], [64, 64], s, flags)  # its own graph cache, so both replay
        ws = plan.workspace()
        wsf = planf.workspace()
        y, mask, p, sigma2 = V.to_device(plan, slices)
        r = (torch.randn(plan.ntot, dtype=torch.complex64, generator=torch.Generator().manual_seed(3)) * 0.1).cuda()
        th = torch.full((plan.batch * plan.nbands,), 0.05, dtype=torch.float32, device="cuda")
        al = torch.full_like(th, 0.3)
        lam = torch.tensor([0.01, 0.02], dtype=torch.float32, device="cuda")
        x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
        mon = torch.empty(4 * plan.ntot, dtype=torch.complex64, device="cuda")
        obj = torch.empty(6 * plan.batch, dtype=torch.float32, device="cuda")
        xf = torch.empty_like(x)
        reps = []
        for rep in range(3 if flags else 1):
            for t in (x, mon, xf):
                t.fill_(float("nan"))
            obj.fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                plan.vdamp_solve_resume(ws, y, mask, p, sigma2, r, th, None, al, 4, x, None, mon, stream=stream)
            stream.synchronize()
            a = (x.cpu().numpy().copy(), mon.cpu().numpy().copy())
            with torch.cuda.stream(stream):
                planf.fista_solve(wsf, y, mask, lam, 6, xf, objective=obj, stream=stream)
            stream.synchronize()
            reps.append(a + (xf.cpu().numpy().copy(), obj.cpu().numpy().copy()))
        out[name] = reps
        plan.close()
        planf.close()
    for arr in out["eager"][0]:
        assert np.all(np.isfinite(arr))
    for rep, got in enumerate(out["graph"]):
        for a, b in zip(got, out["eager"][0]):
            assert np.array_equal(a, b), rep


def test_mixed_batch_graph_replays_match_eager_bitwise():
    """The ragged batch of 512 slices (128 each of 128^2, 192^2, 256^2 and 320^2, R 4-10,
    25-45 dB, 50 iterations) captured in one hipGraph, whose passes fork their size
    groups onto parallel branches: three replays, with eager work of the program between
    them, against the eager solve."""
    import torch
    from paper_1911_01234_amd import vdamp as V
    slices, s, K = synth.workload_mixed()
    ny = [sl.y.shape[0] for sl in slices]
    nx = [sl.y.shape[1] for sl in slices]
    stream = torch.cuda.Stream()
    out = {}
    for name, flags in (("eager", 0), ("graph", V.VDAMP_FLAG_USE_GRAPH)):
        plan = V.Plan(ny, nx, s, flags)
        ws = plan.workspace()
        y, mask, p, sigma2 = V.to_device(plan, slices)
        x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
        tr = torch.empty(K * plan.batch * plan.nbands * 3, dtype=torch.float32, device="cuda")
        reps = []
        for rep in range(3 if flags else 1):
            x.fill_(float("nan"))
            tr.fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                plan.vdamp_solve(ws, y, mask, p, sigma2, K, x, tr, stream=stream)
            stream.synchronize()
            reps.append((x.cpu().numpy().copy(), tr.cpu().numpy().copy()))
        out[name] = reps
        plan.close()
    assert np.all(np.isfinite(out["eager"][0][0])) and np.all(np.isfinite(out["eager"][0][1]))
    for rep, (gx, gt) in enumerate(out["graph"]):
        assert np.array_equal(gx, out["eager"][0][0]), rep
        assert np.array_equal(gt, out["eager"][0][1]), rep

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

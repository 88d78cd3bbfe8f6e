"""vdamp_solve_noalloc (the entry point for callers that cannot allocate) through the C
ABI against vdamp_solve with a caller workspace: two calls in a row, the second with a
smaller plan, must give the same results bit for bit (the same kernels run on the same
inputs; only the workspace differs), and a plan whose workspace exceeds the library's
array is refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

from paper_1911_01234_amd import synth

pytestmark = pytest.mark.gpu


def _solve_both(slices, s, K):
    import torch
    from paper_1911_01234_amd import vdamp as V
    lib = V.load_library()
    plan = V.Plan([sl.y.shape[0] for sl in slices], [sl.y.shape[1] for sl in slices], s)
    assert plan.workspace_bytes <= V.VDAMP_NOALLOC_MAX_WORKSPACE
    y, mask, p, sigma2 = V.to_device(plan, slices)
    x_ref = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    t_ref = torch.empty(K * plan.batch * plan.nbands * 3, dtype=torch.float32, device="cuda")
    plan.vdamp_solve(plan.workspace(), y, mask, p, sigma2, K, x_ref, t_ref)
    x = torch.full((plan.ntot,), float("nan"), dtype=torch.complex64, device="cuda")
    t = torch.full_like(t_ref, float("nan"))
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.vdamp_solve_noalloc(plan._h, stream, y.data_ptr(), mask.data_ptr(), p.data_ptr(),
                                 sigma2.data_ptr(), K, x.data_ptr(), t.data_ptr())
    assert st == 0, lib.vdamp_last_error().decode()
    torch.cuda.synchronize()
    assert torch.equal(x, x_ref)
    assert torch.equal(t, t_ref)
    plan.close()


def test_noalloc_matches_workspace_solve_twice_smaller_second():
    first = [synth.workload_single256(R)[0][0] for R in (4.0, 6.0, 8.0)] + \
            [synth.make_slice(3, 5, 192, 192, 16, 6.0, 6.0, 16, 35.0)]
    _solve_both(first, 4, 12)
    _solve_both(synth.workload_single64()[0], 3, 8)


def test_noalloc_refuses_a_plan_beyond_its_array():
    import torch
    from paper_1911_01234_amd import vdamp as V
    lib = V.load_library()
    plan = V.Plan([256] * 40, [256] * 40, 4)  # 2.6 M pixels: about 74 MB of workspace
    assert plan.workspace_bytes > V.VDAMP_NOALLOC_MAX_WORKSPACE
    x = torch.empty(plan.ntot, dtype=torch.complex64, device="cuda")
    d = torch.empty(plan.ntot, dtype=torch.float32, device="cuda")
    st = lib.vdamp_solve_noalloc(plan._h, None, x.data_ptr(), d.data_ptr(), d.data_ptr(), d.data_ptr(), 2,
                                 x.data_ptr(), None)
    assert st == 4 and b"vdamp_solve_noalloc" in lib.vdamp_last_error()

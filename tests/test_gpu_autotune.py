"""Plan-time tuning (VDAMP_FLAG_AUTOTUNE) and the plan description.

The tuner picks, per size group, between kernels that compute the same transforms
(four-step register FFT or in-LDS Stockham FFT) and the same threshold search (size
classes that differ only in how the FP64 walk sums are grouped).  A tuned plan must
therefore solve to the default plan's result up to FP32 rounding, and both follow the
oracle (Algorithm 1 in FP64) on the same seeded inputs."""
import numpy as np
import pytest

from oracle import vdamp_ref as o
from paper_1911_01234_amd import synth

from gpu_helpers import rel_l2, run_vdamp

pytestmark = pytest.mark.gpu


def test_describe_default_plan():
    from paper_1911_01234_amd import vdamp as V
    plan = V.Plan([256, 320], [256, 320], 4)
    d = plan.describe()
    print(d)
    assert "slices 2, levels 4" in d
    assert "rows nx=320" in d and "rows nx=256" in d and "cols ny=256" in d
    assert "four-step M=16" in d and "four-step M=20" in d
    assert "sure class 3: 3 bands" in d  # the three 160x160 bands of the 320 slice
    assert "autotune" not in d
    plan.close()


def test_autotuned_plan_matches_default_and_oracle():
    """A tuned plan of the mixed batch (2 slices each of 128^2 .. 320^2): its x_hat after
    two iterations within 1e-5 of the default plan's (different FFT algorithms and
    threshold-search groupings, the same arithmetic up to FP32 rounding), and, for every
    slice, one step from the oracle's FP32-rounded state at k = 0 and 1 at the parity gate
    (r, tau, x_hat to 1e-5; theta and alpha to the tolerances the iterate's implies)."""
    from paper_1911_01234_amd import vdamp as V
    from gpu_helpers import fp32_state, run_resume
    from test_gpu_parity import TOL_ITER, one_step_check, oracle_run
    slices, s, _ = synth.workload_mixed(n_per_size=2)
    K = 2
    g0 = run_vdamp(slices, s, K)
    g1 = run_vdamp(slices, s, K, flags=V.VDAMP_FLAG_AUTOTUNE)
    plan = g1["plan"]
    d = plan.describe()
    print(d)
    assert "autotune:" in d
    for n in (128, 192, 256, 320):
        assert f"rows nx={n} (four-step" in d and f"cols ny={n} (four-step" in d
    assert "sure N_b=16384 (class 2" in d  # the 256 slices' finest bands: classes 2 and 3
    worst = 0.0
    for i in range(len(slices)):
        e = rel_l2(g1["x_hat"][i], g0["x_hat"][i])
        worst = max(worst, e)
        assert e <= TOL_ITER, (i, slices[i].y.shape, e)
    print(f"tuned vs default x_hat: worst rel L2 {worst:.2e}")
    trajs = [oracle_run(sl, s, 3) for sl in slices]
    for k in (0, 1):
        states = {b: fp32_state(tr["r"][k], tr["theta"][k], tr["alpha"][k]) for b, tr in enumerate(trajs)}
        g = run_resume(plan, slices, states, 1)
        for b, sl in enumerate(slices):
            e, et, fl = one_step_check(sl, s, states[b], g, b, k, what=f"tuned slice {b}")
            print(f"k={k} slice {b} {sl.y.shape}: r {e:.2e} tau {et:.2e} flips {fl}")

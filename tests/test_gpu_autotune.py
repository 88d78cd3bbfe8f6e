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
    from paper_1911_01234_amd import vdamp as V
    slices, s, _ = synth.workload_mixed(n_per_size=2)
    K = 2
    g0 = run_vdamp(slices, s, K)
    g1 = run_vdamp(slices, s, K, flags=V.VDAMP_FLAG_AUTOTUNE)
    d = g1["plan"].describe()
    print(d)
    assert "autotune:" in d
    for n in (128, 192, 256, 320):
        assert f"rows nx={n} (four-step" in d and f"cols ny={n} (four-step" in d
    assert "sure N_b=16384 (class 2" in d  # the 256 slices' finest bands: classes 2 and 3
    worst = 0.0
    for i in range(len(slices)):
        e = rel_l2(g1["x_hat"][i], g0["x_hat"][i])
        worst = max(worst, e)
        assert e <= 1e-4, (i, slices[i].y.shape, e)
    print(f"tuned vs default x_hat: worst rel L2 {worst:.2e}")
    for i in range(len(slices)):
        sl = slices[i]
        ref = o.vdamp(sl.y, sl.mask, sl.p, sl.sigma2, s, K)
        et = np.max(np.abs(g1["trace"][:, i, :, 0] - ref["tau"]) / ref["tau"])
        assert et <= 1e-4, (i, sl.y.shape, et)

"""Whole-iteration pins of the oracle on the 256x256 recipe (Section 3 experiments):
colored state evolution (predicted tau vs measured per-subband error, the analogue of
the per-subband NMSE figure), Gaussianity of the effective noise (the analogue of the
quantile-quantile figure), and VDAMP ahead of FISTA (the abstract's claim)."""
import numpy as np
import pytest
from scipy import stats

from oracle import vdamp_ref as o
from paper_1911_01234_amd import synth


def _run(R, iters):
    sl, s, _ = synth.workload_single256(R)
    sl = sl[0]
    out = o.vdamp(sl.y, sl.mask, sl.p, sl.sigma2, s, iters, record=True)
    return sl, s, out


@pytest.mark.parametrize("R", [4.0, 6.0, 8.0])
def test_colored_state_evolution(R):
    """r_k = w0 + CN(0, Sigma_k^2) with Sigma diagonal, constant per subband (eqs. 5-6),
    and tau_k tracks that variance: |10 log10(N_b tau_b) - 10 log10 ||r_b - w0_b||^2|
    stays small for k = 0..20.  Under the model ||r_b - w0_b||^2 / tau_b is a sum of N_b
    unit-mean exponentials, whose relative standard deviation is 1/sqrt(N_b), i.e.
    (10/ln 10)/sqrt(N_b) dB; the bound for bands of N_b >= 1024 coefficients is four of
    those (0.54 dB at 1024, 0.27 dB at 4096, 0.14 dB at 16384), and 1.5 dB for the
    smaller, signal-dominated bands.  The measured deviations scale as 1/sqrt(N_b)
    (about 0.5, 0.17 and 0.07 dB at the three sizes), the signature of that sampling
    spread rather than of a bias."""
    sl, s, out = _run(R, 21)
    ny, nx = sl.y.shape
    w0 = o.haar_analysis(sl.x0, s)
    bl = o.bands(ny, nx, s)
    Nb = np.array([(rs.stop - rs.start) * (cs.stop - cs.start) for (rs, cs, _, _) in bl])
    for k, r in enumerate(out["r"]):
        err = np.array([np.sum(np.abs(r[rs, cs] - w0[rs, cs]) ** 2) for (rs, cs, _, _) in bl])
        dev = np.abs(10 * np.log10(Nb * out["tau"][k]) - 10 * np.log10(err))
        tol = np.where(Nb >= 1024, 4.0 * (10.0 / np.log(10.0)) / np.sqrt(Nb), 1.5)
        assert (dev <= tol).all(), (k, dev)


def test_effective_noise_is_gaussian():
    sl, s, out = _run(8.0, 3)
    ny, nx = sl.y.shape
    w0 = o.haar_analysis(sl.x0, s)
    for k in range(3):
        r = out["r"][k]
        for b, (rs, cs, _, _) in enumerate(o.bands(ny, nx, s)):
            if (rs.stop - rs.start) * (cs.stop - cs.start) < 4096:
                continue
            e = (r[rs, cs] - w0[rs, cs]).ravel() / np.sqrt(out["tau"][k][b] / 2)
            assert stats.kstest(e.real, "norm").statistic <= 0.05
            assert stats.kstest(e.imag, "norm").statistic <= 0.05


@pytest.mark.slow
@pytest.mark.parametrize("R", [4.0, 6.0, 8.0])
def test_vdamp_converges_faster_than_fista(R):
    """At equal compute time VDAMP is ahead of FISTA (abstract; Section 3).  The paper's
    per-iteration times are 0.091 s (VDAMP) and 0.065 s (FISTA), so 10 VDAMP iterations
    cost about 14 FISTA iterations.  FISTA gets its best lambda for that budget from
    the sweep lambda_max 10^(-j/4), j = 4..20, chosen with the ground truth as in the
    paper's exhaustive search.  (With a lambda tuned on the ground truth for long runs,
    FISTA's final NMSE on these phantoms is close to VDAMP's: that comparison is
    reported, not asserted.)"""
    sl, s, _ = synth.workload_single256(R)
    sl = sl[0]
    v = o.vdamp(sl.y, sl.mask, sl.p, sl.sigma2, s, 10)
    nv = o.nmse_db(v["x_hat"], sl.x0)
    lam_max = np.abs(o.haar_analysis(o.ifft2u(sl.y), s)).max()
    best = np.inf
    for j in range(4, 21):
        f = o.fista(sl.y, sl.mask, lam_max * 10 ** (-j / 4), s, 14)
        best = min(best, o.nmse_db(f["x_hat"], sl.x0))
    assert nv < best - 2.0, (nv, best)

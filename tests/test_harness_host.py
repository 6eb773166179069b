"""Host-side parts of the Section 5.2 and Section 6.3 harnesses (no GPU):
the parameter grids are the paper's, and the curve sampling is what the
summaries print."""
import pytest

pytest.importorskip("torch")

from paper_2602_17494_amd import quality as q
from paper_2602_17494_amd import validate as v


def test_parameter_grids_are_the_papers():
    assert q.DELTAS == (0.001, 0.002, 0.005, 0.01, 0.02, 0.04, 0.08, 0.15, 0.3, 0.6, 1.2, 2.5, 5.0, 10.0)
    # IRV2: 1e-6, 3e-6, ..., 3e2, 1e3
    assert len(q.ALPHAS_IRV2) == 19
    assert q.ALPHAS_IRV2[0] == pytest.approx(1e-6) and q.ALPHAS_IRV2[-1] == pytest.approx(1e3)
    assert all(b / a == pytest.approx(3.0) or b / a == pytest.approx(10.0 / 3.0)
               for a, b in zip(q.ALPHAS_IRV2, q.ALPHAS_IRV2[1:]))
    # IRV1: 1/30, 1/10, 1/3, 1, ..., 1e3, 1e4/3
    assert len(q.ALPHAS_IRV1) == 11
    assert q.ALPHAS_IRV1[0] == pytest.approx(1 / 30) and q.ALPHAS_IRV1[-1] == pytest.approx(1e4 / 3)
    assert q.EPS_IRV1 == (10.0, 1.0, 0.1, 1e-2, 1e-3, 1e-4, 1e-7, 1e-10, 1e-13)


def test_curve_samples():
    assert v._samples(0) == [0]
    assert v._samples(7) == [0, 1, 2, 5, 7]
    assert v._samples(2000) == [0, 1, 2, 5, 10, 20, 50, 100, 200, 500, 1000, 2000]


def test_summary_subtracts_the_reference_energy():
    res = {"tfs": {"ref_energy": 1.0, "dd": [5.0, 3.0, 2.0]}, "seconds": 0.0}
    for name in ("irv2", "irv1"):
        res[name] = {"ref_energy": 2.0, "dd_tau_dd": [4.0, 3.0, 1.5], "dd_tau_ref": [4.0, 3.0, 2.5],
                     "image_maxabs_dd_vs_ref": 0.1, "image_psnr_dd_vs_ref": 20.0}
    s = v.summary(res)
    assert s["tfs_dd"] == {0: 4.0, 1: 2.0, 2: 1.0}
    assert s["irv2_dd_tau_dd"][2] == -0.5 and s["irv1_dd_tau_ref"][2] == 0.5

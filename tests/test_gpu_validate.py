"""The per-sweep energy history (tvs_energy_history) and the domain-
decomposition validation protocol of Section 6.3 (paper_2602_17494_amd.validate)
through the C-ABI.

* The history of a 3 x 3 Schwarz solve (shared stripes of 4 rows and 3
  columns, alpha-hat = 0.25, the paper's validation layout) equals the FP64
  oracle's energy after every sweep, for both steps, to 1e-10 relative.
* The protocol on a small image: the DD energies of Step 1 approach the
  single-domain reference energy; Step 2 fed the reference tangent field
  approaches the reference Step-2 energy, closer than when fed the DD
  tangent field (the perturbed problem the paper describes)."""
import numpy as np
import pytest

import synth
from oracle import schwarz as osw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
LAY = (3, 3, 4, 3)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_17494_amd import Context
    c = Context(0)
    yield c
    c.close()


def test_energy_history_matches_oracle(ctx):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    n2, n1, sweeps, inner = 40, 60, 6, 10
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 9)
    d0 = torch.tensor(d64, device=DEV)
    prm, L, its = make_params(0.15, 10.0), make_layout(*LAY, 0.25), make_iters(sweeps, inner)
    assert ctx.energy_history() == []
    tau, _ = ctx.step1(d0, prm, L, its)
    h1 = ctx.energy_history()
    ctx.step2(d0, tau, prm, L, its)
    h2 = ctx.energy_history()
    tau_o, _, o1 = osw.step1_schwarz(d64, 0.15, osw.Layout(n2, n1, *LAY, step=1), sweeps, inner)
    _, _, o2 = osw.step2_schwarz(d64, tau_o, 10.0, osw.Layout(n2, n1, *LAY, step=2), sweeps, inner)
    assert len(h1) == sweeps + 1 and len(h2) == sweeps + 1
    # the oracle records the energy after each sweep; entry 0 is D(p^0 = 0)
    np.testing.assert_allclose(h1[1:], o1, rtol=1e-10)
    np.testing.assert_allclose(h2[1:], o2, rtol=1e-10)
    # a call without statistics leaves no history
    ctx.step1(d0, prm, L, its, stats=False)
    assert ctx.energy_history() == []


def test_validation_protocol_small(ctx):
    from paper_2602_17494_amd.validate import protocol, summary
    _, noisy = synth.noisy_image(48, 72, 0.1, 10)
    d0 = torch.tensor(noisy, device=DEV)
    res = protocol(ctx, d0, inner=10, sweeps=300, ref_iters=20000)
    s = summary(res)
    print(s, flush=True)
    tfs = res["tfs"]["dd"]
    e1 = res["tfs"]["ref_energy"]
    # Step 1: the DD energies decrease towards the reference energy
    assert tfs[-1] - e1 < 1e-3 * (tfs[1] - e1)
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(tfs[1:], tfs[2:]))
    for name in ("irv2", "irv1"):
        r = res[name]
        gap_ref = abs(r["dd_tau_ref"][-1] - r["ref_energy"])
        gap_dd = abs(r["dd_tau_dd"][-1] - r["ref_energy"])
        # with the reference tangent field DD Step 2 reaches the reference energy
        assert gap_ref < 1e-3 * abs(r["dd_tau_ref"][1] - r["ref_energy"]) + 1e-12
        assert gap_ref <= gap_dd
        # the DD and non-DD images are close (the paper: visually alike)
        assert r["image_psnr_dd_vs_ref"] > 40.0

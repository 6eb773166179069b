"""Schwarz versus single domain at convergence, on the GPU (float64), with
the paper's protocol of feeding the same tau to Step 2.

Both primals are strongly convex (TFS with modulus 1/delta on K, the IRV2
image problem with modulus alpha), so a dual iterate with duality gap G lies
within sqrt(2 delta G), resp. sqrt(2 G / alpha), of the unique primal
solution in the l2 norm.  The decomposed and the plain results must therefore
lie within the sum of their two radii of each other, whatever the iteration
counts; the decomposed radius must shrink as sweeps are added."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_17494_amd import Context
    c = Context(0)
    yield c
    c.close()


def test_schwarz_agrees_with_single_domain(ctx):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    n = 96
    _, d64 = synth.noisy_f32(n, n, 0.1, 41)
    delta, alpha = synth.params_for_sigma(0.1)
    prm = make_params(delta, alpha)
    d0 = torch.tensor(d64, device=DEV)
    plain, dd = make_layout(1, 1, 0, 0), make_layout(2, 2, 4, 4)
    # Step 1
    tau_p, st_p = ctx.step1(d0, prm, plain, make_iters(1, 20000))
    r_p = np.sqrt(2 * delta * max(st_p["gap"], 0.0))
    rads = []
    for sweeps in (10, 40):
        tau_d, st_d = ctx.step1(d0, prm, dd, make_iters(sweeps, 500))
        torch.cuda.synchronize()
        assert st_p["gap"] >= -1e-9 and st_d["gap"] >= -1e-9
        r_d = np.sqrt(2 * delta * max(st_d["gap"], 0.0))
        dist = float(torch.linalg.vector_norm(tau_p - tau_d))
        assert dist <= r_p + r_d + 1e-9
        rads.append(r_d)
    assert rads[1] < 0.8 * rads[0]
    # Step 2 from the same tau
    d_p, s2_p = ctx.step2(d0, tau_p, prm, plain, make_iters(1, 20000))
    q_p = np.sqrt(2 * max(s2_p["gap"], 0.0) / alpha)
    rads = []
    for sweeps in (10, 40):
        d_d, s2_d = ctx.step2(d0, tau_p, prm, dd, make_iters(sweeps, 500))
        torch.cuda.synchronize()
        q_d = np.sqrt(2 * max(s2_d["gap"], 0.0) / alpha)
        dist2 = float(torch.linalg.vector_norm(d_p - d_d))
        assert dist2 <= q_p + q_d + 1e-9
        rads.append(q_d)
    assert rads[1] < 0.8 * rads[0]

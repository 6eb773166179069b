"""The 512 x 512 workload: a float32 image (sigma = 0.1) solved plain
(single domain) and with a 2 x 2 overlapping Schwarz layout (8-pixel shared
stripes).

* Reduced counts: the HIP path against the FP64 oracle element by element.
* Full counts (plain: 10 000 dual iterations per step; Schwarz: 20 sweeps x
  500 inner), where the oracle is too slow: the float32 run against the
  float64 run of the same kernels (1e-4 on the image), tau divergence free
  (float64, 1e-10), non-negative gaps."""
import numpy as np
import pytest

import synth
from oracle import operators as op
from oracle import schwarz as osw
from oracle import solvers as osv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 512
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_17494_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def image():
    _, d64 = synth.noisy_f32(N, N, 0.1, 2)
    return d64


def solve(ctx, d64, dtype, lay, sweeps, inner):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    delta, alpha = synth.params_for_sigma(0.1)
    d0 = torch.tensor(d64, dtype=dtype, device=DEV)
    tau = torch.empty((2, N + 1, N + 1), dtype=dtype, device=DEV)
    d, st = ctx.schwarz_solve(d0, make_params(delta, alpha), make_layout(*lay), make_iters(sweeps, inner),
                              tau_out=tau)
    torch.cuda.synchronize()
    return d.double().cpu().numpy(), tau.double().cpu().numpy(), st


@pytest.mark.parametrize("dtype,tol_d,tol_tau", [(torch.float64, 1e-10, 1e-10), (torch.float32, 1e-4, 1e-5)])
def test_512_reduced_counts_against_oracle(ctx, image, dtype, tol_d, tol_tau):
    delta, alpha = synth.params_for_sigma(0.1)
    # Schwarz 2 x 2, s = 8: 2 sweeps x 3 inner
    lay = (2, 2, 8, 8)
    d, tau, st = solve(ctx, image, dtype, lay, 2, 3)
    tau_o, _, h1 = osw.step1_schwarz(image, delta, osw.Layout(N, N, *lay, step=1), 2, 3)
    d_o, _, h2 = osw.step2_schwarz(image, tau_o, alpha, osw.Layout(N, N, *lay, step=2), 2, 3)
    assert np.abs(tau - tau_o).max() < tol_tau
    assert np.abs(d - d_o).max() < tol_d
    # plain: 40 dual iterations per step
    d, tau, _ = solve(ctx, image, dtype, (1, 1, 0, 0), 1, 40)
    d_p, tau_p, _, _ = osv.tv_stokes_plain(image, delta, alpha, 40, 40)
    assert np.abs(tau - tau_p).max() < tol_tau
    assert np.abs(d - d_p).max() < tol_d


def test_512_full_counts_properties(ctx, image):
    for lay, sweeps, inner in (((2, 2, 8, 8), 20, 500), ((1, 1, 0, 0), 1, 10000)):
        d32, _, st32 = solve(ctx, image, torch.float32, lay, sweeps, inner)
        d64, tau64, st64 = solve(ctx, image, torch.float64, lay, sweeps, inner)
        assert np.abs(d32 - d64).max() < 1e-4
        assert np.abs(op.div(tau64)).max() < 1e-10
        for st in (st32, st64):
            assert st[0]["gap"] >= 0 and st[1]["gap"] >= 0

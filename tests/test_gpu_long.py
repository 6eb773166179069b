"""Grids whose inverse-Laplacian transforms are too long for two LDS buffers
(the one-buffer FFT engine): the plain single-domain solve at 2600 x 2600
(Omega-tilde 2601^2, 5400-point transforms) and at 4096 x 4096 (8640-point
transforms, the largest image side of the serving workload) against the
FP64 oracle at reduced counts, a non-square grid where only one axis needs
the long engine, a Schwarz job at 4096 x 4096 equal to its one-shot solve,
and the refusal of sides beyond the limit."""
import numpy as np
import pytest

import synth
from oracle import schwarz as osw
from oracle import solvers as sv

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


def plain(ctx, d64, dtype, sweeps, inner):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    n2, n1 = d64.shape
    d0 = torch.tensor(d64, dtype=dtype, device=DEV)
    tau = torch.empty((2, n2 + 1, n1 + 1), dtype=dtype, device=DEV)
    d, st = ctx.schwarz_solve(d0, make_params(0.15, 10.0), make_layout(), make_iters(sweeps, inner),
                              tau_out=tau)
    torch.cuda.synchronize()
    return d.double().cpu().numpy(), tau.double().cpu().numpy()


@pytest.mark.parametrize("n2,n1", [(2600, 2600), (2600, 700), (4096, 4096)])
def test_plain_long_transforms_against_oracle(ctx, n2, n1):
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 77)
    # the plain layout runs Algorithm 1 and the ROF iteration: 1 sweep x 2
    tau_o = sv.tfs_tau(sv.chambolle_tfs(sv.tfs_data(d64, 0.15), 2), sv.tfs_data(d64, 0.15), 0.15)
    f2 = sv.irv2_data(d64, sv.irv2_potential(tau_o, n2, n1), 10.0)
    d_o = sv.irv2_image(d64, sv.chambolle_rof(f2, 2), 10.0)
    for dtype, tol_d, tol_t in ((torch.float64, 1e-10, 1e-10), (torch.float32, 1e-4, 1e-5)):
        d, tau = plain(ctx, d64, dtype, 1, 2)
        print(f"{n2}x{n1} {dtype}: |tau - oracle| = {np.abs(tau - tau_o).max():.2e}, "
              f"|d - oracle| = {np.abs(d - d_o).max():.2e}", flush=True)
        assert np.abs(tau - tau_o).max() < tol_t
        assert np.abs(d - d_o).max() < tol_d


def test_schwarz_job_4096_equals_one_shot(ctx):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    n = 4096
    _, d64 = synth.noisy_f32(n, n, 0.2, 78)
    delta, alpha = synth.params_for_sigma(0.2)
    d0 = torch.tensor(d64, dtype=torch.float32, device=DEV)
    prm, L, its = make_params(delta, alpha), make_layout(16, 16, 16, 16), make_iters(2, 3)
    tau_ref = torch.empty((2, n + 1, n + 1), dtype=torch.float32, device=DEV)
    d_ref, st_ref = ctx.schwarz_solve(d0, prm, L, its, tau_out=tau_ref)
    job = ctx.job(d0, prm, L, its)
    while not job.done:
        ctx.batch_sweep([job])
    d, tau, st = job.result()
    torch.cuda.synchronize()
    assert torch.equal(d, d_ref) and torch.equal(tau, tau_ref)
    assert st[1]["energy"] == st_ref[1]["energy"]
    assert np.isfinite([st_ref[0]["energy"], st_ref[1]["energy"]]).all()
    job.close()


def test_sides_beyond_the_limit_are_refused(ctx):
    from paper_2602_17494_amd import TVS_EINVAL, TvsError, make_iters, make_layout, make_params
    d0 = torch.zeros((5120, 8), dtype=torch.float32, device=DEV)
    with pytest.raises(TvsError) as e:
        ctx.schwarz_solve(d0, make_params(0.15, 10.0), make_layout(), make_iters(1, 1))
    assert e.value.code == TVS_EINVAL
    with pytest.raises(TvsError) as e:
        ctx.job(d0, make_params(0.15, 10.0), make_layout(), make_iters(1, 1))
    assert e.value.code == TVS_EINVAL
    u = torch.zeros((2, 5121, 8), dtype=torch.float32, device=DEV)
    with pytest.raises(TvsError) as e:
        ctx.project_div_free(u)
    assert e.value.code == TVS_EINVAL

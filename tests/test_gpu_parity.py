"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle on
identical seeded inputs, element by element.

Tolerances: float64 runs must match to 1e-10 max-abs and float32 runs to
1e-4 max-abs on the reconstructed image (the stated targets); the
intermediate tangent field and projections use bounds derived from float32
rounding of the FFT-based inverse Laplacian (a few 1e-6 relative to the data,
see the individual tests)."""
import numpy as np
import pytest

import synth
from oracle import operators as op
from oracle import schwarz as osw
from oracle import solvers as osv

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


def run_case(ctx, n2, n1, lay, sweeps, inner, dtype, sigma=0.1, seed=1, variant=0):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    _, d64 = synth.noisy_f32(n2, n1, sigma, seed)
    delta, alpha = synth.params_for_sigma(sigma)
    d0 = torch.tensor(d64, dtype=dtype, device=DEV)
    tau = torch.empty((2, n2 + 1, n1 + 1), dtype=dtype, device=DEV)
    prm = make_params(delta, alpha, variant=variant)
    d, st = ctx.schwarz_solve(d0, prm, make_layout(*lay), make_iters(sweeps, inner), tau_out=tau)
    torch.cuda.synchronize()
    return d64, delta, alpha, d.cpu().numpy(), tau.cpu().numpy(), st


def oracle_case(d64, delta, alpha, lay, sweeps, inner):
    n2, n1 = d64.shape
    l1 = osw.Layout(n2, n1, *lay, step=1)
    l2 = osw.Layout(n2, n1, *lay, step=2)
    tau, _, h1 = osw.step1_schwarz(d64, delta, l1, sweeps, inner)
    d, _, h2 = osw.step2_schwarz(d64, tau, alpha, l2, sweeps, inner)
    return d, tau, h1, h2


@pytest.mark.parametrize("n2,n1", [(5, 7), (33, 65), (97, 130), (257, 200)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_projection(ctx, n2, n1, dtype):
    rng = np.random.default_rng(n2 * 1000 + n1)
    u = rng.standard_normal((2, n2, n1))
    t = torch.float64 if dtype == "f64" else torch.float32
    out = ctx.project_div_free(torch.tensor(u, dtype=t, device=DEV)).cpu().numpy()
    ref = op.project_k(u.astype(np.float32).astype(np.float64) if dtype == "f32" else u)
    tol = 1e-12 if dtype == "f64" else 2e-5
    assert np.abs(out - ref).max() < tol
    if dtype == "f64":
        assert np.abs(op.div(out)).max() < 1e-12


# (n2, n1, layout, sweeps, inner): plain and decomposed, square and not,
# sides that leave ragged tails of the 64-wide thread tiles
CASES = [
    (24, 28, (1, 1, 0, 0), 2, 3),
    (24, 28, (2, 2, 4, 4), 3, 4),
    (37, 70, (2, 3, 4, 3), 2, 3),
    (70, 37, (3, 2, 5, 4), 2, 3),
    (64, 64, (2, 2, 8, 8), 2, 5),
    (100, 131, (4, 4, 6, 6), 2, 2),
    (150, 200, (2, 2, 6, 8), 2, 2),   # frames wider than 64 columns (padded pitch)
    (90, 140, (1, 1, 0, 0), 2, 3),    # single domain, padded pitch
    (544, 544, (2, 2, 8, 8), 1, 3),   # 277-point Green boxes: 576-point transforms (compile-time passes)
    (496, 496, (2, 2, 8, 8), 1, 3),   # 254-point boxes: 512-point transforms (compile-time passes)
    (632, 632, (2, 2, 8, 8), 1, 2),   # 322-point boxes: 648-point transforms (compile-time passes)
]


@pytest.mark.parametrize("n2,n1,lay,sweeps,inner", CASES)
def test_schwarz_solve_f64(ctx, n2, n1, lay, sweeps, inner):
    d64, delta, alpha, d, tau, st = run_case(ctx, n2, n1, lay, sweeps, inner, torch.float64)
    d_ref, tau_ref, h1, h2 = oracle_case(d64, delta, alpha, lay, sweeps, inner)
    assert np.abs(tau - tau_ref).max() < 1e-10
    assert np.abs(d - d_ref).max() < 1e-10
    assert st[0]["energy"] == pytest.approx(h1[-1], rel=1e-10)
    assert st[1]["energy"] == pytest.approx(h2[-1], rel=1e-10)


@pytest.mark.parametrize("n2,n1,lay,sweeps,inner", CASES)
def test_schwarz_solve_f32(ctx, n2, n1, lay, sweeps, inner):
    d64, delta, alpha, d, tau, st = run_case(ctx, n2, n1, lay, sweeps, inner, torch.float32)
    d_ref, tau_ref, h1, h2 = oracle_case(d64, delta, alpha, lay, sweeps, inner)
    assert np.abs(d - d_ref).max() < 1e-4
    # tau feeds a row integral of up to N1 terms into d; bound it tighter
    assert np.abs(tau - tau_ref).max() < 1e-5
    assert st[0]["energy"] == pytest.approx(h1[-1], rel=1e-5)


def test_plain_64_config_f64(ctx):
    # the 64 x 64 workload: plain single-domain, 200 dual iterations per step
    d64, delta, alpha, d, tau, st = run_case(ctx, 64, 64, (1, 1, 0, 0), 1, 200, torch.float64, seed=1)
    d_ref, tau_ref, _, _ = osv.tv_stokes_plain(d64, delta, alpha, 200, 200)
    assert np.abs(tau - tau_ref).max() < 1e-10
    assert np.abs(d - d_ref).max() < 1e-10
    assert np.abs(op.div(tau)).max() < 1e-12


def test_step2_alone_and_irv1(ctx):
    from paper_2602_17494_amd import make_iters, make_layout, make_params, TVS_IRV1
    n2, n1 = 30, 41
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 5)
    rng = np.random.default_rng(6)
    tau = 0.2 * rng.standard_normal((2, n2 + 1, n1 + 1))
    lay = (2, 2, 4, 4)
    d0 = torch.tensor(d64, device=DEV)
    t = torch.tensor(tau, device=DEV)
    d, st = ctx.step2(d0, t, make_params(0.15, 10.0), make_layout(*lay), make_iters(3, 4))
    l2 = osw.Layout(n2, n1, *lay, step=2)
    d_ref, _, _ = osw.step2_schwarz(d64, tau, 10.0, l2, 3, 4)
    assert np.abs(d.cpu().numpy() - d_ref).max() < 1e-10
    # IRV1: xi from tau, f = alpha d0 - div xi, d = d0 - (div p + div xi)/alpha
    d1, _ = ctx.step2(d0, t, make_params(0.15, 10.0, eps=1e-3, variant=TVS_IRV1),
                      make_layout(*lay), make_iters(3, 4))
    xi = osv.irv1_xi(tau, n2, n1, 1e-3)
    f = osv.irv1_data(d64, xi, 10.0)
    p, _, _ = osw.schwarz(l2, osw.inner_rof, f, 1, 3, 4)
    d1_ref = osv.irv1_image(d64, p, xi, 10.0)
    assert np.abs(d1.cpu().numpy() - d1_ref).max() < 1e-10


def test_constant_image_is_fixed_point(ctx):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    for t in (torch.float32, torch.float64):
        d0 = torch.full((40, 50), 0.625, dtype=t, device=DEV)
        tau = torch.empty((2, 41, 51), dtype=t, device=DEV)
        d, _ = ctx.schwarz_solve(d0, make_params(0.15, 10.0), make_layout(2, 2, 4, 4),
                                 make_iters(3, 5), tau_out=tau)
        torch.cuda.synchronize()
        assert torch.all(tau == 0) and torch.all(d == 0.625)


def test_dual_feasibility_and_gap(ctx):
    # |p| <= 1 is not observable through the ABI; the duality gaps it
    # implies are >= 0, and they shrink with more iterations
    gaps = []
    for inner in (5, 50):
        _, _, _, _, _, st = run_case(ctx, 48, 40, (2, 2, 4, 4), 4, inner, torch.float64, seed=9)
        assert st[0]["gap"] >= -1e-9 and st[1]["gap"] >= -1e-9
        gaps.append(st[0]["gap"])
    assert gaps[1] < gaps[0]


def test_tolerance_stop(ctx):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    _, d64 = synth.noisy_f32(32, 32, 0.1, 3)
    d0 = torch.tensor(d64, device=DEV)
    _, st = ctx.step1(d0, make_params(0.15, 10.0), make_layout(1, 1, 0, 0),
                      make_iters(1000, 10, tol=1e-3))
    assert 1 <= st["sweeps_done"] < 1000 and st["residual"] < 1e-3


def test_invalid_arguments_are_rejected(ctx):
    from paper_2602_17494_amd import TvsError, make_iters, make_layout, make_params
    d0 = torch.zeros((16, 16), device=DEV)
    with pytest.raises(TvsError):
        ctx.step1(d0, make_params(0.15, 10.0, t=0.2), make_layout(), make_iters(1, 1))
    with pytest.raises(TvsError):
        ctx.step1(d0, make_params(0.15, 10.0), make_layout(4, 4, 8, 8), make_iters(1, 1))
    with pytest.raises(TvsError):
        ctx.step1(d0, make_params(-1.0, 10.0), make_layout(), make_iters(1, 1))
    with pytest.raises(TvsError):
        ctx.step1(d0, make_params(0.15, 10.0), make_layout(), make_iters(0, 1))

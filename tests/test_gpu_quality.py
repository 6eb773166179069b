"""Quality measures and the parameter-selection experiment of Section 5.2,
through the C-ABI, against the FP64 oracle on identical seeded inputs.

* tvs_quality (PSNR, MSSIM, MSE from FP64 moments) against oracle.quality on
  the same arrays: only the summation order differs, so 1e-12 relative.
* tvs_tangent_field against the oracle's tau_0: the same two differences.
* The delta sweep (Perf of the tangent field) and the IRV2 / IRV1 sweeps
  (PSNR, MSSIM of the image) on the 64 x 64 workload with 200 dual
  iterations per step: each side runs its own chain from the same image, so
  the measures agree to the FP64 parity of the solves (tau and d within
  1e-10), and the selected parameters are the same."""
import numpy as np
import pytest

import synth
from oracle import quality as oq
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


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n2,n1", [(1, 1), (1, 9), (37, 53), (513, 260), (2048, 2048)])
def test_quality_matches_oracle(ctx, dtype, n2, n1):
    print(f"quality {n2}x{n1} {dtype}", flush=True)
    gt = synth.clean_image(max(n2, 2), max(n1, 2), 3)[:n2, :n1]
    _, noisy = synth.noisy_image(max(n2, 2), max(n1, 2), 0.1, 3)
    noisy = noisy[:n2, :n1]
    np_dt = np.float64 if dtype == torch.float64 else np.float32
    x, r = noisy.astype(np_dt), gt.astype(np_dt)
    got = ctx.quality(torch.tensor(x, device=DEV), torch.tensor(r, device=DEV))
    xo, ro = x.astype(np.float64), r.astype(np.float64)
    assert got["mse"] == pytest.approx(oq.mse(xo, ro), rel=1e-12)
    assert got["psnr"] == pytest.approx(oq.psnr(xo, ro), rel=1e-12)
    assert got["mssim"] == pytest.approx(oq.mssim(xo, ro), rel=1e-12, abs=1e-14)


def test_quality_identical_and_constant(ctx):
    a = torch.tensor(synth.clean_image(31, 45, 4), device=DEV)
    got = ctx.quality(a, a)
    assert got["psnr"] == float("inf") and got["mse"] == 0.0
    assert got["mssim"] == pytest.approx(1.0, abs=1e-15)
    c = torch.full((16, 16), 0.25, dtype=torch.float64, device=DEV)
    got = ctx.quality(c + 0.1, c)
    # constant images: the structure factor is c2 / c2 and MSE = 0.01
    assert got["psnr"] == pytest.approx(20.0, rel=1e-12)
    want = (2 * 0.35 * 0.25 + 1e-4) / (0.35 ** 2 + 0.25 ** 2 + 1e-4)
    assert got["mssim"] == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_tangent_field_matches_oracle(ctx, dtype):
    n2, n1 = 45, 70
    gt = synth.clean_image(n2, n1, 8)
    np_dt = np.float64 if dtype == torch.float64 else np.float32
    g = gt.astype(np_dt)
    got = ctx.tangent_field(torch.tensor(g, device=DEV)).double().cpu().numpy()
    want = oq.tangent_gt(g.astype(np.float64))
    assert got.shape == (2, n2 + 1, n1 + 1)
    assert np.abs(got - want).max() <= (0.0 if dtype == torch.float64 else 2e-7)


N, SIGMA, SEED, IT = 64, 0.1, 1, 200
DELTAS = (0.02, 0.08, 0.15, 0.3, 0.6)
ALPHAS = (1.0, 3.0, 10.0, 30.0)
EPSS = (1e-1, 1e-3)


@pytest.fixture(scope="module")
def images():
    gt, noisy = synth.noisy_image(N, N, SIGMA, SEED)
    return gt, noisy


def oracle_tau(noisy, delta):
    f1 = osv.tfs_data(noisy, delta)
    return osv.tfs_tau(osv.chambolle_tfs(f1, IT), f1, delta)


def test_delta_sweep_matches_oracle(ctx, images):
    from paper_2602_17494_amd import make_iters, make_layout
    from paper_2602_17494_amd.quality import tfs_sweep
    gt, noisy = images
    g, d0 = torch.tensor(gt, device=DEV), torch.tensor(noisy, device=DEV)
    rows, best, tau = tfs_sweep(ctx, g, d0, DELTAS, make_layout(), make_iters(1, IT))
    tg = oq.tangent_gt(gt)
    want = [oq.perf_tau(oracle_tau(noisy, dl), tg) for dl in DELTAS]
    for row, w in zip(rows, want):
        assert row["perf"] == pytest.approx(w, abs=1e-6)
    assert best == int(np.argmax(want))
    assert abs(want[best] - sorted(want)[-2]) > 1e-3  # the choice is not a near tie
    assert torch.equal(tau, ctx.step1(d0, _params(DELTAS[best], 1.0), make_layout(), make_iters(1, IT))[0])


def _params(delta, alpha, **kw):
    from paper_2602_17494_amd import make_params
    return make_params(delta, alpha, **kw)


def test_step2_sweeps_match_oracle(ctx, images):
    from paper_2602_17494_amd import make_iters, make_layout
    from paper_2602_17494_amd.quality import irv1_sweep, irv2_sweep
    gt, noisy = images
    delta = 0.15
    g, d0 = torch.tensor(gt, device=DEV), torch.tensor(noisy, device=DEV)
    tau, _ = ctx.step1(d0, _params(delta, 1.0), make_layout(), make_iters(1, IT))
    rows2, p2, s2 = irv2_sweep(ctx, g, d0, tau, delta, ALPHAS, make_layout(), make_iters(1, IT))
    rows1, p1, s1 = irv1_sweep(ctx, g, d0, tau, delta, ALPHAS, EPSS, make_layout(), make_iters(1, IT))

    tau_o = oracle_tau(noisy, delta)
    gpot = osv.irv2_potential(tau_o, N, N)
    want2 = []
    for alpha in ALPHAS:
        f2 = osv.irv2_data(noisy, gpot, alpha)
        d = osv.irv2_image(noisy, osv.chambolle_rof(f2, IT), alpha)
        want2.append((oq.psnr(d, gt), oq.mssim(d, gt)))
    for row, (ps, ms) in zip(rows2, want2):
        assert row["psnr"] == pytest.approx(ps, abs=1e-7)
        assert row["mssim"] == pytest.approx(ms, abs=1e-9)
    assert p2 == int(np.argmax([w[0] for w in want2])) and s2 == int(np.argmax([w[1] for w in want2]))

    want1 = []
    for alpha in ALPHAS:
        for eps in EPSS:
            xi = osv.irv1_xi(tau_o, N, N, eps)
            f = osv.irv1_data(noisy, xi, alpha)
            d = osv.irv1_image(noisy, osv.chambolle_rof(f, IT), xi, alpha)
            want1.append((oq.psnr(d, gt), oq.mssim(d, gt)))
    for row, (ps, ms) in zip(rows1, want1):
        assert row["psnr"] == pytest.approx(ps, abs=1e-7)
        assert row["mssim"] == pytest.approx(ms, abs=1e-9)
    assert p1 == int(np.argmax([w[0] for w in want1])) and s1 == int(np.argmax([w[1] for w in want1]))


def test_experiment_end_to_end(ctx, images):
    """The whole selection with tolerance stops: best entries are the
    extremes of their tables and every solve ran at least one sweep."""
    from paper_2602_17494_amd import make_iters, make_layout
    from paper_2602_17494_amd.quality import experiment
    gt, noisy = images
    res = experiment(ctx, torch.tensor(gt, device=DEV), torch.tensor(noisy, device=DEV), make_layout(),
                     make_iters(50, 20, 1e-7), DELTAS, ALPHAS, ALPHAS, EPSS)
    assert res["tfs"]["best"]["perf"] == max(r["perf"] for r in res["tfs"]["rows"])
    assert res["irv2"]["best_psnr"]["psnr"] == max(r["psnr"] for r in res["irv2"]["rows"])
    assert res["irv1"]["best_mssim"]["mssim"] == max(r["mssim"] for r in res["irv1"]["rows"])
    assert all(r["sweeps"] >= 1 for r in res["tfs"]["rows"] + res["irv2"]["rows"] + res["irv1"]["rows"])
    # denoising helps: the best reconstruction beats the noisy observation
    assert res["irv2"]["best_psnr"]["psnr"] > res["noisy"]["psnr"] + 3.0


def test_quality_argument_errors(ctx):
    a = torch.zeros((4, 5), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        ctx.quality(a, torch.zeros((4, 6), dtype=torch.float64, device=DEV))
    with pytest.raises(TypeError):
        ctx.quality(a, torch.zeros((4, 5), dtype=torch.float32, device=DEV))
    with pytest.raises(ValueError):
        ctx.quality(torch.zeros(5, dtype=torch.float64, device=DEV), torch.zeros(5, dtype=torch.float64, device=DEV))

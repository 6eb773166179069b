"""The block-DCT realisation of LP_m (eq. invLaplLowCapLong; tvs_set_local_projection
with TVS_LP_BLOCKDCT) through the C-ABI.

It computes the same operator as the image method, so the whole Schwarz solve
is held to the same bars: against the FP64 oracle element by element (1e-10 in
float64, 1e-4 on the image in float32), on square and non-square grids with
ragged tails, and against the image-method solve of the same input."""
import numpy as np
import pytest

import synth
from oracle import schwarz as osw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctxs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_17494_amd import TVS_LP_BLOCKDCT, Context
    bd, im = Context(0), Context(0)
    bd.set_local_projection(TVS_LP_BLOCKDCT)
    yield bd, im
    bd.close()
    im.close()


def solve(ctx, d64, dtype, lay, sweeps, inner):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    n2, n1 = d64.shape
    delta, alpha = synth.params_for_sigma(0.1)
    d0 = torch.tensor(d64, dtype=dtype, device=DEV)
    tau = torch.empty((2, n2 + 1, n1 + 1), dtype=dtype, device=DEV)
    d, st = ctx.schwarz_solve(d0, make_params(delta, alpha), make_layout(*lay), make_iters(sweeps, inner),
                              tau_out=tau)
    torch.cuda.synchronize()
    return d.double().cpu().numpy(), tau.double().cpu().numpy(), st


def oracle(d64, lay, sweeps, inner):
    n2, n1 = d64.shape
    delta, alpha = synth.params_for_sigma(0.1)
    tau, _, h1 = osw.step1_schwarz(d64, delta, osw.Layout(n2, n1, *lay, step=1), sweeps, inner)
    d, _, _ = osw.step2_schwarz(d64, tau, alpha, osw.Layout(n2, n1, *lay, step=2), sweeps, inner)
    return d, tau, h1


CASES = [
    (24, 28, (2, 2, 4, 4), 3, 4),
    (37, 70, (2, 3, 4, 3), 2, 3),
    (70, 37, (3, 2, 5, 4), 2, 3),
    (150, 200, (2, 2, 6, 8), 2, 2),
]


@pytest.mark.parametrize("n2,n1,lay,sweeps,inner", CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_blockdct_against_oracle_and_image_method(ctxs, n2, n1, lay, sweeps, inner, dtype):
    print(f"blockdct {n2}x{n1} layout={lay} {sweeps}x{inner} {dtype}", flush=True)
    bd, im = ctxs
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 3)
    d, tau, st = solve(bd, d64, dtype, lay, sweeps, inner)
    d_ref, tau_ref, h1 = oracle(d64, lay, sweeps, inner)
    d_im, tau_im, _ = solve(im, d64, dtype, lay, sweeps, inner)
    if dtype == torch.float64:
        assert np.abs(tau - tau_ref).max() < 1e-10
        assert np.abs(d - d_ref).max() < 1e-10
        assert np.abs(d - d_im).max() < 1e-10
        assert st[0]["energy"] == pytest.approx(h1[-1], rel=1e-10)
    else:
        assert np.abs(tau - tau_ref).max() < 1e-5
        assert np.abs(d - d_ref).max() < 1e-4
        assert np.abs(d - d_im).max() < 1e-4


_ORACLE = {}


def oracle_cached(d64, lay, sweeps, inner, key):
    if key not in _ORACLE:
        _ORACLE[key] = oracle(d64, lay, sweeps, inner)
    return _ORACLE[key]


# 8 x 8 layouts: 64 boxes and 7 x 7 or 6 x 8 frequency blocks, summed one
# block at a time (every partial sum of W and O accumulates), in uneven
# groups, and in the automatic grouping
GROUP_CASES = [
    (320, 320, (8, 8, 4, 4), (1, 1)),
    (320, 320, (8, 8, 4, 4), (0, 0)),
    (288, 352, (8, 8, 4, 4), (2, 3)),
    (288, 352, (8, 8, 4, 4), (1, 1)),
]


@pytest.mark.parametrize("n2,n1,lay,groups", GROUP_CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_blockdct_frequency_groups_against_oracle(ctxs, n2, n1, lay, groups, dtype):
    print(f"blockdct groups {groups} {n2}x{n1} layout={lay} {dtype}", flush=True)
    bd, _ = ctxs
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 5)
    bd.set_block_groups(*groups)
    try:
        d, tau, st = solve(bd, d64, dtype, lay, 1, 2)
    finally:
        bd.set_block_groups(0, 0)
    d_ref, tau_ref, h1 = oracle_cached(d64, lay, 1, 2, (n2, n1, lay))
    if dtype == torch.float64:
        assert np.abs(tau - tau_ref).max() < 1e-10
        assert np.abs(d - d_ref).max() < 1e-10
        assert st[0]["energy"] == pytest.approx(h1[-1], rel=1e-10)
    else:
        assert np.abs(tau - tau_ref).max() < 1e-5
        assert np.abs(d - d_ref).max() < 1e-4


def test_block_groups_rejected_outside_range(ctxs):
    from paper_2602_17494_amd import TvsError
    bd, _ = ctxs
    for g in ((-1, 0), (0, 65)):
        with pytest.raises(TvsError) as e:
            bd.set_block_groups(*g)
        assert e.value.code == -1  # TVS_EINVAL


def test_blockdct_512_reduced_counts(ctxs):
    """The 512 x 512 workload's 2 x 2 layout (8-pixel stripes) at 1 sweep x
    5 inner: float32 block-DCT against the float64 oracle."""
    bd, _ = ctxs
    _, d64 = synth.noisy_f32(512, 512, 0.1, 2)
    lay = (2, 2, 8, 8)
    d, tau, _ = solve(bd, d64, torch.float32, lay, 1, 5)
    d_ref, tau_ref, _ = oracle(d64, lay, 1, 5)
    assert np.abs(tau - tau_ref).max() < 1e-5
    assert np.abs(d - d_ref).max() < 1e-4


def test_jobs_keep_the_image_method(ctxs):
    """A context switched to the block formula still runs jobs (recorded as
    graphs) with the image method: a job equals the image-method solve bit
    for bit."""
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    bd, im = ctxs
    _, d64 = synth.noisy_f32(40, 56, 0.1, 4)
    d0 = torch.tensor(d64, dtype=torch.float32, device=DEV)
    prm, L, its = make_params(0.15, 10.0), make_layout(2, 2, 4, 4), make_iters(2, 3)
    job = bd.job(d0, prm, L, its)
    while not job.done:
        bd.batch_sweep([job])
    torch.cuda.synchronize()
    d_job, _, _ = job.result()
    d_im, _ = im.schwarz_solve(d0, prm, L, its)
    torch.cuda.synchronize()
    assert torch.equal(d_job, d_im)
    job.close()


def test_unknown_local_projection_rejected(ctxs):
    from paper_2602_17494_amd import TvsError
    bd, _ = ctxs
    with pytest.raises(TvsError) as e:
        bd.set_local_projection(7)
    assert e.value.code == -1  # TVS_EINVAL


@pytest.mark.parametrize("dtype,tol_d,tol_tau", [(torch.float64, 1e-10, 1e-10), (torch.float32, 1e-4, 1e-5)])
def test_blockdct_2048_reduced_counts_against_oracle(ctxs, dtype, tol_d, tol_tau):
    """The 2048 x 2048 workload's 8 x 8 layout with the block formula in its
    automatic grouping (2 x 8 frequency blocks per group, 4 row groups whose
    partial sums accumulate), at 2 sweeps x 2 inner against the FP64 oracle's
    stored values (tests/golden/make_golden_2048.py, sigma = 0.1)."""
    import os
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_2048_s2i2_sigma0.1.npz")
    g = np.load(golden)
    meta = g["meta"]
    n = 2048
    print(f"blockdct 2048 golden {dtype}", flush=True)
    bd, _ = ctxs
    _, d64 = synth.noisy_f32(n, n, 0.1, int(meta[1]))
    delta, alpha = synth.params_for_sigma(0.1)
    d0 = torch.tensor(d64, dtype=dtype, device=DEV)
    tau = torch.empty((2, n + 1, n + 1), dtype=dtype, device=DEV)
    d, st = bd.schwarz_solve(d0, make_params(delta, alpha), make_layout(8, 8, 16, 16),
                             make_iters(int(meta[2]), int(meta[3])), tau_out=tau)
    torch.cuda.synchronize()
    d = d.double().cpu().numpy()
    tau = tau.double().cpu().numpy()
    ii, jj = g["ii"], g["jj"]
    assert np.abs(tau[0, ii, jj] - g["tau1"]).max() < tol_tau
    assert np.abs(tau[1, ii, jj] - g["tau2"]).max() < tol_tau
    assert np.abs(d[np.minimum(ii, n - 1), np.minimum(jj, n - 1)] - g["d"]).max() < tol_d
    w0 = int(g["win0"])
    w = slice(w0, w0 + g["d_win"].shape[0])
    assert np.abs(d[w, w] - g["d_win"]).max() < tol_d
    assert np.abs(tau[:, w, w] - g["tau_win"]).max() < tol_tau
    assert np.abs(d.sum(axis=1) - g["d_rowsum"]).max() < tol_d * n
    assert np.abs(tau[1].sum(axis=1) - g["tau2_rowsum"]).max() < tol_tau * n

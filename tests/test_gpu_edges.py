"""Edge cases of the HIP path through the C-ABI, against the FP64 oracle:
the smallest images the method accepts (2 x 2, thin strips), the maximum
number of subdomains per axis (32), minimal overlaps, and the error paths
(too-small images, non-finite data)."""
import numpy as np
import pytest

import synth
from oracle import schwarz as osw

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


EDGE = [
    (2, 2, (1, 1, 0, 0)),     # the smallest image
    (3, 3, (1, 1, 0, 0)),
    (2, 9, (1, 1, 0, 0)),     # one-row-pair strips
    (9, 2, (1, 1, 0, 0)),
    (2, 64, (1, 4, 0, 4)),    # a strip split along x only
    (24, 200, (1, 32, 0, 2)),  # 32 subdomains along an axis (the maximum)
    (5, 40, (2, 3, 1, 3)),    # overlap of one pixel, cores of three
]


@pytest.mark.parametrize("n2,n1,lay", EDGE)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_edge_shapes_against_oracle(ctx, n2, n1, lay, dtype):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 3)
    t = torch.float64 if dtype == "f64" else torch.float32
    d0 = torch.tensor(d64, dtype=t, device=DEV)
    tau = torch.empty((2, n2 + 1, n1 + 1), dtype=t, device=DEV)
    d, st = ctx.schwarz_solve(d0, make_params(0.15, 10.0), make_layout(*lay), make_iters(2, 3),
                              tau_out=tau)
    torch.cuda.synchronize()
    l1 = osw.Layout(n2, n1, *lay, step=1)
    l2 = osw.Layout(n2, n1, *lay, step=2)
    tau_ref, _, h1 = osw.step1_schwarz(d64, 0.15, l1, 2, 3)
    d_ref, _, h2 = osw.step2_schwarz(d64, tau_ref, 10.0, l2, 2, 3)
    tol_d, tol_tau = (1e-10, 1e-10) if dtype == "f64" else (1e-4, 1e-5)
    assert np.abs(tau.double().cpu().numpy() - tau_ref).max() < tol_tau
    assert np.abs(d.double().cpu().numpy() - d_ref).max() < tol_d
    if dtype == "f64":
        assert st[0]["energy"] == pytest.approx(h1[-1], rel=1e-10)
        assert st[1]["energy"] == pytest.approx(h2[-1], rel=1e-10)


def test_rejects_images_below_two_by_two(ctx):
    from paper_2602_17494_amd import TvsError, make_iters, make_layout, make_params
    for shape in ((1, 5), (5, 1)):
        d0 = torch.zeros(shape, device=DEV)
        with pytest.raises(TvsError):
            ctx.schwarz_solve(d0, make_params(0.15, 10.0), make_layout(), make_iters(1, 1))


def test_rejects_non_finite_data(ctx):
    from paper_2602_17494_amd import TvsError, make_iters, make_layout, make_params
    _, d64 = synth.noisy_f32(16, 20, 0.1, 4)
    d64[3, 5] = np.nan
    d0 = torch.tensor(d64, device=DEV)
    with pytest.raises(TvsError) as e:
        ctx.schwarz_solve(d0, make_params(0.15, 10.0), make_layout(2, 2, 2, 2), make_iters(2, 2))
    assert e.value.code == -4  # TVS_ENONFINITE

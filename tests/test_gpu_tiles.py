"""The workgroup shapes the tuner chooses between change speed only: a solve
with every forced choice of stencil run length (1, 2, 4 rows per thread, both
steps) and of Green-pass workgroup shape (row pairs and columns per
workgroup) equals, bit for bit, the solve with the tuner's choice; on the
576-point compile-time passes, on runtime-descriptor passes and on the plain
single-domain layout, in both dtypes; and jobs batched together give the
same bits under any forced choice."""
import itertools

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


def solve(ctx, d0, lay, its):
    from paper_2602_17494_amd import make_params
    n2, n1 = d0.shape
    tau = torch.empty((2, n2 + 1, n1 + 1), dtype=d0.dtype, device=DEV)
    d, _ = ctx.schwarz_solve(d0, make_params(0.15, 10.0), lay, its, tau_out=tau)
    torch.cuda.synchronize()
    return d, tau


CASES = [(544, 544, (2, 2, 8, 8)),   # 277-point boxes: 576-point compile-time passes
         (150, 230, (3, 2, 5, 7)),   # runtime transform descriptors
         (70, 90, (1, 1, 0, 0))]     # the plain layout (whole-grid plan in the inner loop)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n2,n1,lay", CASES)
def test_every_tile_choice_gives_the_same_bits(ctx, n2, n1, lay, dtype):
    from paper_2602_17494_amd import make_iters, make_layout
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 71)
    d0 = torch.tensor(d64, dtype=dtype, device=DEV)
    L, its = make_layout(*lay), make_iters(2, 3)
    ctx.set_tiles()
    d_ref, tau_ref = solve(ctx, d0, L, its)
    tuned = ctx.get_tiles((n2, n1), dtype, L)
    assert tuned[0] in (1, 2, 4) and tuned[1] in (1, 2, 4) and tuned[4] in (1, 2, 4)
    assert tuned[2] > 0 and tuned[3] > 0
    choices = [(run, rows, cols) for run, rows, cols in itertools.product((1, 2, 4), (2, 8, 16), (1, 3, 4))]
    for run, rows, cols in choices[::3] + [(4, 16, 4), (1, 2, 1)]:
        ctx.set_tiles(run, {1: 4, 2: 1, 4: 2}[run], rows, cols, run)
        d, tau = solve(ctx, d0, L, its)
        assert torch.equal(d, d_ref) and torch.equal(tau, tau_ref), (run, rows, cols)
    ctx.set_tiles()


def test_batched_jobs_under_forced_tiles(ctx):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    _, d64 = synth.noisy_f32(120, 140, 0.1, 72)
    d0 = torch.tensor(d64, dtype=torch.float32, device=DEV)
    prm, L, its = make_params(0.15, 10.0), make_layout(2, 3, 6, 6), make_iters(2, 3)
    ctx.set_tiles()
    d_ref, tau_ref = solve(ctx, d0, L, its)
    for tiles in [(1, 4, 16, 1, 4), (4, 1, 2, 4, 1)]:
        ctx.set_tiles(*tiles)
        jobs = [ctx.job(d0, prm, L, its) for _ in range(3)]
        while not all(j.done for j in jobs):
            ctx.batch_sweep([j for j in jobs if not j.done])
        for j in jobs:
            d, tau, _ = j.result()
            torch.cuda.synchronize()
            assert torch.equal(d, d_ref) and torch.equal(tau, tau_ref), tiles
            j.close()
    ctx.set_tiles()


def test_tile_arguments_are_checked(ctx):
    from paper_2602_17494_amd import TVS_EINVAL, TvsError
    for bad in [(3, 0, 0, 0, 0), (0, 5, 0, 0, 0), (0, 0, -1, 0, 0), (0, 0, 0, 65, 0), (0, 0, 0, 0, 8)]:
        with pytest.raises(TvsError) as e:
            ctx.set_tiles(*bad)
        assert e.value.code == TVS_EINVAL

"""Checkpoint and resume of jobs (tvs_job_export_state / tvs_job_import_state)
through the C-ABI.

A job exported between two sweeps and re-created from the blob must finish
exactly as the uninterrupted solve does: its image, tau and FP64 statistics
are compared bit for bit with the one-shot tvs_schwarz_solve of the same
image, for checkpoints inside Step 1, at the Step-1/Step-2 boundary, inside
Step 2 and after the end, in both dtypes, in the Schwarz and the single-domain
layout, and into a second context.  Malformed blobs are rejected before any
device work."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SWEEPS, INNER = 3, 4


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_17494_amd import Context
    c = Context(0)
    yield c
    c.close()


def one_shot(ctx, d0, prm, lay, its):
    n2, n1 = d0.shape
    tau = torch.empty((2, n2 + 1, n1 + 1), dtype=d0.dtype, device=DEV)
    d, st = ctx.schwarz_solve(d0, prm, lay, its, tau_out=tau)
    torch.cuda.synchronize()
    return d, tau, st


def finish(ctx, job):
    while not job.done:
        ctx.batch_sweep([job])
    torch.cuda.synchronize()
    return job.result()


def same_result(got, ref, stats_ref):
    d, tau, st = got
    d_ref, tau_ref = ref
    torch.cuda.synchronize()
    assert torch.equal(d, d_ref) and torch.equal(tau, tau_ref)
    for a, b in zip(st, stats_ref):
        for k in ("energy", "gap", "residual", "sweeps_done"):
            assert a[k] == b[k], k


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n2,n1,lay", [(40, 56, (2, 2, 4, 4)), (33, 30, (1, 1, 0, 0))])
@pytest.mark.parametrize("at", [1, SWEEPS, SWEEPS + 1, 2 * SWEEPS])
def test_resume_equals_uninterrupted(ctx, dtype, n2, n1, lay, at):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    print(f"resume dtype={dtype} shape={n2}x{n1} layout={lay} checkpoint after {at} sweeps", flush=True)
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 21)
    d0 = torch.tensor(d64, dtype=dtype, device=DEV)
    prm, L, its = make_params(0.15, 10.0), make_layout(*lay), make_iters(SWEEPS, INNER)
    d_ref, tau_ref, st_ref = one_shot(ctx, d0, prm, L, its)

    job = ctx.job(d0, prm, L, its)
    for _ in range(at):
        ctx.batch_sweep([job])
    status = job.status()
    blob = job.export_state()
    assert blob.dtype == np.uint8 and bytes(blob[:8]) == b"TVSJOBST"
    # exporting leaves the job as it was: it still finishes as the one-shot solve
    same_result(finish(ctx, job), (d_ref, tau_ref), st_ref)
    job.close()

    back = ctx.import_job(blob.tobytes())
    assert back.status() == status and back.shape == (n2, n1) and back.dtype == dtype
    same_result(finish(ctx, back), (d_ref, tau_ref), st_ref)
    back.close()


def test_resume_in_another_context_and_batch(ctx):
    """A blob taken mid-Step-2 resumes in a fresh context, in a batch with a
    job that never stopped."""
    from paper_2602_17494_amd import Context, make_iters, make_layout, make_params
    n2, n1 = 48, 64
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 22)
    d0 = torch.tensor(d64, dtype=torch.float32, device=DEV)
    prm, L, its = make_params(0.15, 10.0), make_layout(2, 3, 4, 4), make_iters(SWEEPS, INNER)
    d_ref, tau_ref, st_ref = one_shot(ctx, d0, prm, L, its)
    job = ctx.job(d0, prm, L, its)
    for _ in range(SWEEPS + 2):
        ctx.batch_sweep([job])
    blob = job.export_state()
    job.close()
    c2 = Context(0)
    try:
        back = c2.import_job(blob)
        fresh = c2.job(d0, prm, L, its)
        while not (back.done and fresh.done):
            c2.batch_sweep([j for j in (back, fresh) if not j.done])
        torch.cuda.synchronize()
        same_result(back.result(), (d_ref, tau_ref), st_ref)
        same_result(fresh.result(), (d_ref, tau_ref), st_ref)
        back.close()
        fresh.close()
    finally:
        c2.close()


def test_resume_with_tolerance(ctx):
    """The stopping test of a tolerance-driven run reads the restored energy
    history."""
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    n2, n1 = 40, 40
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 23)
    d0 = torch.tensor(d64, dtype=torch.float64, device=DEV)
    prm, L = make_params(0.15, 10.0), make_layout(2, 2, 4, 4)
    # a tolerance the Step-1 residual passes within 4 sweeps
    _, _, st4 = one_shot(ctx, d0, prm, L, make_iters(4, 6))
    its = make_iters(12, 6, tol=1.5 * st4[0]["residual"])
    d_ref, tau_ref, st_ref = one_shot(ctx, d0, prm, L, its)
    assert st_ref[0]["sweeps_done"] <= 4
    job = ctx.job(d0, prm, L, its)
    for _ in range(2):
        ctx.batch_sweep([job])
    back = ctx.import_job(job.export_state())
    job.close()
    same_result(finish(ctx, back), (d_ref, tau_ref), st_ref)
    back.close()


def test_malformed_blobs_rejected(ctx):
    from paper_2602_17494_amd import TvsError, make_iters, make_layout, make_params
    _, d64 = synth.noisy_f32(24, 28, 0.1, 24)
    d0 = torch.tensor(d64, dtype=torch.float32, device=DEV)
    job = ctx.job(d0, make_params(0.15, 10.0), make_layout(2, 2, 4, 4), make_iters(2, 2))
    ctx.batch_sweep([job])
    blob = job.export_state()
    job.close()

    def rejected(b):
        with pytest.raises(TvsError) as e:
            ctx.import_job(b)
        assert e.value.code == -1  # TVS_EINVAL

    rejected(blob[:100])                     # shorter than its header
    rejected(blob[:-4])                      # truncated arrays
    bad = blob.copy(); bad[0] ^= 1           # magic
    rejected(bad)
    bad = blob.copy(); bad[8] += 1           # version
    rejected(bad)
    bad = blob.copy(); bad[28] += 1          # N2 no longer matches the arrays
    rejected(bad)
    bad = blob.copy(); bad[24] = 7           # dtype
    rejected(bad)
    # section sizes that add up but do not match the job's arrays (the
    # section table is the last 48 bytes of the header)
    hb = int(blob[12:16].view(np.uint32)[0])
    bad = blob.copy()
    sec = bad[hb - 48:hb].view(np.uint64)
    sec[1] += 8
    sec[2] -= 8
    rejected(bad)
    # the intact blob still resumes
    ctx.import_job(blob).close()

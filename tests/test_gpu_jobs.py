"""Jobs (resident state, one Schwarz sweep per batch call), batches of uneven
images and the continuous-batching server, through the C-ABI.

A job runs the launches of tvs_schwarz_solve in the same order, so its
results are compared bit for bit with the one-shot solve of the same image,
alone and in a mix; two small cases are also checked against the FP64
oracle."""
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


def one_shot(ctx, d0, prm, lay, its):
    n2, n1 = d0.shape
    tau = torch.empty((2, n2 + 1, n1 + 1), dtype=d0.dtype, device=DEV)
    d, st = ctx.schwarz_solve(d0, prm, lay, its, tau_out=tau)
    torch.cuda.synchronize()
    return d, tau, st


def run_jobs(ctx, jobs):
    rounds = 0
    while not all(j.done for j in jobs):
        ctx.batch_sweep([j for j in jobs if not j.done])
        rounds += 1
    torch.cuda.synchronize()
    return rounds


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n2,n1,lay", [(40, 56, (2, 2, 4, 4)), (33, 30, (1, 1, 0, 0))])
def test_job_equals_one_shot(ctx, dtype, n2, n1, lay):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 11)
    d0 = torch.tensor(d64, dtype=dtype, device=DEV)
    prm, L, its = make_params(0.15, 10.0), make_layout(*lay), make_iters(3, 4)
    d_ref, tau_ref, st_ref = one_shot(ctx, d0, prm, L, its)
    job = ctx.job(d0, prm, L, its)
    assert job.status() == (1, 0, False)
    rounds = run_jobs(ctx, [job])
    assert rounds == 2 * 3
    d, tau, st = job.result()
    torch.cuda.synchronize()
    assert torch.equal(d, d_ref) and torch.equal(tau, tau_ref)
    for a, b in zip(st, st_ref):
        assert a["energy"] == b["energy"] and a["gap"] == b["gap"] and a["sweeps_done"] == 3
    job.close()


def test_footprint_and_busy(ctx):
    from paper_2602_17494_amd import TVS_EBUSY, TvsError, job_footprint, make_iters, make_layout, make_params
    n2, n1 = 48, 64
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 12)
    for dtype in (torch.float32, torch.float64):
        d0 = torch.tensor(d64, dtype=dtype, device=DEV)
        L, its = make_layout(2, 3, 4, 4), make_iters(2, 2)
        job = ctx.job(d0, make_params(0.15, 10.0), L, its)
        fp = job_footprint((n2, n1), dtype, L, its)
        assert fp == job.bytes() + 8 * (n2 + 2) * (n1 + 2)
        with pytest.raises(TvsError) as e:
            job.result()
        assert e.value.code == TVS_EBUSY
        job.close()


def test_batch_of_uneven_images(ctx):
    """A batch of images of uneven sizes and layouts, advanced together one
    sweep per call: every result equals the image solved alone."""
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    rng = np.random.default_rng(4)
    sizes = [32, 48, 64, 96]
    specs = []
    for k in range(8):
        n = int(rng.choice(sizes))
        m = 2 if n <= 48 else 4
        sigma = float(rng.choice([0.05, 0.1, 0.2]))
        specs.append((n, m, sigma, 100 + k))
    its = make_iters(2, 3)
    jobs, refs, imgs = [], [], []
    for n, m, sigma, seed in specs:
        _, d64 = synth.noisy_f32(n, n, sigma, seed)
        delta, alpha = synth.params_for_sigma(sigma)
        d0 = torch.tensor(d64, dtype=torch.float32, device=DEV)
        prm, L = make_params(delta, alpha), make_layout(m, m, 4, 4)
        refs.append(one_shot(ctx, d0, prm, L, its))
        jobs.append(ctx.job(d0, prm, L, its))
        imgs.append((d64, delta, alpha, (m, m, 4, 4)))
    run_jobs(ctx, jobs)
    for job, (d_ref, tau_ref, _) in zip(jobs, refs):
        d, tau, _ = job.result()
        torch.cuda.synchronize()
        assert torch.equal(d, d_ref) and torch.equal(tau, tau_ref)
        job.close()
    # the first two against the FP64 oracle (float32 bar)
    for (d64, delta, alpha, lay), (d_ref, _, _) in list(zip(imgs, refs))[:2]:
        n = d64.shape[0]
        tau_o, _, _ = osw.step1_schwarz(d64, delta, osw.Layout(n, n, *lay, step=1), 2, 3)
        d_o, _, _ = osw.step2_schwarz(d64, tau_o, alpha, osw.Layout(n, n, *lay, step=2), 2, 3)
        assert np.abs(d_ref.double().cpu().numpy() - d_o).max() < 1e-4


def test_batch_mix_of_the_64_image_workload_shapes(ctx):
    """One job at each side of the 64-image workload (128, 256, 512, 1024)
    with its layout (4 x 4 with 8-pixel stripes up to 256, 8 x 8 with 8 at
    512 and 16 at 1024), float32, reduced counts, advanced together: each
    result equals its one-shot solve bit for bit, and the 128 and 256 images
    match the FP64 oracle within the float32 bar."""
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    specs = [(128, (4, 4, 8, 8)), (256, (4, 4, 8, 8)), (512, (8, 8, 8, 8)), (1024, (8, 8, 16, 16))]
    its = make_iters(2, 3)
    jobs, refs, imgs = [], [], []
    for k, (n, lay) in enumerate(specs):
        _, d64 = synth.noisy_f32(n, n, 0.1, 400 + k)
        delta, alpha = synth.params_for_sigma(0.1)
        d0 = torch.tensor(d64, dtype=torch.float32, device=DEV)
        prm, L = make_params(delta, alpha), make_layout(*lay)
        refs.append(one_shot(ctx, d0, prm, L, its))
        jobs.append(ctx.job(d0, prm, L, its))
        imgs.append((d64, delta, alpha, lay))
    run_jobs(ctx, jobs)
    for job, (d_ref, tau_ref, _) in zip(jobs, refs):
        d, tau, _ = job.result()
        torch.cuda.synchronize()
        assert torch.equal(d, d_ref) and torch.equal(tau, tau_ref)
        job.close()
    for (d64, delta, alpha, lay), (d_ref, tau_ref, _) in list(zip(imgs, refs))[:2]:
        n = d64.shape[0]
        tau_o, _, _ = osw.step1_schwarz(d64, delta, osw.Layout(n, n, *lay, step=1), 2, 3)
        d_o, _, _ = osw.step2_schwarz(d64, tau_o, alpha, osw.Layout(n, n, *lay, step=2), 2, 3)
        assert np.abs(tau_ref.double().cpu().numpy() - tau_o).max() < 1e-5
        assert np.abs(d_ref.double().cpu().numpy() - d_o).max() < 1e-4


def test_serving_loop_interleaves_and_matches_alone(ctx):
    """Poisson arrivals of uneven requests through the continuous-batching
    server with a budget that holds only a few jobs: every result equals the
    request solved alone, the budget is never exceeded, and requests run
    interleaved."""
    from paper_2602_17494_amd import job_footprint, make_iters, make_layout, make_params
    from paper_2602_17494_amd.serve import Request, latency_summary, serve
    rng = np.random.default_rng(5)
    its = make_iters(3, 5)
    reqs, refs, t = [], {}, 0.0
    for k in range(10):
        t += float(rng.exponential(0.002))
        n = int(rng.integers(32, 97))
        sigma = float(rng.uniform(0.05, 0.2))
        _, d64 = synth.noisy_f32(n, n, sigma, 200 + k)
        delta, alpha = synth.params_for_sigma(sigma)
        d0 = torch.tensor(d64, dtype=torch.float32, device=DEV)
        m = max(1, min(4, round(n / 32)))
        prm, L = make_params(delta, alpha), make_layout(m, m, 0 if m == 1 else 4, 0 if m == 1 else 4)
        refs[k] = one_shot(ctx, d0, prm, L, its)
        reqs.append(Request(k, d0, prm, L, its, arrival=t))
    fps = [job_footprint(tuple(r.d0.shape), r.d0.dtype, r.layout, r.iters) for r in reqs]
    budget = int(2.5 * max(fps))
    results, srv = serve(ctx, reqs, budget)
    assert sorted(r.rid for r in results) == list(range(10))
    assert srv.peak_in_use <= budget
    assert srv.rounds < sum(2 * its.sweeps for _ in reqs)  # rounds served several jobs at once
    for r in results:
        d_ref, tau_ref, _ = refs[r.rid]
        assert torch.equal(r.d, d_ref) and torch.equal(r.tau, tau_ref)
        assert r.finished >= r.admitted >= 0
    lat = latency_summary(results)
    assert lat["n"] == 10 and lat["p99"] >= lat["p50"] > 0


def test_graph_replays_match_eager_sweeps(ctx):
    """Sweep bodies are replayed from recorded graphs (kernel timing off) or
    run eagerly (timing on).  Two jobs on the same image, advanced one sweep
    at a time with synchronisations and eager work of their own between the
    replays (five sweeps with an even inner count replay one graph four
    times per step): both equal the one-shot solve bit for bit."""
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    _, d64 = synth.noisy_f32(52, 44, 0.1, 21)
    d0 = torch.tensor(d64, dtype=torch.float32, device=DEV)
    prm, L, its = make_params(0.15, 10.0), make_layout(2, 2, 4, 4), make_iters(5, 4)
    d_ref, tau_ref, _ = one_shot(ctx, d0, prm, L, its)
    graph_job = ctx.job(d0, prm, L, its)
    ctx.timing(True)
    eager_job = ctx.job(d0, prm, L, its)
    ctx.timing(False)
    while not graph_job.done:
        ctx.batch_sweep([graph_job])
        torch.cuda.synchronize()
        ctx.timing(True)
        ctx.batch_sweep([eager_job])
        ctx.timing(False)
        torch.cuda.synchronize()
        assert graph_job.status()[:2] == eager_job.status()[:2]
    ctx.timing_reset()
    for job in (graph_job, eager_job):
        d, tau, _ = job.result()
        torch.cuda.synchronize()
        assert torch.equal(d, d_ref) and torch.equal(tau, tau_ref)
        job.close()


def test_nonfinite_job_fails_alone(ctx):
    """A job whose image holds a NaN fails at the end of Step 1 with
    TVS_ENONFINITE; the batch call goes on, and the healthy job in the same
    batch still equals its one-shot solve bit for bit."""
    from paper_2602_17494_amd import TvsError, make_iters, make_layout, make_params
    n2, n1 = 40, 56
    _, d64 = synth.noisy_f32(n2, n1, 0.1, 13)
    good = torch.tensor(d64, dtype=torch.float32, device=DEV)
    bad = good.clone()
    bad[7, 9] = float("nan")
    prm, L, its = make_params(0.15, 10.0), make_layout(2, 2, 4, 4), make_iters(2, 3)
    d_ref, tau_ref, _ = one_shot(ctx, good, prm, L, its)
    jb, jg = ctx.job(bad, prm, L, its), ctx.job(good, prm, L, its)
    rounds = 0
    while not (jb.done and jg.done):
        ctx.batch_sweep([j for j in (jb, jg) if not j.done])
        rounds += 1
    torch.cuda.synchronize()
    assert jb.failed and jb.status()[0] == -1 and not jg.failed
    with pytest.raises(TvsError) as e:
        jb.result()
    assert e.value.code == -4  # TVS_ENONFINITE
    with pytest.raises(TvsError):
        jb.export_state()
    d, tau, _ = jg.result()
    torch.cuda.synchronize()
    assert torch.equal(d, d_ref) and torch.equal(tau, tau_ref)
    jb.close()
    jg.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_solves_are_deterministic(ctx, dtype):
    """The same solve twice, and once more in a fresh context, gives the same
    bits: every reduction has a fixed order and no kernel races."""
    from paper_2602_17494_amd import Context, make_iters, make_layout, make_params
    _, d64 = synth.noisy_f32(70, 90, 0.1, 14)
    d0 = torch.tensor(d64, dtype=dtype, device=DEV)
    prm, L, its = make_params(0.15, 10.0), make_layout(3, 3, 4, 6), make_iters(2, 4)
    a = one_shot(ctx, d0, prm, L, its)
    b = one_shot(ctx, d0, prm, L, its)
    with Context(0) as c2:
        c = one_shot(c2, d0, prm, L, its)
    for x in (b, c):
        assert torch.equal(a[0], x[0]) and torch.equal(a[1], x[1])
        assert a[2][0]["energy"] == x[2][0]["energy"] and a[2][1]["gap"] == x[2][1]["gap"]

"""The continuous-batching loop (paper_2602_17494_amd.serve) on the host,
with a stand-in context whose jobs finish after a fixed number of sweeps:
admission in arrival order within the byte budget, one batch call per
round over the live jobs, retirement, progress reports.  Footprints come
from the library's host-side tvs_job_footprint."""
import pytest

torch = pytest.importorskip("torch")


class FakeJob:
    def __init__(self, sweeps):
        self.left = sweeps
        self.closed = False

    @property
    def done(self):
        return self.left == 0

    def result(self):
        return torch.zeros(1), torch.zeros(1), [{}, {}]

    def close(self):
        self.closed = True


class FakeCtx:
    device = "cpu"

    def __init__(self, sweeps):
        self.sweeps, self.created, self.batches = sweeps, [], []

    def job(self, d0, params, layout, iters):
        j = FakeJob(self.sweeps)
        self.created.append(j)
        return j

    def batch_sweep(self, jobs):
        self.batches.append(len(jobs))
        for j in jobs:
            assert not j.done
            j.left -= 1

    def synchronize(self):
        pass


def make_requests(sizes, arrivals):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    from paper_2602_17494_amd.serve import Request
    return [Request(k, torch.zeros((n, n), dtype=torch.float32), make_params(0.15, 10.0),
                    make_layout(2, 2, 8, 8), make_iters(3, 5), arrival=a)
            for k, (n, a) in enumerate(zip(sizes, arrivals))]


def test_admission_within_budget_and_fifo():
    from paper_2602_17494_amd import job_footprint, make_iters, make_layout
    from paper_2602_17494_amd.serve import Server
    sizes = [64, 128, 64, 96, 64]
    fp = [job_footprint((n, n), torch.float32, make_layout(2, 2, 8, 8), make_iters(3, 5)) for n in sizes]
    budget = fp[0] + fp[1]          # the first two fit together, the third must wait
    ctx = FakeCtx(sweeps=2)
    srv = Server(ctx, budget)
    for r in make_requests(sizes, [0.0] * 5):
        srv.submit(r)
    order, t = [], [0.0]
    while srv.queue or srv.live:
        done = srv.round(lambda: t[0])
        order += [res.rid for res in done]
        assert srv.in_use <= budget and srv.peak_in_use <= budget
    assert order == [0, 1, 2, 3, 4]  # equal-length jobs admitted in order finish in order
    assert all(j.closed for j in ctx.created)
    assert srv.in_use == 0


def test_request_over_budget_rejected():
    from paper_2602_17494_amd.serve import Server
    srv = Server(FakeCtx(1), budget=1)
    with pytest.raises(ValueError):
        srv.submit(make_requests([64], [0.0])[0])


def test_serve_reports_progress_and_latencies():
    from paper_2602_17494_amd.serve import serve
    ctx = FakeCtx(sweeps=3)
    seen = []
    reqs = make_requests([64] * 7, [0.0, 0.0, 0.001, 0.002, 0.002, 0.003, 0.003])
    results, srv = serve(ctx, reqs, budget=1 << 40, progress=seen.append, every=2)
    assert sorted(r.rid for r in results) == list(range(7))
    # reported whenever the finished count crosses a multiple of `every`
    assert seen == sorted(set(seen)) and seen[-1] == 7
    assert all(b // 2 > a // 2 for a, b in zip([0] + seen, seen))
    assert all(r.finished >= r.admitted >= r.arrival - 1e-9 for r in results)
    assert max(ctx.batches) > 1      # requests arriving together share batch calls

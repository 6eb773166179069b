"""The continuous-batching loop (paper_2602_17494_amd.serve) on the host,
with a stand-in context whose jobs finish after a fixed number of sweeps:
admission in arrival order within the byte budget, one batch call per
round over the live jobs, retirement, progress reports.  Footprints come
from the library's host-side tvs_job_footprint."""
import pytest

torch = pytest.importorskip("torch")


class FakeJob:
    def __init__(self, sweeps, fail=False):
        self.left = sweeps
        self.closed = False
        self.fail = fail

    @property
    def done(self):
        return self.left == 0

    @property
    def failed(self):
        return self.fail and self.left == 0

    def result(self):
        if self.failed:
            from paper_2602_17494_amd import TvsError
            raise TvsError(-4, "step 1: non-finite energy or gap")
        return torch.zeros(1), torch.zeros(1), [{}, {}]

    def close(self):
        self.closed = True


class FakeCtx:
    device = "cpu"

    def __init__(self, sweeps, fail_ids=()):
        self.sweeps, self.created, self.batches = sweeps, [], []
        self.fail_ids = set(fail_ids)

    def job(self, d0, params, layout, iters):
        j = FakeJob(self.sweeps, fail=len(self.created) in self.fail_ids)
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
    assert not srv.submit(make_requests([64], [0.0])[0])
    out = srv.round(lambda: 0.0)
    assert len(out) == 1 and out[0].d is None and "over the budget" in out[0].error
    assert not srv.queue and not srv.live


def test_unsupported_shape_refused_alone():
    """A request whose shape the library refuses (image sides above 5119) is
    retired with the library's message; the others are served."""
    from paper_2602_17494_amd.serve import serve
    reqs = make_requests([64, 64, 64], [0.0, 0.0, 0.0])
    reqs[1].d0 = torch.zeros((5120, 64), dtype=torch.float32)
    ctx = FakeCtx(sweeps=2)
    results, srv = serve(ctx, reqs, budget=1 << 40)
    by = {r.rid: r for r in results}
    assert sorted(by) == [0, 1, 2]
    assert by[1].d is None and "5120" in by[1].error
    assert by[0].d is not None and by[2].d is not None
    assert len(ctx.created) == 2 and srv.in_use == 0


def test_max_live_serves_one_at_a_time():
    from paper_2602_17494_amd.serve import serve
    ctx = FakeCtx(sweeps=2)
    results, srv = serve(ctx, make_requests([64] * 4, [0.0] * 4), budget=1 << 40, max_live=1)
    assert [r.rid for r in results] == [0, 1, 2, 3]
    assert max(ctx.batches) == 1


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


def test_failed_job_is_retired_alone():
    """A job that fails (the library reports non-finite statistics) ends as a
    result carrying the error; the others finish normally."""
    from paper_2602_17494_amd.serve import serve
    ctx = FakeCtx(sweeps=2, fail_ids={1})
    results, srv = serve(ctx, make_requests([64] * 3, [0.0] * 3), budget=1 << 40)
    by = {r.rid: r for r in results}
    assert by[1].d is None and "non-finite" in by[1].error
    assert by[0].error == "" and by[2].error == "" and by[0].d is not None
    assert srv.in_use == 0 and all(j.closed for j in ctx.created)


def test_cancel_queued_and_running():
    from paper_2602_17494_amd import job_footprint, make_iters, make_layout
    from paper_2602_17494_amd.serve import Server
    fp = job_footprint((64, 64), torch.float32, make_layout(2, 2, 8, 8), make_iters(3, 5))
    ctx = FakeCtx(sweeps=3)
    srv = Server(ctx, budget=2 * fp)
    for r in make_requests([64] * 4, [0.0] * 4):
        srv.submit(r)
    srv.round(lambda: 0.0)                    # admits 0 and 1, sweeps them once
    assert [r.rid for r, _, _ in srv.live] == [0, 1]
    assert srv.cancel(1) and srv.in_use == fp and ctx.created[1].closed
    assert srv.cancel(3) and [r.rid for r in srv.queue] == [2]
    assert not srv.cancel(3) and not srv.cancel(99)
    done = []
    while srv.queue or srv.live:
        done += [r.rid for r in srv.round(lambda: 0.0)]
    assert sorted(done) == [0, 2]

"""Continuous batching of TV-Stokes denoise requests on one GPU.

Each request is a job of the HIP library (tvs_job_*): its dual variables and
plans stay resident on the device between Schwarz sweeps.  The server loop
admits waiting requests in arrival order while the sum of the admitted jobs'
device footprints stays within a byte budget, advances every live job by one
sweep per round (one tvs_batch_sweep call), and retires the jobs that have
finished, so that requests arriving while others run join the next round and
their work interleaves on the device with the running ones.  A job computes
exactly what a one-shot tvs_schwarz_solve of its image computes.  A request
whose job fails (non-finite data) is retired with its error and does not
disturb the others; so is a request the library refuses (a shape it does not
support, a footprint over the budget), at submission or at admission.
Queued or running requests can be cancelled.
"""
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from .tvs import Context, Job, TvsError, job_footprint


@dataclass
class Request:
    rid: int
    d0: torch.Tensor          # GPU image, float32 or float64
    params: object            # tvs_params
    layout: object            # tvs_layout
    iters: object             # tvs_iters
    arrival: float = 0.0      # seconds after the start of the run
    footprint: int = 0


@dataclass
class Result:
    rid: int
    d: torch.Tensor           # None if the job failed
    tau: torch.Tensor         # None if the job failed
    stats: list
    arrival: float
    admitted: float
    finished: float
    error: str = ""           # the library's message if the job failed

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclass
class Server:
    ctx: Context
    budget: int                       # device bytes the live jobs may hold
    queue: list = field(default_factory=list)
    live: list = field(default_factory=list)   # (request, job, admitted time)
    in_use: int = 0
    peak_in_use: int = 0
    rounds: int = 0
    max_live: int = 0                 # > 0: at most this many live jobs
    peak_probe: int = 0               # largest value of serve()'s probe
    refused: list = field(default_factory=list)  # results of refused requests, not yet returned

    def _refuse(self, req, now, msg):
        self.refused.append(Result(req.rid, None, None, [], req.arrival, now, now, msg))

    def submit(self, req: Request, now=0.0):
        """Queue a request; False (and a result carrying the reason, returned
        by the next round) if the library refuses its shape or its footprint
        exceeds the whole budget."""
        try:
            req.footprint = job_footprint(tuple(req.d0.shape), req.d0.dtype, req.layout, req.iters)
        except TvsError as e:
            self._refuse(req, now, str(e))
            return False
        if req.footprint > self.budget:
            self._refuse(req, now, f"needs {req.footprint} bytes, over the budget of {self.budget}")
            return False
        self.queue.append(req)
        return True

    def _admit(self, now):
        while (self.queue and self.in_use + self.queue[0].footprint <= self.budget
               and (self.max_live <= 0 or len(self.live) < self.max_live)):
            req = self.queue.pop(0)
            try:
                job = self.ctx.job(req.d0, req.params, req.layout, req.iters)
            except TvsError as e:
                self._refuse(req, now, str(e))
                continue
            self.in_use += req.footprint
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.live.append((req, job, now))

    def round(self, now_fn):
        """Admit what fits, advance every live job by one sweep, retire the
        finished ones; returns their results (and those of requests refused
        since the last round)."""
        self._admit(now_fn())
        refused, self.refused = self.refused, []
        if not self.live:
            return refused
        self.ctx.batch_sweep([job for _, job, _ in self.live])
        self.rounds += 1
        self.ctx.synchronize()
        out, keep = [], []
        for req, job, adm in self.live:
            if job.done:
                if job.failed:
                    try:
                        job.result()
                        err = "failed"
                    except TvsError as e:
                        err = str(e)
                    out.append(Result(req.rid, None, None, [], req.arrival, adm, now_fn(), err))
                else:
                    d, tau, st = job.result()
                    self.ctx.synchronize()
                    out.append(Result(req.rid, d, tau, st, req.arrival, adm, now_fn()))
                job.close()
                self.in_use -= req.footprint
            else:
                keep.append((req, job, adm))
        self.live = keep
        return refused + out

    def cancel(self, rid):
        """Drop request `rid`, queued or running (its job is freed); False if
        it is unknown or already finished."""
        for i, req in enumerate(self.queue):
            if req.rid == rid:
                del self.queue[i]
                return True
        for i, (req, job, _) in enumerate(self.live):
            if req.rid == rid:
                job.close()
                self.in_use -= req.footprint
                del self.live[i]
                return True
        return False


def serve(ctx, requests, budget, clock=time.perf_counter, progress=None, every=50, max_live=0, probe=None):
    """Run `requests` (with arrival offsets in seconds) through a server
    with the given byte budget (and at most max_live live jobs, if > 0) in
    real time; returns the results in completion order and the server (for
    its counters).  progress, if given, is called with the number of
    finished requests every `every`; probe, if given, after every round,
    and the largest value it returns is kept as srv.peak_probe (for example
    the device bytes in use)."""
    pending = sorted(requests, key=lambda r: r.arrival)
    srv = Server(ctx, budget, max_live=max_live)
    t0 = clock()
    now = lambda: clock() - t0
    done = []
    while pending or srv.queue or srv.live or srv.refused:
        while pending and pending[0].arrival <= now():
            srv.submit(pending.pop(0), now())
        if not srv.queue and not srv.live and not srv.refused:
            time.sleep(max(0.0, min(0.01, pending[0].arrival - now())))
            continue
        before = len(done)
        done.extend(srv.round(now))
        if probe is not None:
            srv.peak_probe = max(srv.peak_probe, probe())
        if progress and len(done) // every > before // every:
            progress(len(done))
    return done, srv


def latency_summary(results):
    lat = np.array([r.latency for r in results])
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "mean": float(lat.mean()), "n": int(lat.size)}

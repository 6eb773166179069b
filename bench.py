#!/usr/bin/env python3
"""Throughput benchmark of the TV-Stokes hot path on one MI355X.

One step = one full solve of the workload: Step 1 (TFS dual iterations with
the divergence-free projection) and Step 2 (IRV2 dual iterations), each as
`sweeps` outer iterations of the overlapping Schwarz method with `inner`
subdomain iterations, on a 2048 x 2048 float32 image (sigma = 0.1) split
into 8 x 8 subdomains with a 16-pixel shared stripe; FP64 only in the energy,
residual and duality-gap reductions.  The input image is resident in device
memory before the timed region starts.

value = pixel-iterations per second / 1e6, counting each global grid point
once per dual iteration: (|Omega-tilde| + |Omega|) * sweeps * inner per step.

Also reported: p50/p99 latency of one solve, the roofline of the dominant
kernel (achieved algorithmic GB/s from HIP events around its launches), the
same solve in float64 (error of the float32 image against it) and the plain
single-domain float64 solve with the same number of dual iterations per step,
and the FP64 CPU oracle timed on a bounded sample of the workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TIMING_EVERY = 16
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--sigma", type=float, default=0.1)
    ap.add_argument("--layout", type=int, nargs=4, default=[8, 8, 16, 16], metavar=("M2", "M1", "SY", "SX"))
    ap.add_argument("--sweeps", type=int, default=20)
    ap.add_argument("--inner", type=int, default=500)
    ap.add_argument("--no-compare", action="store_true", help="skip the float64 comparator solves")
    ap.add_argument("--tiles", type=int, nargs=5, default=None, metavar=("RUN1", "RUN1D", "ROWS", "COLS", "RUN2"),
                    help="force the workgroup shapes instead of tuning them (profiling runs: no tuning launches)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="host cores (worker processes) for the CPU oracle baseline, at most os.cpu_count()")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (counter calibration)")
    ap.add_argument("--batch", action="store_true",
                    help="instead: a batch of 64 images of uneven sizes as resident jobs, one "
                         "batch call per Schwarz sweep, against solving them one by one")
    ap.add_argument("--serve", action="store_true",
                    help="instead: Poisson arrivals (sides 256-4096) through the continuous-batching "
                         "server, FP32 Schwarz jobs against plain single-domain FP64 jobs")
    ap.add_argument("--requests", type=int, default=24, help="requests in --serve mode")
    ap.add_argument("--serve-parts", default="fp32,plain,fifo",
                    help="servers --serve runs (comma list of fp32, plain, fifo)")
    ap.add_argument("--timing", action="store_true",
                    help="--batch: time one launch in 16 of each kernel class (eager launches, no graphs)")
    ap.add_argument("--burst", type=int, default=24,
                    help="--serve: requests of the capacity (burst) runs, the first of the Poisson ones")
    ap.add_argument("--lp-compare", action="store_true",
                    help="instead: time one Step-1 inner iteration with the image-method LP_m and "
                         "with the block-DCT formula (float32, the bench workload's layout)")
    return ap.parse_args()


def batch_mode(args):
    """64 images, sides uniform in {128, 256, 512, 1024}, float32; layout 4x4
    with s = 8 up to 256, 8x8 from 512 (s = 16 at 1024); every image a job,
    all advanced by one sweep per batch call until all are done.  Compared with
    the same images solved one after another (tvs_schwarz_solve)."""
    import numpy as np
    import torch
    import synth
    from paper_2602_17494_amd import Context, make_iters, make_layout, make_params
    ctx = Context(0)
    rng = np.random.default_rng(4)
    its = make_iters(args.sweeps, args.inner)
    work = []
    for k in range(64):
        n = int(rng.choice([128, 256, 512, 1024]))
        lay = (4, 4, 8, 8) if n <= 256 else (8, 8, 16 if n == 1024 else 8, 16 if n == 1024 else 8)
        _, d64 = synth.noisy_f32(n, n, args.sigma, 4000 + k)
        delta, alpha = synth.params_for_sigma(args.sigma)
        work.append((torch.tensor(d64, dtype=torch.float32, device="cuda:0"),
                     make_params(delta, alpha), make_layout(*lay)))
    pix = sum(((d.shape[0] + 1) ** 2 + d.shape[0] ** 2) for d, _, _ in work) * args.sweeps * args.inner
    # one by one (plans cached in the context after a first pass)
    for d0, prm, lay in work:
        ctx.schwarz_solve(d0, prm, lay, make_iters(1, 1), stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d0, prm, lay in work:
        ctx.schwarz_solve(d0, prm, lay, its, stats=False)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    # as jobs: creation (plans, copies) outside the timed region
    jobs = [ctx.job(d0, prm, lay, its) for d0, prm, lay in work]
    torch.cuda.synchronize()
    if args.timing:
        # per-class kernel times (launched eagerly: no graph while timing)
        ctx.timing_reset()
        ctx.timing(True, every=TIMING_EVERY)
    t0 = time.perf_counter()
    calls = 0
    while True:
        live = [j for j in jobs if not j.done]
        if not live:
            break
        ctx.batch_sweep(live)
        calls += 1
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    kernels = None
    if args.timing:
        ctx.timing(False)
        kernels = {k: {"timed_launches": v[0], "avg_us": round(v[1] / v[0] * 1e3, 2) if v[0] else None,
                       "total_ms_est": round(v[1] * TIMING_EVERY, 1)}
                   for k, v in sorted(ctx.timing_read().items(), key=lambda kv: -kv[1][1])}
    out = {"metric": "Mpix*iter/s, batch of 64 uneven images (FP32 Schwarz, both steps)",
           "value": round(pix / t_batch / 1e6, 1), "unit": "Mpix*iter/s",
           "seconds": round(t_batch, 3), "batch_calls": calls,
           "one_by_one": {"seconds": round(t_seq, 3), "mpix_iter_s": round(pix / t_seq / 1e6, 1)},
           "megapixels": round(sum(d.numel() for d, _, _ in work) / 1e6, 2),
           "sweeps": args.sweeps, "inner": args.inner, "dtype": "f32", "data": "synthetic"}
    if kernels is not None:
        out["kernels"] = kernels
    for j in jobs:
        j.close()
    print(json.dumps(out), flush=True)


def serve_mode(args):
    """Serving workload: Poisson arrivals of denoise requests, image side
    uniform in [256, 4096], sigma uniform in [0.05, 0.2], served twice on the
    same arrivals, each time through the continuous-batching server
    (paper_2602_17494_amd.serve, admission by footprint within 64 GB, one
    batch call per round over all live jobs, 10 sweeps x 100 inner
    iterations per step):
      * FP32 Schwarz jobs with FP64 reductions, layout M = clamp(round(N /
        256), 1, 16) per axis, 16-pixel shared stripes;
      * the plain single-domain FP64 solve as jobs (layout 1 x 1: 10 x 100
        is exactly 1000 Chambolle iterations per step);
      * and the plain FP64 solve served first come, first served, one
        request at a time as a one-shot solve in a context of its own with
        the workgroup shapes given (no tuning): batching cannot help a
        whole-grid solve, so this is the comparator's own best server, and
        the speedups are taken against the better of the two.
    The arrival rate is 0.7 of the plain FP64 capacity, measured first as
    one-at-a-time plain solves of a sample of sides (fitted to a + b N^2 and
    averaged over the side distribution).  Latencies are measured in real
    time for both servers; the device bytes in use are sampled after every
    round.  At that load both servers keep up with the arrivals, so their
    served pixel-iterations per second only restate the offered load; the
    capacity of each is measured separately as a burst: the first
    --burst requests all arriving at once, served to the last."""
    import numpy as np
    import torch
    import synth
    from paper_2602_17494_amd import Context, make_iters, make_layout, make_params
    from paper_2602_17494_amd.serve import Request, latency_summary, serve
    rng = np.random.default_rng(5)
    its = make_iters(10, 100)
    lo, hi = 256, 4096
    specs = []
    for k in range(args.requests):
        n = int(rng.integers(lo, hi + 1))
        sigma = float(rng.uniform(0.05, 0.2))
        m = max(1, min(16, round(n / 256)))
        specs.append((k, n, sigma, m))
    # plain FP64 capacity: one-at-a-time solves of a sample of sides
    sample_n = [256, 768, 1280, 1792, 2304, 2816, 3328, 3840, 4096]
    ts = []
    with Context(0) as pc:
        for n in sample_n:
            _, d64 = synth.noisy_f32(n, n, 0.1, 90 + n)
            d0 = torch.tensor(d64, dtype=torch.float64, device="cuda:0")
            prm = make_params(*synth.params_for_sigma(0.1))
            pc.schwarz_solve(d0, prm, make_layout(), make_iters(1, 1), stats=False)  # plans
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pc.schwarz_solve(d0, prm, make_layout(), its, stats=False)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            del d0
            print(f"serve: plain FP64 service time at {n}^2: {ts[-1]:.3f} s", file=sys.stderr, flush=True)
    coef = np.polyfit(np.array(sample_n, dtype=float) ** 2, np.array(ts), 1)
    mean_service = float(np.mean([np.polyval(coef, float(n) ** 2) for _, n, _, _ in specs]))
    rate = 0.7 / mean_service
    arrivals, t = [], 0.0
    for _ in specs:
        t += float(rng.exponential(1.0 / rate))
        arrivals.append(t)
    imgs = {k: synth.noisy_f32(n, n, sigma, 5000 + k)[0] for k, n, sigma, _ in specs}
    free0, total_mem = torch.cuda.mem_get_info(0)

    def used():
        return free0 - torch.cuda.mem_get_info(0)[0]

    def run(kind, burst=0):
        reqs = []
        sel = list(zip(specs, arrivals))[:burst] if burst else list(zip(specs, arrivals))
        for (k, n, sigma, m), a in sel:
            a = 0.0 if burst else a
            delta, alpha = synth.params_for_sigma(sigma)
            if kind == "fp32_schwarz":
                d0 = torch.tensor(imgs[k], dtype=torch.float32, device="cuda:0")
                lay = make_layout(m, m, 16 if m > 1 else 0, 16 if m > 1 else 0)
            else:
                d0 = torch.tensor(imgs[k], dtype=torch.float64, device="cuda:0")
                lay = make_layout()
            reqs.append(Request(k, d0, make_params(delta, alpha), lay, its, arrival=a))
        torch.cuda.synchronize()
        with Context(0) as ctx:
            t0 = time.perf_counter()
            results, srv = serve(ctx, reqs, 64 << 30, probe=used,
                                 progress=lambda done: print(f"serve {kind}: {done} of {len(reqs)} requests "
                                                             "served", file=sys.stderr, flush=True), every=10)
            wall = time.perf_counter() - t0
        ok = [r for r in results if not r.error]
        pix = sum(((r.d.shape[0] + 1) ** 2 + r.d.shape[0] ** 2) for r in ok) * 10 * 100
        lat = latency_summary(ok)
        rec = {"served": len(ok), "refused_or_failed": len(results) - len(ok),
               "latency_s": {"p50": round(lat["p50"], 4), "p99": round(lat["p99"], 4),
                             "mean": round(lat["mean"], 4)},
               "throughput_mpix_iter_s": round(pix / wall / 1e6, 1), "wall_s": round(wall, 2),
               "rounds": srv.rounds, "peak_footprint_bytes": srv.peak_in_use,
               "peak_device_bytes_measured": int(srv.peak_probe)}
        del reqs, results
        torch.cuda.synchronize()
        return rec

    def run_fifo(burst=0):
        """The plain FP64 solve, first come first served in real time: sleep
        until the next arrival when idle, then a one-shot solve in a fresh
        context (its plans are freed with it) with the shapes given."""
        sel = sorted(list(zip(specs, arrivals))[:burst] if burst else list(zip(specs, arrivals)),
                     key=lambda sa: 0.0 if burst else sa[1])
        lat, pix = [], 0
        t0 = time.perf_counter()
        for i, ((k, n, sigma, m), a) in enumerate(sel):
            a = 0.0 if burst else a
            now = time.perf_counter() - t0
            if now < a:
                time.sleep(a - now)
            delta, alpha = synth.params_for_sigma(sigma)
            d0 = torch.tensor(imgs[k], dtype=torch.float64, device="cuda:0")
            with Context(0) as ctx:
                ctx.set_tiles(2, 2, 8, 3, 2)  # every shape given: no timing launches
                ctx.schwarz_solve(d0, make_params(delta, alpha), make_layout(), its, stats=False)
                torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0 - a)
            pix += ((n + 1) ** 2 + n ** 2) * 10 * 100
            del d0
            if (i + 1) % 10 == 0:
                print(f"serve fp64_fifo: {i + 1} of {len(sel)} requests served", file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        lat = np.array(lat)
        return {"served": len(sel), "refused_or_failed": 0,
                "latency_s": {"p50": round(float(np.percentile(lat, 50)), 4),
                              "p99": round(float(np.percentile(lat, 99)), 4), "mean": round(float(lat.mean()), 4)},
                "throughput_mpix_iter_s": round(pix / wall / 1e6, 1), "wall_s": round(wall, 2)}

    parts = set(args.serve_parts.split(","))
    nb = min(args.burst, len(specs))
    out = {"metric": "continuous-batching serving: p50/p99 latency and throughput, FP32 Schwarz jobs against "
                     "the plain single-domain FP64 solve (as jobs, and first come first served) on the same arrivals",
           "requests": len(specs), "sides": [lo, hi], "rate_per_s": round(rate, 4),
           "plain_fp64_mean_service_s": round(mean_service, 4),
           "plain_fp64_service_fit_s": {"a": float(coef[1]), "b_per_px": float(coef[0])},
           "iterations_per_step": "10 sweeps x 100 inner", "burst_requests": nb}
    for name, part, fn in (("fp32_schwarz", "fp32", lambda b: run("fp32_schwarz", b)),
                           ("fp64_plain", "plain", lambda b: run("fp64_plain", b)),
                           ("fp64_plain_fifo", "fifo", run_fifo)):
        if part in parts:
            rec = fn(0)
            rec["burst_capacity"] = fn(nb)
            out[name] = rec
    if "fp32_schwarz" in out:
        comps = [out[c] for c in ("fp64_plain", "fp64_plain_fifo") if c in out]
        if comps:
            best_p99 = min(c["latency_s"]["p99"] for c in comps)
            best_cap = max(c["burst_capacity"]["throughput_mpix_iter_s"] for c in comps)
            out["p99_speedup"] = round(best_p99 / out["fp32_schwarz"]["latency_s"]["p99"], 2)
            out["capacity_speedup"] = round(out["fp32_schwarz"]["burst_capacity"]["throughput_mpix_iter_s"] /
                                            best_cap, 2)
    out.update({"device_bytes_total": int(total_mem), "data": "synthetic"})
    print(json.dumps(out), flush=True)


def lp_compare_mode(args):
    """Step 1 with 1 sweep and K inner iterations, for K = 2 and K = 12, with
    each realisation of LP_m; the time of one inner iteration is the
    difference over the 10 extra iterations (the set-up and the sweep's
    global parts cancel).  For the block formula the four batched products
    are also timed with HIP events and priced against the FP32 matrix peak."""
    import torch

    import synth
    from paper_2602_17494_amd import TVS_LP_BLOCKDCT, TVS_LP_IMAGE, Context, make_iters, make_layout, make_params

    n = args.size
    delta, _ = synth.params_for_sigma(args.sigma)
    _, d64 = synth.noisy_f32(n, n, args.sigma, 31)
    dev = torch.device("cuda", 0)
    d0 = torch.tensor(d64, dtype=torch.float32, device=dev)
    prm, lay = make_params(delta, 1.0), make_layout(*args.layout)
    out, taus = {}, {}
    for name, kind in (("image", TVS_LP_IMAGE), ("blockdct", TVS_LP_BLOCKDCT)):
        ctx = Context(0)
        ctx.set_local_projection(kind)
        t = {}
        for k in (2, 12):
            ctx.step1(d0, prm, lay, make_iters(1, k), stats=False)  # plans, warm-up
            torch.cuda.synchronize()
            reps = []
            for _ in range(3):
                t0 = time.perf_counter()
                tau, _ = ctx.step1(d0, prm, lay, make_iters(1, k), stats=False)
                torch.cuda.synchronize()
                reps.append(time.perf_counter() - t0)
            t[k] = min(reps)
            taus[name] = tau
        per_inner = (t[12] - t[2]) / 10
        rec = {"ms_per_inner": per_inner * 1e3, "ctx_bytes": ctx.bytes()}
        if kind == TVS_LP_BLOCKDCT:
            ctx.timing(True, 1)
            ctx.step1(d0, prm, lay, make_iters(1, 4), stats=False)
            torch.cuda.synchronize()
            launches, ms, flops = ctx.timing_read()["s1_bdct"]
            ctx.timing(False)
            tf = flops / (ms * 1e-3) / 1e12
            rec.update({"apply_ms": ms / launches, "tflops": tf, "fp32_peak_tflops": FP32_PEAK_TFLOPS,
                        "frac": tf / FP32_PEAK_TFLOPS})
        out[name] = rec
        ctx.close()
    diff = float((taus["image"].double() - taus["blockdct"].double()).abs().max())
    print(json.dumps({"metric": "ms per Step-1 inner iteration", "workload": f"{n}x{n} float32 Schwarz "
                      f"{args.layout[0]}x{args.layout[1]} s={args.layout[2]}", "image": out["image"],
                      "blockdct": out["blockdct"], "slowdown": out["blockdct"]["ms_per_inner"] /
                      out["image"]["ms_per_inner"], "max_abs_tau_diff": diff}))


def calibrate_copy():
    """A plain copy of known size: under rocprofv3 --pmc its FETCH_SIZE and
    WRITE_SIZE per dispatch give the factor from counter KiB to bytes."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": n * 4, "bytes_written": n * 4}), flush=True)


def copy_bandwidth():
    """HBM bandwidth a plain device copy reaches on this GPU (1 GiB read and
    1 GiB written per copy, best of 5, HIP events on the current stream):
    the practical ceiling next to the 8 TB/s published peak."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2 * n * 4 / (best * 1e-3) / 1e9


def _code_only(text):
    """C++ source without comments and blank space, so that editing a comment
    does not invalidate measurements taken on the same code."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(csrc=None, read=None):
    """Hash of the code of every HIP source of the library (comments and
    spacing ignored): the kernels, and the host orchestration, which sets the
    frame pitch, the subdomain and Green-box geometry and the launch sequence
    that decide the counted traffic."""
    csrc = csrc or os.path.join(ROOT, "paper_2602_17494_amd", "csrc")
    names = sorted(os.listdir(csrc)) if read is None else sorted(read)
    h = hashlib.sha256()
    for name in names:
        if read is None:
            with open(os.path.join(csrc, name), encoding="utf-8") as f:
                text = f.read()
        else:
            text = read[name]
        h.update(name.encode())
        h.update(_code_only(text).encode())
    return h.hexdigest()[:16]


def read_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it is missing or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(kernel)
    return None if ent is None else ent.get("hbm_bytes_per_launch")


def read_valu_issue(kernel):
    """VALU instruction-issue time per launch of `kernel` (timer name) from the
    committed rocprofv3 SQ counters, or None when missing or taken on other
    code: SQ_INSTS_VALU * 4 cycles over the 1024 SIMDs at 2.4 GHz, the time
    the kernel needs for its vector instructions alone."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            name = json.load(f)["kernels"][kernel]["kernel"]
        with open(os.path.join(ROOT, "profiles", "sq_counters.json")) as f:
            rec = json.load(f)
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(name)
    return None if ent is None else ent.get("valu_issue_us")


def _cpu_sample(n, sigma, lay, m):
    """One worker of the CPU baseline: subdomain m's inner loops of both steps
    (see cpu_baseline), single-threaded; returns the four timings."""
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    import numpy as np

    import synth
    from oracle import schwarz as osw
    from oracle import solvers as osv

    _, d64 = synth.noisy_f32(n, n, sigma, 31)
    delta, alpha = synth.params_for_sigma(sigma)
    m2, m1, sy, sx = lay
    l1 = osw.Layout(n, n, m2, m1, sy, sx, step=1)
    l2 = osw.Layout(n, n, m2, m1, sy, sx, step=2)
    f1 = osv.tfs_data(d64, delta)
    p1 = np.zeros((2, 2) + l1.shape)
    # an untimed first call of each loop takes the one-time costs (transform
    # plans, first touches of the arrays)
    osw.inner_tfs_local(l1, m, p1, np.zeros_like(p1), f1, 1, 0.125)
    t = []
    for iters in (1, 3):
        t0 = time.perf_counter()
        osw.inner_tfs_local(l1, m, p1, np.zeros_like(p1), f1, iters, 0.125)
        t.append(time.perf_counter() - t0)
    s1_iter = max((t[1] - t[0]) / 2, 1e-9)
    s1_sweep = max(t[0] - s1_iter, 0.0)
    f2 = alpha * d64
    p2 = np.zeros((1, 2) + l2.shape)
    osw.inner_rof(l2, m, p2, np.zeros_like(p2), f2, 1, 0.125)
    t2 = []
    for iters in (1, 3):
        t0 = time.perf_counter()
        osw.inner_rof(l2, m, p2, np.zeros_like(p2), f2, iters, 0.125)
        t2.append(time.perf_counter() - t0)
    s2_iter = max((t2[1] - t2[0]) / 2, 1e-9)
    s2_sweep = max(t2[0] - s2_iter, 0.0)
    return s1_iter, s1_sweep, s2_iter, s2_sweep


def cpu_baseline(n, sigma, lay, workers):
    """Time the FP64 oracle on a bounded sample of the workload, on `workers`
    host cores: each worker process runs one interior subdomain's inner loop
    of each step (Algorithm 5 for Step 1, Algorithm 3 for Step 2) at 1 and at
    3 inner iterations after an untimed first call, single-threaded, which separates
    its per-sweep set-up from its per-iteration cost.  The subdomains of a
    sweep are independent (Algorithm 2), so the workers solve them
    side by side: the full workload takes sweeps x ceil(subdomains /
    workers) rounds of the mean per-subdomain time measured while all
    workers ran at once."""
    import multiprocessing as mp

    from oracle import schwarz as osw

    m2, m1, sy, sx = lay
    count = osw.Layout(n, n, m2, m1, sy, sx, step=1).count
    interior = [a * m1 + b for a in range(1, max(2, m2 - 1)) for b in range(1, max(2, m1 - 1))]
    interior = [m for m in interior if m < count] or [0]
    subs = [interior[k % len(interior)] for k in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.starmap(_cpu_sample, [(n, sigma, tuple(lay), m) for m in subs])
    wall = time.perf_counter() - t0
    mean = [sum(r[k] for r in res) / len(res) for k in range(4)]
    return mean + [count, wall]


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.batch or args.serve or args.lp_compare:
        import torch
        if not torch.cuda.is_available():
            print("no GPU available", file=sys.stderr)
            sys.exit(1)
        (batch_mode if args.batch else serve_mode if args.serve else lp_compare_mode)(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design note only", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2602_17494_amd import Context, make_iters, make_layout, make_params

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    n = args.size
    delta, alpha = synth.params_for_sigma(args.sigma)
    _, d64 = synth.noisy_f32(n, n, args.sigma, 31)
    ctx = Context(0)
    if args.tiles:
        ctx.set_tiles(*args.tiles)
    dev = torch.device("cuda", 0)
    d0 = torch.tensor(d64, dtype=torch.float32, device=dev)
    tau = torch.empty((2, n + 1, n + 1), dtype=torch.float32, device=dev)
    d = torch.empty_like(d0)
    prm = make_params(delta, alpha)
    lay = make_layout(*args.layout)
    its = make_iters(args.sweeps, args.inner)
    pix_iters = ((n + 1) * (n + 1) + n * n) * args.sweeps * args.inner

    for _ in range(args.warmup):
        ctx.schwarz_solve(d0, prm, lay, its, d_out=d, tau_out=tau)
    torch.cuda.synchronize()
    ctx.timing_reset()
    # HIP events around one launch in TIMING_EVERY of each kernel class, over
    # the whole timed region (timing every launch would add two event
    # records to each of the ~10^5 launches of a solve)
    ctx.timing(True, every=TIMING_EVERY)
    lat = []
    stats = None
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        _, stats = ctx.schwarz_solve(d0, prm, lay, its, d_out=d, tau_out=tau)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    ctx.timing(False)
    timing = ctx.timing_read()
    value = pix_iters * args.steps / total / 1e6

    # dominant kernel class: largest total time
    dom = max(timing.items(), key=lambda kv: kv[1][1])
    dname, (dlaunch, dms, dbytes) = dom
    achieved = (dbytes / dlaunch) / (dms / dlaunch * 1e-3) / 1e9
    # the committed counters were taken on the default workload only
    profiled = (n == 2048 and list(args.layout) == [8, 8, 16, 16])
    traffic = read_traffic(dname) if profiled else None
    valu_us = read_valu_issue(dname) if profiled else None
    breakdown = {k: {"timed_launches": v[0], "avg_us": round(v[1] / v[0] * 1e3, 2) if v[0] else None,
                     "gbs": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
                 for k, v in sorted(timing.items(), key=lambda kv: -kv[1][1])}

    out = {
        "metric": f"Mpix*iter/s at {n}^2 (FP32 Schwarz, both TV-Stokes steps)",
        "value": round(value, 1),
        "unit": "Mpix*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{n}x{n} float32 image (seeded piecewise-smooth + Gaussian noise "
                         f"sigma={args.sigma}), TFS + IRV2, {args.layout[0]}x{args.layout[1]} "
                         f"subdomains, shared stripe {args.layout[2]}x{args.layout[3]} px, "
                         f"{args.sweeps} sweeps x {args.inner} inner iterations per step, "
                         "FP64 energy/residual/gap reductions"),
            "delta": delta, "alpha": alpha, "t": 0.125,
        },
        "latency_s": {"p50": round(float(np.percentile(lat, 50)), 4),
                      "p99": round(float(np.percentile(lat, 99)), 4)},
        "per_step": {
            "step1_seconds": round(stats[0]["seconds"], 4),
            "step2_seconds": round(stats[1]["seconds"], 4),
            "step1_mpix_iter_s": round((n + 1) ** 2 * args.sweeps * args.inner / stats[0]["seconds"] / 1e6, 1),
            "step2_mpix_iter_s": round(n * n * args.sweeps * args.inner / stats[1]["seconds"] / 1e6, 1),
            "energy": [stats[0]["energy"], stats[1]["energy"]],
            "gap": [stats[0]["gap"], stats[1]["gap"]],
            "residual": [stats[0]["residual"], stats[1]["residual"]],
        },
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes_per_launch": dbytes / dlaunch,
                     "avg_launch_us": round(dms / dlaunch * 1e3, 2),
                     "valu_issue_us": valu_us,
                     "valu_issue_frac": None if valu_us is None else round(valu_us / (dms / dlaunch * 1e3), 3),
                     "copy_gbs": round(copy_bandwidth(), 1)},
        "kernels": breakdown,
    }
    t1 = tuple(args.tiles) if args.tiles else ctx.get_tiles((n, n), torch.float32, lay)
    out["tiles"] = {"forced": bool(args.tiles), "step1_update_run": t1[0], "step1_vecdiv_run": t1[1], "green_rows": t1[2],
                    "green_cols": t1[3], "step2_update_run": t1[4]}

    if not args.no_compare:
        d_f32 = d.double().cpu()
        d064 = torch.tensor(d64, dtype=torch.float64, device=dev)
        t0 = time.perf_counter()
        d_f64, _ = ctx.schwarz_solve(d064, prm, lay, its)
        torch.cuda.synchronize()
        t_f64 = time.perf_counter() - t0
        err = float((d_f32 - d_f64.cpu()).abs().max())
        t0 = time.perf_counter()
        d_plain, st_plain = ctx.schwarz_solve(d064, prm, make_layout(1, 1, 0, 0), its)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        out["compare"] = {
            "f64_same_layout": {"seconds": round(t_f64, 3),
                                "mpix_iter_s": round(pix_iters / t_f64 / 1e6, 1),
                                "max_abs_err_f32_image": err},
            "f64_plain_single_domain": {"seconds": round(t_plain, 3),
                                        "mpix_iter_s": round(pix_iters / t_plain / 1e6, 1),
                                        "step1_seconds": round(st_plain[0]["seconds"], 3),
                                        "step2_seconds": round(st_plain[1]["seconds"], 3)},
            "speedup_vs_f64_plain": round(t_plain / (total / args.steps), 2),
        }

    if not args.no_cpu:
        workers = max(1, min(args.cpu_workers, os.cpu_count() or 1))
        s1_iter, s1_sweep, s2_iter, s2_sweep, nsub, wall = cpu_baseline(n, args.sigma, args.layout, workers)
        rounds = -(-nsub // workers)
        t_full = args.sweeps * rounds * ((s1_sweep + args.inner * s1_iter) + (s2_sweep + args.inner * s2_iter))
        out["cpu_baseline"] = {
            "value": round(pix_iters / t_full / 1e6, 3), "unit": "Mpix*iter/s", "cores": workers,
            "kind": "oracle",
            "sample": (f"FP64 numpy/scipy oracle, {workers} single-threaded worker processes on "
                       f"{workers} host cores (of {os.cpu_count()}), each on an interior subdomain of the "
                       f"{n}^2 {args.layout[0]}x{args.layout[1]} workload: Step-1 inner loop (Alg. 5) at "
                       "1 and 3 iterations, Step-2 inner loop (Alg. 3) at 1 and 3 iterations, side by "
                       f"side; scaled to {args.sweeps} sweeps x {rounds} rounds of {workers} subdomains "
                       f"x {args.inner} inner; {wall:.1f} s wall"),
            "seconds_full_workload_estimate": round(t_full, 1),
        }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

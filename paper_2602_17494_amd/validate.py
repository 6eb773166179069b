"""The domain-decomposition validation protocol of Section 6.3 on one GPU.

Reference: the single-domain (non-DD) solve of each step with many dual
iterations (the paper uses 10^6 per step).  DD: a 3 x 3 decomposition with
shared stripes of 4 rows and 3 columns and relaxation alpha-hat = 0.25, 10
inner iterations per Schwarz sweep.  Reported per step, as energy curves
D(p^n) - D(p*) over the sweeps n:
* Step 1 (TFS), which must approach the reference energy;
* Step 2 for IRV2 and IRV1, once with the DD tangent field (a perturbed
  problem: its energy need not reach the reference one) and once with the
  reference tangent field (which must reach it).
The DD and non-DD images are compared as well (max-abs and PSNR of one
against the other).  Every solve and measure runs in the HIP library; this
module only calls it and collects the curves.  The paper's image is not
available: the command line uses a seeded synthetic 270 x 480 image at
sigma^2 = 0.01.
"""
import argparse
import json
import time

from .tvs import TVS_IRV1, TVS_IRV2, make_iters, make_layout, make_params


def _samples(n):
    """Sweep indices 0, 1, 2, 5, 10, 20, 50, ... up to n, and n."""
    out, k = [], 1
    while k <= n:
        for m in (1, 2, 5):
            if m * k <= n:
                out.append(m * k)
        k *= 10
    return sorted(set([0] + out + [n]))


def protocol(ctx, d0, delta=0.15, alpha=10.0, mu=0.1, eps=1e-3, layout=(3, 3, 4, 3), alpha_hat=0.25,
             inner=10, sweeps=2000, ref_iters=100000):
    """Run the protocol on the GPU image d0; returns a dict of curves
    (full per-sweep lists) and the reference energies."""
    plain, dd = make_layout(), make_layout(*layout, alpha_hat)
    ref_its, dd_its = make_iters(1, ref_iters), make_iters(sweeps, inner)
    variants = {"irv2": make_params(delta, alpha, variant=TVS_IRV2),
                "irv1": make_params(delta, 1.0 / mu, eps=eps, variant=TVS_IRV1)}
    t0 = time.perf_counter()
    out = {"layout": list(layout), "alpha_hat": alpha_hat, "inner": inner, "sweeps": sweeps,
           "ref_iters": ref_iters}
    # Step 1
    tau_ref, st = ctx.step1(d0, variants["irv2"], plain, ref_its)
    e1_ref = st["energy"]
    tau_dd, _ = ctx.step1(d0, variants["irv2"], dd, dd_its)
    out["tfs"] = {"ref_energy": e1_ref, "dd": ctx.energy_history()}
    # Step 2, both variants, with the DD and with the reference tangent field
    for name, prm in variants.items():
        d_ref, st = ctx.step2(d0, tau_ref, prm, plain, ref_its)
        e_ref = st["energy"]
        d_dd, _ = ctx.step2(d0, tau_dd, prm, dd, dd_its)
        h_dd = ctx.energy_history()
        d_dr, _ = ctx.step2(d0, tau_ref, prm, dd, dd_its)
        h_dr = ctx.energy_history()
        q = ctx.quality(d_dd, d_ref)
        out[name] = {"ref_energy": e_ref, "dd_tau_dd": h_dd, "dd_tau_ref": h_dr,
                     "image_maxabs_dd_vs_ref": float((d_dd - d_ref).abs().max()),
                     "image_psnr_dd_vs_ref": q["psnr"]}
    out["seconds"] = time.perf_counter() - t0
    return out


def summary(res):
    """The curves at logarithmically spaced sweeps, as D(p^n) - D(p*)."""
    def curve(h, e):
        return {n: h[n] - e for n in _samples(len(h) - 1)}
    s = {"tfs_dd": curve(res["tfs"]["dd"], res["tfs"]["ref_energy"])}
    for name in ("irv2", "irv1"):
        r = res[name]
        s[name + "_dd_tau_dd"] = curve(r["dd_tau_dd"], r["ref_energy"])
        s[name + "_dd_tau_ref"] = curve(r["dd_tau_ref"], r["ref_energy"])
        s[name + "_image_maxabs"] = r["image_maxabs_dd_vs_ref"]
        s[name + "_image_psnr"] = r["image_psnr_dd_vs_ref"]
    s["seconds"] = res["seconds"]
    return s


def main(argv=None):
    import torch

    import synth
    from .tvs import Context

    ap = argparse.ArgumentParser(description="Section 6.3 DD validation on a synthetic image")
    ap.add_argument("--n2", type=int, default=270)
    ap.add_argument("--n1", type=int, default=480)
    ap.add_argument("--sigma2", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=10)
    ap.add_argument("--dtype", choices=("f32", "f64"), default="f64")
    ap.add_argument("--sweeps", type=int, default=2000)
    ap.add_argument("--inner", type=int, default=10)
    ap.add_argument("--ref-iters", type=int, default=100000)
    a = ap.parse_args(argv)
    _, noisy = synth.noisy_image(a.n2, a.n1, a.sigma2 ** 0.5, a.seed)
    ctx = Context(0)
    d0 = torch.tensor(noisy, dtype=torch.float64 if a.dtype == "f64" else torch.float32, device=ctx.device)
    res = protocol(ctx, d0, inner=a.inner, sweeps=a.sweeps, ref_iters=a.ref_iters)
    print(json.dumps({"n2": a.n2, "n1": a.n1, "sigma2": a.sigma2, "dtype": a.dtype, **summary(res)}))
    ctx.close()


if __name__ == "__main__":
    main()

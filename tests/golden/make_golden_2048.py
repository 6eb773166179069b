"""Write tests/golden/oracle_2048_s2i2_sigma{0.05,0.1,0.2}.npz: the FP64 oracle
on the 2048 x 2048 workload (8 x 8 subdomains, 16-pixel shared stripes) at
reduced counts (2 sweeps x 2 inner iterations per step) for one noise level:
sigma = 0.05, 0.1, 0.2 with seeds 30, 31, 32 and the parameters of
synth.params_for_sigma.  Stored: d and tau at 4096 fixed random points, d and
tau on a 96 x 96 window across the corner where four subdomains overlap, the
row and column sums of d and of tau_2 (every pixel enters them), and the
per-sweep energies.  Calls only oracle/ and synth.  Takes a few minutes per
noise level on one CPU core.

    python tests/golden/make_golden_2048.py 0.05 0.1 0.2
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import schwarz as osw  # noqa: E402

N = 2048
SEEDS = {0.05: 30, 0.1: 31, 0.2: 32}
LAYOUT = (8, 8, 16, 16)
SWEEPS, INNER = 2, 2
# top-left corner of the window: the core cut floor(4 * 2049 / 8) = 1024 of
# both axes lies at its centre, inside the shared stripes of four subdomains
WIN0, WIN = 1024 - 48, 96


def path_for(sigma):
    return os.path.join(HERE, f"oracle_2048_s2i2_sigma{sigma}.npz")


def make(sigma):
    t0 = time.time()
    seed = SEEDS[sigma]
    _, d64 = synth.noisy_f32(N, N, sigma, seed)
    delta, alpha = synth.params_for_sigma(sigma)
    l1 = osw.Layout(N, N, *LAYOUT, step=1)
    l2 = osw.Layout(N, N, *LAYOUT, step=2)
    tau, _, h1 = osw.step1_schwarz(d64, delta, l1, SWEEPS, INNER)
    print(f"sigma {sigma}: step 1 done after {time.time() - t0:.0f} s", flush=True)
    d, _, h2 = osw.step2_schwarz(d64, tau, alpha, l2, SWEEPS, INNER)
    print(f"sigma {sigma}: step 2 done after {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(2048)
    ii = rng.integers(0, N + 1, 4096)
    jj = rng.integers(0, N + 1, 4096)
    di = np.minimum(ii, N - 1)
    dj = np.minimum(jj, N - 1)
    w = slice(WIN0, WIN0 + WIN)
    np.savez_compressed(
        path_for(sigma),
        ii=ii, jj=jj, tau1=tau[0, ii, jj], tau2=tau[1, ii, jj], d=d[di, dj],
        win0=np.array(WIN0), d_win=d[w, w], tau_win=tau[:, w, w],
        d_rowsum=d.sum(axis=1), d_colsum=d.sum(axis=0),
        tau2_rowsum=tau[1].sum(axis=1), tau2_colsum=tau[1].sum(axis=0),
        energy1=np.array(h1), energy2=np.array(h2),
        meta=np.array([N, seed, SWEEPS, INNER] + list(LAYOUT)), sigma=sigma,
        params=np.array([delta, alpha]))
    print(f"sigma {sigma}: written after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for a in (sys.argv[1:] or ["0.05", "0.1", "0.2"]):
        make(float(a))

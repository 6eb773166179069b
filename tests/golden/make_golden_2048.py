"""Write tests/golden/oracle_2048_s2i2.npz: the FP64 oracle on the 2048 x 2048
workload (seed 31, sigma = 0.1, 8 x 8 subdomains, 16-pixel shared stripes)
at reduced counts (2 sweeps x 2 inner iterations per step), sampled at fixed
pixels, plus the row sums of d and of tau_2.  Calls only oracle/ and synth.
Takes a few minutes on one CPU core."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import schwarz as osw  # noqa: E402

N, SIGMA, SEED = 2048, 0.1, 31
LAYOUT = (8, 8, 16, 16)
SWEEPS, INNER = 2, 2


def main():
    t0 = time.time()
    _, d64 = synth.noisy_f32(N, N, SIGMA, SEED)
    delta, alpha = synth.params_for_sigma(SIGMA)
    l1 = osw.Layout(N, N, *LAYOUT, step=1)
    l2 = osw.Layout(N, N, *LAYOUT, step=2)
    tau, _, h1 = osw.step1_schwarz(d64, delta, l1, SWEEPS, INNER)
    print(f"step 1 done after {time.time() - t0:.0f} s", flush=True)
    d, _, h2 = osw.step2_schwarz(d64, tau, alpha, l2, SWEEPS, INNER)
    print(f"step 2 done after {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(2048)
    ii = rng.integers(0, N + 1, 4096)
    jj = rng.integers(0, N + 1, 4096)
    di = np.minimum(ii, N - 1)
    dj = np.minimum(jj, N - 1)
    np.savez_compressed(
        os.path.join(HERE, "oracle_2048_s2i2.npz"),
        ii=ii, jj=jj, tau1=tau[0, ii, jj], tau2=tau[1, ii, jj], d=d[di, dj],
        d_rowsum=d.sum(axis=1), tau2_rowsum=tau[1].sum(axis=1),
        energy1=np.array(h1), energy2=np.array(h2),
        meta=np.array([N, SEED, SWEEPS, INNER] + list(LAYOUT)), sigma=SIGMA)
    print(f"written after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()

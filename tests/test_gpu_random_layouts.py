"""Seeded random shapes and layouts, FP64 through the C-ABI against the FP64
oracle to 1e-10 (both steps, both variants).  The cases are drawn once from
a fixed seed: image sides 6-90, up to 4 subdomains per axis, shared stripes
from 1 up to the core width, relaxation alpha-hat from the colouring rule or
drawn from (0, 1], a few sweeps and inner iterations.  They reach tile tails,
frame pitches and stripe placements that the hand-picked cases do not."""
import numpy as np
import pytest

import synth
from oracle import schwarz as osw
from oracle import solvers as osv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def draw_cases(count, seed=20261202):
    rng = np.random.default_rng(seed)
    cases = []
    while len(cases) < count:
        n2, n1 = int(rng.integers(6, 91)), int(rng.integers(6, 91))
        m2, m1 = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        # cores floor(k n / M) on the (n+1)-point axis must be >= max(s, 2)
        c2, c1 = (n2 + 1) // m2, (n1 + 1) // m1
        if (m2 > 1 and c2 < 3) or (m1 > 1 and c1 < 3):
            continue
        s_y = int(rng.integers(1, c2 + 1)) if m2 > 1 else 0
        s_x = int(rng.integers(1, c1 + 1)) if m1 > 1 else 0
        ahat = float(rng.choice([0.0, rng.uniform(0.2, 1.0)]))
        variant = int(rng.integers(0, 2))
        cases.append((n2, n1, (m2, m1, s_y, s_x), ahat, variant, int(rng.integers(1, 4)),
                      int(rng.integers(1, 5))))
    return cases


CASES = draw_cases(12)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_17494_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}-a{c[3]:.2f}-v{c[4]}" for c in CASES])
def test_random_layout_against_oracle(ctx, case):
    from paper_2602_17494_amd import make_iters, make_layout, make_params
    n2, n1, lay, ahat, variant, sweeps, inner = case
    print("case", case, flush=True)
    _, d64 = synth.noisy_f32(n2, n1, 0.1, n2 * 131 + n1)
    delta, alpha = synth.params_for_sigma(0.1)
    d0 = torch.tensor(d64, device=DEV)
    tau = torch.empty((2, n2 + 1, n1 + 1), dtype=torch.float64, device=DEV)
    prm = make_params(delta, alpha, eps=1e-3, variant=variant)
    d, _ = ctx.schwarz_solve(d0, prm, make_layout(*lay, ahat), make_iters(sweeps, inner), tau_out=tau)
    torch.cuda.synchronize()
    l1 = osw.Layout(n2, n1, *lay, step=1)
    l2 = osw.Layout(n2, n1, *lay, step=2)
    a1 = ahat if ahat > 0 else None
    f1 = osv.tfs_data(d64, delta)
    p1, _, _ = osw.schwarz(l1, osw.inner_tfs_local, f1, 2, sweeps, inner, alpha_hat=a1)
    tau_ref = osv.tfs_tau(p1, f1, delta)
    if variant == 0:
        g = osv.irv2_potential(tau_ref, n2, n1)
        f2 = osv.irv2_data(d64, g, alpha)
        p2, _, _ = osw.schwarz(l2, osw.inner_rof, f2, 1, sweeps, inner, alpha_hat=a1)
        d_ref = osv.irv2_image(d64, p2, alpha)
    else:
        xi = osv.irv1_xi(tau_ref, n2, n1, 1e-3)
        f2 = osv.irv1_data(d64, xi, alpha)
        p2, _, _ = osw.schwarz(l2, osw.inner_rof, f2, 1, sweeps, inner, alpha_hat=a1)
        d_ref = osv.irv1_image(d64, p2, xi, alpha)
    assert np.abs(tau.cpu().numpy() - tau_ref).max() < 1e-10
    assert np.abs(d.cpu().numpy() - d_ref).max() < 1e-10

"""Pins of the oracle's overlapping Schwarz decomposition (Section 6):
partition-of-unity properties (i)-(iii), exactness of the localized inner
loop (Algorithm 5 equals Algorithm 4), the single-subdomain case reducing to
Algorithm 1, and convergence of the decomposition to the single-domain
solution (the paper's validation protocol, with the same tau fed to Step 2)."""
import numpy as np
import pytest

import synth
from oracle import operators as op
from oracle import schwarz as sw
from oracle import solvers as sv

LAYOUTS = [(64, 64, 2, 2, 8, 8), (2048, 2048, 8, 8, 16, 16), (270, 480, 3, 3, 4, 3),
           (512, 512, 2, 2, 8, 8), (40, 30, 1, 3, 0, 5), (33, 47, 4, 2, 5, 2)]


@pytest.mark.parametrize("n2,n1,m2,m1,sy,sx", LAYOUTS)
@pytest.mark.parametrize("step", [1, 2])
def test_partition_of_unity(n2, n1, m2, m1, sy, sx, step):
    lay = sw.Layout(n2, n1, m2, m1, sy, sx, step=step)
    total = np.zeros(lay.shape)
    for (i0, i1, j0, j1), th in zip(lay.boxes, lay.thetas):
        total += th
        inside = np.zeros(lay.shape, bool)
        inside[i0:i1, j0:j1] = True
        assert np.all(th[inside] > 0) and np.all(th[~inside] == 0)   # (ii)
        gx, gy = op.grad(th)
        smin = min(s for s in (sy, sx) if s > 0) if max(sy, sx) > 0 else 1
        assert max(np.abs(gx).max(), np.abs(gy).max()) <= 1.0 / smin + 1e-15  # (iii)
    assert np.abs(total - 1.0).max() < 1e-15                          # (i)
    assert lay.count == m2 * m1


def test_layout_of_the_2048_config():
    lay = sw.Layout(2048, 2048, 8, 8, 16, 16, step=1)
    sides = sorted({b[1] - b[0] for b in lay.boxes})
    assert sides == [264, 265, 272]
    assert lay.alpha_hat() == 0.25
    assert sw.Layout(64, 64, 1, 1, 0, 0).alpha_hat() == 1.0
    assert sw.Layout(64, 64, 1, 2, 0, 4).alpha_hat() == 0.5


def test_core_narrower_than_overlap_is_rejected():
    with pytest.raises(ValueError):
        sw.Layout(20, 20, 4, 4, 8, 8)


def test_localized_inner_loop_equals_global_one():
    # Algorithm 5 is Algorithm 4 written on the subdomain: same iterates.
    _, d0 = synth.noisy_image(14, 19, 0.1, 21)
    lay = sw.Layout(14, 19, 2, 3, 4, 3, step=1)
    f = sv.tfs_data(d0, 0.15)
    rng = np.random.default_rng(22)
    p = rng.uniform(-0.6, 0.6, (2, 2) + lay.shape)
    for m in range(lay.count):
        q = lay.thetas[m] * rng.uniform(-0.6, 0.6, p.shape)
        a = sw.inner_tfs_global(lay, m, p, q, f, 7, 0.125)
        b = sw.inner_tfs_local(lay, m, p, q, f, 7, 0.125)
        assert np.abs(a - b).max() <= 1e-12


def test_single_subdomain_is_algorithm_1():
    _, d0 = synth.noisy_image(11, 13, 0.1, 23)
    lay1 = sw.Layout(11, 13, 1, 1, 0, 0, step=1)
    tau_s, p_s, _ = sw.step1_schwarz(d0, 0.15, lay1, 4, 5)
    f = sv.tfs_data(d0, 0.15)
    p_a = sv.chambolle_tfs(f, 20)
    assert np.array_equal(p_s, p_a)
    lay2 = sw.Layout(11, 13, 1, 1, 0, 0, step=2)
    d_s, p2_s, _ = sw.step2_schwarz(d0, tau_s, 10.0, lay2, 4, 5)
    g = sv.irv2_potential(tau_s, 11, 13)
    p2_a = sv.chambolle_rof(sv.irv2_data(d0, g, 10.0), 20)
    assert np.array_equal(p2_s, p2_a)


def test_sweep_prologue_rewrites():
    # The subdomain data can be formed from one global projection per sweep:
    # omega_m = R_{m,+}(f - P_K vecdiv p) + LP_m(vecdiv(theta_m p)) because
    # sum_{l != m} theta_l = 1 - theta_m (property (i)); for Step 2 the
    # frozen part only enters through div((1 - theta_m) p) - f near the
    # subdomain.  Both forms must agree with the literal ones.
    _, d0 = synth.noisy_image(15, 18, 0.1, 24)
    lay = sw.Layout(15, 18, 2, 2, 4, 4, step=1)
    f = sv.tfs_data(d0, 0.15)
    rng = np.random.default_rng(25)
    p = rng.uniform(-1, 1, (2, 2) + lay.shape)
    r = f - sv.tfs_apply(p)
    for m in range(lay.count):
        box_p = op.grow_box(lay.boxes[m], lay.shape)
        lit = op.restrict(f - sv.tfs_apply(sw.others_sum(lay, m, p)), box_p)
        z = op.restrict(op.vecdiv(lay.thetas[m] * p), box_p)
        alt = op.restrict(r, box_p) + sw.local_projection(z, box_p, lay.shape)
        assert np.abs(lit - alt).max() < 1e-12
    lay2 = sw.Layout(15, 18, 2, 2, 4, 4, step=2)
    f2 = rng.standard_normal(lay2.shape)
    p2 = rng.uniform(-1, 1, (1, 2) + lay2.shape)
    for m in range(lay2.count):
        w = sw.others_sum(lay2, m, p2)
        lit = op.div(w[0]) - f2
        alt = op.div((1 - lay2.thetas[m]) * p2[0]) - f2
        assert np.abs(lit - alt).max() < 1e-13


def test_step2_schwarz_converges_to_single_domain():
    # The paper's protocol: feed the same tau to Step 2 and compare the
    # decomposed and the plain solve.  The primal is alpha-strongly convex,
    # so ||u(p) - u*||_2 <= sqrt(2 gap(p) / alpha) for any feasible p: the
    # decomposed and the plain results must lie within the sum of their two
    # radii of each other, and the decomposed gap must shrink.
    _, d0 = synth.noisy_image(12, 12, 0.1, 26)
    tau = np.zeros((2, 13, 13))
    alpha = 10.0
    lay = sw.Layout(12, 12, 2, 2, 4, 4, step=2)
    g = sv.irv2_potential(tau, 12, 12)
    f2 = sv.irv2_data(d0, g, alpha)

    def radius(p):
        u = (f2 - op.div(p[0])) / alpha
        gap = sv.gap_rof(p, u)
        assert gap >= -1e-12
        return np.sqrt(2 * max(gap, 0.0) / alpha)

    p_ref = sv.chambolle_rof(f2, 40000)
    d_ref = sv.irv2_image(d0, p_ref, alpha)
    rad = []
    p = q = None
    for chunk in (50, 950):
        p, q, _ = sw.schwarz(lay, sw.inner_rof, f2, 1, chunk, 10, p0=p, q0=q)
        rad.append(radius(p))
        dist = np.sqrt(np.sum((sv.irv2_image(d0, p, alpha) - d_ref) ** 2))
        assert dist <= rad[-1] + radius(p_ref) + 1e-12
    assert rad[1] < 0.1 * rad[0] and rad[1] < 2e-3


def test_step1_schwarz_converges_to_single_domain():
    # Same argument for TFS: the primal is (1/delta)-strongly convex on K,
    # so ||tau(p) - tau*||_2 <= sqrt(2 delta gap(p)).
    _, d0 = synth.noisy_image(8, 8, 0.1, 27)
    delta = 0.15
    f = sv.tfs_data(d0, delta)

    def radius(p):
        gap = sv.gap_tfs(p, sv.tfs_tau(p, f, delta))
        assert gap >= -1e-12
        return np.sqrt(2 * delta * max(gap, 0.0))

    p_ref = sv.chambolle_tfs(f, 30000)
    tau_ref = sv.tfs_tau(p_ref, f, delta)
    lay = sw.Layout(8, 8, 2, 2, 2, 2, step=1)
    rad = []
    p = q = None
    for chunk in (100, 1400):
        p, q, _ = sw.schwarz(lay, sw.inner_tfs_local, f, 2, chunk, 10, p0=p, q0=q)
        rad.append(radius(p))
        dist = np.sqrt(np.sum((sv.tfs_tau(p, f, delta) - tau_ref) ** 2))
        assert dist <= rad[-1] + radius(p_ref) + 1e-12
    assert rad[1] < 0.3 * rad[0] and rad[1] < 1e-2

"""Pins of the oracle's single-domain dual solvers (Section 4.2) and the
TV-Stokes pipeline: independent solvers on tiny grids, closed-form special
cases and invariants that the paper's mathematics fixes."""
import numpy as np
import pytest

import synth
from oracle import operators as op
from oracle import solvers as sv
from tests import bruteforce as bf


def pdhg_rof(f, alpha, iters, h=1.0):
    """Chambolle-Pock primal-dual iteration (accelerated for the alpha-strongly
    convex data term) for min_u sum |grad u| + alpha/2 ||u - f||^2; an
    algorithm independent of Chambolle's projection iteration."""
    u = f.copy()
    ubar = u.copy()
    y = np.zeros((2,) + f.shape)
    tau_s, sig = 0.25, 0.5  # tau * sigma * ||grad||^2 <= 1 with ||grad||^2 <= 8
    for _ in range(iters):
        y = y + sig * op.grad(ubar, h)
        nrm = np.maximum(1.0, np.sqrt(y[0] ** 2 + y[1] ** 2))
        y = y / nrm
        u_new = (u + tau_s * op.div(y, h) + tau_s * alpha * f) / (1 + tau_s * alpha)
        th = 1.0 / np.sqrt(1.0 + 2 * alpha * tau_s)
        tau_s, sig = th * tau_s, sig / th
        ubar = u_new + th * (u_new - u)
        u = u_new
    return u


@pytest.mark.parametrize("seed,alpha", [(7, 10.0), (8, 3.0)])
def test_rof_matches_bruteforce_4x4(seed, alpha):
    rng = np.random.default_rng(seed)
    d0 = rng.uniform(0, 1, (4, 4))
    u_bf, _ = bf.rof_bruteforce(d0, alpha)
    p = sv.chambolle_rof(alpha * d0, 20000)
    d = sv.irv2_image(d0, p, alpha)
    assert np.abs(d - u_bf).max() < 1e-8


@pytest.mark.parametrize("seed,delta", [(7, 0.15)])
def test_tfs_matches_bruteforce_4x4(seed, delta):
    rng = np.random.default_rng(seed)
    d0 = rng.uniform(0, 1, (4, 4))
    tau_bf, ptau0, _ = bf.tfs_bruteforce(sv.tau0(d0), delta)
    f = sv.tfs_data(d0, delta)
    assert np.abs(delta * f - ptau0).max() < 1e-13
    p = sv.chambolle_tfs(f, 50000)
    tau = sv.tfs_tau(p, f, delta)
    assert np.abs(tau - tau_bf).max() < 1e-6


def rof_objective(u, f, alpha):
    g = op.grad(u)
    return float(np.sqrt(g[0] ** 2 + g[1] ** 2).sum() + 0.5 * alpha * np.sum((u - f) ** 2))


def test_rof_matches_pdhg():
    # Both iterations converge slowly (O(1/n)-like), so the primal images are
    # compared to 1e-4 and the primal objective to 1e-7 relative; a dropped
    # term or a wrong sign moves either by orders of magnitude more.
    _, d0 = synth.noisy_image(12, 10, 0.1, 11)
    alpha = 10.0
    u_cp = pdhg_rof(d0, alpha, 6000)
    p = sv.chambolle_rof(alpha * d0, 20000)
    d = sv.irv2_image(d0, p, alpha)
    assert np.abs(d - u_cp).max() < 1e-4
    e_cp, e_ch = rof_objective(u_cp, d0, alpha), rof_objective(d, d0, alpha)
    assert abs(e_cp - e_ch) < 1e-7 * abs(e_ch)


def test_tau_divergence_free_and_dual_feasible():
    # spec pins on the 64 x 64 workload: div tau = 0 to 1e-12 and the
    # pointwise constraint |p_k| <= 1 (up to rounding) at every iteration.
    _, d0 = synth.noisy_f32(64, 64, 0.1, 1)
    delta, alpha = synth.params_for_sigma(0.1)
    f1 = sv.tfs_data(d0, delta)
    worst = [0.0]

    def cb(_, p):
        worst[0] = max(worst[0], float(np.sqrt(p[:, 0] ** 2 + p[:, 1] ** 2).max()))

    p1 = sv.chambolle_tfs(f1, 200, callback=cb)
    tau = sv.tfs_tau(p1, f1, delta)
    assert np.abs(op.div(tau)).max() < 1e-12
    assert worst[0] <= 1.0 + 1e-12
    g = sv.irv2_potential(tau, 64, 64)
    p2 = sv.chambolle_rof(sv.irv2_data(d0, g, alpha), 200, callback=cb)
    assert worst[0] <= 1.0 + 1e-12
    d = sv.irv2_image(d0, p2, alpha)
    assert np.isfinite(d).all()


def test_constant_image_is_fixed_point():
    d0 = np.full((9, 11), 0.375)
    d, tau, p1, p2 = sv.tv_stokes_plain(d0, 0.15, 10.0, 50, 50)
    assert np.all(tau == 0) and np.all(p1 == 0) and np.all(p2 == 0)
    assert np.all(d == 0.375)


def test_potential_integrates_divergence_free_field():
    # g exists because div tau = 0 on Omega-tilde: its backward y-difference
    # (first-row and interior rule) equals -tau_1 on Omega.
    _, d0 = synth.noisy_image(13, 17, 0.1, 12)
    f1 = sv.tfs_data(d0, 0.15)
    p = sv.chambolle_tfs(f1, 100)
    tau = sv.tfs_tau(p, f1, 0.15)
    g = sv.irv2_potential(tau, 13, 17)
    dyg = np.vstack([g[:1], g[1:] - g[:-1]])
    assert np.abs(dyg + tau[0, :13, :17]).max() < 1e-12
    dxg = np.hstack([g[:, :1], g[:, 1:] - g[:, :-1]])
    assert np.abs(dxg - tau[1, :13, :17]).max() < 1e-12


def test_energies_decrease_and_gaps_vanish():
    _, d0 = synth.noisy_image(10, 12, 0.1, 13)
    f1 = sv.tfs_data(d0, 0.15)
    es = []
    sv.chambolle_tfs(f1, 300, callback=lambda _, p: es.append(sv.energy_tfs(p, f1)))
    assert all(b <= a * (1 + 1e-12) + 1e-15 for a, b in zip(es, es[1:]))
    gaps = []
    for it in (200, 20000):
        p = sv.chambolle_tfs(f1, it)
        gaps.append(sv.gap_tfs(p, sv.tfs_tau(p, f1, 0.15)))
    assert gaps[1] >= -1e-12 and gaps[1] < 1e-3 * gaps[0]
    f2 = 10.0 * d0
    er = []
    p2 = sv.chambolle_rof(f2, 3000, callback=lambda _, p: er.append(sv.energy_rof(p, f2)))
    assert all(b <= a * (1 + 1e-12) + 1e-15 for a, b in zip(er, er[1:]))
    u = (f2 - op.div(p2[0])) / 10.0
    g_late = sv.gap_rof(p2, u)
    p_early = sv.chambolle_rof(f2, 30)
    g_early = sv.gap_rof(p_early, (f2 - op.div(p_early[0])) / 10.0)
    assert g_late >= -1e-12 and g_late < 1e-2 * g_early


def test_stop_residual_scale():
    assert sv.stop_residual(4.0, 1.0, 8, 2) == pytest.approx(1.0 / 4.0)


def test_irv1_xi_is_in_unit_ball():
    rng = np.random.default_rng(14)
    tau = rng.standard_normal((2, 7, 8))
    xi = sv.irv1_xi(tau, 6, 7, 1e-3)
    assert np.sqrt(xi[0] ** 2 + xi[1] ** 2).max() < 1.0
    # xi is parallel to (tau_2, -tau_1)
    assert np.abs(xi[0] * (-tau[0, :6, :7]) - xi[1] * tau[1, :6, :7]).max() < 1e-14


# --- orientation of tau_0 and the IRV1 maps ---------------------------------

def test_tau0_of_a_ramp():
    # d = a x + b y (x = column j, y = row i): the Neumann backward differences
    # are a and b inside their interior ranges, so tau_0 = (-D_y d, D_x d) is
    # (-b, a) there (text after eq. ir2dualdis); a swapped or sign-flipped
    # component gives another constant.
    a, b = 2.0, 5.0
    i, j = np.mgrid[0:6, 0:7]
    t0 = sv.tau0(a * j + b * i)
    assert np.all(t0[0, 1:6, 0:7] == -b)
    assert np.all(t0[1, 0:6, 1:7] == a)


def test_potential_of_tau0_recovers_the_image():
    # (D^-_x, D^-_y) g = (R tau)^perp = (tau_2, -tau_1); for tau = tau_0 =
    # (-D_y d, D_x d) the right side is the gradient of d, so g is d up to its
    # first column: g = d - d[:, :1] on Omega (eq. def:backdiffNeumann and the
    # definition of g after eq. ir2dualdis).  A flipped tau_0 gives -(d - d0).
    # (The y-equation does not hold for tau_0 itself: D^{neum-}_x is 0 in the
    # first column, so tau_0 is not divergence-free on the boundary ring.)
    rng = np.random.default_rng(21)
    d = rng.standard_normal((9, 12))
    g = sv.irv2_potential(sv.tau0(d), 9, 12)
    assert np.abs(g - (d - d[:, :1])).max() < 1e-13


def test_xi_of_hand_built_fields():
    # eq. eq:defXi2:discrete: xi = tau^perp / sqrt(|tau^perp|^2 + eps) with
    # tau^perp = R_Omega (tau_2, -tau_1).  With |tau| = 1 and eps = 3 the root
    # is exactly 2; eps outside the root, or a swapped or flipped component,
    # gives other values.
    tau = np.zeros((2, 4, 5))
    tau[0, :, :] = 1.0          # tau = (1, 0): tau^perp = (0, -1)
    tau[0, 1, 2], tau[1, 1, 2] = 0.0, 1.0   # tau = (0, 1): tau^perp = (1, 0)
    xi = sv.irv1_xi(tau, 3, 4, 3.0)
    assert xi.shape == (2, 3, 4)
    want = np.zeros((2, 3, 4))
    want[1] = -0.5
    want[0, 1, 2], want[1, 1, 2] = 0.5, 0.0
    assert np.array_equal(xi, want)


@pytest.mark.parametrize("a,b,eps", [(0.3, -1.2, 1e-3), (-2.0, 0.5, 0.25)])
def test_xi_of_constant_field(a, b, eps):
    tau = np.stack([np.full((6, 7), a), np.full((6, 7), b)])
    xi = sv.irv1_xi(tau, 5, 6, eps)
    r = np.sqrt(a * a + b * b + eps)
    assert np.abs(xi[0] - b / r).max() < 1e-15
    assert np.abs(xi[1] + a / r).max() < 1e-15


def _div_xi_bruteforce(xi):
    # div by the explicit matrix of tests/bruteforce.py (div = -grad^T)
    _, n2, n1 = xi.shape
    dmat = bf.divergence_matrix(n2, n1)
    return (dmat @ np.concatenate([xi[0].ravel(), xi[1].ravel()])).reshape(n2, n1)


@pytest.mark.parametrize("seed,alpha,eps", [(31, 10.0, 1e-3), (32, 3.0, 0.5)])
def test_irv1_matches_bruteforce_4x4(seed, alpha, eps):
    # IRV1 (eq. ir1dualdis with eq. eq:tau_hat) solves the ROF problem of
    # eq. IRPXi_ROF, whose data is d0 - div xi / alpha.  The SLSQP solver of
    # that ROF dual, fed the data built here with its own xi and div, must
    # give the same image as the oracle's chain xi -> data -> Chambolle ->
    # image.
    rng = np.random.default_rng(seed)
    d0 = rng.uniform(0, 1, (4, 4))
    tau = rng.standard_normal((2, 5, 5))
    tp1, tp2 = tau[1, :4, :4], -tau[0, :4, :4]
    root = np.sqrt(tp1 ** 2 + tp2 ** 2 + eps)
    xi_ref = np.stack([tp1 / root, tp2 / root])
    u_bf, _ = bf.rof_bruteforce(d0 - _div_xi_bruteforce(xi_ref) / alpha, alpha)
    xi = sv.irv1_xi(tau, 4, 4, eps)
    p = sv.chambolle_rof(sv.irv1_data(d0, xi, alpha), 20000)
    d = sv.irv1_image(d0, p, xi, alpha)
    assert np.abs(d - u_bf).max() < 1e-8

"""Single-domain dual solvers of Section 4.2 and the TV-Stokes pipeline,
float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np

from . import operators as op


def tau0(d0, h=1.0):
    """Tangent field of the observed image on Omega-tilde,
    tau_0 = (-D^{neum-}_y d0, D^{neum-}_x d0) (text after eq. ir2dualdis)."""
    return np.stack([-op.dy_neum(d0, h), op.dx_neum(d0, h)])


def tfs_data(d0, delta, h=1.0):
    """f = delta^{-1} P_K tau_0, the data term of the TFS dual (eq. tfsdualdis).

    Reading: Algorithm 1 prints delta^{-1} tau_0 inside its update, while the
    problem it solves (eq. tfsdualdis, Corollary Cor:tfsdual with
    eq. tfs_dualPK) uses delta^{-1} P_K tau_0.  The oracle follows the
    problem statement."""
    return op.project_k(tau0(d0, h), h) / delta


def chambolle_step(p, psi, t):
    """The semi-implicit update shared by all dual iterations (Algorithm 1,
    second line of the loop): p_k <- (p_k + t psi_k)/(1 + t |psi_k|) with the
    Euclidean norm of each 2-vector psi_k taken pointwise."""
    nrm = np.sqrt(psi[:, 0] ** 2 + psi[:, 1] ** 2)[:, None]
    return (p + t * psi) / (1.0 + t * nrm)


def tfs_apply(p, h=1.0):
    """Lambda p = P_K vecdiv p of the TFS dual (eq. tfsdualdis)."""
    w = op.vecdiv(p, h)
    return op.project_k(w, h)


def chambolle_tfs(f, iters, t=0.125, h=1.0, p0=None, callback=None):
    """Algorithm 1 (alg:chambTfs): p^0 = 0, then
    psi = vecgrad(P_K vecdiv p - f) and the pointwise update, for a fixed
    number of iterations.  f lives on Omega-tilde, shape (2, N2+1, N1+1)."""
    c, n2, n1 = f.shape
    p = np.zeros((c, 2, n2, n1)) if p0 is None else p0.copy()
    for it in range(iters):
        psi = op.vecgrad(tfs_apply(p, h) - f, h)
        p = chambolle_step(p, psi, t)
        if callback is not None:
            callback(it, p)
    return p


def tfs_tau(p, f, delta, h=1.0):
    """Primal recovery tau = P_K tau_0 - delta P_K vecdiv p = delta (f -
    P_K vecdiv p) (Corollary Cor:tfsdual with eq. tfs_dualPK)."""
    return delta * (f - tfs_apply(p, h))


def irv2_potential(tau, n2, n1, h=1.0):
    """The IRV2 potential g on Omega with (D^-_x, D^-_y) g = (R_Omega tau)^perp
    (text after eq. ir2dualdis), i.e. D^-_x g = tau_2 and D^-_y g = -tau_1.

    Reading: D^-_x at the last column is -g_{N1-1}/h, which cannot be
    integrated; the interior rule is used at every column, so g is the row-wise
    prefix sum h sum_{j' <= j} tau_2[i, j'] with g = 0 before the first
    column.  The constant of g does not matter for d = d0 - div p / alpha."""
    t2 = tau[1, :n2, :n1]
    return h * np.cumsum(t2, axis=1)


def irv2_data(d0, g, alpha):
    """f = alpha (d0 - g), the data term of the IRV2 dual (eq. ir2dualdis)."""
    return alpha * (d0 - g)


def chambolle_rof(f, iters, t=0.125, h=1.0, p0=None, callback=None):
    """Chambolle's iteration for min_{|p| <= 1} ||div p - f||^2 (eq.
    ir2dualdis): psi = grad(div p - f), then the pointwise update.  p has
    shape (1, 2, n2, n1)."""
    n2, n1 = f.shape
    p = np.zeros((1, 2, n2, n1)) if p0 is None else p0.copy()
    for it in range(iters):
        psi = op.grad(op.div(p[0], h) - f, h)[None]
        p = chambolle_step(p, psi, t)
        if callback is not None:
            callback(it, p)
    return p


def irv2_image(d0, p, alpha, h=1.0):
    """Reconstructed image d = d0 - div p / alpha (Section 3.3, the formula
    after eq. modifiedStep2_2_dual)."""
    return d0 - op.div(p[0], h) / alpha


# --- IRV1 (the other reconstruction variant) --------------------------------

def irv1_xi(tau, n2, n1, eps):
    """xi = tau_perp / sqrt(|tau_perp|^2 + eps) with tau_perp = R_Omega(tau_2,
    -tau_1) (eq. eq:defXi2:discrete)."""
    tp = np.stack([tau[1, :n2, :n1], -tau[0, :n2, :n1]])
    nrm = np.sqrt(tp[0] ** 2 + tp[1] ** 2 + eps)
    return tp / nrm


def irv1_data(d0, xi, alpha, h=1.0):
    """f = alpha d0 - div xi (eq. ir1dualdis)."""
    return alpha * d0 - op.div(xi, h)


def irv1_image(d0, p, xi, alpha, h=1.0):
    """d = d0 - (div p + div xi)/alpha (eq. eq:tau_hat)."""
    return d0 - (op.div(p[0], h) + op.div(xi, h)) / alpha


# --- energies, stopping residual, duality gap --------------------------------

def energy_tfs(p, f, h=1.0):
    """D_TFS(p) = ||P_K vecdiv p - f||^2 with the h^2-weighted norm (eq.
    tfsdualdis)."""
    r = tfs_apply(p, h) - f
    return float(h * h * np.sum(r * r))


def energy_rof(p, f, h=1.0):
    """D(p) = ||div p - f||^2 (eq. ir2dualdis / ir1dualdis)."""
    r = op.div(p[0], h) - f
    return float(h * h * np.sum(r * r))


def stop_residual(e_prev, e_next, npoints, channels):
    """|D(p^n)^(1/2) - D(p^{n+1})^(1/2)| / (channels |Gamma|)^(1/2), the
    left side of the stopping tests of Section 5.2 divided by their scale
    (2|Omega-tilde|)^(1/2) for TFS and |Omega|^(1/2) for IRV; comparing it with
    T = 1e-7 is the paper's test."""
    return abs(np.sqrt(e_prev) - np.sqrt(e_next)) / np.sqrt(channels * npoints)


def gap_tfs(p, tau, h=1.0):
    """Duality gap of TFS: sum_k sum (|grad tau_k| + grad tau_k . p_k).

    The paper states no gap; this follows from its duality theorem: with
    |p_k| <= 1 every term is >= 0, and all vanish exactly at the optimum where
    p_k = -grad tau_k / |grad tau_k| wherever grad tau_k != 0."""
    g = op.vecgrad(tau, h)
    nrm = np.sqrt(g[:, 0] ** 2 + g[:, 1] ** 2)
    dot = g[:, 0] * p[:, 0] + g[:, 1] * p[:, 1]
    return float(h * h * np.sum(nrm + dot))


def gap_rof(p, u, h=1.0):
    """Duality gap of the ROF dual: sum (|grad u| + grad u . p) with the
    primal u = (f - div p)/alpha (same derivation as gap_tfs)."""
    g = op.grad(u, h)
    nrm = np.sqrt(g[0] ** 2 + g[1] ** 2)
    dot = g[0] * p[0, 0] + g[1] * p[0, 1]
    return float(h * h * np.sum(nrm + dot))


# --- the plain single-domain pipeline ----------------------------------------

def tv_stokes_plain(d0, delta, alpha, it1, it2, t=0.125, h=1.0):
    """Plain single-domain TV-Stokes with IRV2: Step 1 by Algorithm 1 on
    Omega-tilde, the potential g, Step 2 by Chambolle's ROF iteration on
    Omega.  Returns (d, tau, p1, p2)."""
    n2, n1 = d0.shape
    f1 = tfs_data(d0, delta, h)
    p1 = chambolle_tfs(f1, it1, t, h)
    tau = tfs_tau(p1, f1, delta, h)
    g = irv2_potential(tau, n2, n1, h)
    f2 = irv2_data(d0, g, alpha)
    p2 = chambolle_rof(f2, it2, t, h)
    d = irv2_image(d0, p2, alpha, h)
    return d, tau, p1, p2

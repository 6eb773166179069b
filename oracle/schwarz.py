"""Overlapping Schwarz decomposition of Section 6, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A layout is (M2, M1, s_y, s_x): M2 x M1 subdomains, and a stripe of width s
shared by neighbouring subdomains.  Everything is defined on Omega-tilde (the
Step-1 grid); the Step-2 subdomains are Omega_m = Omega-tilde_m cut to Omega,
as the paper suggests after Algorithm 2.
"""
import numpy as np

from . import operators as op
from . import solvers as sv


# ---------------------------------------------------------------------------
# Subdomains and partition of unity (Section 6.1, properties (i)-(iii))
# ---------------------------------------------------------------------------

def axis_cuts(n, m_count):
    """Core cuts floor(k n / M), k = 0..M, of one axis of length n."""
    return [(k * n) // m_count for k in range(m_count + 1)]


def axis_intervals(n, m_count, s):
    """Half-open intervals [start, end) of the M subdomains of one axis of
    Omega-tilde (length n).

    Reading of "overlap s": s is the width of the stripe shared by two
    neighbours, centred on the core cut c_k as [c_k - floor(s/2),
    c_k + ceil(s/2)).  Needs every core to be at least s wide."""
    cuts = axis_cuts(n, m_count)
    lo, hi = s // 2, s - s // 2
    for m in range(m_count):
        if cuts[m + 1] - cuts[m] < max(s, 2):
            raise ValueError("core narrower than the overlap")
    out = []
    for m in range(m_count):
        a = 0 if m == 0 else cuts[m] - lo
        b = n if m == m_count - 1 else cuts[m + 1] + hi
        out.append((a, b))
    return out


def axis_theta(n, m_count, s, m):
    """One-dimensional partition-of-unity weight of subdomain m on an axis of
    length n.

    Reading: the paper fixes only properties (i)-(iii) of Section 6.1.  The
    oracle takes linear ramps across each shared stripe: at offset q = 0..s-1
    inside a stripe the right neighbour gets (q + 1/2)/s and the left one the
    rest; the core outside the stripes gets 1.  The weight is positive on the
    whole subdomain and the weights add up to one at every point."""
    cuts = axis_cuts(n, m_count)
    lo, hi = s // 2, s - s // 2
    a, b = axis_intervals(n, m_count, s)[m]
    th = np.zeros(n)
    x = np.arange(a, b)
    th[a:b] = 1.0
    if m > 0:
        left = (x < cuts[m] + hi)
        q = x[left] - (cuts[m] - lo)
        th[x[left]] = (q + 0.5) / s
    if m < m_count - 1:
        right = (x >= cuts[m + 1] - lo)
        q = x[right] - (cuts[m + 1] - lo)
        th[x[right]] = 1.0 - (q + 0.5) / s
    return th


class Layout:
    """The subdomains Omega-tilde_m of an (N2+1) x (N1+1) grid and their
    weights theta_m (Section 6.1).  ``step`` 1 works on Omega-tilde, 2 on
    Omega (the same subdomains cut to the first N2 rows and N1 columns)."""

    def __init__(self, n2, n1, m2, m1, s_y, s_x, step=1):
        self.nt2, self.nt1 = n2 + 1, n1 + 1
        self.m2, self.m1 = m2, m1
        iy = axis_intervals(self.nt2, m2, s_y)
        ix = axis_intervals(self.nt1, m1, s_x)
        ty = [axis_theta(self.nt2, m2, s_y, a) for a in range(m2)]
        tx = [axis_theta(self.nt1, m1, s_x, a) for a in range(m1)]
        if step == 1:
            self.shape = (self.nt2, self.nt1)
        else:
            self.shape = (n2, n1)
        g2, g1 = self.shape
        self.boxes = []
        self.thetas = []
        for a in range(m2):
            for b in range(m1):
                i0, i1 = iy[a][0], min(iy[a][1], g2)
                j0, j1 = ix[b][0], min(ix[b][1], g1)
                self.boxes.append((i0, i1, j0, j1))
                self.thetas.append(np.outer(ty[a][:g2], tx[b][:g1]))

    @property
    def count(self):
        return len(self.boxes)

    def alpha_hat(self):
        """Relaxation weight from the colouring rule after Algorithm 2:
        1 for one subdomain, 1/2 for a single row or column of subdomains,
        1/4 otherwise."""
        if self.m1 == 1 and self.m2 == 1:
            return 1.0
        if self.m1 == 1 or self.m2 == 1:
            return 0.5
        return 0.25


def others_sum(layout, m, p):
    """sum_{l != m} theta_l p, the frozen part in Algorithms 2-5."""
    w = np.zeros_like(p)
    for l, th in enumerate(layout.thetas):
        if l != m:
            w += th * p
    return w


def theta_update(v, psi, theta, t):
    """Weighted update of Algorithm 3: v_k <- (theta v_k + t theta psi_k) /
    (theta + t |psi_k|) per channel k.  Outside supp theta the new v is 0
    (reading: the printed formula is 0/0 there when psi = 0)."""
    nrm = np.sqrt(psi[:, 0] ** 2 + psi[:, 1] ** 2)[:, None]
    num = theta * v + t * theta * psi
    den = np.broadcast_to(theta + t * nrm, num.shape)
    pos = np.broadcast_to(theta > 0, num.shape)
    out = np.zeros_like(v)
    out[pos] = num[pos] / den[pos]
    return out


# ---------------------------------------------------------------------------
# Inner loops
# ---------------------------------------------------------------------------

def inner_rof(layout, m, p, q, f, iters, t, h=1.0):
    """Algorithm 3 (alg:tfsparinner) for the ROF dual (Lambda = div, c = 1)
    on global arrays: psi = Lambda^*(-Lambda(v + sum_{l != m} theta_l p) + f)
    with Lambda^* = -grad, then the theta-weighted update."""
    th = layout.thetas[m]
    w = others_sum(layout, m, p)
    v = q.copy()
    for _ in range(iters):
        psi = -op.grad(-op.div((v + w)[0], h) + f, h)[None]
        v = theta_update(v, psi, th, t)
    return v


def inner_tfs_global(layout, m, p, q, f, iters, t, h=1.0):
    """Algorithm 4 (alg:tfsparinnertfs): omega = f - P_K vecdiv sum_{l != m}
    theta_l p, then psi = vecgrad(P_K vecdiv v - omega) and the
    theta-weighted update, everything on all of Omega-tilde."""
    th = layout.thetas[m]
    omega = f - sv.tfs_apply(others_sum(layout, m, p), h)
    v = q.copy()
    for _ in range(iters):
        psi = op.vecgrad(sv.tfs_apply(v, h) - omega, h)
        v = theta_update(v, psi, th, t)
    return v


def local_projection(z, box_p, shape, h=1.0):
    """LP_m z = R_{A} P_K E_{A} z for A = box_p (the projection of locally
    supported data, restricted to the same rectangle), by its plain
    definition: extend by zero, project globally, restrict."""
    return op.restrict(op.project_k(op.extend(z, box_p, shape), h), box_p)


def inner_tfs_local(layout, m, p, q, f, iters, t, h=1.0):
    """Algorithm 5 (alg:tfsparinnertfsloc), the localized TFS inner loop.

    v_loc lives on Omega-tilde_m, z = vecdiv of (v_loc extended by zero to
    A = Omega-tilde_{m,+}) with the rectangle's own divergence, y = LP_m z,
    psi_loc = the part on Omega-tilde_m of vecgrad_A (y - omega_loc), and the
    theta-weighted update.  omega_loc is R_A of the omega of Algorithm 4."""
    shape = layout.shape
    box = layout.boxes[m]
    box_p = op.grow_box(box, shape)
    i0, i1, j0, j1 = box
    a0, a1, b0, b1 = box_p
    th = op.restrict(layout.thetas[m], box)
    omega = f - sv.tfs_apply(others_sum(layout, m, p), h)
    omega_loc = op.restrict(omega, box_p)
    v = op.restrict(q, box)
    ni, nj = i1 - i0, j1 - j0
    for _ in range(iters):
        vp = np.zeros(v.shape[:2] + (a1 - a0, b1 - b0))
        vp[..., :ni, :nj] = v
        z = op.vecdiv(vp, h)
        y = local_projection(z, box_p, shape, h)
        psi = op.vecgrad(y - omega_loc, h)[..., :ni, :nj]
        v = theta_update(v, psi, th, t)
    return op.extend(v, box, shape)


# ---------------------------------------------------------------------------
# Algorithm 2 (alg:disalgsubsp)
# ---------------------------------------------------------------------------

def schwarz(layout, inner, f, channels, sweeps, iters, t=0.125, h=1.0,
            alpha_hat=None, energy=None, p0=None, q0=None):
    """Algorithm 2: for every subdomain m, q_m <- inner(m, p^n, q_m) (warm
    start from the previous sweep), then p^{n+1} = (1 - a) p^n + a sum_m q_m.

    Reading: q_m before the first sweep is theta_m p^0 = 0 (the paper warm
    starts from q_m^n and leaves n = 0 open).  Returns p, the list of q_m and
    the energy after each sweep (when ``energy`` is given)."""
    a = layout.alpha_hat() if alpha_hat is None else alpha_hat
    g2, g1 = layout.shape
    p = np.zeros((channels, 2, g2, g1)) if p0 is None else p0.copy()
    q = ([np.zeros_like(p) for _ in range(layout.count)] if q0 is None
         else [x.copy() for x in q0])
    hist = []
    for _ in range(sweeps):
        q = [inner(layout, m, p, q[m], f, iters, t, h) for m in range(layout.count)]
        p = (1.0 - a) * p + a * sum(q)
        if energy is not None:
            hist.append(energy(p))
    return p, q, hist


def step1_schwarz(d0, delta, layout, sweeps, iters, t=0.125, h=1.0, local=True):
    """Step 1 (TFS) by Algorithm 2 on Omega-tilde with the localized inner
    loop (Algorithm 5) or the global one (Algorithm 4).  Returns tau, p and
    the energy history."""
    f = sv.tfs_data(d0, delta, h)
    inner = inner_tfs_local if local else inner_tfs_global
    p, _, hist = schwarz(layout, inner, f, 2, sweeps, iters, t, h,
                         energy=lambda pp: sv.energy_tfs(pp, f, h))
    return sv.tfs_tau(p, f, delta, h), p, hist


def step2_schwarz(d0, tau, alpha, layout, sweeps, iters, t=0.125, h=1.0):
    """Step 2 (IRV2) by Algorithm 2 on Omega with the inner loop of
    Algorithm 3.  Returns d, p and the energy history."""
    n2, n1 = d0.shape
    g = sv.irv2_potential(tau, n2, n1, h)
    f = sv.irv2_data(d0, g, alpha)
    p, _, hist = schwarz(layout, inner_rof, f, 1, sweeps, iters, t, h,
                         energy=lambda pp: sv.energy_rof(pp, f, h))
    return sv.irv2_image(d0, p, alpha, h), p, hist


def tv_stokes_schwarz(d0, delta, alpha, m2, m1, s_y, s_x, sweeps, iters,
                      t=0.125, h=1.0):
    """Both TV-Stokes steps (IRV2) inside Algorithm 2 with the same
    splitting for both steps.  Returns (d, tau)."""
    n2, n1 = d0.shape
    l1 = Layout(n2, n1, m2, m1, s_y, s_x, step=1)
    l2 = Layout(n2, n1, m2, m1, s_y, s_x, step=2)
    tau, _, _ = step1_schwarz(d0, delta, l1, sweeps, iters, t, h)
    d, _, _ = step2_schwarz(d0, tau, alpha, l2, sweeps, iters, t, h)
    return d, tau

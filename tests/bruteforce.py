"""Independent convex solvers for tiny grids, used to pin the oracle.

They share nothing with the oracle's iteration: the difference matrices are
built here from scratch with explicit loops, the divergence-free subspace
comes from an SVD null space, and the minimisation is scipy's SLSQP on the
dual problems (a convex quadratic with one disc constraint per pixel and
field).  The primal results they return are unique even where p is not."""
import numpy as np
import scipy.linalg
import scipy.optimize


def forward_diff_matrices(n2, n1, h=1.0):
    """Sparse-free dense matrices of the forward differences with a zero last
    column / row, acting on row-major vectors of an n2 x n1 image."""
    n = n2 * n1
    gx = np.zeros((n, n))
    gy = np.zeros((n, n))
    for i in range(n2):
        for j in range(n1):
            r = i * n1 + j
            if j + 1 < n1:
                gx[r, r + 1] += 1.0 / h
                gx[r, r] -= 1.0 / h
            if i + 1 < n2:
                gy[r, r + n1] += 1.0 / h
                gy[r, r] -= 1.0 / h
    return gx, gy


def _dual_qp(lam, f, nfields, n):
    """min_p ||lam p - f||^2 subject to |p_{k,i}|^2 <= 1 for every field k and
    pixel i, by SLSQP.  p is stacked as [p_1x, p_1y, p_2x, p_2y, ...]."""
    def obj(v):
        r = lam @ v - f
        return float(r @ r)

    def obj_grad(v):
        return 2.0 * lam.T @ (lam @ v - f)

    def cons(v):
        q = v.reshape(nfields, 2, n)
        return (1.0 - q[:, 0] ** 2 - q[:, 1] ** 2).ravel()

    def cons_jac(v):
        q = v.reshape(nfields, 2, n)
        jac = np.zeros((nfields * n, nfields * 2 * n))
        for k in range(nfields):
            for i in range(n):
                jac[k * n + i, (2 * k) * n + i] = -2 * q[k, 0, i]
                jac[k * n + i, (2 * k + 1) * n + i] = -2 * q[k, 1, i]
        return jac

    v0 = np.zeros(nfields * 2 * n)
    res = scipy.optimize.minimize(
        obj, v0, jac=obj_grad, method="SLSQP",
        constraints=[{"type": "ineq", "fun": cons, "jac": cons_jac}],
        options={"ftol": 1e-20, "maxiter": 10000})
    return res.x, res


def divergence_matrix(n2, n1, h=1.0):
    """div = -(grad)^T acting on (u1, u2) stacked, for an n2 x n1 grid."""
    gx, gy = forward_diff_matrices(n2, n1, h)
    return -np.hstack([gx.T, gy.T])


def rof_bruteforce(f_img, alpha, h=1.0):
    """Solve min_{|p| <= 1} ||div p - alpha f||^2 by SLSQP and return the
    primal u = f - div p / alpha (unique although p is not)."""
    n2, n1 = f_img.shape
    dmat = divergence_matrix(n2, n1, h)
    f = alpha * f_img.ravel()
    p, res = _dual_qp(dmat, f, 1, n2 * n1)
    u = (f - dmat @ p) / alpha
    return u.reshape(n2, n1), res


def tfs_bruteforce(tau0, delta, h=1.0):
    """Solve min_{|p_k| <= 1} ||P vecdiv p - P tau0 / delta||^2 by SLSQP, with
    P = Z Z^T the orthogonal projector onto null(div) from an SVD basis Z.
    Returns (tau = P tau0 - delta P vecdiv p, P tau0, result)."""
    _, n2, n1 = tau0.shape
    n = n2 * n1
    dmat = divergence_matrix(n2, n1, h)
    z = scipy.linalg.null_space(dmat)
    proj = z @ z.T
    vdiv = np.zeros((2 * n, 4 * n))
    vdiv[:n, :2 * n] = dmat
    vdiv[n:, 2 * n:] = dmat
    lam = proj @ vdiv
    ptau0 = proj @ tau0.reshape(2 * n)
    p, res = _dual_qp(lam, ptau0 / delta, 2, n)
    tau = ptau0 - delta * (lam @ p)
    return tau.reshape(2, n2, n1), ptau0.reshape(2, n2, n1), res

"""Discrete operators of Section 4.1 (Notations), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions.  A scalar image on a grid Gamma with #Gamma_y = n2 rows and
#Gamma_x = n1 columns is a numpy array of shape (n2, n1); row index i <-> y,
column index j <-> x, both 0-based here (the paper counts from 1).  A vector
field u = (u1, u2) (x-component, y-component) has shape (2, n2, n1).  A dual
variable of X(Gamma, 2 x c) has shape (c, 2, n2, n1): p[k] = p_k is the
k-th 2-vector field, p[k, 0] its x- and p[k, 1] its y-component.
"""
import numpy as np
import scipy.fft


# ---------------------------------------------------------------------------
# Finite differences (Section 4.1, definition of D^+_x, D^+_y, D^-_x, D^-_y)
# ---------------------------------------------------------------------------

def dxp(d, h=1.0):
    """Forward difference in x: (d_{i,j+1} - d_{i,j})/h, and 0 in the last
    column (Section 4.1, D^+_{x,Omega})."""
    out = np.zeros_like(d, dtype=np.float64)
    out[:, :-1] = (d[:, 1:] - d[:, :-1]) / h
    return out


def dyp(d, h=1.0):
    """Forward difference in y: (d_{i+1,j} - d_{i,j})/h, and 0 in the last
    row (Section 4.1, D^+_{y,Omega})."""
    out = np.zeros_like(d, dtype=np.float64)
    out[:-1, :] = (d[1:, :] - d[:-1, :]) / h
    return out


def dxm(d, h=1.0):
    """Backward difference in x with the paper's boundary rule (Section 4.1,
    D^-_{x,Omega}): first column d_{i,1}/h, interior (d_{i,j} - d_{i,j-1})/h,
    last column -d_{i,N1-1}/h.  Needs at least two columns."""
    n1 = d.shape[1]
    assert n1 >= 2
    out = np.empty_like(d, dtype=np.float64)
    out[:, 0] = d[:, 0]
    out[:, 1:n1 - 1] = d[:, 1:n1 - 1] - d[:, 0:n1 - 2]
    out[:, n1 - 1] = -d[:, n1 - 2]
    return out / h


def dym(d, h=1.0):
    """Backward difference in y with the paper's boundary rule (Section 4.1,
    D^-_{y,Omega}): first row d_{1,j}/h, interior (d_{i,j} - d_{i-1,j})/h,
    last row -d_{N2-1,j}/h.  Needs at least two rows."""
    n2 = d.shape[0]
    assert n2 >= 2
    out = np.empty_like(d, dtype=np.float64)
    out[0, :] = d[0, :]
    out[1:n2 - 1, :] = d[1:n2 - 1, :] - d[0:n2 - 2, :]
    out[n2 - 1, :] = -d[n2 - 2, :]
    return out / h


def dx_neum(d, h=1.0):
    """Neumann backward difference in x, Omega -> Omega-tilde (eq.
    def:backdiffNeumann).  Output has shape (N2+1, N1+1): zero in the first
    and last column; (d_{i,j} - d_{i,j-1})/h in the interior columns for the
    image rows; the extra last row mirrors the last image row."""
    n2, n1 = d.shape
    out = np.zeros((n2 + 1, n1 + 1))
    out[:n2, 1:n1] = d[:, 1:n1] - d[:, 0:n1 - 1]
    out[n2, 1:n1] = d[n2 - 1, 1:n1] - d[n2 - 1, 0:n1 - 1]
    return out / h


def dy_neum(d, h=1.0):
    """Neumann backward difference in y, Omega -> Omega-tilde (eq.
    def:backdiffNeumann): zero in the first and last row; (d_{i,j} -
    d_{i-1,j})/h in the interior rows for the image columns; the extra last
    column mirrors the last image column."""
    n2, n1 = d.shape
    out = np.zeros((n2 + 1, n1 + 1))
    out[1:n2, :n1] = d[1:n2, :] - d[0:n2 - 1, :]
    out[1:n2, n1] = d[1:n2, n1 - 1] - d[0:n2 - 1, n1 - 1]
    return out / h


# ---------------------------------------------------------------------------
# Gradient, divergence and their channel-wise versions (eqs. defGradDis,
# defDivDis and the multi-gradient / multi-divergence after them)
# ---------------------------------------------------------------------------

def grad(d, h=1.0):
    """Discrete gradient (D^+_x d, D^+_y d), eq. defGradDis; shape (2,n2,n1)."""
    return np.stack([dxp(d, h), dyp(d, h)])


def div(u, h=1.0):
    """Discrete divergence D^-_x u1 + D^-_y u2, eq. defDivDis."""
    return dxm(u[0], h) + dym(u[1], h)


def vecgrad(u, h=1.0):
    """Channel-wise gradient of a c-channel image u (shape (c,n2,n1)); result
    has shape (c, 2, n2, n1)."""
    return np.stack([grad(u[k], h) for k in range(u.shape[0])])


def vecdiv(p, h=1.0):
    """Channel-wise divergence of p (shape (c,2,n2,n1)); shape (c,n2,n1)."""
    return np.stack([div(p[k], h) for k in range(p.shape[0])])


def laplacian(d, h=1.0):
    """Neumann Laplacian div(grad d) on the grid of d (Section 4.1)."""
    return div(grad(d, h), h)


# ---------------------------------------------------------------------------
# DCT and the Moore-Penrose inverse of the Laplacian (eqs. form:DCTmat,
# eq:DCT2D, eq:DCT2Dinv, form:DiscInvLapl, form:DiscInvLaplTild)
# ---------------------------------------------------------------------------

def dct_matrix(n):
    """Orthonormal DCT-II matrix C_N of eq. form:DCTmat:
    row 0 is sqrt(1/N), row k >= 1 is sqrt(2/N) cos(k (2l+1) pi / (2N))."""
    k = np.arange(n)[:, None]
    l = np.arange(n)[None, :]
    c = np.sqrt(2.0 / n) * np.cos(k * (2 * l + 1) * np.pi / (2 * n))
    c[0, :] = np.sqrt(1.0 / n)
    return c


def sigma(n, h=1.0):
    """sigma_{N,j} = (2/h) sin((j-1) pi / (2N)), j = 1..N (0-based index k =
    j-1 here), from the text after eq. form:DiscInvLaplTild."""
    return (2.0 / h) * np.sin(np.arange(n) * np.pi / (2 * n))


def inv_lambda(n2, n1, h=1.0):
    """Diagonal of the spectral pseudo-inverse of eq. form:DiscInvLaplTild:
    0 at the constant mode, -1/(sigma^2 + sigma^2) elsewhere.

    Reading: the printed subscripts pair the row index with N1 and the column
    index with N2.  With the 2-D DCT C_{N2} d C_{N1}^T of eq. eq:DCT2D the
    row frequency belongs to N2 and the column frequency to N1, so the
    diagonal is taken as -1/(sigma_{N2,i}^2 + sigma_{N1,j}^2).  Only this
    reading equals pinv(Laplacian) on non-square grids (pinned in tests)."""
    s2 = sigma(n2, h) ** 2
    s1 = sigma(n1, h) ** 2
    lam = s2[:, None] + s1[None, :]
    out = np.zeros((n2, n1))
    nz = lam > 0
    out[nz] = -1.0 / lam[nz]
    return out


_DENSE_MAX = 600


def dct2(d):
    """2-D DCT C_{N2} d C_{N1}^T (eq. eq:DCT2D).  Dense matrices for small
    sides; scipy's orthonormal DCT-II (the same matrix) above that."""
    n2, n1 = d.shape
    if max(n2, n1) <= _DENSE_MAX:
        return dct_matrix(n2) @ d @ dct_matrix(n1).T
    return scipy.fft.dctn(d, type=2, norm="ortho")


def idct2(d):
    """Inverse 2-D DCT C_{N2}^T d C_{N1} (eq. eq:DCT2Dinv)."""
    n2, n1 = d.shape
    if max(n2, n1) <= _DENSE_MAX:
        return dct_matrix(n2).T @ d @ dct_matrix(n1)
    return scipy.fft.idctn(d, type=2, norm="ortho")


def inv_laplacian(d, h=1.0):
    """Moore-Penrose inverse of the Neumann Laplacian through the DCT,
    (Delta)^dagger d = C^{-1} (Delta-tilde)^dagger C d (eq. form:DiscInvLapl)."""
    n2, n1 = d.shape
    return idct2(inv_lambda(n2, n1, h) * dct2(d))


def inv_laplacian_blocks(d_a, box_a, box_b, shape, row_blocks, col_blocks, h=1.0):
    """R_B (Delta)^dagger E_A d by the block formula of eq. invLaplLowCapLong
    (Section 6.2.2).  row_blocks and col_blocks are disjoint decompositions
    of the frequency rows [0, n2) and columns [0, n1) into half-open ranges
    (the blocks A-tilde_lambda of eq. def:2DDs are their products); box_a,
    box_b = (i0, i1, j0, j1) are A_k and B_m.  The result is the sum over
    lambda = (lambda2, lambda1) of
        [C_{N2}]_{lambda2,B}^T  Lambda_lambda o ([C_{N2}]_{lambda2,A} d [C_{N1}]_{lambda1,A}^T)  [C_{N1}]_{lambda1,B},
    where [C]_{l,A} holds the rows of frequency block l and the columns of A
    (Figure fig:matvisualization) and Lambda_lambda is the block of the
    diagonal of eq. form:DiscInvLaplTild on A-tilde_lambda; the middle factor
    is diagonal, so of the double sum over lambda, lambda' in eq.
    locglobprojpart3 only lambda' = lambda remains."""
    n2, n1 = shape
    c2, c1 = dct_matrix(n2), dct_matrix(n1)
    lam = inv_lambda(n2, n1, h)
    ai0, ai1, aj0, aj1 = box_a
    bi0, bi1, bj0, bj1 = box_b
    out = np.zeros((bi1 - bi0, bj1 - bj0))
    for r0, r1 in row_blocks:
        for q0, q1 in col_blocks:
            forward = c2[r0:r1, ai0:ai1] @ d_a @ c1[q0:q1, aj0:aj1].T
            out += c2[r0:r1, bi0:bi1].T @ (lam[r0:r1, q0:q1] * forward) @ c1[q0:q1, bj0:bj1]
    return out


def project_k(u, h=1.0):
    """Orthogonal projection onto K^h = null(div) on the grid of u (eq.
    formula:PKh): P u = u - grad (Delta)^dagger div u.  u has shape
    (2, n2, n1)."""
    return u - grad(inv_laplacian(div(u, h), h), h)


# ---------------------------------------------------------------------------
# Restriction and extension by zero (Section 4.1 and Section 6.2.1)
# ---------------------------------------------------------------------------

def restrict(u, box):
    """R_A: the sub-rectangle box = (i0, i1, j0, j1) (half-open) of the last
    two axes of u."""
    i0, i1, j0, j1 = box
    return u[..., i0:i1, j0:j1].copy()


def extend(u_loc, box, shape):
    """E_A: zero extension of data on box = (i0, i1, j0, j1) to a grid of
    shape (n2, n1) (last two axes)."""
    i0, i1, j0, j1 = box
    out = np.zeros(u_loc.shape[:-2] + tuple(shape))
    out[..., i0:i1, j0:j1] = u_loc
    return out


def grow_box(box, shape):
    """A_+ of Section 6.2.1: the rectangle grown by one row below and one
    column to the right, clipped at the grid (reading: the printed names of
    the two stripes are swapped and their union misses the corner; the
    rectangle grown by one row and one column is what the localization
    identities need)."""
    i0, i1, j0, j1 = box
    return (i0, min(i1 + 1, shape[0]), j0, min(j1 + 1, shape[1]))

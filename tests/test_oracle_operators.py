"""Pins of the oracle's discrete operators (Section 4.1) against facts that
do not come from the oracle itself: adjointness stated in the paper, the
textbook DCT-II (scipy), numpy's pseudo-inverse, an SVD null-space
projector, and closed forms for special inputs."""
import numpy as np
import pytest
import scipy.fft
import scipy.linalg

from oracle import operators as op

SHAPES = [(5, 7), (7, 5), (4, 9), (2, 3), (6, 6)]


def as_matrix(f, shape_in):
    n = int(np.prod(shape_in))
    cols = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        cols.append(np.asarray(f(e.reshape(shape_in))).ravel())
    return np.array(cols).T


@pytest.mark.parametrize("shape", SHAPES)
def test_div_is_minus_grad_adjoint(shape):
    # Section 4.1: div = -(grad)^*, and D^- = -(D^+)^T per axis.
    g = as_matrix(op.grad, shape)
    d = as_matrix(op.div, (2,) + shape)
    assert np.abs(d + g.T).max() == 0.0
    gx = as_matrix(op.dxp, shape)
    dx = as_matrix(op.dxm, shape)
    assert np.abs(dx + gx.T).max() == 0.0


@pytest.mark.parametrize("shape", SHAPES)
def test_vecdiv_is_minus_vecgrad_adjoint(shape):
    g = as_matrix(op.vecgrad, (2,) + shape)
    d = as_matrix(op.vecdiv, (2, 2) + shape)
    assert np.abs(d + g.T).max() == 0.0


def test_forward_difference_closed_form():
    # A linear ramp has constant forward differences except on the last
    # column / row where D^+ is zero.
    n2, n1 = 6, 8
    yy, xx = np.mgrid[0:n2, 0:n1].astype(float)
    d = 0.3 * xx - 0.7 * yy + 2.0
    gx, gy = op.grad(d, h=0.5)
    assert np.allclose(gx[:, :-1], 0.6) and np.all(gx[:, -1] == 0)
    assert np.allclose(gy[:-1, :], -1.4) and np.all(gy[-1, :] == 0)


@pytest.mark.parametrize("n", [1, 2, 5, 8, 13, 64])
def test_dct_matrix_is_scipy_dct2_ortho(n):
    c = op.dct_matrix(n)
    ref = scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0)
    assert np.abs(c - ref).max() < 1e-14
    assert np.abs(c @ c.T - np.eye(n)).max() < 1e-13


def test_dct_dense_and_fast_paths_agree():
    rng = np.random.default_rng(3)
    d = rng.standard_normal((37, 41))
    dense = op.dct_matrix(37) @ d @ op.dct_matrix(41).T
    fast = scipy.fft.dctn(d, type=2, norm="ortho")
    assert np.abs(dense - fast).max() < 1e-12
    assert np.abs(op.idct2(op.dct2(d)) - d).max() < 1e-12


@pytest.mark.parametrize("shape", [(5, 7), (7, 5), (4, 9), (3, 3), (8, 2)])
def test_inv_laplacian_is_pinv(shape):
    # Pins the eigenvalue pairing (row frequency <-> N2, column <-> N1):
    # on non-square grids only that reading equals the pseudo-inverse.
    lap = as_matrix(op.laplacian, shape)
    inv = as_matrix(op.inv_laplacian, shape)
    assert np.abs(inv - np.linalg.pinv(lap)).max() < 1e-12


def test_inv_laplacian_large_grid_property():
    # scipy DCT path (sides above the dense limit): Delta Delta^+ b = b - mean b.
    rng = np.random.default_rng(4)
    b = rng.standard_normal((611, 605))
    phi = op.inv_laplacian(b)
    assert abs(phi.mean()) < 1e-10
    assert np.abs(op.laplacian(phi) - (b - b.mean())).max() < 1e-9


@pytest.mark.parametrize("shape", [(5, 7), (6, 4), (3, 3)])
def test_projection_is_svd_nullspace_projector(shape):
    # eq. formula:PKh and Proposition prop:DisProj: the unique orthogonal
    # projection onto null(div).  Compare with Z Z^T from an SVD basis.
    p = as_matrix(op.project_k, (2,) + shape)
    d = as_matrix(op.div, (2,) + shape)
    z = scipy.linalg.null_space(d)
    assert np.abs(z @ z.T - p).max() < 1e-12
    assert np.abs(p @ p - p).max() < 1e-12
    assert np.abs(p - p.T).max() < 1e-12
    assert np.abs(d @ p).max() < 1e-12


def test_neumann_differences_special_cases():
    n2, n1 = 5, 6
    yy, xx = np.mgrid[0:n2, 0:n1].astype(float)
    d = 0.25 * xx + 1.5 * yy
    dx = op.dx_neum(d)
    dy = op.dy_neum(d)
    assert dx.shape == (n2 + 1, n1 + 1)
    # zero on the first and last column / row, constant slope inside,
    # including the mirrored extra row / column
    assert np.all(dx[:, 0] == 0) and np.all(dx[:, n1] == 0)
    assert np.allclose(dx[:, 1:n1], 0.25)
    assert np.all(dy[0, :] == 0) and np.all(dy[n2, :] == 0)
    assert np.allclose(dy[1:n2, :], 1.5)
    # a constant image has no tangent field
    assert np.all(op.dx_neum(np.full((4, 4), 0.7)) == 0)


def test_neumann_difference_telescopes_to_image():
    # summing D^{neum-}_x d along a row recovers d up to its first column
    rng = np.random.default_rng(5)
    d = rng.standard_normal((6, 9))
    dx = op.dx_neum(d)
    rec = np.cumsum(dx[:6, :9], axis=1)
    assert np.abs(rec - (d - d[:, :1])).max() < 1e-13


def test_rotated_gradient_is_divergence_free_inside():
    # tau_0 = (-D_y d, D_x d): mixed backward differences commute, so
    # div tau_0 vanishes away from the boundary ring of Omega-tilde, but in
    # general not on it (which is why P_K tau_0 is needed).
    rng = np.random.default_rng(6)
    d = rng.standard_normal((7, 8))
    tau0 = np.stack([-op.dy_neum(d), op.dx_neum(d)])
    dv = op.div(tau0)
    assert np.abs(dv[1:-2, 1:-2]).max() < 1e-13
    assert np.abs(dv).max() > 1e-3


def test_grow_box():
    assert op.grow_box((0, 4, 2, 5), (10, 10)) == (0, 5, 2, 6)
    assert op.grow_box((6, 10, 7, 10), (10, 10)) == (6, 10, 7, 10)


def _random_cuts(rng, n):
    """A random disjoint decomposition of [0, n) into half-open ranges."""
    k = int(rng.integers(1, min(n, 6) + 1))
    cuts = np.sort(rng.choice(np.arange(1, n), size=k - 1, replace=False)) if k > 1 else np.array([], int)
    edges = [0] + [int(c) for c in cuts] + [n]
    return list(zip(edges[:-1], edges[1:]))


@pytest.mark.parametrize("seed", range(6))
def test_block_formula_is_restricted_inverse_laplacian(seed):
    """Eq. invLaplLowCapLong summed over random disjoint frequency blocks,
    with data on a box A read on another box B, equals the definition
    R_B (Delta)^dagger E_A d on non-square grids.  A != B and unequal block
    sizes make a transposed or swapped DCT block, or A's columns used on the
    output side, fail."""
    rng = np.random.default_rng(70 + seed)
    n2, n1 = int(rng.integers(7, 23)), int(rng.integers(7, 23))
    while n1 == n2:
        n1 = int(rng.integers(7, 23))

    def box():
        i0, j0 = int(rng.integers(0, n2 - 2)), int(rng.integers(0, n1 - 2))
        return (i0, int(rng.integers(i0 + 1, n2 + 1)), j0, int(rng.integers(j0 + 1, n1 + 1)))

    a, b = box(), box()
    d_a = rng.standard_normal((a[1] - a[0], a[3] - a[2]))
    h = float(rng.choice([1.0, 0.5]))
    ref = op.restrict(op.inv_laplacian(op.extend(d_a, a, (n2, n1)), h), b)
    got = op.inv_laplacian_blocks(d_a, a, b, (n2, n1), _random_cuts(rng, n2), _random_cuts(rng, n1), h)
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_block_formula_single_block_and_single_frequencies():
    """The two extreme decompositions, one block and one block per frequency,
    give the same operator."""
    rng = np.random.default_rng(77)
    n2, n1 = 11, 16
    a, b = (2, 9, 3, 12), (0, 6, 5, 16)
    d_a = rng.standard_normal((7, 9))
    one = op.inv_laplacian_blocks(d_a, a, b, (n2, n1), [(0, n2)], [(0, n1)])
    each = op.inv_laplacian_blocks(d_a, a, b, (n2, n1), [(i, i + 1) for i in range(n2)],
                                   [(j, j + 1) for j in range(n1)])
    ref = op.restrict(op.inv_laplacian(op.extend(d_a, a, (n2, n1))), b)
    assert np.abs(one - ref).max() < 1e-12 and np.abs(each - ref).max() < 1e-12

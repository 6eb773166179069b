"""Pins of the oracle's quality measures (Section 5.2): exact rational
arithmetic on small grids, closed forms for shifted and rescaled images, and
the invariants the definitions fix."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import quality as q


def mssim_exact(x, ref):
    """The MSSIM formula in exact rational arithmetic, with plain loops; the
    constants c1 = (1/100)^2 and c2 = (3/100)^2 are exact rationals too."""
    xs = [Fraction(v) for v in np.ravel(x)]
    rs = [Fraction(v) for v in np.ravel(ref)]
    n = len(xs)
    mx, mr = sum(xs) / n, sum(rs) / n
    vx = sum((a - mx) ** 2 for a in xs) / n
    vr = sum((b - mr) ** 2 for b in rs) / n
    cv = sum((a - mx) * (b - mr) for a, b in zip(xs, rs)) / n
    c1, c2 = Fraction(1, 100) ** 2, Fraction(3, 100) ** 2
    return (2 * mx * mr + c1) * (2 * cv + c2) / ((mx * mx + mr * mr + c1) * (vx + vr + c2))


def mse_exact(x, ref):
    d = [(Fraction(a) - Fraction(b)) ** 2 for a, b in zip(np.ravel(x), np.ravel(ref))]
    return sum(d) / len(d)


def dyadic(rng, shape):
    """Values k/64 in [0, 1]: exact in binary, so Fraction(v) is the value."""
    return rng.integers(0, 65, size=shape) / 64.0


@pytest.mark.parametrize("shape", [(3, 4), (5, 2), (1, 7)])
def test_against_exact_rationals(shape):
    rng = np.random.default_rng(7)
    x, ref = dyadic(rng, shape), dyadic(rng, shape)
    assert q.mssim(x, ref) == pytest.approx(float(mssim_exact(x, ref)), rel=1e-14, abs=1e-15)
    m = float(mse_exact(x, ref))
    assert q.mse(x, ref) == pytest.approx(m, rel=1e-15)
    assert q.psnr(x, ref) == pytest.approx(-10.0 * np.log10(m), rel=1e-14)


def test_psnr_closed_form_and_identity():
    ref = np.random.default_rng(1).random((9, 11))
    for c in (0.5, 0.1, 1e-3):
        # MSE of a constant offset c is c^2, so PSNR = -20 log10 c
        assert q.psnr(ref + c, ref) == pytest.approx(-20.0 * np.log10(c), rel=1e-12)
    assert q.psnr(ref, ref) == float("inf")


def test_mssim_identity_symmetry_and_bounds():
    rng = np.random.default_rng(2)
    a, b = rng.random((8, 6)), rng.random((8, 6))
    assert q.mssim(a, a) == pytest.approx(1.0, abs=1e-15)
    const = np.full((4, 5), 0.3)
    assert q.mssim(const, const) == pytest.approx(1.0, abs=1e-15)
    assert q.mssim(a, b) == pytest.approx(q.mssim(b, a), rel=1e-15)
    assert -1.0 <= q.mssim(a, b) <= 1.0
    assert q.mssim(a, 1.0 - a) < 0  # anti-correlated structure


def test_mssim_shift_closed_form():
    """x = ref + c: equal variances and cov = var, so the structure factor is
    1 and MSSIM = (2 m (m + c) + c1) / (m^2 + (m + c)^2 + c1)."""
    ref = np.random.default_rng(3).random((10, 7))
    m, c1 = ref.mean(), 1e-4
    for c in (0.2, -0.05):
        want = (2 * m * (m + c) + c1) / (m * m + (m + c) ** 2 + c1)
        assert q.mssim(ref + c, ref) == pytest.approx(want, rel=1e-13)


def test_mssim_contrast_closed_form():
    """x = m + k (ref - m): equal means, so the luminance factor is 1 and
    MSSIM = (2 k v + c2) / ((1 + k^2) v + c2), v the variance of ref."""
    ref = np.random.default_rng(4).random((6, 9))
    m, v, c2 = ref.mean(), ref.var(), 9e-4
    for k in (0.5, 2.0, -1.0):
        want = (2 * k * v + c2) / ((1 + k * k) * v + c2)
        assert q.mssim(m + k * (ref - m), ref) == pytest.approx(want, rel=1e-12)


def test_perf_of_tangent_fields():
    gt = synth.clean_image(20, 24, 5)
    tg = q.tangent_gt(gt)
    assert tg.shape == (2, 21, 25)
    # offset c in both components: each PSNR is -20 log10 c, and each MSSIM
    # follows the shift closed form
    c = 0.01
    want = 0.0
    for k in range(2):
        m = tg[k].mean()
        ms = (2 * m * (m + c) + 1e-4) / (m * m + (m + c) ** 2 + 1e-4)
        want += 0.5 * (-20.0 * np.log10(c)) + 10.0 * ms
    assert q.perf_tau(tg + c, tg) == pytest.approx(want, rel=1e-12)
    # a field closer to the truth scores higher
    rng = np.random.default_rng(6)
    noise = rng.standard_normal(tg.shape)
    assert q.perf_tau(tg + 0.01 * noise, tg) > q.perf_tau(tg + 0.05 * noise, tg)

"""Image-quality measures of Section 5.2 (Comparison of IRV1 and IRV2,
Numerical Experiments), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* PSNR: minus ten times the decimal logarithm of the mean squared error over
  the grid (the paper fixes the maximal pixel value R = 1, so no peak term).
* MSSIM: the single-window structural similarity of the whole grid, built from
  the two means, the two variances and the covariance, all normalised by the
  point count (not by the count minus one), with c1 = (k1 R)^2, c2 = (k2 R)^2,
  k1 = 0.01, k2 = 0.03, R = 1.
* Perf of a tangent field: per component, half its PSNR plus ten times its
  MSSIM (20 * MSSIM / 2), summed over the two components, against the
  tangent field of the ground truth.

Readings: the ground-truth tangent field is tau_0 of the clean image (the same
Neumann differences that give tau_0 of the observation); a tangent field is
compared on its own grid Omega-tilde, so its point count is (N2+1)(N1+1).
"""
import numpy as np

from . import solvers as sv

K1, K2, R = 0.01, 0.03, 1.0


def mse(x, ref):
    """Mean of the squared pointwise differences."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.mean((x - ref) ** 2))


def psnr(x, ref):
    """PSNR(x, ref) = -10 log10 MSE(x, ref); +inf when x equals ref."""
    m = mse(x, ref)
    return float("inf") if m == 0.0 else float(-10.0 * np.log10(m))


def mssim(x, ref):
    """The paper's MSSIM of x against ref (one window: the whole grid)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    c1, c2 = (K1 * R) ** 2, (K2 * R) ** 2
    mx, mr = x.mean(), ref.mean()
    vx = np.mean((x - mx) ** 2)
    vr = np.mean((ref - mr) ** 2)
    cov = np.mean((x - mx) * (ref - mr))
    return float((2 * mx * mr + c1) * (2 * cov + c2) / ((mx * mx + mr * mr + c1) * (vx + vr + c2)))


def tangent_gt(gt, h=1.0):
    """Tangent field of the ground-truth image (reading: tau_0 of it)."""
    return sv.tau0(np.asarray(gt, dtype=np.float64), h)


def perf_tau(tau, tau_gt):
    """Perf = sum over the two components of PSNR/2 + 20 * MSSIM/2."""
    return float(sum(0.5 * psnr(tau[k], tau_gt[k]) + 20.0 * 0.5 * mssim(tau[k], tau_gt[k]) for k in range(2)))

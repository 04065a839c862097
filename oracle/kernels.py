"""Triweight kernel and its cumulative integral (Appendix B).

Test infrastructure (see the package docstring).

Readings:
  * Eq. triweight gives the kernel per unit z = (x - mu)/sigma; as a density
    in x it carries a factor 1/sigma, which the printed form omits.
  * Eq. terf prints "0 otherwise" for the cumulative kernel.  Because p(-3) = 0
    and p(3) = 1, the only consistent reading is 0 for z < -3 and 1 for z > 3.
  * The kernel is twice continuously differentiable at |z| = 3, not smooth to
    all orders as the appendix states; finite-difference checks keep away from
    the clip points.
"""

from __future__ import annotations

import numpy as np


def triweight_pdf(z):
    """T(z) = 35/96 (1 - (z/3)^2)^3 for |z| <= 3, else 0 (Eq. triweight)."""
    z = np.asarray(z, dtype=np.float64)
    u = 1.0 - (z / 3.0) ** 2
    return np.where(np.abs(z) <= 3.0, (35.0 / 96.0) * u**3, 0.0)


def triweight_cdf_poly(z):
    """The polynomial p(z) of Eq. terf, valid on [-3, 3]."""
    z = np.asarray(z, dtype=np.float64)
    return (0.5 + (35.0 / 96.0) * z - (35.0 / 864.0) * z**3
            + (7.0 / 2592.0) * z**5 - (5.0 / 69984.0) * z**7)


def triweight_cdf(z):
    """T_erf(z): 0 for z < -3, p(z) on [-3, 3], 1 for z > 3 (Eq. terf)."""
    z = np.asarray(z, dtype=np.float64)
    out = np.where(z < -3.0, 0.0, np.where(z > 3.0, 1.0, triweight_cdf_poly(np.clip(z, -3.0, 3.0))))
    return out


def triweight_blend(young, old, t):
    """young + (old - young) t for a transition weight t = T_erf(...), taken
    as old where t is exactly 1: both asymptotes are then reproduced exactly,
    and so is a value that does not change (old = young)."""
    young = np.asarray(young, dtype=np.float64)
    old = np.asarray(old, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return np.where(t == 1.0, old, young + (old - young) * t)


def triweight_cdf_x(x, mu, sigma):
    """T_erf(x | mu, sigma) = T_erf((x - mu)/sigma), with +-inf handled."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        z = (x - mu) / sigma
    z = np.where(np.isposinf(x), np.inf, np.where(np.isneginf(x), -np.inf, z))
    return triweight_cdf(z)

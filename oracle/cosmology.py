"""Cosmic time and distance modulus for flat wCDM (Section 2.2.1).

The paper converts rest-frame to apparent magnitudes with the distance modulus
D_mod(z) of a flat wCDM cosmology (text after Eq. restmag), and observes each
galaxy at the cosmic time t(z) that sets the upper limit of its star-formation
history (Section 3.1, Eq. mstartot).  Radiation is neglected.

Test infrastructure (see the package docstring).
"""

from __future__ import annotations

import numpy as np
from scipy import integrate

from .constants import C_KM_S, HUBBLE_TIME_GYR_KMS_MPC


def hubble_e(z, om0: float, w0: float = -1.0):
    """E(z) = H(z)/H0 for flat wCDM."""
    zp1 = 1.0 + np.asarray(z, dtype=np.float64)
    return np.sqrt(om0 * zp1**3 + (1.0 - om0) * zp1 ** (3.0 * (1.0 + w0)))


def hubble_time_gyr(h: float) -> float:
    return HUBBLE_TIME_GYR_KMS_MPC / (100.0 * h)


def age_at_z(z, om0: float = 0.3, h: float = 0.7, w0: float = -1.0):
    """Cosmic time t(z) in Gyr.

    For w0 = -1 (flat LCDM) the closed form
      t(z) = 2 / (3 H0 sqrt(OL)) * asinh( sqrt(OL/Om) (1+z)^{-3/2} )
    is used; otherwise t(z) = (1/H0) int_z^inf dz' / ((1+z') E(z')) by
    adaptive quadrature.
    """
    z = np.asarray(z, dtype=np.float64)
    th = hubble_time_gyr(h)
    if w0 == -1.0:
        ol = 1.0 - om0
        return (2.0 / (3.0 * np.sqrt(ol))) * th * np.arcsinh(
            np.sqrt(ol / om0) * (1.0 + z) ** -1.5)
    out = np.empty_like(z)
    for idx, zz in np.ndenumerate(z):
        val, _ = integrate.quad(lambda x: 1.0 / ((1.0 + x) * hubble_e(x, om0, w0)),
                                float(zz), np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
        out[idx] = th * val
    return out


def age_at_z_quadrature(z, om0: float = 0.3, h: float = 0.7, w0: float = -1.0):
    """t(z) straight from its defining integral (used to pin the closed form)."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    th = hubble_time_gyr(h)
    out = np.empty_like(z)
    for i, zz in enumerate(z):
        val, _ = integrate.quad(lambda x: 1.0 / ((1.0 + x) * hubble_e(x, om0, w0)),
                                float(zz), np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
        out[i] = th * val
    return out


def comoving_distance_mpc(z, om0: float = 0.3, h: float = 0.7, w0: float = -1.0):
    """Line-of-sight comoving distance (c/H0) int_0^z dz'/E(z') in Mpc."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    dh = C_KM_S / (100.0 * h)
    out = np.empty_like(z)
    for i, zz in enumerate(z):
        val, _ = integrate.quad(lambda x: 1.0 / hubble_e(x, om0, w0), 0.0, float(zz),
                                epsabs=0.0, epsrel=1e-12, limit=200)
        out[i] = dh * val
    return out


def luminosity_distance_mpc(z, om0: float = 0.3, h: float = 0.7, w0: float = -1.0):
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    return (1.0 + z) * comoving_distance_mpc(z, om0, h, w0)


def distance_modulus(z, om0: float = 0.3, h: float = 0.7, w0: float = -1.0):
    """D_mod(z) = 5 log10( d_L / 10 pc ) with d_L in Mpc (-inf at z = 0)."""
    dl = luminosity_distance_mpc(z, om0, h, w0)
    with np.errstate(divide="ignore"):
        return 5.0 * np.log10(dl) + 25.0

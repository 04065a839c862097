"""Redshifted filter integrals and apparent AB magnitudes (Section 2.2.1).

Test infrastructure (see the package docstring).

Eq. restmag gives the absolute magnitude through a filter T_Q as the ratio of
two integrals over d lambda / lambda, discretised by trapezoidal sums.  For
the observer frame, the rest-frame SED is moved to lambda_obs = (1+z)
lambda_rest before the integral, and the apparent magnitude is
m = M' + D_mod(z) - 2.5 log10(1+z).

Readings:
  * "Simple interpolation" is read as resampling the filter curve onto the
    redshifted SED grid by linear interpolation, with zero transmission outside
    the tabulated filter.  Numerator and denominator use the same grid, so a
    flat f_nu spectrum gives its exact value.
  * The trapezoid runs in lambda (not ln lambda) over T L / lambda, as printed.
  * Parts of a band outside the SED grid contribute nothing.
  * A band with zero denominator gives NaN; a zero numerator gives +inf.
"""

from __future__ import annotations

import numpy as np

from .constants import AB0_LSUN_PER_HZ


def filter_on_grid(lam_obs, filt_wave, filt_trans):
    """T(lambda_obs) by linear interpolation, zero outside the table."""
    return np.interp(lam_obs, filt_wave, filt_trans, left=0.0, right=0.0)


def band_integrals(wave_rest, sed_row, z, filt_wave, filt_trans):
    """(num[b], den[b]) for one galaxy.

    num_b = trapz( T_b(l_obs) * L(l_rest) / l_obs, l_obs )
    den_b = trapz( T_b(l_obs) / l_obs, l_obs ),   l_obs = (1+z) l_rest.
    """
    lam_obs = (1.0 + z) * np.asarray(wave_rest, dtype=np.float64)
    n_band = filt_wave.shape[0]
    num = np.empty(n_band)
    den = np.empty(n_band)
    for b in range(n_band):
        t = filter_on_grid(lam_obs, filt_wave[b], filt_trans[b])
        num[b] = np.trapezoid(t * sed_row / lam_obs, lam_obs)
        den[b] = np.trapezoid(t / lam_obs, lam_obs)
    return num, den


def apparent_mag(num, den, dmod, z):
    """m = -2.5 log10( num / (AB0 den) ) + D_mod(z) - 2.5 log10(1+z).

    Reading: at z = 0 the observable is the absolute magnitude M of
    Eq. restmag itself (a source at 10 pc; the population of the Section 4.1
    benchmark is observed at z = 0), so the distance terms apply for z > 0
    only; dmod is ignored there.
    """
    num = np.asarray(num, dtype=np.float64)
    den = np.asarray(den, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = num / (AB0_LSUN_PER_HZ * den)
        m_abs = -2.5 * np.log10(ratio)
    m_abs = np.where(den == 0.0, np.nan, m_abs)
    dmod = np.asarray(dmod, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    if m_abs.ndim == 2:
        dmod = dmod[:, None]
        z = z[:, None]
    with np.errstate(invalid="ignore"):
        offset = np.where(z > 0.0, dmod - 2.5 * np.log10(1.0 + z), 0.0)
    return m_abs + offset

"""Dust attenuation (Section 3.4, Eqs. attenuation, salim, kzero, uvbump) and
its dependence on stellar age (Section 3.4.1, Eq. agedep_dust_csp).

Test infrastructure (see the package docstring).

F_att(lambda) = 10^(-0.4 A_lambda),  A_lambda = A_V/4.05 * k_lambda,
k_lambda = k0(lambda) (lambda/5500 A)^delta + D_lambda,
D_lambda = E_b (lambda dl)^2 / ((lambda^2 - lambda_b^2)^2 + (lambda dl)^2).

Readings:
  * Eq. kzero prints the Calzetti curve below 0.15 micron and the Leitherer
    curve above it.  The cited Salim et al. parameterisation and the ranges over
    which the two curves were fitted (Leitherer et al. 2002: 0.097-0.18 micron;
    Calzetti et al. 2000: 0.12-2.2 micron) imply the reverse, which is the
    default here: Leitherer below 0.15 micron, Calzetti at and above it.  The
    printed order is available with k0_reading="printed".
  * Calzetti's two branches meet at 0.63 micron without being continuous; the
    ultraviolet-optical branch is used below 0.63 micron.  Both curves are
    extrapolated outside their fitted ranges.
  * The bump amplitude E_b is a free per-galaxy parameter ("bump"); the
    paper's tie E_b = -1.9 delta + 0.85 is the special case bump = that value.
  * The coefficients of the two k0 curves come from the cited publications
    (Calzetti et al. 2000, Eq. 4; Leitherer et al. 2002, Eq. 14), not from the
    paper's text.
  * Age-dependent attenuation: A_V and delta move from their young-star
    values (the per-galaxy av, delta) to old-star values (av_old, delta_old)
    through the cumulative triweight of log10 age, X_i = X_young + (X_old -
    X_young) T_erf((log10 tau_i - pivot) / width) (Appendix B, Eq. terf).  The
    paper names neither the centre nor the width; the default centre is
    log10 tau = 7 (10 Myr, the birth-cloud time scale of the model it cites)
    and the width a population-wide scalar.  The bump amplitude stays
    age-independent: the paper lets only A_V and delta vary.
"""

from __future__ import annotations

import numpy as np

from .constants import (DRUDE_CENTRE_ANGSTROM, DRUDE_WIDTH_ANGSTROM, K0_SWITCH_MICRON,
                        LAMBDA_V_ANGSTROM, R_V_SALIM)


def k_calzetti00(lam_micron):
    """Calzetti et al. (2000) starburst attenuation curve k(lambda), R_V = 4.05."""
    x = np.asarray(lam_micron, dtype=np.float64)
    uv = 2.659 * (-2.156 + 1.509 / x - 0.198 / x**2 + 0.011 / x**3) + 4.05
    ir = 2.659 * (-1.857 + 1.040 / x) + 4.05
    return np.where(x < 0.63, uv, ir)


def k_leitherer02(lam_micron):
    """Leitherer et al. (2002) far-UV attenuation curve k(lambda)."""
    x = np.asarray(lam_micron, dtype=np.float64)
    return 5.472 + 0.671 / x - 9.218e-3 / x**2 + 2.620e-3 / x**3


def k0(lam_angstrom, reading: str = "salim"):
    """Baseline curve k0(lambda) of Eq. kzero (see the module readings)."""
    x = np.asarray(lam_angstrom, dtype=np.float64) / 1.0e4
    if reading == "salim":
        return np.where(x < K0_SWITCH_MICRON, k_leitherer02(x), k_calzetti00(x))
    if reading == "printed":
        return np.where(x < K0_SWITCH_MICRON, k_calzetti00(x), k_leitherer02(x))
    raise ValueError(reading)


def drude_bump(lam_angstrom, amplitude):
    """D_lambda of Eq. uvbump with E_b = amplitude (broadcasts)."""
    lam = np.asarray(lam_angstrom, dtype=np.float64)
    ld = lam * DRUDE_WIDTH_ANGSTROM
    return amplitude * ld**2 / ((lam**2 - DRUDE_CENTRE_ANGSTROM**2) ** 2 + ld**2)


def k_lambda(lam_angstrom, delta, bump, reading: str = "salim"):
    """k_lambda[g, l] = k0 (lambda/lambda_V)^delta + D_lambda (Eq. salim)."""
    lam = np.asarray(lam_angstrom, dtype=np.float64)[None, :]
    delta = np.atleast_1d(np.asarray(delta, dtype=np.float64))[:, None]
    bump = np.atleast_1d(np.asarray(bump, dtype=np.float64))[:, None]
    return k0(lam, reading) * (lam / LAMBDA_V_ANGSTROM) ** delta + drude_bump(lam, bump)


def age_dependent_parameters(av, delta, av_old, delta_old, lg_age, pivot, width):
    """(A_V[g, i], delta[g, i]) of the age-dependent attenuation (Section
    3.4.1): each moves from its young-star value to its old-star value with
    T_erf((log10 tau_i - pivot) / width)."""
    from .kernels import triweight_blend, triweight_cdf
    t = triweight_cdf((np.asarray(lg_age, dtype=np.float64) - pivot) / width)[None, :]
    col = lambda v: np.atleast_1d(np.asarray(v, dtype=np.float64))[:, None]
    return (triweight_blend(col(av), col(av_old), t),
            triweight_blend(col(delta), col(delta_old), t))


def attenuation(lam_angstrom, av, delta, bump, reading: str = "salim"):
    """F_att[g, l] = 10^(-0.4 A_V/4.05 k_lambda) (Eqs. attenuation, salim)."""
    av = np.atleast_1d(np.asarray(av, dtype=np.float64))[:, None]
    a_lam = av / R_V_SALIM * k_lambda(lam_angstrom, delta, bump, reading)
    return 10.0 ** (-0.4 * a_lam)

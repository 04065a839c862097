"""Star-formation history, mass formed and age-bin masses (Section 3.1).

Test infrastructure (see the package docstring).

The SSP block is tabulated at discrete ages, so the continuous composite
spectrum (Eq. csp) becomes a sum over age bins weighted by the mass formed in
each bin (Eq. cspsum, with the total mass formed of Eq. mstartot).  The mass
formed up to time t is the trapezoid integral of the tabulated SFR
(Section 2.2.1 discretises integrals with trapezoidal sums).

Readings:
  * The shared time grid t_table (Gyr) starts after the Big Bang; no stars form
    before t_table[0] and the SFR is linear between grid points, so the mass
    formed is piecewise linear between cumulative-trapezoid nodes and is held
    at its last value after t_table[-1].
  * Bin edges (the text after Eq. cspsum is garbled): ages are binned at the
    geometric midpoints of adjacent SSP ages, with the youngest bin starting at
    age 0 and the oldest extending to infinite age.  With these edges the bin
    masses telescope to the total mass formed up to t_obs.
  * Masses are masses formed (the footnote to Eq. spsagedef); the surviving-
    mass fits of Appendix A are out of scope.
  * The parametric SFR stand-in for Diffstar is
      SFR(t) = A (t/tau)^alpha exp(-t/tau) (1 - q Phi((t - t_q)/0.5 Gyr))
    with Phi the standard normal CDF.
"""

from __future__ import annotations

import numpy as np
from scipy import special

from .constants import SFH_QUENCH_WIDTH_GYR, YR_PER_GYR


def sfr_from_params(t_table, sfh_params):
    """Tabulate SFR [M_sun/yr] on t_table [Gyr] for params [5, n_gal].

    Returns [n_gal, n_t].
    """
    t = np.asarray(t_table, dtype=np.float64)[None, :]
    a, tau, alpha, q, tq = (np.asarray(p, dtype=np.float64)[:, None] for p in sfh_params)
    base = a * (t / tau) ** alpha * np.exp(-t / tau)
    quench = 1.0 - q * special.ndtr((t - tq) / SFH_QUENCH_WIDTH_GYR)
    return base * quench


def cumulative_mass(t_table, sfr):
    """Mass formed up to each grid time, M_cum[g, n] in M_sun (Eq. mstartot).

    M_cum[:, 0] = 0 and M_cum[:, n] = 1e9 * sum_{m<n} (SFR_m + SFR_{m+1})/2
    * (t_{m+1} - t_m).
    """
    t = np.asarray(t_table, dtype=np.float64)
    sfr = np.atleast_2d(np.asarray(sfr, dtype=np.float64))
    dt = np.diff(t)
    seg = 0.5 * (sfr[:, :-1] + sfr[:, 1:]) * dt[None, :] * YR_PER_GYR
    out = np.zeros_like(sfr)
    out[:, 1:] = np.cumsum(seg, axis=1)
    return out


def mass_formed_at(t, t_table, mcum_row):
    """M(t) for one galaxy: 0 for t <= t_table[0], linear interpolation of the
    cumulative nodes inside the grid, the last node after it."""
    t = np.asarray(t, dtype=np.float64)
    tt = np.asarray(t_table, dtype=np.float64)
    out = np.interp(t, tt, mcum_row)
    return np.where(t <= tt[0], 0.0, out)


def age_bin_edges_yr(lg_age):
    """Age-bin edges [n_age + 1] in years: 0, geometric midpoints, +inf."""
    a = np.asarray(lg_age, dtype=np.float64)
    edges = np.empty(a.size + 1)
    edges[0] = 0.0
    edges[1:-1] = 10.0 ** (0.5 * (a[:-1] + a[1:]))
    edges[-1] = np.inf
    return edges


def age_bin_masses(t_obs, t_table, sfr, lg_age):
    """Mass formed in each SSP age bin, m_age[g, i] in M_sun (Eq. cspsum).

    Bin i collects stars with ages in [edge_i, edge_{i+1}), i.e. formed at
    cosmic times in (t_obs - edge_{i+1}/1e9, t_obs - edge_i/1e9].
    m_age = M_star(t_obs) * P_SFH(tau_i | t_obs).
    """
    t_obs = np.atleast_1d(np.asarray(t_obs, dtype=np.float64))
    mcum = cumulative_mass(t_table, sfr)
    edges_gyr = age_bin_edges_yr(lg_age) / YR_PER_GYR
    n_gal = t_obs.size
    out = np.empty((n_gal, edges_gyr.size - 1))
    for g in range(n_gal):
        t_edge = t_obs[g] - edges_gyr            # decreasing cosmic times
        m_edge = mass_formed_at(t_edge, t_table, mcum[g])
        out[g] = m_edge[:-1] - m_edge[1:]
    return out


def total_mass_formed(t_obs, t_table, sfr):
    """M_star(t_obs) (Eq. mstartot) for each galaxy."""
    t_obs = np.atleast_1d(np.asarray(t_obs, dtype=np.float64))
    mcum = cumulative_mass(t_table, sfr)
    return np.array([mass_formed_at(t_obs[g], t_table, mcum[g]) for g in range(t_obs.size)])

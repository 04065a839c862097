"""Age-dependent metallicity distribution weights (Section 3.2).

Test infrastructure (see the package docstring).

At fixed stellar age the MDF is a triweight kernel in log10 Z (a clipped
log-normal, Section 3.2.1), and the weight of SSP metallicity j is the kernel
mass inside bin j, a difference of cumulative kernels (Appendix B, Eq. terf).
The centre of the MDF depends on age (Section 3.2.2, Eq. agedep_mdf); the
workloads give it as a linear slope in log age, and Section 3.2.2 also moves
it from a young-age to an old-age value through the cumulative triweight
T_erf of log10 age (Appendix B, Eq. terf).

Readings:
  * Metallicity bins are bounded by the midpoints of adjacent SSP log10 Z
    values, with the lowest bin open to -inf and the highest to +inf, so the
    weights over j sum to one for every age.
  * mu_i = lgmet + slope * (log10 tau_i - pivot) with pivot log10 tau = 9.0;
    slope = 0 gives the uncorrelated MDF of Eq. simple_mdf.
  * Transition model: mu_i = lgmet + (lgmet_old - lgmet) T_erf((log10 tau_i -
    pivot) / width), lgmet being the young-age centre.  The paper names
    neither the centre nor the width of the transition; the centre is the
    same pivot (log10 tau = 9.0) and the width a population-wide scalar in dex
    (the transition runs over +-3 widths).
  * "log-normal" in the workload text is read as the triweight-clipped
    log-normal the paper uses.
"""

from __future__ import annotations

import numpy as np

from .kernels import triweight_blend, triweight_cdf, triweight_cdf_x


def met_bin_edges(lgz):
    """[n_met + 1] edges in log10 Z: -inf, midpoints, +inf."""
    z = np.asarray(lgz, dtype=np.float64)
    edges = np.empty(z.size + 1)
    edges[0] = -np.inf
    edges[1:-1] = 0.5 * (z[:-1] + z[1:])
    edges[-1] = np.inf
    return edges


def transition_weight(lg_age, pivot, width):
    """T_erf((lg_age_i - pivot) / width): 0 for the young asymptote, 1 for the
    old one (Eq. terf)."""
    a = np.asarray(lg_age, dtype=np.float64)
    return triweight_cdf((a - pivot) / width)


def mdf_centres(lgmet, lg_age, slope, pivot, lgmet_old=None, width=None):
    """Linear model: mu[g, i] = lgmet_g + slope * (lg_age_i - pivot).
    Transition model (lgmet_old given): mu[g, i] = lgmet_g + (lgmet_old_g -
    lgmet_g) T_erf((lg_age_i - pivot) / width)."""
    lgmet = np.atleast_1d(np.asarray(lgmet, dtype=np.float64))
    a = np.asarray(lg_age, dtype=np.float64)
    if lgmet_old is None:
        return lgmet[:, None] + slope * (a[None, :] - pivot)
    old = np.atleast_1d(np.asarray(lgmet_old, dtype=np.float64))
    t = transition_weight(a, pivot, width)
    return triweight_blend(lgmet[:, None], old[:, None], t[None, :])


def mdf_weights(lgmet, sigma, lgz, lg_age, slope=0.1, pivot=9.0, lgmet_old=None, width=None):
    """P[g, j, i] = T_erf(e_{j+1} | mu_gi, sigma_g) - T_erf(e_j | mu_gi, sigma_g)."""
    lgmet = np.atleast_1d(np.asarray(lgmet, dtype=np.float64))
    sigma = np.atleast_1d(np.asarray(sigma, dtype=np.float64))
    edges = met_bin_edges(lgz)
    mu = mdf_centres(lgmet, lg_age, slope, pivot, lgmet_old, width)   # [g, i]
    cdf = triweight_cdf_x(edges[None, :, None], mu[:, None, :], sigma[:, None, None])
    return cdf[:, 1:, :] - cdf[:, :-1, :]

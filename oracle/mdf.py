"""Age-dependent metallicity distribution weights (Section 3.2).

Test infrastructure (see the package docstring).

At fixed stellar age the MDF is a triweight kernel in log10 Z (a clipped
log-normal, Section 3.2.1), and the weight of SSP metallicity j is the kernel
mass inside bin j, a difference of cumulative kernels (Appendix B, Eq. terf).
The centre of the MDF depends on age (Section 3.2.2, Eq. agedep_mdf); the
workloads give it as a linear slope in log age.

Readings:
  * Metallicity bins are bounded by the midpoints of adjacent SSP log10 Z
    values, with the lowest bin open to -inf and the highest to +inf, so the
    weights over j sum to one for every age.
  * mu_i = lgmet + slope * (log10 tau_i - pivot) with pivot log10 tau = 9.0;
    slope = 0 gives the uncorrelated MDF of Eq. simple_mdf.
  * "log-normal" in the workload text is read as the triweight-clipped
    log-normal the paper uses.
"""

from __future__ import annotations

import numpy as np

from .kernels import triweight_cdf_x


def met_bin_edges(lgz):
    """[n_met + 1] edges in log10 Z: -inf, midpoints, +inf."""
    z = np.asarray(lgz, dtype=np.float64)
    edges = np.empty(z.size + 1)
    edges[0] = -np.inf
    edges[1:-1] = 0.5 * (z[:-1] + z[1:])
    edges[-1] = np.inf
    return edges


def mdf_centres(lgmet, lg_age, slope, pivot):
    """mu[g, i] = lgmet_g + slope * (lg_age_i - pivot)."""
    lgmet = np.atleast_1d(np.asarray(lgmet, dtype=np.float64))
    a = np.asarray(lg_age, dtype=np.float64)
    return lgmet[:, None] + slope * (a[None, :] - pivot)


def mdf_weights(lgmet, sigma, lgz, lg_age, slope=0.1, pivot=9.0):
    """P[g, j, i] = T_erf(e_{j+1} | mu_gi, sigma_g) - T_erf(e_j | mu_gi, sigma_g)."""
    lgmet = np.atleast_1d(np.asarray(lgmet, dtype=np.float64))
    sigma = np.atleast_1d(np.asarray(sigma, dtype=np.float64))
    edges = met_bin_edges(lgz)
    mu = mdf_centres(lgmet, lg_age, slope, pivot)                  # [g, i]
    cdf = triweight_cdf_x(edges[None, :, None], mu[:, None, :], sigma[:, None, None])
    return cdf[:, 1:, :] - cdf[:, :-1, :]

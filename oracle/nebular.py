"""Nebular ionization axis and emission-line equivalent widths (Section 3.3,
Eq. nebsed; Section 2.2.2, Eq. eqw).

Test infrastructure (see the package docstring).

With the ionization parameter u = log10 U_s as a third SSP axis, the
composite SED sums over (age, metallicity, ionization) cells, the weight of a
cell being the age-bin mass times the metallicity weight times an ionization
weight P_neb(u_k).  P_neb is a triweight kernel in u, handled exactly as the
MDF: the weight of grid point k is the kernel mass inside its bin.

The equivalent width of a line is the integral, over a window around the
line, of the SED's excess over its continuum relative to the continuum; the
continuum is a least-squares quadratic fitted to the SED around the line with
the line window masked out.

Readings:
  * Ionization bins are bounded by the midpoints of adjacent grid values of u,
    the lowest open to -inf and the highest to +inf (the metallicity reading),
    so the weights sum to one.  The distribution's centre and width are per
    galaxy; the paper's example uses width 0.25 dex.
  * The SSP block with the ionization axis is indexed [met, age, u, lambda].
  * The neighbourhood in which the continuum is fitted is a window of
    half-width fit_half_width around the line centre; the points of the line
    window, |lambda - centre| <= half_width, are masked out of the fit, every
    other grid point of the neighbourhood counts with equal weight.
  * The paper writes the continuum both as L_0(lambda') inside the integral
    and as its value at the line centre.  Here L_0(lambda') is the fitted
    quadratic evaluated at lambda' (the usual definition; for a flat
    continuum the two agree).
  * The integral is the trapezoid rule over the SED grid points inside the
    closed line window, in rest-frame Angstrom.  Emission gives a positive
    width.  Fewer than three fit points or two window points give NaN.

Gradients (the paper differentiates line strengths with respect to u_s):
the ionization weights are differentiable in the distribution's centre and
width, the SED is linear in them, and the width is a smooth function of the
SED, so d(width)/d(u_s) is the width's tangent along
dL/du_s = sum_k dP_k/du_s L_k, with L_k the SED of ionization point k alone.
"""

from __future__ import annotations

import numpy as np

from .kernels import triweight_cdf_x, triweight_pdf


def ion_bin_edges(lgu):
    """[n_u + 1] edges in u = log10 U_s: -inf, midpoints, +inf."""
    u = np.asarray(lgu, dtype=np.float64)
    edges = np.empty(u.size + 1)
    edges[0] = -np.inf
    edges[1:-1] = 0.5 * (u[:-1] + u[1:])
    edges[-1] = np.inf
    return edges


def ionization_weights(lgu_s, sigma_u, lgu):
    """P_neb[g, k] = T_erf(e_{k+1} | u_g, sigma_g) - T_erf(e_k | u_g, sigma_g)."""
    centre = np.atleast_1d(np.asarray(lgu_s, dtype=np.float64))
    sigma = np.atleast_1d(np.asarray(sigma_u, dtype=np.float64))
    edges = ion_bin_edges(lgu)
    cdf = triweight_cdf_x(edges[None, :], centre[:, None], sigma[:, None])
    return cdf[:, 1:] - cdf[:, :-1]


def ionization_weight_derivatives(lgu_s, sigma_u, lgu):
    """(dP/du_s, dP/dsigma_u) [g, n_u] of the ionization weights.

    With z_e = (e - u_s)/sigma and T the triweight density, the weight of bin
    k is T_erf(z_{k+1}) - T_erf(z_k), so dP_k/du_s = -(T(z_{k+1}) -
    T(z_k))/sigma and dP_k/dsigma = -(z_{k+1} T(z_{k+1}) - z_k T(z_k))/sigma;
    the infinite outer edges contribute nothing."""
    centre = np.atleast_1d(np.asarray(lgu_s, dtype=np.float64))
    sigma = np.atleast_1d(np.asarray(sigma_u, dtype=np.float64))
    edges = ion_bin_edges(lgu)
    with np.errstate(invalid="ignore"):
        z = (edges[None, :] - centre[:, None]) / sigma[:, None]
    finite = np.isfinite(z)
    zf = np.where(finite, z, 0.0)
    t = np.where(finite, triweight_pdf(zf), 0.0)
    zt = np.where(finite, zf * t, 0.0)
    d_u = -(t[:, 1:] - t[:, :-1]) / sigma[:, None]
    d_s = -(zt[:, 1:] - zt[:, :-1]) / sigma[:, None]
    return d_u, d_s


def sed_nebular(w, p_neb, lum):
    """Eq. nebsed: L[g, l] = sum_{j,i,k} W[g, j, i] P_neb[g, k] L_SSP[j, i, k, l].

    w [g, n_met, n_age] (age-bin mass times metallicity weight), p_neb
    [g, n_u], lum [n_met, n_age, n_u, n_wave].  The joint weight is formed
    densely and contracted with one matrix product."""
    n_met, n_age, n_u, n_wave = lum.shape
    joint = w[:, :, :, None] * p_neb[:, None, None, :]
    return joint.reshape(w.shape[0], -1) @ lum.reshape(n_met * n_age * n_u, n_wave)


def line_windows(wave, centre, half_width, fit_half_width):
    """Boolean masks over the grid: the line window and the continuum points
    (inside the neighbourhood, outside the line window)."""
    lam = np.asarray(wave, dtype=np.float64)
    d = np.abs(lam - centre)
    in_line = d <= half_width
    in_fit = (d <= fit_half_width) & ~in_line
    return in_line, in_fit


def continuum_fit(wave, spec, centre, fit_half_width, in_fit):
    """Least-squares coefficients (c0, c1, c2) of the quadratic continuum in
    x = (lambda - centre) / fit_half_width over the continuum points."""
    x = (np.asarray(wave, dtype=np.float64)[in_fit] - centre) / fit_half_width
    design = np.stack([np.ones_like(x), x, x * x], axis=1)
    coef, *_ = np.linalg.lstsq(design, np.asarray(spec, dtype=np.float64)[in_fit], rcond=None)
    return coef


def equivalent_width_jvp(wave, spec, dspec, centre, half_width, fit_half_width):
    """(W, dW) for every row: Eq. eqw and its derivative along a tangent
    dspec of the SED.  The fit is linear in the SED, so the continuum's
    tangent is the same least-squares fit of dspec; the ratio's derivative is
    (dL L_0 - L dL_0) / L_0^2, integrated with the same trapezoid rule."""
    lam = np.asarray(wave, dtype=np.float64)
    spec = np.atleast_2d(np.asarray(spec, dtype=np.float64))
    dspec = np.atleast_2d(np.asarray(dspec, dtype=np.float64))
    in_line, in_fit = line_windows(lam, centre, half_width, fit_half_width)
    w = np.full(spec.shape[0], np.nan)
    dw = np.full(spec.shape[0], np.nan)
    if in_fit.sum() < 3 or in_line.sum() < 2:
        return w, dw
    xl = (lam[in_line] - centre) / fit_half_width
    for g in range(spec.shape[0]):
        c = continuum_fit(lam, spec[g], centre, fit_half_width, in_fit)
        dc = continuum_fit(lam, dspec[g], centre, fit_half_width, in_fit)
        cont = c[0] + c[1] * xl + c[2] * xl * xl
        dcont = dc[0] + dc[1] * xl + dc[2] * xl * xl
        line = spec[g, in_line]
        w[g] = np.trapezoid((line - cont) / cont, lam[in_line])
        dw[g] = np.trapezoid((dspec[g, in_line] * cont - line * dcont) / (cont * cont), lam[in_line])
    return w, dw


def equivalent_width(wave, spec, centre, half_width, fit_half_width):
    """Eq. eqw for every row of spec [n_gal, n_wave] (rest frame); [n_gal]."""
    lam = np.asarray(wave, dtype=np.float64)
    spec = np.atleast_2d(np.asarray(spec, dtype=np.float64))
    in_line, in_fit = line_windows(lam, centre, half_width, fit_half_width)
    out = np.full(spec.shape[0], np.nan)
    if in_fit.sum() < 3 or in_line.sum() < 2:
        return out
    xl = (lam[in_line] - centre) / fit_half_width
    for g in range(spec.shape[0]):
        c0, c1, c2 = continuum_fit(lam, spec[g], centre, fit_half_width, in_fit)
        cont = c0 + c1 * xl + c2 * xl * xl
        ratio = (spec[g, in_line] - cont) / cont
        out[g] = np.trapezoid(ratio, lam[in_line])
    return out

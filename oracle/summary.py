"""Population summary of the forward model (Section 4.1) and its gradient.

Test infrastructure (see the package docstring).

The Section 4.1 pipeline selects red galaxies with a colour cut and evaluates
a histogram of r-band magnitude over the selected sample.  To carry gradients
from such a summary back to every galaxy (the population-level target that
the discussion in Section 4.1 points to), both steps are smoothed with the
triweight kernel of Appendix B:

  colour weight   w_g = T_erf((c_g - c_cut) / s_c),  c_g = m_a - m_b
  bin membership  B_k(m) = T_erf((e_{k+1} - m) / s_m) - T_erf((e_k - m) / s_m)
  histogram       H_k = sum_g w_g B_k(m_g)

T_erf is the cumulative triweight in units of its width (support +-3).
Readings:
  * "red" means the colour above the cut (redder = larger m_a - m_b with a
    bluer than b).
  * Zero widths give the paper's hard selection (w = 1 for c > c_cut, else 0)
    and the plain histogram with bins [e_k, e_{k+1}), the last bin closed on
    the right; the summary is then piecewise constant and its gradient zero.
  * A galaxy whose colour or magnitude is not finite contributes nothing.
"""

from __future__ import annotations

import numpy as np

from .kernels import triweight_cdf, triweight_pdf


def _finite(c, m):
    return np.isfinite(c) & np.isfinite(m)


def colour_weight(colour, cut, width):
    """w = T_erf((c - cut)/width), or the hard cut c > cut for width 0."""
    c = np.asarray(colour, dtype=np.float64)
    if width == 0.0:
        return (c > cut).astype(np.float64)
    return triweight_cdf((c - cut) / width)


def bin_membership(m, edges, width):
    """B[g, k]: the smoothed indicator of bin k, or the hard one for width 0."""
    m = np.asarray(m, dtype=np.float64)[:, None]
    e = np.asarray(edges, dtype=np.float64)
    if width == 0.0:
        lo, hi = e[None, :-1], e[None, 1:]
        inside = (m >= lo) & (m < hi)
        inside[:, -1] |= (m[:, 0] == e[-1])
        return inside.astype(np.float64)
    t = triweight_cdf((e[None, :] - m) / width)
    return t[:, 1:] - t[:, :-1]


def histogram(mags, band_a, band_b, cut, colour_width, band_m, edges, mag_width):
    """H[k] = sum_g w_g B_k(m_g) (float64)."""
    mags = np.asarray(mags, dtype=np.float64)
    c = mags[:, band_a] - mags[:, band_b]
    m = mags[:, band_m]
    ok = _finite(c, m)
    w = colour_weight(np.where(ok, c, 0.0), cut, colour_width) * ok
    b = bin_membership(np.where(ok, m, 0.0), edges, mag_width)
    return (w[:, None] * b).sum(axis=0)


def histogram_vjp(mags, band_a, band_b, cut, colour_width, band_m, edges, mag_width, hist_bar):
    """d(sum_k hbar_k H_k)/d mags, [n_gal, n_band] (zero for zero widths)."""
    mags = np.asarray(mags, dtype=np.float64)
    out = np.zeros_like(mags)
    if colour_width == 0.0 or mag_width == 0.0:
        return out
    hb = np.asarray(hist_bar, dtype=np.float64)
    c = mags[:, band_a] - mags[:, band_b]
    m = mags[:, band_m]
    ok = _finite(c, m)
    c = np.where(ok, c, 0.0)
    m = np.where(ok, m, 0.0)
    w = colour_weight(c, cut, colour_width)
    dw = triweight_pdf((c - cut) / colour_width) / colour_width
    b = bin_membership(m, edges, mag_width)
    e = np.asarray(edges, dtype=np.float64)
    # d/dm of T_erf((e - m)/s) is -pdf((e - m)/s)/s
    dt = -triweight_pdf((e[None, :] - m[:, None]) / mag_width) / mag_width
    db = dt[:, 1:] - dt[:, :-1]
    g_w = (b * hb[None, :]).sum(axis=1) * ok
    g_m = w * (db * hb[None, :]).sum(axis=1) * ok
    out[:, band_a] += g_w * dw
    out[:, band_b] -= g_w * dw
    out[:, band_m] += g_m
    return out

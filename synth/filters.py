"""Six LSST-like observed-frame filter transmission curves.

The paper integrates through LSST-like optical bands (Sections 3.1 and 4.1);
the real curves are not shipped here, so each band is a Gaussian transmission
curve tabulated on a uniform observed-frame wavelength grid spanning the centre
plus or minus two FWHM.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class FilterSet:
    """wave, trans: [n_band, n_pts] float64, observed-frame Angstrom and
    transmission probability."""

    wave: np.ndarray
    trans: np.ndarray

    @property
    def n_band(self) -> int:
        return int(self.wave.shape[0])

    @property
    def n_pts(self) -> int:
        return int(self.wave.shape[1])


def make_filters(n_band: int = 6, n_pts: int = 500, centre_range=(3600.0, 9700.0),
                 fwhm_range=(800.0, 1500.0), half_span_fwhm: float = 2.0) -> FilterSet:
    centres = np.linspace(centre_range[0], centre_range[1], n_band)
    fwhms = np.linspace(fwhm_range[0], fwhm_range[1], n_band)
    wave = np.empty((n_band, n_pts))
    trans = np.empty((n_band, n_pts))
    for b, (c, f) in enumerate(zip(centres, fwhms)):
        w = np.linspace(c - half_span_fwhm * f, c + half_span_fwhm * f, n_pts)
        wave[b] = w
        trans[b] = np.exp(-4.0 * np.log(2.0) * ((w - c) / f) ** 2)
    return FilterSet(wave=wave, trans=trans)


def make_tophat_filters(edges, n_pts: int = 2001) -> FilterSet:
    """Top-hat bands (transmission 1 inside [lo, hi]) for closed-form tests."""
    wave = np.empty((len(edges), n_pts))
    trans = np.ones((len(edges), n_pts))
    for b, (lo, hi) in enumerate(edges):
        wave[b] = np.linspace(lo, hi, n_pts)
    return FilterSet(wave=wave, trans=trans)

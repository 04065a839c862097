"""Seeded synthetic SSP spectral block L_SSP(lambda | tau_age, Z).

The paper takes the SSP block as a precomputed, fixed input (Section 2.1,
Eq. sspdef and the text after Eq. cspsum); its own tables come from FSPS with
MILES spectra, which are not available here.  This module builds a stand-in of
the same shape and units (L_sun/Hz per M_sun formed) from a few blackbodies and
Gaussian line features whose strengths vary smoothly with age and metallicity.
The result is strictly positive.  Nothing here is part of the method.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Physical constants used only to shape the synthetic spectra.
_HC_OVER_K_ANGSTROM_K = 1.438776877e8      # h c / k_B in Angstrom * Kelvin
_H_OVER_K_SECONDS_K = 4.799243073e-11      # h / k_B in second * Kelvin
_C_ANGSTROM_PER_S = 2.99792458e18


@dataclass(frozen=True)
class SspTable:
    """An SSP block on fixed (log10 Z, log10 age, wavelength) grids.

    lgz:    [n_met]  log10 Z (absolute metal mass fraction), ascending
    lg_age: [n_age]  log10 of the stellar age in years, ascending
    wave:   [n_wave] rest-frame wavelength in Angstrom, ascending
    lum:    [n_met, n_age, n_wave] float32, L_sun/Hz per M_sun formed
    """

    lgz: np.ndarray
    lg_age: np.ndarray
    wave: np.ndarray
    lum: np.ndarray

    @property
    def shape(self):
        return self.lum.shape


def _blackbody_per_hz(wave_angstrom: np.ndarray, temp_k: np.ndarray) -> np.ndarray:
    """Blackbody spectral shape normalised to unit integral over frequency.

    Returns b_nu with int b_nu dnu = 1 (units 1/Hz), broadcasting temp_k
    against wave_angstrom.
    """
    x = _HC_OVER_K_ANGSTROM_K / (wave_angstrom * temp_k)
    shape = (15.0 / np.pi**4) * (_H_OVER_K_SECONDS_K / temp_k)
    with np.errstate(over="ignore"):
        return shape * x**3 / np.expm1(x)


def make_ssp(n_wave: int = 1000, wave_lo: float = 1.0e3, wave_hi: float = 2.0e4,
             n_met: int = 12, n_age: int = 94, seed: int = 1,
             lgz_range=(-4.5, -1.3), lg_age_range=(5.5, 10.15),
             scale: float = 5.75) -> SspTable:
    """Build the synthetic SSP block.

    Grids: log10 Z uniform on lgz_range (n_met points), log10 age uniform on
    lg_age_range (n_age points), rest wavelengths log-spaced on
    [wave_lo, wave_hi] (n_wave points).  The overall scale puts the median
    r-band magnitude of the small 100-galaxy population near 22.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lgz = np.linspace(lgz_range[0], lgz_range[1], n_met)
    lg_age = np.linspace(lg_age_range[0], lg_age_range[1], n_age)
    wave = np.geomspace(wave_lo, wave_hi, n_wave)

    # Normalised age and metallicity coordinates in [0, 1].
    xa = ((lg_age - lg_age_range[0]) / (lg_age_range[1] - lg_age_range[0]))[None, :, None]
    yz = ((lgz - lgz_range[0]) / (lgz_range[1] - lgz_range[0]))[:, None, None]
    lam = wave[None, None, :]

    l_bol = 10.0 ** (3.0 - 3.3 * xa)                      # L_sun per M_sun
    w_hot = np.exp(-6.0 * xa)
    w_warm = 0.5 * np.exp(-2.0 * xa)
    w_cool = 0.3 + 0.4 * xa
    w_sum = w_hot + w_warm + w_cool
    t_hot = 3.5e4 * 10.0 ** (-0.6 * xa) * (1.0 - 0.10 * yz)
    t_warm = 9.0e3 * 10.0 ** (-0.2 * xa) * (1.0 - 0.05 * yz)
    t_cool = 4.5e3 * 10.0 ** (-0.08 * xa) * (1.0 - 0.05 * yz)

    spec = l_bol * (w_hot * _blackbody_per_hz(lam, t_hot)
                    + w_warm * _blackbody_per_hz(lam, t_warm)
                    + w_cool * _blackbody_per_hz(lam, t_cool)) / w_sum

    # Ten emission and ten absorption features.
    n_lines = 10
    for kind in ("emission", "absorption"):
        centres = np.exp(rng.uniform(np.log(1200.0), np.log(9000.0), n_lines))
        widths = centres * rng.uniform(0.002, 0.006, n_lines)
        if kind == "emission":
            amps = rng.uniform(0.5, 5.0, n_lines)
        else:
            amps = rng.uniform(0.05, 0.5, n_lines)
        for c, s, a in zip(centres, widths, amps):
            profile = np.exp(-0.5 * ((lam - c) / s) ** 2)
            if kind == "emission":
                spec = spec * (1.0 + a * np.exp(-5.0 * xa) * profile)
            else:
                spec = spec * (1.0 - a * (0.3 + 0.7 * xa) * (0.5 + 0.5 * yz) * profile)

    lum = (spec * scale).astype(np.float32)
    # Flush anything that underflowed float32 to the smallest normal so the
    # block stays strictly positive.
    tiny = np.finfo(np.float32).tiny
    lum = np.where(lum < tiny, tiny, lum).astype(np.float32)
    return SspTable(lgz=lgz, lg_age=lg_age, wave=wave, lum=np.ascontiguousarray(lum))

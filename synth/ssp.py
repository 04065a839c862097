"""Seeded synthetic SSP spectral block L_SSP(lambda | tau_age, Z), optionally
with a third axis, the nebular ionization parameter u = log10 U_s.

The paper takes the SSP block as a precomputed, fixed input (Section 2.1,
Eq. sspdef and the text after Eq. cspsum); its own tables come from FSPS with
MILES spectra, which are not available here.  This module builds a stand-in of
the same shape and units (L_sun/Hz per M_sun formed) from a few blackbodies and
Gaussian line features whose strengths vary smoothly with age and metallicity.
The result is strictly positive.  Nothing here is part of the method.

make_ssp_nebular adds the ionization axis of Section 3.3: nebular emission
lines at their rest wavelengths on top of the stellar block, present only for
young ages, with strengths that move with u the way the usual diagnostic
lines do ([OIII] up with u, [OII], [NII] and [SII] down, the Balmer lines
flat).  Their shapes and numbers are stand-ins chosen for structure, not
photoionization results.
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
    lum:    [n_met, n_age, n_wave] float32, L_sun/Hz per M_sun formed, or
            [n_met, n_age, n_u, n_wave] with the ionization axis
    lgu:    [n_u] log10 U_s, ascending, or None without the axis
    """

    lgz: np.ndarray
    lg_age: np.ndarray
    wave: np.ndarray
    lum: np.ndarray
    lgu: np.ndarray | None = None

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


# Rest wavelengths (Angstrom) of the nebular lines of the stand-in, with the
# equivalent width (Angstrom, on the young stellar continuum) at u = -3 and
# the slope of its log with u.  A second slope scales with metallicity.
NEBULAR_LINES = (
    # name,        centre,   EW(u=-3), dlog EW / du, dlog EW / dy
    ("Lya",        1215.67,  200.0,    0.0,          -0.2),
    ("[OII]3727",  3727.42,  150.0,   -0.4,           0.1),
    ("Hbeta",      4862.68,  100.0,    0.0,          -0.1),
    ("[OIII]4959", 4960.30,   33.3,    0.6,          -0.3),
    ("[OIII]5007", 5008.24,  100.0,    0.6,          -0.3),
    ("Halpha",     6564.61,  300.0,    0.0,          -0.1),
    ("[NII]6584",  6585.27,   60.0,   -0.3,           0.4),
    ("[SII]6717",  6718.29,   40.0,   -0.5,           0.2),
)


def make_ssp_nebular(n_u: int = 7, lgu_range=(-4.0, -1.0), n_wave: int = 1000,
                     wave_lo: float = 1.0e3, wave_hi: float = 2.0e4, n_met: int = 12,
                     n_age: int = 94, seed: int = 1, lgz_range=(-4.5, -1.3),
                     lg_age_range=(5.5, 10.15), scale: float = 5.75,
                     line_sigma_pixels: float = 2.0) -> SspTable:
    """SSP block with the ionization axis: lum [n_met, n_age, n_u, n_wave].

    The stellar part is make_ssp's block (same arguments and seed).  For cell
    (j, i, k) with young-age factor f = exp(-tau_i / 3 Myr), u = lgu_k and
    normalised metallicity y in [0, 1], the spectrum is the stellar one times
    a weak nebular-continuum factor 1 + 0.05 f (u + 2.5), plus, per line, a
    Gaussian in wavelength (sigma = line_sigma_pixels grid steps at the line)
    of area f EW(u, y) times the stellar continuum at the line centre, with
    log10 EW = log10 EW(-3) + s_u (u + 3) + s_y (y - 0.5).  u on lgu_range
    (n_u points, uniform); n_u = 1 takes the lower end.
    """
    base = make_ssp(n_wave=n_wave, wave_lo=wave_lo, wave_hi=wave_hi, n_met=n_met, n_age=n_age,
                    seed=seed, lgz_range=lgz_range, lg_age_range=lg_age_range, scale=scale)
    lgu = np.linspace(lgu_range[0], lgu_range[1], n_u) if n_u > 1 else np.array([lgu_range[0]])
    wave = base.wave
    stellar = base.lum.astype(np.float64)                                   # [j, i, l]
    f_age = np.exp(-(10.0 ** base.lg_age) / 3.0e6)[None, :, None, None]    # [1, i, 1, 1]
    yz = ((base.lgz - lgz_range[0]) / (lgz_range[1] - lgz_range[0]))[:, None, None, None]
    u = lgu[None, None, :, None]
    spec = stellar[:, :, None, :] * (1.0 + 0.05 * f_age * (u + 2.5))
    dlnl = np.log(wave_hi / wave_lo) / (n_wave - 1)
    lam = wave[None, None, None, :]
    for _, centre, ew3, s_u, s_y in NEBULAR_LINES:
        if not (wave[0] < centre < wave[-1]):
            continue
        n0 = int(np.argmin(np.abs(wave - centre)))
        cont = stellar[:, :, n0][:, :, None, None]                          # [j, i, 1, 1]
        ew = ew3 * 10.0 ** (s_u * (u + 3.0) + s_y * (yz - 0.5))
        sig = line_sigma_pixels * centre * dlnl
        profile = np.exp(-0.5 * ((lam - centre) / sig) ** 2) / (sig * np.sqrt(2.0 * np.pi))
        spec = spec + f_age * ew * cont * profile
    lum = spec.astype(np.float32)
    tiny = np.finfo(np.float32).tiny
    lum = np.where(lum < tiny, tiny, lum).astype(np.float32)
    return SspTable(lgz=base.lgz, lg_age=base.lg_age, wave=wave, lum=np.ascontiguousarray(lum),
                    lgu=lgu)


def make_line_spectra(n: int, wave: np.ndarray, lines, seed: int = 5) -> np.ndarray:
    """[n, n_wave] float32 spectra on `wave`: smooth positive continua (a
    random power law in wavelength with a weak ripple) times, at each
    (centre, half_width, ...) of `lines`, a Gaussian line of sigma half_width/4
    and random strength in [-0.5, 20] times the continuum (absorption to
    strong emission).  Stand-in input for equivalent-width checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    wave = np.asarray(wave, dtype=np.float64)
    x = np.log(wave / 5000.0)
    spec = (rng.uniform(0.5, 2.0, (n, 1)) * np.exp(rng.uniform(-2, 1, (n, 1)) * x)
            * (1.0 + 0.1 * np.sin(rng.uniform(3, 9, (n, 1)) * x)))
    for line in lines:
        c, h = float(line[0]), float(line[1])
        amp = rng.uniform(-0.5, 20.0, (n, 1))
        spec = spec * (1.0 + amp * np.exp(-0.5 * ((wave - c) / (0.25 * h)) ** 2))
    return (np.abs(spec) + 1e-3).astype(np.float32)

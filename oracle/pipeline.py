"""The forward hot path, end to end, in float64 (Sections 2-3).

Test infrastructure (see the package docstring).

  weights   W[g, j, i] = m_age[g, i] * P[g, j, i]   (Eqs. cspsum, agedep_mdf)
  sed       L[g, l] = sum_{j,i} W[g, j, i] L_SSP[j, i, l]   (Eqs. cspdeftheta,
            full_mdf), optionally times F_att (Eq. attenuation); with the
            ionization axis also summed over u with P_neb (Eq. nebsed)
  band_sums num/den of Eq. restmag on the redshifted grid
  mags      apparent AB magnitudes (Section 2.2.1)

The contraction is a plain matrix product (a library primitive); galaxies are
processed in blocks only to bound memory.  Nothing is windowed or skipped.

quantize_bf16_rne is the reference for the BF16 storage of the SSP block: each
(met, age) row is divided by its power-of-two scale s_k (the smallest power of
two not below the row maximum) and rounded to bfloat16 with
round-to-nearest-even.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cosmology, dust, mdf, nebular, photometry, sfh


@dataclass
class OracleInputs:
    lgz: np.ndarray          # [n_met]
    lg_age: np.ndarray       # [n_age]
    wave: np.ndarray         # [n_wave] rest-frame Angstrom
    lum: np.ndarray          # [n_met, n_age, n_wave] float64 (or [.., n_u, n_wave])
    filt_wave: np.ndarray    # [n_band, n_pts]
    filt_trans: np.ndarray   # [n_band, n_pts]
    t_table: np.ndarray      # [n_t] Gyr
    sfr: np.ndarray          # [n_gal, n_t] M_sun/yr
    z: np.ndarray
    lgmet: np.ndarray
    sigma_z: np.ndarray
    av: np.ndarray
    delta: np.ndarray
    bump: np.ndarray
    lgmet_slope: float = 0.1
    lg_age_pivot: float = 9.0
    lgmet_old: np.ndarray | None = None   # transition MDF: old-age centre per galaxy
    mdf_width: float = 0.5                # transition width in dex
    av_old: np.ndarray | None = None      # age-dependent dust: old-star A_V and delta
    delta_old: np.ndarray | None = None
    dust_pivot: float = 7.0               # its transition centre (log10 yr) and width (dex)
    dust_width: float = 0.25
    lgu_grid: np.ndarray | None = None    # ionization axis of the SSP block [n_u]
    lgu: np.ndarray | None = None         # per-galaxy ionization centre and width
    sigma_u: np.ndarray | None = None
    om0: float = 0.3
    h: float = 0.7
    w0: float = -1.0
    k0_reading: str = "salim"
    sfh_params: np.ndarray | None = None

    @property
    def n_gal(self):
        return int(self.z.shape[0])

    def subset(self, idx):
        idx = np.asarray(idx)
        kw = dict(self.__dict__)
        for name in ("sfr", "z", "lgmet", "sigma_z", "av", "delta", "bump"):
            kw[name] = getattr(self, name)[idx]
        for name in ("lgmet_old", "av_old", "delta_old", "lgu", "sigma_u"):
            if getattr(self, name) is not None:
                kw[name] = getattr(self, name)[idx]
        if self.sfh_params is not None:
            kw["sfh_params"] = self.sfh_params[:, idx]
        return OracleInputs(**kw)


def prepare_inputs(ssp, filters, pop, sfr=None, om0=0.3, h=0.7, w0=-1.0,
                   k0_reading="salim") -> OracleInputs:
    """Collect generator outputs; tabulate the SFR from the parametric history
    when no table is given (the oracle's own step, see oracle.sfh)."""
    if sfr is None:
        sfr = sfh.sfr_from_params(pop.t_table, pop.sfh_params)
    return OracleInputs(
        lgz=np.asarray(ssp.lgz, np.float64), lg_age=np.asarray(ssp.lg_age, np.float64),
        wave=np.asarray(ssp.wave, np.float64), lum=np.asarray(ssp.lum, np.float64),
        filt_wave=np.asarray(filters.wave, np.float64),
        filt_trans=np.asarray(filters.trans, np.float64),
        t_table=np.asarray(pop.t_table, np.float64), sfr=np.asarray(sfr, np.float64),
        z=np.asarray(pop.z, np.float64), lgmet=np.asarray(pop.lgmet, np.float64),
        sigma_z=np.asarray(pop.sigma_z, np.float64), av=np.asarray(pop.av, np.float64),
        delta=np.asarray(pop.delta, np.float64), bump=np.asarray(pop.bump, np.float64),
        lgmet_slope=float(pop.lgmet_slope), lg_age_pivot=float(pop.lg_age_pivot),
        lgmet_old=(None if getattr(pop, "lgmet_old", None) is None
                   else np.asarray(pop.lgmet_old, np.float64)),
        mdf_width=float(getattr(pop, "mdf_width", 0.5)),
        av_old=(None if getattr(pop, "av_old", None) is None else np.asarray(pop.av_old, np.float64)),
        delta_old=(None if getattr(pop, "delta_old", None) is None
                   else np.asarray(pop.delta_old, np.float64)),
        dust_pivot=float(getattr(pop, "dust_pivot", 7.0)),
        dust_width=float(getattr(pop, "dust_width", 0.25)),
        lgu_grid=(None if getattr(ssp, "lgu", None) is None else np.asarray(ssp.lgu, np.float64)),
        lgu=(None if getattr(pop, "lgu", None) is None else np.asarray(pop.lgu, np.float64)),
        sigma_u=(None if getattr(pop, "sigma_u", None) is None
                 else np.asarray(pop.sigma_u, np.float64)),
        om0=om0, h=h, w0=w0, k0_reading=k0_reading,
        sfh_params=np.asarray(pop.sfh_params, np.float64))


def observation_times(inp: OracleInputs):
    return cosmology.age_at_z(inp.z, inp.om0, inp.h, inp.w0)


def weights(inp: OracleInputs, return_parts: bool = False):
    """W[g, j, i] in M_sun: age-bin masses times metallicity weights."""
    t_obs = observation_times(inp)
    m_age = sfh.age_bin_masses(t_obs, inp.t_table, inp.sfr, inp.lg_age)       # [g, i]
    p_met = mdf.mdf_weights(inp.lgmet, inp.sigma_z, inp.lgz, inp.lg_age,
                            inp.lgmet_slope, inp.lg_age_pivot,
                            inp.lgmet_old, inp.mdf_width)                       # [g, j, i]
    w = m_age[:, None, :] * p_met
    if return_parts:
        return w, m_age, p_met, t_obs
    return w


def ionization_weights(inp: OracleInputs):
    """P_neb[g, k] over the SSP block's ionization axis (Eq. nebsed)."""
    if inp.lgu is None or inp.sigma_u is None:
        raise ValueError("the SSP block has an ionization axis: lgu and sigma_u are needed")
    return nebular.ionization_weights(inp.lgu, inp.sigma_u, inp.lgu_grid)


def sed_ion_tangent(inp: OracleInputs, which: str = "lgu", apply_dust: bool = False,
                    block: int = 64):
    """dL/d(lgu) or dL/d(sigma_u) [n_gal, n_wave]: the SED sum of Eq. nebsed
    with the ionization weights replaced by their derivatives (each galaxy's
    SED depends only on its own distribution)."""
    if inp.lgu_grid is None:
        raise ValueError("the SSP block has no ionization axis")
    if apply_dust and inp.av_old is not None:
        raise NotImplementedError("age-dependent attenuation with the ionization tangent")
    out = np.empty((inp.n_gal, inp.lum.shape[-1]))
    for s in range(0, inp.n_gal, block):
        sub = inp.subset(np.arange(s, min(s + block, inp.n_gal)))
        d_u, d_s = nebular.ionization_weight_derivatives(sub.lgu, sub.sigma_u, inp.lgu_grid)
        spec = nebular.sed_nebular(weights(sub), d_u if which == "lgu" else d_s, inp.lum)
        if apply_dust:
            spec = spec * dust.attenuation(inp.wave, sub.av, sub.delta, sub.bump, inp.k0_reading)
        out[s:s + sub.n_gal] = spec
    return out


def sed(inp: OracleInputs, apply_dust: bool = False, block: int = 256):
    """Rest-frame composite SED [n_gal, n_wave] in L_sun/Hz."""
    n_met, n_age = inp.lum.shape[:2]
    n_wave = inp.lum.shape[-1]
    neb = inp.lgu_grid is not None
    table = None if neb else inp.lum.reshape(n_met * n_age, n_wave)
    out = np.empty((inp.n_gal, n_wave))
    if apply_dust and inp.av_old is not None:
        return _sed_age_dependent_dust(inp)
    if neb:
        block = min(block, 64)
    for s in range(0, inp.n_gal, block):
        sub = inp.subset(np.arange(s, min(s + block, inp.n_gal)))
        if neb:
            spec = nebular.sed_nebular(weights(sub), ionization_weights(sub), inp.lum)
        else:
            spec = weights(sub).reshape(sub.n_gal, n_met * n_age) @ table
        if apply_dust:
            spec = spec * dust.attenuation(inp.wave, sub.av, sub.delta, sub.bump, inp.k0_reading)
        out[s:s + sub.n_gal] = spec
    return out


def _sed_age_dependent_dust(inp: OracleInputs, block: int = 8):
    """Eq. agedep_dust_csp: the attenuation moves inside the sum over ages,
    L(lambda) = sum_i F_att(lambda | tau_i) sum_j W[j, i] L_SSP[j, i, lambda],
    with A_V and delta of age i from dust.age_dependent_parameters."""
    out = np.empty((inp.n_gal, inp.lum.shape[2]))
    for s in range(0, inp.n_gal, block):
        sub = inp.subset(np.arange(s, min(s + block, inp.n_gal)))
        w = weights(sub)                                                     # [g, j, i]
        if inp.lgu_grid is not None:
            per_age = np.einsum("gji,gk,jikl->gil", w, ionization_weights(sub), inp.lum)
        else:
            per_age = np.einsum("gji,jil->gil", w, inp.lum)                  # [g, i, l]
        av_i, delta_i = dust.age_dependent_parameters(
            sub.av, sub.delta, sub.av_old, sub.delta_old, inp.lg_age, inp.dust_pivot, inp.dust_width)
        for r in range(sub.n_gal):
            f = dust.attenuation(inp.wave, av_i[r], delta_i[r], np.full(av_i.shape[1], sub.bump[r]),
                                 inp.k0_reading)                             # [i, l]
            out[s + r] = np.sum(f * per_age[r], axis=0)
    return out


def band_sums(inp: OracleInputs, block: int = 256):
    """(num, den) [n_gal, n_band] of Eq. restmag for the dust-attenuated SED."""
    n_band = inp.filt_wave.shape[0]
    num = np.empty((inp.n_gal, n_band))
    den = np.empty((inp.n_gal, n_band))
    for s in range(0, inp.n_gal, block):
        idx = np.arange(s, min(s + block, inp.n_gal))
        spec = sed(inp.subset(idx), apply_dust=True, block=block)
        for r, g in enumerate(idx):
            num[g], den[g] = photometry.band_integrals(inp.wave, spec[r], inp.z[g],
                                                       inp.filt_wave, inp.filt_trans)
    return num, den


def mags(inp: OracleInputs, block: int = 256, return_sums: bool = False):
    """Apparent AB magnitudes [n_gal, n_band]."""
    num, den = band_sums(inp, block)
    dmod = cosmology.distance_modulus(inp.z, inp.om0, inp.h, inp.w0)
    m = photometry.apparent_mag(num, den, dmod, inp.z)
    if return_sums:
        return m, num, den
    return m


def mags_ion_tangent(inp: OracleInputs, which: str = "lgu"):
    """dm/d(lgu) or dm/d(sigma_u) [n_gal, n_band]: m_b = -2.5 log10 num_b +
    terms free of the ionization distribution, and num_b is linear in the
    attenuated SED, so dm_b = -2.5 / ln 10 num_b(dL) / num_b(L) with dL the SED
    tangent of sed_ion_tangent."""
    num, _ = band_sums(inp)
    dspec = sed_ion_tangent(inp, which, apply_dust=True)
    dnum = np.empty_like(num)
    for g in range(inp.n_gal):
        dnum[g], _ = photometry.band_integrals(inp.wave, dspec[g], inp.z[g], inp.filt_wave,
                                               inp.filt_trans)
    return -2.5 / np.log(10.0) * dnum / num


def bf16_row_scales(lum_rows_f32):
    """Smallest power of two >= each row maximum, as float32 [rows]."""
    x = np.asarray(lum_rows_f32, dtype=np.float32)
    row_max = x.max(axis=1).astype(np.float64)
    mant, expo = np.frexp(row_max)           # row_max = mant * 2**expo, mant in [0.5, 1)
    expo = np.where(mant == 0.5, expo - 1, expo)
    return np.ldexp(np.float32(1.0), expo).astype(np.float32)


def quantize_bf16_rne(lum_rows_f32):
    """(bf16 bits [rows, cols] uint16, scale [rows] float32).

    q = bf16_rne(x / s_row); the division by a power of two is exact except
    where it produces a subnormal, which float32 division rounds the same way
    on any IEEE implementation.
    """
    x = np.asarray(lum_rows_f32, dtype=np.float32)
    s = bf16_row_scales(x)
    y = (x / s[:, None]).astype(np.float32)
    bits = y.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((bits >> 16) & 1)
    q = ((bits + bias) >> 16).astype(np.uint16)
    return q, s


def bf16_to_f32(bits):
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32)

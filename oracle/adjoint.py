"""Hand-written reverse-mode gradient of the magnitudes, in float64.

Test infrastructure (see the package docstring).

The paper obtains gradients by differentiating through the SSP weights
(Section 2.1: with the SSP block fixed, dL/dtheta follows from dP/dtheta) and
through the analytic attenuation (Section 3.4).  This module writes the
vector-Jacobian product out by hand, one step per forward step, in reverse
order: magnitudes -> band integrals -> attenuated SED -> (dust parameters,
SED) -> SSP weights -> (metallicity weights -> lgmet, sigma_Z) and (age-bin
masses -> cumulative mass -> tabulated SFR -> parametric SFH).

Every step is checked against central finite differences of the forward
oracle in the CPU tests.  The observation redshift is data and gets no
gradient.
"""

from __future__ import annotations

import numpy as np
from scipy import special

from . import cosmology, dust, mdf, nebular, photometry, sfh
from .constants import (LAMBDA_V_ANGSTROM, R_V_SALIM, SFH_QUENCH_WIDTH_GYR, YR_PER_GYR)
from .kernels import triweight_pdf
from .pipeline import OracleInputs

LN10 = np.log(10.0)


def trapezoid_weights(x):
    """w such that sum(w * y) equals the trapezoid integral of y over x."""
    x = np.asarray(x, dtype=np.float64)
    dx = np.diff(x)
    w = np.zeros_like(x)
    w[:-1] += 0.5 * dx
    w[1:] += 0.5 * dx
    return w


def _sfr_param_vjp(t_table, params, sfr_bar):
    """Pull SFR_bar[n] back to (A, tau, alpha, q, t_q) for one galaxy."""
    a, tau, alpha, q, tq = params
    t = np.asarray(t_table, dtype=np.float64)
    base = a * (t / tau) ** alpha * np.exp(-t / tau)
    v = (t - tq) / SFH_QUENCH_WIDTH_GYR
    quench = 1.0 - q * special.ndtr(v)
    s = base * quench
    d_a = base * quench / a
    d_tau = s * (-alpha / tau + t / tau**2)
    d_alpha = s * np.log(t / tau)
    d_q = -base * special.ndtr(v)
    pdf = np.exp(-0.5 * v * v) / np.sqrt(2.0 * np.pi)
    d_tq = base * q * pdf / SFH_QUENCH_WIDTH_GYR
    return np.array([np.dot(sfr_bar, d) for d in (d_a, d_tau, d_alpha, d_q, d_tq)])


def mags_vjp(inp: OracleInputs, mags_bar):
    """Vector-Jacobian product of the magnitudes.

    Returns a dict with float64 arrays:
      sfr_bar [n_gal, n_t], sfh_params_bar [5, n_gal] (only when
      inp.sfh_params is set), lgmet_bar, sigma_bar, av_bar, delta_bar,
      bump_bar [n_gal], and lgmet_old_bar [n_gal] for the transition MDF
      (d mu_i / d lgmet = 1 - T_i and d mu_i / d lgmet_old = T_i with
      T_i = T_erf((log10 tau_i - pivot) / width)).
    With the ionization axis (Eq. nebsed) each galaxy contracts against its
    own table sum_k P_k L[:, :, k, :], and lgu_bar, sigma_u_bar [n_gal] follow
    from P_bar_k = sum_{j,i} W[j, i] (L[j, i, k, :] . spec_bar) through the
    derivatives of the ionization weights.
    With the age-dependent attenuation (Section 3.4.1, Eq. agedep_dust_csp)
    every age has its own attenuation F_i, so W_bar[j, i] = sum_l G F_i L, with
    G the cotangent of the attenuated SED, and the dust cotangents collect per
    age, split between young- and old-star parameters by 1 - T_i and T_i
    (av_old_bar and delta_old_bar are added).
    """
    if inp.av_old is not None:
        if inp.lgu_grid is not None:
            raise NotImplementedError("age-dependent attenuation with the ionization axis")
        return _mags_vjp_age_dust(inp, mags_bar)
    mags_bar = np.atleast_2d(np.asarray(mags_bar, dtype=np.float64))
    n_gal = inp.n_gal
    n_met, n_age = inp.lum.shape[:2]
    n_wave = inp.lum.shape[-1]
    neb = inp.lgu_grid is not None
    table = None if neb else inp.lum.reshape(n_met * n_age, n_wave)
    n_band = inp.filt_wave.shape[0]
    t_table = np.asarray(inp.t_table, dtype=np.float64)
    n_t = t_table.size
    dt = np.diff(t_table)

    t_obs = cosmology.age_at_z(inp.z, inp.om0, inp.h, inp.w0)
    age_edges_gyr = sfh.age_bin_edges_yr(inp.lg_age) / YR_PER_GYR
    met_edges = mdf.met_bin_edges(inp.lgz)
    lam = np.asarray(inp.wave, dtype=np.float64)
    k0 = dust.k0(lam, inp.k0_reading)
    log_ratio = np.log(lam / LAMBDA_V_ANGSTROM)
    drude_unit = dust.drude_bump(lam, 1.0)

    out = {k: np.zeros(n_gal) for k in ("lgmet_bar", "sigma_bar", "av_bar", "delta_bar", "bump_bar")}
    terf_mdf = inp.lgmet_old is not None
    if terf_mdf:
        out["lgmet_old_bar"] = np.zeros(n_gal)
        t_age = mdf.transition_weight(inp.lg_age, inp.lg_age_pivot, inp.mdf_width)    # [i]
    if neb:
        out["lgu_bar"] = np.zeros(n_gal)
        out["sigma_u_bar"] = np.zeros(n_gal)
        p_neb_all = nebular.ionization_weights(inp.lgu, inp.sigma_u, inp.lgu_grid)      # [g, k]
        dp_u, dp_s = nebular.ionization_weight_derivatives(inp.lgu, inp.sigma_u, inp.lgu_grid)
    out["sfr_bar"] = np.zeros((n_gal, n_t))
    if inp.sfh_params is not None:
        out["sfh_params_bar"] = np.zeros((5, n_gal))

    for g in range(n_gal):
        # ---- forward recomputation for this galaxy ----
        parts = _galaxy_weights(inp, g, t_obs, age_edges_gyr, met_edges)
        w = parts["w"].reshape(-1)
        if neb:
            table = np.einsum("k,jikl->jil", p_neb_all[g], inp.lum).reshape(n_met * n_age, n_wave)
        spec = w @ table                                                             # [l]
        kdust = k0 * np.exp(inp.delta[g] * log_ratio) + inp.bump[g] * drude_unit
        att = 10.0 ** (-0.4 * inp.av[g] / R_V_SALIM * kdust)
        lam_obs = (1.0 + inp.z[g]) * lam
        tw = trapezoid_weights(lam_obs) / lam_obs
        tb = np.stack([photometry.filter_on_grid(lam_obs, inp.filt_wave[b], inp.filt_trans[b])
                       for b in range(n_band)])                                     # [b, l]
        num = tb @ (tw * att * spec)

        # ---- reverse sweep ----
        num_bar = mags_bar[g] * (-2.5 / (LN10 * num))                                # [b]
        g_l = (num_bar @ tb) * tw                                                    # [l]
        spec_bar = g_l * att
        att_bar = g_l * spec
        dlnf_dk = -0.4 * LN10 * inp.av[g] / R_V_SALIM
        out["av_bar"][g] = np.sum(att_bar * att * (-0.4 * LN10 / R_V_SALIM) * kdust)
        out["delta_bar"][g] = np.sum(att_bar * att * dlnf_dk * k0
                                     * np.exp(inp.delta[g] * log_ratio) * log_ratio)
        out["bump_bar"][g] = np.sum(att_bar * att * dlnf_dk * drude_unit)

        w_bar = (table @ spec_bar).reshape(n_met, n_age)                             # [j, i]
        if neb:
            per_point = np.einsum("jikl,l->jik", inp.lum, spec_bar)                  # [j, i, k]
            p_neb_bar = np.einsum("ji,jik->k", w.reshape(n_met, n_age), per_point)
            out["lgu_bar"][g] = np.dot(p_neb_bar, dp_u[g])
            out["sigma_u_bar"][g] = np.dot(p_neb_bar, dp_s[g])
        _pullback_weights(inp, g, w_bar, parts, out)
    return out


def _galaxy_weights(inp: OracleInputs, g, t_obs, age_edges_gyr, met_edges):
    """Forward pieces of galaxy g's weights that the pull-back needs: the
    cumulative mass, the age-edge times, age-bin masses, MDF centres, the
    standardised bin edges u and the weights P, W."""
    t_table = np.asarray(inp.t_table, dtype=np.float64)
    terf_mdf = inp.lgmet_old is not None
    mcum = sfh.cumulative_mass(t_table, inp.sfr[g:g + 1])[0]
    t_edge = t_obs[g] - age_edges_gyr
    m_edge = sfh.mass_formed_at(t_edge, t_table, mcum)
    m_age = m_edge[:-1] - m_edge[1:]
    mu = mdf.mdf_centres(inp.lgmet[g], inp.lg_age, inp.lgmet_slope, inp.lg_age_pivot,
                         None if not terf_mdf else inp.lgmet_old[g:g + 1], inp.mdf_width)[0]
    sig = inp.sigma_z[g]
    with np.errstate(invalid="ignore"):
        u = (met_edges[:, None] - mu[None, :]) / sig                                  # [e, i]
    u = np.where(np.isinf(met_edges)[:, None], np.sign(met_edges)[:, None] * np.inf, u)
    p_met = mdf.mdf_weights(inp.lgmet[g], sig, inp.lgz, inp.lg_age, inp.lgmet_slope,
                            inp.lg_age_pivot, None if not terf_mdf else inp.lgmet_old[g:g + 1],
                            inp.mdf_width)[0]                                         # [j, i]
    return {"t_edge": t_edge, "m_age": m_age, "u": u, "p_met": p_met, "sig": sig,
            "w": m_age[None, :] * p_met}


def _pullback_weights(inp: OracleInputs, g, w_bar, parts, out):
    """W_bar [j, i] of galaxy g -> MDF parameters, age-bin masses, the
    cumulative mass, the SFR table and the parametric history."""
    t_table = np.asarray(inp.t_table, dtype=np.float64)
    n_t = t_table.size
    dt = np.diff(t_table)
    n_met, n_age = w_bar.shape
    m_age, p_met, u, sig, t_edge = (parts["m_age"], parts["p_met"], parts["u"], parts["sig"],
                                    parts["t_edge"])
    m_age_bar = np.sum(w_bar * p_met, axis=0)                                        # [i]
    p_bar = w_bar * m_age[None, :]                                                   # [j, i]
    cdf_bar = np.zeros((n_met + 1, n_age))
    cdf_bar[1:] += p_bar
    cdf_bar[:-1] -= p_bar
    u_bar = cdf_bar * triweight_pdf(np.where(np.isfinite(u), u, 0.0)) * np.isfinite(u)
    u_fin = np.where(np.isfinite(u), u, 0.0)
    mu_bar = np.sum(u_bar, axis=0) * (-1.0 / sig)                                    # [i]
    if inp.lgmet_old is not None:
        t_age = mdf.transition_weight(inp.lg_age, inp.lg_age_pivot, inp.mdf_width)
        out["lgmet_bar"][g] = np.sum(mu_bar * (1.0 - t_age))
        out["lgmet_old_bar"][g] = np.sum(mu_bar * t_age)
    else:
        out["lgmet_bar"][g] = np.sum(mu_bar)
    out["sigma_bar"][g] = np.sum(u_bar * (-u_fin / sig))

    # mass at each age edge -> cumulative nodes -> SFR table
    edge_bar = np.zeros(n_age + 1)
    edge_bar[:-1] += m_age_bar
    edge_bar[1:] -= m_age_bar
    mcum_bar = np.zeros(n_t)
    for e in range(n_age + 1):
        te = t_edge[e]
        if not (te > t_table[0]):
            continue
        if te >= t_table[-1]:
            mcum_bar[-1] += edge_bar[e]
            continue
        n = int(np.searchsorted(t_table, te, side="right") - 1)
        f = (te - t_table[n]) / (t_table[n + 1] - t_table[n])
        mcum_bar[n] += (1.0 - f) * edge_bar[e]
        mcum_bar[n + 1] += f * edge_bar[e]
    suffix = np.cumsum(mcum_bar[::-1])[::-1]                                         # sum_{m>=n}
    sfr_bar = np.zeros(n_t)
    sfr_bar[1:] += 0.5 * YR_PER_GYR * dt * suffix[1:]
    sfr_bar[:-1] += 0.5 * YR_PER_GYR * dt * suffix[1:]
    out["sfr_bar"][g] = sfr_bar
    if inp.sfh_params is not None:
        out["sfh_params_bar"][:, g] = _sfr_param_vjp(t_table, inp.sfh_params[:, g], sfr_bar)


def _mags_vjp_age_dust(inp: OracleInputs, mags_bar):
    """mags_vjp with the age-dependent attenuation: per galaxy, per age i,
    F_i = 10^(-0.4 A_V,i k(lambda | delta_i) / 4.05) with A_V,i, delta_i the
    transition blends of Eq. agedep_dust_csp.  The weights' part of the
    reverse sweep is shared with the age-independent case through W_bar."""
    from .dust import age_dependent_parameters
    mags_bar = np.atleast_2d(np.asarray(mags_bar, dtype=np.float64))
    n_gal = inp.n_gal
    n_band = inp.filt_wave.shape[0]
    n_t = np.asarray(inp.t_table).size
    lam = np.asarray(inp.wave, dtype=np.float64)
    k0 = dust.k0(lam, inp.k0_reading)
    log_ratio = np.log(lam / LAMBDA_V_ANGSTROM)
    drude_unit = dust.drude_bump(lam, 1.0)
    t_obs = cosmology.age_at_z(inp.z, inp.om0, inp.h, inp.w0)
    age_edges_gyr = sfh.age_bin_edges_yr(inp.lg_age) / YR_PER_GYR
    met_edges = mdf.met_bin_edges(inp.lgz)
    t_age = mdf.transition_weight(inp.lg_age, inp.dust_pivot, inp.dust_width)        # [i]
    av_i, delta_i = age_dependent_parameters(inp.av, inp.delta, inp.av_old, inp.delta_old,
                                             inp.lg_age, inp.dust_pivot, inp.dust_width)
    keys = ("lgmet_bar", "sigma_bar", "av_bar", "delta_bar", "bump_bar", "av_old_bar",
            "delta_old_bar")
    out = {k: np.zeros(n_gal) for k in keys}
    if inp.lgmet_old is not None:
        out["lgmet_old_bar"] = np.zeros(n_gal)
    out["sfr_bar"] = np.zeros((n_gal, n_t))
    if inp.sfh_params is not None:
        out["sfh_params_bar"] = np.zeros((5, n_gal))
    c = -0.4 * LN10 / R_V_SALIM
    for g in range(n_gal):
        parts = _galaxy_weights(inp, g, t_obs, age_edges_gyr, met_edges)
        w = parts["w"]                                                                # [j, i]
        per_age = np.einsum("ji,jil->il", w, inp.lum)                                 # [i, l]
        pw = np.exp(delta_i[g][:, None] * log_ratio[None, :])                          # (l/5500)^delta_i
        kd = k0[None, :] * pw + inp.bump[g] * drude_unit[None, :]
        att = 10.0 ** (-0.4 * av_i[g][:, None] / R_V_SALIM * kd)                      # [i, l]
        spec = np.sum(att * per_age, axis=0)
        lam_obs = (1.0 + inp.z[g]) * lam
        tw = trapezoid_weights(lam_obs) / lam_obs
        tb = np.stack([photometry.filter_on_grid(lam_obs, inp.filt_wave[b], inp.filt_trans[b])
                       for b in range(n_band)])
        num = tb @ (tw * spec)
        num_bar = mags_bar[g] * (-2.5 / (LN10 * num))
        g_l = (num_bar @ tb) * tw                                                     # [l]
        w_bar = np.einsum("l,il,jil->ji", g_l, att, inp.lum)
        # d att_i / d A_V,i = att_i c k_i, / d delta_i = att_i c A_V,i k0 pw ln(l/5500),
        # / d bump = att_i c A_V,i D
        base = g_l[None, :] * att * per_age                                           # [i, l]
        m_av = np.sum(base * c * kd, axis=1)                                          # [i]
        m_delta = np.sum(base * c * av_i[g][:, None] * k0[None, :] * pw * log_ratio[None, :],
                         axis=1)
        m_bump = np.sum(base * c * av_i[g][:, None] * drude_unit[None, :], axis=1)
        out["av_bar"][g] = np.sum((1.0 - t_age) * m_av)
        out["av_old_bar"][g] = np.sum(t_age * m_av)
        out["delta_bar"][g] = np.sum((1.0 - t_age) * m_delta)
        out["delta_old_bar"][g] = np.sum(t_age * m_delta)
        out["bump_bar"][g] = np.sum(m_bump)
        _pullback_weights(inp, g, w_bar, parts, out)
    return out

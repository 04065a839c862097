"""torch.autograd.Function over the fused magnitudes and their hand-written
adjoint (dsps_mags / dsps_mags_vjp).  Forward keeps only the per-galaxy band
sums and dust moments (5 x n_band floats; the band sums alone under the
age-dependent attenuation); backward needs no SED."""

from __future__ import annotations

import torch

from . import api


class DspsMags(torch.autograd.Function):
    """mags = DspsMags.apply(ssp, filters, cosmo, t_table, sfh_params, sfr, z,
    lgmet, sigma_z, av, delta, bump, slope, pivot, lgmet_old, mdf_width,
    av_old, delta_old, dust_pivot, dust_width)

    Exactly one of sfh_params [5, n_gal] (float64) and sfr [n_gal, n_t]
    (float64) is a tensor, the other None; lgmet_old (float32) selects the
    transition MDF, or is None; av_old and delta_old (float32, both or
    neither) select the age-dependent attenuation (an SSP block created with
    age_major=True).  Gradients flow to sfh_params or sfr, lgmet, lgmet_old,
    sigma_z, av, delta, bump, av_old and delta_old; z and t_table get none.
    """

    @staticmethod
    def forward(ctx, ssp, filters, cosmo, t_table, sfh_params, sfr, z, lgmet, sigma_z, av, delta,
                bump, slope=0.1, pivot=9.0, lgmet_old=None, mdf_width=0.5, av_old=None,
                delta_old=None, dust_pivot=7.0, dust_width=0.25):
        pop = api.DevicePopulation(t_table.contiguous(),
                                   None if sfr is None else sfr.detach().contiguous(),
                                   None if sfh_params is None else sfh_params.detach().contiguous(),
                                   z.detach().contiguous(), lgmet.detach().contiguous(),
                                   sigma_z.detach().contiguous(), av.detach().contiguous(),
                                   delta.detach().contiguous(), bump.detach().contiguous(),
                                   float(slope), float(pivot),
                                   None if lgmet_old is None else lgmet_old.detach().contiguous(),
                                   float(mdf_width),
                                   None if av_old is None else av_old.detach().contiguous(),
                                   None if delta_old is None else delta_old.detach().contiguous(),
                                   float(dust_pivot), float(dust_width))
        if pop.av_old is None:
            mags, bands, moments = api.mags(ssp, filters, cosmo, pop, precision="fp32",
                                            with_moments=True)
        else:   # per-age attenuation: no moments, the adjoint forms the dust sums itself
            mags, bands = api.mags(ssp, filters, cosmo, pop, precision="fp32", with_bands=True)
            moments = None
        ctx.ssp, ctx.filters, ctx.cosmo, ctx.pop = ssp, filters, cosmo, pop
        ctx.save_for_backward(bands, moments)
        return mags

    @staticmethod
    def backward(ctx, mags_bar):
        bands, moments = ctx.saved_tensors
        pop = ctx.pop
        want = []
        if pop.sfh_params is not None and ctx.needs_input_grad[4]:
            want.append("sfh_params")
        if pop.sfr is not None and ctx.needs_input_grad[5]:
            want.append("sfr")
        names = ["lgmet", "sigma_z", "av", "delta", "bump"]
        for i, k in enumerate(names):
            if ctx.needs_input_grad[7 + i]:
                want.append(k)
        if pop.lgmet_old is not None and ctx.needs_input_grad[14]:
            want.append("lgmet_old")
        if pop.av_old is not None:
            for i, k in ((16, "av_old"), (17, "delta_old")):
                if ctx.needs_input_grad[i]:
                    want.append(k)
        g = api.mags_vjp(ctx.ssp, ctx.filters, ctx.cosmo, pop, mags_bar, bands=bands, moments=moments,
                         want=tuple(want))
        return (None, None, None, None, g.get("sfh_params"), g.get("sfr"), None,
                g.get("lgmet"), g.get("sigma_z"), g.get("av"), g.get("delta"), g.get("bump"),
                None, None, g.get("lgmet_old"), None, g.get("av_old"), g.get("delta_old"), None,
                None)


def dsps_mags(ssp, filters, cosmo, pop: api.DevicePopulation, sfh_params=None, sfr=None,
              lgmet=None, sigma_z=None, av=None, delta=None, bump=None, lgmet_old=None,
              av_old=None, delta_old=None):
    """Differentiable magnitudes; tensors not given are taken from `pop`."""
    return DspsMags.apply(ssp, filters, cosmo, pop.t_table,
                          sfh_params if sfh_params is not None else pop.sfh_params,
                          sfr if sfr is not None else pop.sfr, pop.z,
                          lgmet if lgmet is not None else pop.lgmet,
                          sigma_z if sigma_z is not None else pop.sigma_z,
                          av if av is not None else pop.av, delta if delta is not None else pop.delta,
                          bump if bump is not None else pop.bump, pop.lgmet_slope, pop.lg_age_pivot,
                          lgmet_old if lgmet_old is not None else pop.lgmet_old, pop.mdf_width,
                          av_old if av_old is not None else pop.av_old,
                          delta_old if delta_old is not None else pop.delta_old,
                          pop.dust_pivot, pop.dust_width)


class PopSummary(torch.autograd.Function):
    """hist = PopSummary.apply(mags, spec): the Section 4.1 summary of a
    population's magnitudes, differentiable w.r.t. the magnitudes (chain it
    after dsps_mags for gradients w.r.t. every galaxy's parameters)."""

    @staticmethod
    def forward(ctx, mags, spec):
        ctx.spec = spec
        m = mags.detach().contiguous()
        ctx.save_for_backward(m)
        return api.pop_summary(m, spec)

    @staticmethod
    def backward(ctx, hist_bar):
        (m,) = ctx.saved_tensors
        return api.pop_summary_vjp(m, ctx.spec, hist_bar), None

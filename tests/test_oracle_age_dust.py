"""Pins for the oracle's age-dependent attenuation (Section 3.4.1, Eq.
agedep_dust_csp): A_V and delta move from young-star to old-star values with
the cumulative triweight of log10 age, and the attenuation sits inside the
sum over ages.  Each test checks the oracle against something other than its
own formula: the age-independent model in the limits where every age shares
one set of dust parameters, a brute-force loop on a tiny grid, the hard-step
limit, the midpoint of the transition and the sign of the physical effect.
CPU only."""

import numpy as np
import pytest

import oracle
import synth
from oracle import dust
from synth.ssp import SspTable


def _inputs(ssp, filters, n=6, seed=61, **kw):
    pop = synth.make_population(n, n_t=100, z_range=(0.1, 1.0), seed=seed, age_dust=True, **kw)
    return pop, oracle.prepare_inputs(ssp, filters, pop)


def _age_independent(inp, av, delta):
    kw = dict(inp.__dict__)
    kw.update(av=np.asarray(av, np.float64), delta=np.asarray(delta, np.float64), av_old=None,
              delta_old=None)
    return oracle.OracleInputs(**kw)


def test_equal_young_and_old_is_age_independent(small_ssp, filters6):
    pop, inp = _inputs(small_ssp, filters6)
    inp.av_old, inp.delta_old = inp.av.copy(), inp.delta.copy()
    got = oracle.sed(inp, apply_dust=True)
    ref = oracle.sed(_age_independent(inp, inp.av, inp.delta), apply_dust=True)
    np.testing.assert_allclose(got, ref, rtol=1e-12)


@pytest.mark.parametrize("side", ["old", "young"])
def test_whole_grid_on_one_side_is_age_independent(small_ssp, filters6, side):
    pop, inp = _inputs(small_ssp, filters6)
    # every SSP age more than 3 widths from the centre
    inp.dust_pivot = 0.0 if side == "old" else 20.0
    got = oracle.mags(inp)
    av, delta = (inp.av_old, inp.delta_old) if side == "old" else (inp.av, inp.delta)
    ref = oracle.mags(_age_independent(inp, av, delta))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_hard_step_limit_is_two_group_split(small_ssp, filters6):
    pop, inp = _inputs(small_ssp, filters6, n=3)
    a = small_ssp.lg_age
    inp.dust_pivot = 0.5 * (a[30] + a[31])        # between two grid ages
    inp.dust_width = 1e-9
    got = oracle.sed(inp, apply_dust=True)
    w = oracle.weights(inp)                        # [g, j, i]
    young = np.arange(a.size) <= 30
    for g in range(inp.n_gal):
        s_y = np.einsum("ji,jil->l", w[g][:, young], small_ssp.lum[:, young].astype(np.float64))
        s_o = np.einsum("ji,jil->l", w[g][:, ~young], small_ssp.lum[:, ~young].astype(np.float64))
        f_y = dust.attenuation(small_ssp.wave, inp.av[g], inp.delta[g], inp.bump[g])[0]
        f_o = dust.attenuation(small_ssp.wave, inp.av_old[g], inp.delta_old[g], inp.bump[g])[0]
        np.testing.assert_allclose(got[g], f_y * s_y + f_o * s_o, rtol=1e-12)


def test_centre_of_transition_is_midpoint():
    av_i, d_i = dust.age_dependent_parameters([1.2], [-0.5], [0.4], [0.1],
                                              np.array([6.0, 7.0, 8.0]), 7.0, 0.25)
    assert av_i[0, 0] == 1.2 and d_i[0, 0] == -0.5          # 4 widths below: young
    assert av_i[0, 1] == pytest.approx(0.8, abs=1e-15)      # T_erf(0) = 1/2
    assert d_i[0, 1] == pytest.approx(-0.2, abs=1e-15)
    assert av_i[0, 2] == 0.4 and d_i[0, 2] == 0.1           # 4 widths above: old, exactly


def test_brute_force_tiny_grid():
    rng = np.random.default_rng(3)
    n_met, n_age, n_wave = 3, 7, 40
    lgz = np.linspace(-3.5, -1.5, n_met)
    lg_age = np.linspace(6.0, 9.8, n_age)
    wave = np.geomspace(2000.0, 9000.0, n_wave)
    lum = rng.uniform(0.5, 2.0, (n_met, n_age, n_wave)).astype(np.float32)
    ssp = SspTable(lgz=lgz, lg_age=lg_age, wave=wave, lum=lum)
    flt = synth.make_filters()
    pop = synth.make_population(2, n_t=60, z_range=(0.2, 0.5), seed=9, age_dust=True,
                                dust_pivot=7.2, dust_width=0.6)
    inp = oracle.prepare_inputs(ssp, flt, pop)
    got = oracle.sed(inp, apply_dust=True)
    w = oracle.weights(inp)
    from oracle.kernels import triweight_cdf
    for g in range(2):
        for l in range(n_wave):
            total = 0.0
            for i in range(n_age):
                t = float(triweight_cdf((lg_age[i] - 7.2) / 0.6))
                av = pop.av[g] + (pop.av_old[g] - pop.av[g]) * t
                de = pop.delta[g] + (pop.delta_old[g] - pop.delta[g]) * t
                f = dust.attenuation(wave[l:l + 1], av, de, pop.bump[g])[0, 0]
                for j in range(n_met):
                    total += w[g, j, i] * float(lum[j, i, l]) * f
            assert got[g, l] == pytest.approx(total, rel=1e-12)


def test_more_young_dust_makes_galaxies_fainter(small_ssp, filters6):
    pop, inp = _inputs(small_ssp, filters6, n=4)
    m0 = oracle.mags(inp)
    inp.av = inp.av + 0.5
    m1 = oracle.mags(inp)
    assert np.all(m1 > m0)


def test_adjoint_matches_central_differences(filters6):
    """Every cotangent of the age-dependent model against central differences
    of the FP64 magnitudes, on a grid whose ages straddle the transition."""
    rng = np.random.default_rng(11)
    lgz = np.linspace(-3.5, -1.5, 4)
    lg_age = np.linspace(6.0, 9.8, 12)
    wave = np.geomspace(1500.0, 12000.0, 300)
    lum = rng.uniform(0.5, 2.0, (4, 12, 300)).astype(np.float32)
    ssp = SspTable(lgz=lgz, lg_age=lg_age, wave=wave, lum=lum)
    pop = synth.make_population(3, n_t=70, z_range=(0.1, 0.4), seed=13, age_dust=True,
                                dust_pivot=7.4, dust_width=0.5)
    inp = oracle.prepare_inputs(ssp, filters6, pop)
    m = oracle.mags(inp)
    # targets near the model's own magnitudes keep the loss, and with it the
    # rounding error of the differences, small
    targets = m + rng.normal(0.0, 0.3, m.shape)
    g = oracle.mags_vjp(inp, 2 * (m - targets))

    def loss(mod):
        p2 = oracle.prepare_inputs(ssp, filters6, pop)
        mod(p2)
        p2.sfr = oracle.sfh.sfr_from_params(p2.t_table, p2.sfh_params)
        return np.sum((oracle.mags(p2) - targets) ** 2)

    fields = {"av": "av_bar", "av_old": "av_old_bar", "delta": "delta_bar",
              "delta_old": "delta_old_bar", "bump": "bump_bar", "lgmet": "lgmet_bar",
              "sigma_z": "sigma_bar"}
    for gi in range(pop.n_gal):
        for fld, key in fields.items():
            h = 1e-5
            def shift(p, s):
                arr = getattr(p, fld).copy(); arr[gi] += s * h; setattr(p, fld, arr)
            fd = (loss(lambda p: shift(p, 1)) - loss(lambda p: shift(p, -1))) / (2 * h)
            assert g[key][gi] == pytest.approx(fd, rel=1e-5, abs=1e-7), (fld, gi)
        for k in (0, 2, 4):
            h = 1e-5 * max(1.0, abs(inp.sfh_params[k, gi]))
            def pp(p, s):
                arr = p.sfh_params.copy(); arr[k, gi] += s * h; p.sfh_params = arr
            fd = (loss(lambda p: pp(p, 1)) - loss(lambda p: pp(p, -1))) / (2 * h)
            assert g["sfh_params_bar"][k, gi] == pytest.approx(fd, rel=1e-5, abs=1e-7), (k, gi)


def test_adjoint_equal_young_and_old_splits_the_age_independent_one(small_ssp, filters6):
    """With equal young and old parameters the model is the age-independent
    one: av_bar + av_old_bar and delta_bar + delta_old_bar equal its
    cotangents, and every other cotangent matches."""
    pop, inp = _inputs(small_ssp, filters6, n=4, seed=15)
    inp.av_old, inp.delta_old = inp.av.copy(), inp.delta.copy()
    m = oracle.mags(inp)
    bar = 2 * (m - pop.targets)
    g = oracle.mags_vjp(inp, bar)
    ref = oracle.mags_vjp(_age_independent(inp, inp.av, inp.delta), bar)
    np.testing.assert_allclose(g["av_bar"] + g["av_old_bar"], ref["av_bar"], rtol=1e-9)
    np.testing.assert_allclose(g["delta_bar"] + g["delta_old_bar"], ref["delta_bar"], rtol=1e-9)
    for k in ("bump_bar", "lgmet_bar", "sigma_bar", "sfr_bar", "sfh_params_bar"):
        np.testing.assert_allclose(g[k], ref[k], rtol=1e-9, atol=1e-12 * np.abs(ref[k]).max())

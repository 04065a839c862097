"""Pins for the oracle's nebular ionization axis (Section 3.3, Eq. nebsed) and
the emission-line equivalent width (Section 2.2.2, Eq. eqw).  Each test
checks the oracle against something other than its own formula: the weights
against quadrature of the triweight and their limits, the three-axis SED
against the two-axis path where the axis carries no information and against a
brute-force loop, the equivalent width against lines of known area on
continua the quadratic fit must reproduce.  CPU only."""

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from oracle import kernels, nebular
from synth.ssp import SspTable


# ---------------------------------------------------------------- P_neb
def test_ionization_weights_sum_to_one_and_match_quadrature():
    grid = np.linspace(-4.0, -1.0, 7)
    centre = np.array([-3.3, -2.0, -1.2, -4.6])
    sigma = np.array([0.25, 0.4, 0.1, 0.3])
    p = nebular.ionization_weights(centre, sigma, grid)
    np.testing.assert_allclose(p.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    edges = 0.5 * (grid[:-1] + grid[1:])
    for g in range(centre.size):
        for k in range(1, grid.size - 1):       # interior bins
            lo, hi = edges[k - 1], edges[k]
            clip = [x for x in (centre[g] - 3 * sigma[g], centre[g] + 3 * sigma[g]) if lo < x < hi]
            val, _ = integrate.quad(lambda x: kernels.triweight_pdf((x - centre[g]) / sigma[g])
                                    / sigma[g], lo, hi, epsabs=1e-15, epsrel=1e-14,
                                    points=clip or None, limit=200)
            assert p[g, k] == pytest.approx(val, abs=1e-13)


def test_ionization_weights_narrow_kernel_is_one_hot():
    grid = np.linspace(-4.0, -1.0, 7)
    p = nebular.ionization_weights([-2.45, -3.9, -0.2], [1e-4, 1e-4, 1e-4], grid)
    np.testing.assert_array_equal(p, np.eye(7)[[3, 0, 6]])


def test_ionization_weights_clip_at_three_sigma():
    grid = np.linspace(-4.0, -1.0, 7)                 # bin edges at -3.75, -3.25, ...
    p = nebular.ionization_weights([-2.5], [0.25], grid)
    # support [-3.25, -1.75]: bins 2, 3, 4 only
    assert np.all(p[0, [0, 1, 5, 6]] == 0.0) and np.all(p[0, 2:5] > 0)


# ---------------------------------------------------------------- Eq. nebsed
def _tiny_table(n_u, rng, same_over_u=False):
    lgz = np.linspace(-3.5, -1.5, 3)
    lg_age = np.linspace(6.0, 9.8, 5)
    wave = np.geomspace(2000.0, 9000.0, 30)
    lum = rng.uniform(0.5, 2.0, (3, 5, n_u, 30)).astype(np.float32)
    if same_over_u:
        lum[:] = lum[:, :, :1, :]
    lgu = np.linspace(-3.5, -1.5, n_u) if n_u > 1 else np.array([-2.0])
    return SspTable(lgz=lgz, lg_age=lg_age, wave=wave, lum=lum, lgu=lgu)


def _plain(ssp, k=0):
    return SspTable(lgz=ssp.lgz, lg_age=ssp.lg_age, wave=ssp.wave,
                    lum=np.ascontiguousarray(ssp.lum[:, :, k, :]))


def test_table_constant_over_u_gives_two_axis_sed():
    rng = np.random.default_rng(5)
    ssp = _tiny_table(4, rng, same_over_u=True)
    pop = synth.make_population(6, n_t=60, z_range=(0.2, 0.5), seed=41, nebular=True)
    flt = synth.make_filters()
    got = oracle.sed(oracle.prepare_inputs(ssp, flt, pop), apply_dust=True)
    ref = oracle.sed(oracle.prepare_inputs(_plain(ssp), flt, pop), apply_dust=True)
    np.testing.assert_allclose(got, ref, rtol=1e-13)


def test_single_ionization_point_is_two_axis_path():
    rng = np.random.default_rng(6)
    ssp = _tiny_table(1, rng)
    pop = synth.make_population(5, n_t=60, z_range=(0.2, 0.5), seed=43, nebular=True)
    flt = synth.make_filters()
    got = oracle.mags(oracle.prepare_inputs(ssp, flt, pop))
    ref = oracle.mags(oracle.prepare_inputs(_plain(ssp), flt, pop))
    np.testing.assert_array_equal(got, ref)


def test_narrow_ionization_kernel_selects_one_slab():
    rng = np.random.default_rng(7)
    ssp = _tiny_table(5, rng)
    pop = synth.make_population(4, n_t=60, z_range=(0.2, 0.5), seed=45, nebular=True)
    pop.lgu = ssp.lgu[[0, 2, 4, 1]].copy()
    pop.sigma_u = np.full(4, 1e-4)
    flt = synth.make_filters()
    got = oracle.sed(oracle.prepare_inputs(ssp, flt, pop))
    for g, k in enumerate([0, 2, 4, 1]):
        ref = oracle.sed(oracle.prepare_inputs(_plain(ssp, k), flt, pop.subset([g])))
        np.testing.assert_allclose(got[g], ref[0], rtol=1e-13)


def test_brute_force_tiny_grid():
    rng = np.random.default_rng(8)
    ssp = _tiny_table(4, rng)
    pop = synth.make_population(2, n_t=60, z_range=(0.2, 0.5), seed=47, nebular=True)
    pop.sigma_u = np.array([0.6, 0.3])
    inp = oracle.prepare_inputs(ssp, synth.make_filters(), pop)
    got = oracle.sed(inp)
    w = oracle.weights(inp)
    edges = np.concatenate([[-np.inf], 0.5 * (ssp.lgu[:-1] + ssp.lgu[1:]), [np.inf]])
    for g in range(2):
        pn = [float(kernels.triweight_cdf((edges[k + 1] - pop.lgu[g]) / pop.sigma_u[g])
                    - kernels.triweight_cdf((edges[k] - pop.lgu[g]) / pop.sigma_u[g]))
              for k in range(4)]
        for l in range(ssp.wave.size):
            total = 0.0
            for j in range(3):
                for i in range(5):
                    for k in range(4):
                        total += w[g, j, i] * pn[k] * float(ssp.lum[j, i, k, l])
            assert got[g, l] == pytest.approx(total, rel=1e-12)


def test_higher_ionization_strengthens_oiii_in_the_stand_in():
    """Sign of the paper's Fig. on [OIII]: a larger U_s gives a larger width
    (a property of the synthetic block, checked through the oracle)."""
    ssp = synth.make_ssp_nebular(n_wave=1200, wave_lo=3000.0, wave_hi=8000.0, n_met=4, n_age=20,
                                 lg_age_range=(6.0, 10.0))
    pop = synth.make_population(3, n_t=100, z_range=(0.1, 0.3), seed=49, nebular=True)
    pop.sfh_params[3] = 0.0                            # unquenched: young stars present
    widths = []
    for u in (-3.0, -2.0):
        pop.lgu = np.full(3, u)
        pop.sigma_u = np.full(3, 0.25)
        spec = oracle.sed(oracle.prepare_inputs(ssp, synth.make_filters(), pop))
        widths.append(nebular.equivalent_width(ssp.wave, spec, 5008.24, 40.0, 150.0))
    assert np.all(widths[1] > widths[0]) and np.all(widths[0] > 0)


# ---------------------------------------------------------------- Eq. eqw
def _grid():
    return np.linspace(4800.0, 5200.0, 4001)          # 0.1 Angstrom steps


def test_quadratic_continuum_has_zero_width():
    lam = _grid()
    x = (lam - 5000.0) / 200.0
    spec = np.stack([3.0 + 0.4 * x - 0.7 * x * x, 1e-3 * (2.0 - x + 0.2 * x * x)])
    ew = nebular.equivalent_width(lam, spec, 5000.0, 20.0, 200.0)
    np.testing.assert_allclose(ew, 0.0, atol=1e-11)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_compact_line_on_quadratic_continuum_recovers_its_area(sign):
    # L = Q(lambda) (1 + a T((lambda - c)/s)/s) with the triweight T, which
    # vanishes beyond 3 s: the masked fit sees Q exactly, (L - L0)/L0 is the
    # line term itself, and its integral is a (to the trapezoid error).
    lam = _grid()
    c, s, a = 5003.0, 4.0, 12.0 * sign
    x = (lam - c) / 200.0
    q = 5.0 - 1.2 * x + 0.8 * x * x
    spec = q * (1.0 + a * kernels.triweight_pdf((lam - c) / s) / s)
    ew = nebular.equivalent_width(lam, spec[None], c, 3.0 * s + 0.5, 200.0)
    assert ew[0] == pytest.approx(a, rel=1e-6)


def test_width_is_scale_invariant_and_window_limited():
    lam = _grid()
    c = 5000.0
    spec = 2.0 + 30.0 * np.exp(-0.5 * ((lam - c) / 3.0) ** 2)
    ew1 = nebular.equivalent_width(lam, spec, c, 25.0, 150.0)
    ew2 = nebular.equivalent_width(lam, 7.5 * spec, c, 25.0, 150.0)
    assert ew2[0] == pytest.approx(ew1[0], rel=1e-13)
    # flat continuum: the width of a Gaussian of peak 15 x continuum is
    # 15 sqrt(2 pi) 3 Angstrom
    assert ew1[0] == pytest.approx(15.0 * np.sqrt(2.0 * np.pi) * 3.0, rel=1e-6)


def test_too_few_points_give_nan():
    lam = np.linspace(4990.0, 5010.0, 5)
    ew = nebular.equivalent_width(lam, np.ones((2, 5)), 5000.0, 6.0, 8.0)
    assert np.all(np.isnan(ew))


# ---------------------------------------------------------------- tangents
def test_ionization_weight_derivatives_match_differences_and_sum_to_zero():
    grid = np.linspace(-4.0, -1.0, 7)
    centre = np.array([-3.1, -2.37, -1.6])
    sigma = np.array([0.3, 0.22, 0.45])
    d_u, d_s = nebular.ionization_weight_derivatives(centre, sigma, grid)
    h = 1e-6
    fd_u = (nebular.ionization_weights(centre + h, sigma, grid)
            - nebular.ionization_weights(centre - h, sigma, grid)) / (2 * h)
    fd_s = (nebular.ionization_weights(centre, sigma + h, grid)
            - nebular.ionization_weights(centre, sigma - h, grid)) / (2 * h)
    np.testing.assert_allclose(d_u, fd_u, rtol=0, atol=2e-8)
    np.testing.assert_allclose(d_s, fd_s, rtol=0, atol=2e-8)
    np.testing.assert_allclose(d_u.sum(axis=1), 0.0, atol=1e-14)
    np.testing.assert_allclose(d_s.sum(axis=1), 0.0, atol=1e-14)
    assert np.any(d_u != 0) and np.any(d_s != 0)


@pytest.mark.parametrize("which", ["lgu", "sigma_u"])
def test_sed_tangent_matches_central_difference(which):
    ssp = synth.make_ssp_nebular(n_u=5, lgu_range=(-4.0, -2.0), n_wave=300, wave_lo=3000.0,
                                 wave_hi=8000.0, n_met=4, n_age=12, lg_age_range=(6.0, 10.0))
    pop = synth.make_population(3, n_t=80, z_range=(0.1, 0.3), seed=51, nebular=True)
    flt = synth.make_filters()
    got = oracle.pipeline.sed_ion_tangent(oracle.prepare_inputs(ssp, flt, pop), which,
                                          apply_dust=True)
    h = 1e-5
    vals = getattr(pop, which).copy()
    specs = []
    for sgn in (1.0, -1.0):
        setattr(pop, which, vals + sgn * h)
        specs.append(oracle.sed(oracle.prepare_inputs(ssp, flt, pop), apply_dust=True))
    setattr(pop, which, vals)
    fd = (specs[0] - specs[1]) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 0
    np.testing.assert_allclose(got, fd, rtol=0, atol=1e-6 * scale)


def test_width_tangent_matches_central_difference():
    lam = np.linspace(4800.0, 5200.0, 801)
    spec = synth.make_line_spectra(4, lam, [(5000.0, 30.0)], seed=3).astype(np.float64)
    dspec = synth.make_line_spectra(4, lam, [(5010.0, 20.0)], seed=4).astype(np.float64)
    w, dw = nebular.equivalent_width_jvp(lam, spec, dspec, 5000.0, 30.0, 120.0)
    np.testing.assert_array_equal(w, nebular.equivalent_width(lam, spec, 5000.0, 30.0, 120.0))
    h = 1e-6
    fd = (nebular.equivalent_width(lam, spec + h * dspec, 5000.0, 30.0, 120.0)
          - nebular.equivalent_width(lam, spec - h * dspec, 5000.0, 30.0, 120.0)) / (2 * h)
    np.testing.assert_allclose(dw, fd, rtol=1e-6, atol=1e-8)


def test_oiii_width_gradient_in_u_is_positive_and_matches_differences():
    """The paper's [OIII] example: d W / d log10 U_s > 0 for star-forming
    galaxies, from the SED tangent and the width tangent, against central
    differences of the width."""
    ssp = synth.make_ssp_nebular(n_wave=900, wave_lo=3000.0, wave_hi=8000.0, n_met=4, n_age=20,
                                 lg_age_range=(6.0, 10.0))
    pop = synth.make_population(3, n_t=100, z_range=(0.1, 0.3), seed=53, nebular=True)
    pop.sfh_params[3] = 0.0
    pop.lgu = np.full(3, -2.0)
    pop.sigma_u = np.full(3, 0.25)
    flt = synth.make_filters()
    inp = oracle.prepare_inputs(ssp, flt, pop)
    spec = oracle.sed(inp)
    dspec = oracle.pipeline.sed_ion_tangent(inp, "lgu")
    _, dw = nebular.equivalent_width_jvp(ssp.wave, spec, dspec, 5008.24, 40.0, 150.0)
    h = 1e-5
    ws = []
    for sgn in (1.0, -1.0):
        pop.lgu = np.full(3, -2.0 + sgn * h)
        ws.append(nebular.equivalent_width(ssp.wave, oracle.sed(oracle.prepare_inputs(ssp, flt, pop)),
                                           5008.24, 40.0, 150.0))
    np.testing.assert_allclose(dw, (ws[0] - ws[1]) / (2 * h), rtol=1e-5)
    assert np.all(dw > 0)


@pytest.mark.parametrize("which", ["lgu", "sigma_u"])
def test_magnitude_tangent_matches_central_difference(which):
    ssp = synth.make_ssp_nebular(n_u=5, lgu_range=(-4.0, -2.0), n_wave=400, wave_lo=1500.0,
                                 wave_hi=12000.0, n_met=4, n_age=12, lg_age_range=(6.0, 10.0))
    pop = synth.make_population(3, n_t=80, z_range=(0.1, 0.3), seed=55, nebular=True)
    flt = synth.make_filters()
    got = oracle.pipeline.mags_ion_tangent(oracle.prepare_inputs(ssp, flt, pop), which)
    h = 1e-5
    vals = getattr(pop, which).copy()
    ms = []
    for sgn in (1.0, -1.0):
        setattr(pop, which, vals + sgn * h)
        ms.append(oracle.mags(oracle.prepare_inputs(ssp, flt, pop)))
    setattr(pop, which, vals)
    fd = (ms[0] - ms[1]) / (2 * h)
    np.testing.assert_allclose(got, fd, rtol=1e-5, atol=1e-9 * np.abs(fd).max())
    assert np.abs(fd).max() > 0


# ---------------------------------------------------------------- adjoint
def test_adjoint_over_the_ionization_axis_matches_central_differences():
    ssp = synth.make_ssp_nebular(n_u=5, lgu_range=(-4.0, -2.0), n_wave=400, wave_lo=1500.0,
                                 wave_hi=12000.0, n_met=5, n_age=14, lg_age_range=(6.0, 10.0))
    flt = synth.make_filters()
    pop = synth.make_population(3, n_t=80, z_range=(0.1, 0.5), seed=57, nebular=True)
    inp = oracle.prepare_inputs(ssp, flt, pop)
    m = oracle.mags(inp)
    g = oracle.mags_vjp(inp, 2 * (m - pop.targets))

    def loss(mod):
        p2 = oracle.prepare_inputs(ssp, flt, pop)
        mod(p2)
        p2.sfr = oracle.sfh.sfr_from_params(p2.t_table, p2.sfh_params)
        return np.sum((oracle.mags(p2) - pop.targets) ** 2)

    fields = {"lgu": "lgu_bar", "sigma_u": "sigma_u_bar", "lgmet": "lgmet_bar",
              "sigma_z": "sigma_bar", "av": "av_bar", "delta": "delta_bar", "bump": "bump_bar"}
    for gi in range(pop.n_gal):
        for fld, key in fields.items():
            h = 1e-5
            def shift(p, s):
                arr = getattr(p, fld).copy(); arr[gi] += s * h; setattr(p, fld, arr)
            fd = (loss(lambda p: shift(p, 1)) - loss(lambda p: shift(p, -1))) / (2 * h)
            assert g[key][gi] == pytest.approx(fd, rel=1e-5, abs=1e-7), (fld, gi)
        k = 2                                              # alpha of the parametric history
        h = 1e-5 * max(1.0, abs(inp.sfh_params[k, gi]))
        def pp(p, s):
            arr = p.sfh_params.copy(); arr[k, gi] += s * h; p.sfh_params = arr
        fd = (loss(lambda p: pp(p, 1)) - loss(lambda p: pp(p, -1))) / (2 * h)
        assert g["sfh_params_bar"][k, gi] == pytest.approx(fd, rel=1e-5, abs=1e-7)

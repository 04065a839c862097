"""Pins for the oracle's transition model of the age-dependent MDF (Section
3.2.2, Eq. agedep_mdf, with the cumulative triweight of Appendix B, Eq.
terf): mu_i = lgmet + (lgmet_old - lgmet) T_erf((log10 tau_i - pivot) /
width).  Each test checks the oracle against something other than its own
formula: the uncorrelated special case, exact asymptotes, the midpoint,
quadrature of the triweight density written out here, and finite
differences of the magnitudes.  CPU only."""

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from oracle import mdf


def _density(u):
    """Triweight density per unit u, typed from Eq. triweight."""
    return 35.0 / 96.0 * (1.0 - (u / 3.0) ** 2) ** 3 if abs(u) <= 3.0 else 0.0


def test_equal_centres_reduce_to_uncorrelated_mdf(small_ssp):
    p_t = mdf.mdf_weights([-2.3], [0.25], small_ssp.lgz, small_ssp.lg_age, 0.1, 9.0,
                          lgmet_old=[-2.3], width=0.4)[0]
    p_u = mdf.mdf_weights([-2.3], [0.25], small_ssp.lgz, small_ssp.lg_age, 0.0, 9.0)[0]
    np.testing.assert_array_equal(p_t, p_u)


def test_asymptotes_are_exact_and_centre_is_midpoint():
    lg_age = np.array([6.0, 8.0, 8.15, 9.0, 9.85, 10.0, 10.2])
    width = 0.3                                   # support 9 +- 0.9 dex
    mu = mdf.mdf_centres([-2.0], lg_age, 0.1, 9.0, lgmet_old=[-2.5], width=width)[0]
    assert mu[0] == -2.0 and mu[1] == -2.0        # young asymptote below 8.1
    assert mu[5] == -2.5 and mu[6] == -2.5        # old asymptote above 9.9
    assert mu[3] == pytest.approx(-2.25, abs=1e-15)   # T_erf(0) = 1/2
    assert mu[0] >= mu[2] >= mu[3] >= mu[4] >= mu[5]  # monotone in between
    assert -2.5 < mu[4] < mu[2] < -2.0


def test_interior_transition_equals_density_quadrature():
    lg_age = np.linspace(8.3, 9.7, 9)
    width = 0.35
    mu = mdf.mdf_centres([-1.9], lg_age, 0.1, 9.0, lgmet_old=[-2.6], width=width)[0]
    for a, m in zip(lg_age, mu):
        z = (a - 9.0) / width
        t, _ = integrate.quad(_density, -3.0, min(z, 3.0), epsabs=1e-15, epsrel=1e-13)
        assert m == pytest.approx(-1.9 + (-2.6 + 1.9) * t, abs=1e-13)


def test_weights_sum_to_one_under_transition(small_ssp):
    pop = synth.make_population(32, seed=5, mdf="transition", mdf_width=0.4)
    p = mdf.mdf_weights(pop.lgmet, pop.sigma_z, small_ssp.lgz, small_ssp.lg_age, 0.1, 9.0,
                        lgmet_old=pop.lgmet_old, width=pop.mdf_width)
    assert np.all(p >= 0)
    np.testing.assert_allclose(p.sum(axis=1), 1.0, atol=1e-14)


def test_common_shift_gradient_equals_uncorrelated_gradient(small_ssp, filters6):
    # With lgmet_old = lgmet the weights are the uncorrelated model's, and a
    # shift of both centres is a shift of the uncorrelated centre.
    pop = synth.make_population(3, seed=51, z_range=(0.2, 0.9), mdf="transition")
    pop.lgmet_old = pop.lgmet.copy()
    inp = oracle.prepare_inputs(small_ssp, filters6, pop)
    m = oracle.mags(inp)
    g = oracle.mags_vjp(inp, 2 * (m - pop.targets))
    pop_u = synth.make_population(3, seed=51, z_range=(0.2, 0.9), lgmet_slope=0.0)
    inp_u = oracle.prepare_inputs(small_ssp, filters6, pop_u)
    m_u = oracle.mags(inp_u)
    np.testing.assert_array_equal(m, m_u)
    g_u = oracle.mags_vjp(inp_u, 2 * (m_u - pop_u.targets))
    np.testing.assert_allclose(g["lgmet_bar"] + g["lgmet_old_bar"], g_u["lgmet_bar"],
                               rtol=1e-12, atol=1e-12)


def test_transition_gradients_match_central_differences(small_ssp, filters6):
    pop = synth.make_population(4, seed=53, z_range=(0.1, 1.0), mdf="transition", mdf_width=0.4)
    inp = oracle.prepare_inputs(small_ssp, filters6, pop)
    m = oracle.mags(inp)
    g = oracle.mags_vjp(inp, 2 * (m - pop.targets))

    def loss_at(field, gi, step):
        p2 = oracle.prepare_inputs(small_ssp, filters6, pop)
        arr = getattr(p2, field).copy()
        arr[gi] += step
        setattr(p2, field, arr)
        return np.sum((oracle.mags(p2) - pop.targets) ** 2)

    h = 1e-4
    for gi in range(pop.n_gal):
        for field, key in (("lgmet", "lgmet_bar"), ("lgmet_old", "lgmet_old_bar"),
                           ("sigma_z", "sigma_bar")):
            fd = (loss_at(field, gi, h) - loss_at(field, gi, -h)) / (2 * h)
            assert g[key][gi] == pytest.approx(fd, rel=1e-5, abs=1e-6), (field, gi)

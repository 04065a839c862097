"""Pins for the oracle's primitives: triweight kernel (Appendix B), cosmology
(Section 2.2.1), attenuation curve (Section 3.4) and constants printed in the
paper (tests/golden/paper_constants.json).  CPU only."""

import json
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import constants, cosmology, dust, kernels

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- constants
def test_printed_constants_match_golden():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        gold = json.load(f)["constants"]
    assert constants.AB0_LSUN_PER_HZ == gold["AB0_Lsun_per_Hz"]["value"]
    assert constants.LAMBDA_V_ANGSTROM == gold["lambda_V_Angstrom"]["value"]
    assert constants.R_V_SALIM == gold["attenuation_normalisation"]["value"]
    assert constants.K0_SWITCH_MICRON == gold["k0_switch_micron"]["value"]
    assert constants.DRUDE_WIDTH_ANGSTROM == gold["drude_width_Angstrom"]["value"]
    assert constants.DRUDE_CENTRE_ANGSTROM == gold["drude_centre_Angstrom"]["value"]
    tw = gold["triweight_coefficient"]["value"]
    assert kernels.triweight_pdf(0.0) == pytest.approx(tw[0] / tw[1], rel=1e-15)
    coeffs = gold["terf_polynomial"]["value"]            # [c0, c1, c3, c5, c7] as [num, den]
    z = np.linspace(-3, 3, 13)
    poly = sum((n / d) * z**p for (n, d), p in zip(coeffs, [0, 1, 3, 5, 7]))
    np.testing.assert_allclose(kernels.triweight_cdf_poly(z), poly, rtol=0, atol=1e-15)


def test_ab_zero_point_is_3631_jansky_at_10pc():
    # 3631 Jy * 4 pi (10 pc)^2 / L_sun, with IAU nominal L_sun = 3.828e26 W.
    jy = 1e-26
    pc = 3.0856775814913673e16
    lsun = 3.828e26
    ab0 = 3631 * jy * 4 * np.pi * (10 * pc) ** 2 / lsun
    assert ab0 == pytest.approx(constants.AB0_LSUN_PER_HZ, rel=2e-4)


# ---------------------------------------------------------------- triweight
def test_triweight_unit_mass_and_variance():
    mass, _ = integrate.quad(kernels.triweight_pdf, -3, 3, epsabs=1e-14)
    var, _ = integrate.quad(lambda z: z * z * kernels.triweight_pdf(z), -3, 3, epsabs=1e-14)
    mean, _ = integrate.quad(lambda z: z * kernels.triweight_pdf(z), -3, 3, epsabs=1e-14)
    assert mass == pytest.approx(1.0, abs=1e-13)
    assert var == pytest.approx(1.0, abs=1e-13)
    assert mean == pytest.approx(0.0, abs=1e-14)
    assert kernels.triweight_pdf(3.0001) == 0.0 and kernels.triweight_pdf(-5) == 0.0


def test_triweight_cdf_closed_values():
    # p(z) is the integral of T from -3: check exact rational values.
    assert kernels.triweight_cdf(-3.0) == pytest.approx(0.0, abs=1e-15)
    assert kernels.triweight_cdf(3.0) == pytest.approx(1.0, abs=1e-15)
    assert kernels.triweight_cdf(0.0) == 0.5
    assert kernels.triweight_cdf(1.0) == pytest.approx(57856.0 / 69984.0, abs=1e-15)
    assert kernels.triweight_cdf(-1.0) == pytest.approx(1 - 57856.0 / 69984.0, abs=1e-15)
    # Reading: 0 below -3 and 1 above +3 (the printed "0 otherwise" is only
    # right on the left).
    assert kernels.triweight_cdf(-7.0) == 0.0
    assert kernels.triweight_cdf(7.0) == 1.0
    assert kernels.triweight_cdf(np.inf) == 1.0 and kernels.triweight_cdf(-np.inf) == 0.0


def test_triweight_cdf_is_integral_of_pdf():
    for z in np.linspace(-3.5, 3.5, 29):
        val, _ = integrate.quad(kernels.triweight_pdf, -3.0, min(z, 3.0), epsabs=1e-14) if z > -3 else (0.0, 0)
        assert kernels.triweight_cdf(z) == pytest.approx(val, abs=1e-13)
    z = np.linspace(-2.9, 2.9, 57)
    h = 1e-5
    deriv = (kernels.triweight_cdf(z + h) - kernels.triweight_cdf(z - h)) / (2 * h)
    np.testing.assert_allclose(deriv, kernels.triweight_pdf(z), atol=1e-9)


# ---------------------------------------------------------------- cosmology
def test_age_closed_form_equals_defining_integral():
    zs = np.array([0.0, 0.1, 0.5, 1.0, 2.0, 3.0, 6.0])
    np.testing.assert_allclose(cosmology.age_at_z(zs), cosmology.age_at_z_quadrature(zs), rtol=1e-11)


def test_einstein_de_sitter_limits():
    # Om0 = 1: t = 2/(3 H0) (1+z)^-1.5 and d_L = 2 (c/H0) (1+z) (1 - (1+z)^-0.5).
    h = 0.7
    zs = np.array([0.1, 0.5, 1.0, 3.0])
    th = constants.HUBBLE_TIME_GYR_KMS_MPC / (100 * h)
    t_eds = cosmology.age_at_z_quadrature(zs, om0=1.0, h=h)
    np.testing.assert_allclose(t_eds, 2.0 / 3.0 * th * (1 + zs) ** -1.5, rtol=1e-11)
    dh = constants.C_KM_S / (100 * h)
    dl = cosmology.luminosity_distance_mpc(zs, om0=1.0, h=h)
    np.testing.assert_allclose(dl, 2 * dh * (1 + zs) * (1 - (1 + zs) ** -0.5), rtol=1e-11)


def test_empty_universe_limit():
    # Om0 = 0 with w = -1: E(z) = 1, d_L = (c/H0) z (1+z).
    zs = np.array([0.1, 1.0, 3.0])
    dh = constants.C_KM_S / 70.0
    np.testing.assert_allclose(cosmology.luminosity_distance_mpc(zs, om0=0.0, h=0.7),
                               dh * zs * (1 + zs), rtol=1e-12)


def test_standard_lcdm_values():
    # Flat LCDM, H0 = 70, Om0 = 0.3, no radiation: widely tabulated values.
    assert cosmology.age_at_z(0.0) == pytest.approx(13.4670, abs=2e-4)
    np.testing.assert_allclose(cosmology.distance_modulus([0.1, 1.0]), [38.3152, 44.1002], atol=2e-4)


def test_wcdm_reduces_to_lcdm_at_w_minus_one():
    zs = np.array([0.3, 1.7])
    np.testing.assert_allclose(cosmology.age_at_z(zs, w0=-1.0 + 1e-12),
                               cosmology.age_at_z(zs), rtol=1e-9)


def test_wcdm_w_minus_third_comoving_distance_closed_form():
    # Flat wCDM with w = -1/3: E^2 = Om x^3 + (1 - Om) x^2 with x = 1 + z, so
    # int dz / E = int dx / (x sqrt(Om x + b)), b = 1 - Om, which integrates to
    # (1/sqrt b) ln[(sqrt(Om x + b) - sqrt b) / (sqrt(Om x + b) + sqrt b)].
    om0, h = 0.27, 0.68
    b = 1.0 - om0
    prim = lambda x: np.log((np.sqrt(om0 * x + b) - np.sqrt(b))
                            / (np.sqrt(om0 * x + b) + np.sqrt(b))) / np.sqrt(b)
    zs = np.array([0.05, 0.6, 2.4])
    dc = constants.C_KM_S / (100.0 * h) * (prim(1.0 + zs) - prim(1.0))
    np.testing.assert_allclose(cosmology.comoving_distance_mpc(zs, om0=om0, h=h, w0=-1.0 / 3.0),
                               dc, rtol=1e-11)


# ---------------------------------------------------------------- dust
def test_calzetti_normalisation_at_v():
    # A_V / E(B-V) = R_V: k(lambda_V) equals R_V = 4.05 to the precision of
    # the published fit.
    assert dust.k_calzetti00(0.55) == pytest.approx(4.05, rel=2e-3)
    assert dust.k0(5500.0) == pytest.approx(4.05, rel=2e-3)


def test_k0_branches_meet_at_switch():
    # The two curves agree to 0.3% at 0.15 micron, which is why the
    # parameterisation switches there.
    assert dust.k_leitherer02(0.15) == pytest.approx(dust.k_calzetti00(0.15), rel=3e-3)
    lam = np.array([1000.0, 1400.0, 1600.0, 3000.0])
    k_s = dust.k0(lam, "salim")
    k_p = dust.k0(lam, "printed")
    assert k_s[0] == dust.k_leitherer02(0.1) and k_p[0] == dust.k_calzetti00(0.1)
    assert k_s[3] == dust.k_calzetti00(0.3) and k_p[3] == dust.k_leitherer02(0.3)


def _calzetti_golden():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "calzetti2000_k.json")
    with open(path) as f:
        return json.load(f)


def test_calzetti_near_infrared_branch_published_values():
    # Calzetti et al. (2000) Eq. 4, near-infrared branch (0.63-2.2 micron):
    # hand-evaluated values of the published curve from the seam to the K
    # band.  A changed digit in either coefficient of the branch, or in its
    # 2.659 factor, moves the K-band value by > 1%.
    g = _calzetti_golden()["near_infrared"]
    lam = np.array(g["lambda_micron"])
    np.testing.assert_allclose(dust.k_calzetti00(lam), g["k"], rtol=2e-6)
    # the baseline curve of Eq. kzero takes this branch at and above 0.63 micron
    np.testing.assert_allclose(dust.k0(lam * 1.0e4), g["k"], rtol=2e-6)
    # linear in 1/lambda: equal steps in 1/lambda give equal steps in k
    k = dust.k_calzetti00(np.array([0.7, 1.0, 1.75]))     # 1/lambda = 10/7, 1, 4/7
    assert k[0] - k[1] == pytest.approx(k[1] - k[2], rel=1e-12)


def test_calzetti_branches_meet_at_063_micron():
    # The published curve switches branch at 0.63 micron; the two branches
    # are not continuous there but agree to 0.72% (3.4766 vs 3.5017).
    g = _calzetti_golden()
    uv = dust.k_calzetti00(0.63 - 1e-12)
    ir = dust.k_calzetti00(0.63)
    assert uv == pytest.approx(g["ultraviolet_optical_at_0.63"], rel=2e-6)
    assert ir == pytest.approx(g["near_infrared"]["k"][0], rel=2e-6)
    assert abs(ir / uv - 1.0) < 1e-2
    # the curve stays positive over the whole branch (A_V > 0 always dims)
    lam = np.linspace(0.63, 2.5, 200)
    assert np.all(dust.k_calzetti00(lam) > 0.0)
    assert np.all(np.diff(dust.k_calzetti00(lam)) < 0.0)


def test_attenuation_identity_and_v_band():
    lam = np.geomspace(900, 25000, 50)
    f0 = dust.attenuation(lam, [0.0, 0.0], [-0.3, 0.2], [1.0, 2.0])
    assert np.all(f0 == 1.0)
    # At lambda_V with no bump, A = A_V k0(V)/4.05.
    f = dust.attenuation(np.array([5500.0]), [1.3], [-0.4], [0.0])
    assert -2.5 * np.log10(f[0, 0]) == pytest.approx(1.3 * dust.k0(5500.0) / 4.05, rel=1e-14)


def test_drude_peak_and_half_width():
    eb = 2.3
    assert dust.drude_bump(2175.0, eb) == pytest.approx(eb, rel=1e-15)
    dl = 350.0
    # D = E_b / 2 where |lambda^2 - lambda_b^2| = lambda * dl.
    lam_hi = (dl + np.sqrt(dl**2 + 4 * 2175.0**2)) / 2
    lam_lo = (-dl + np.sqrt(dl**2 + 4 * 2175.0**2)) / 2
    assert dust.drude_bump(lam_hi, eb) == pytest.approx(eb / 2, rel=1e-13)
    assert dust.drude_bump(lam_lo, eb) == pytest.approx(eb / 2, rel=1e-13)
    # The paper's tie E_b = -1.9 delta + 0.85 is the special case bump = E_b.
    delta = -0.25
    assert dust.drude_bump(2175.0, -1.9 * delta + 0.85) == pytest.approx(1.325)


def test_smaller_delta_attenuates_blue_more():
    lam = np.array([2000.0, 5500.0, 9000.0])
    f = dust.attenuation(lam, [1.0, 1.0], [-0.6, 0.2], [0.0, 0.0])
    assert f[0, 0] < f[1, 0]          # more UV attenuation for smaller delta
    assert f[0, 2] > f[1, 2]          # less near-IR attenuation
    assert f[0, 1] == pytest.approx(f[1, 1])

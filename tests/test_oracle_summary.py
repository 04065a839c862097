"""Pins of the oracle's population summary (Section 4.1 colour cut and
magnitude histogram, triweight-smoothed per Appendix B) and its gradient."""

import numpy as np
import pytest

from oracle import summary
from oracle.kernels import triweight_cdf
import synth

A, B, M = 1, 2, 2          # colour g - r, histogram of r
CUT = 0.55


def test_hard_cut_and_histogram_equal_numpy():
    mags = synth.make_mags(5000, seed=3).astype(np.float64)
    edges = np.linspace(-24.0, -16.0, 33)
    # a galaxy exactly on an interior edge and one on the last edge
    mags[0, M] = edges[7]
    mags[1, M] = edges[-1]
    mags[0, A] = mags[0, B] + 1.0
    mags[1, A] = mags[1, B] + 1.0
    h = summary.histogram(mags, A, B, CUT, 0.0, M, edges, 0.0)
    red = (mags[:, A] - mags[:, B]) > CUT
    ref, _ = np.histogram(mags[red, M], bins=edges)
    np.testing.assert_array_equal(h, ref.astype(np.float64))


def test_smooth_tends_to_hard_away_from_edges():
    mags = synth.make_mags(3000, seed=4).astype(np.float64)
    edges = np.linspace(-24.0, -16.0, 17)
    eps = 1e-7
    c = mags[:, A] - mags[:, B]
    dist_edge = np.min(np.abs(mags[:, M][:, None] - edges[None, :]), axis=1)
    keep = (np.abs(c - CUT) > 3 * eps) & (dist_edge > 3 * eps)
    mags = mags[keep]
    hs = summary.histogram(mags, A, B, CUT, eps, M, edges, eps)
    hh = summary.histogram(mags, A, B, CUT, 0.0, M, edges, 0.0)
    np.testing.assert_array_equal(hs, hh)


def test_smoothed_mass_is_conserved_inside_the_range():
    mags = synth.make_mags(2000, seed=5).astype(np.float64)
    s_m = 0.2
    edges = np.linspace(mags[:, M].min() - 4 * s_m, mags[:, M].max() + 4 * s_m, 25)
    h = summary.histogram(mags, A, B, CUT, 0.08, M, edges, s_m)
    w = summary.colour_weight(mags[:, A] - mags[:, B], CUT, 0.08)
    assert h.sum() == pytest.approx(w.sum(), rel=1e-12)
    assert np.all(h >= -1e-15)


def test_colour_weight_limits_and_midpoint():
    s = 0.1
    c = np.array([CUT, CUT + 3 * s, CUT + 5 * s, CUT - 3 * s, CUT - 7 * s, CUT + s])
    w = summary.colour_weight(c, CUT, s)
    assert w[0] == 0.5
    assert w[1] == 1.0 and w[2] == 1.0 and w[3] == 0.0 and w[4] == 0.0
    assert w[5] == pytest.approx(float(triweight_cdf(1.0)), rel=1e-14)
    cc = np.linspace(CUT - 0.5, CUT + 0.5, 101)
    assert np.all(np.diff(summary.colour_weight(cc, CUT, s)) >= 0.0)


def test_single_galaxy_brute_force():
    edges = np.array([-22.0, -21.0, -20.0, -19.0])
    s_m = 0.1                    # 3 s_m < half a bin
    g = np.zeros((3, 6))
    g[:, A] = 1.0                # colour 1.0 - 0 well above the cut
    g[0, M] = -20.5              # centre of bin 1
    g[1, M] = -21.0              # on the edge between bins 0 and 1
    g[2, M] = -25.0              # far outside
    h = summary.histogram(g, A, B, CUT, 0.05, M, edges, s_m)
    np.testing.assert_allclose(h, [0.5, 1.5, 0.0], atol=1e-15)


def test_non_finite_magnitudes_contribute_nothing():
    mags = synth.make_mags(100, seed=6).astype(np.float64)
    edges = np.linspace(-24.0, -16.0, 9)
    h0 = summary.histogram(mags[10:], A, B, CUT, 0.1, M, edges, 0.3)
    bad = mags.copy()
    bad[:5, A] = np.nan
    bad[5:10, M] = np.inf
    h1 = summary.histogram(bad, A, B, CUT, 0.1, M, edges, 0.3)
    np.testing.assert_allclose(h1, h0, rtol=1e-15)
    g = summary.histogram_vjp(bad, A, B, CUT, 0.1, M, edges, 0.3, np.ones(8))
    assert np.all(g[:10] == 0.0)


def test_vjp_matches_central_differences():
    rng = np.random.default_rng(11)
    mags = synth.make_mags(40, seed=8).astype(np.float64)
    edges = np.linspace(-23.5, -16.5, 15)
    args = (A, B, CUT, 0.15, M, edges, 0.4)
    hb = rng.normal(size=14)
    g = summary.histogram_vjp(mags, *args, hb)
    h = 1e-6
    fd = np.zeros_like(mags)
    for i in range(mags.shape[0]):
        for b in range(mags.shape[1]):
            p, q = mags.copy(), mags.copy()
            p[i, b] += h
            q[i, b] -= h
            fd[i, b] = (hb @ summary.histogram(p, *args) - hb @ summary.histogram(q, *args)) / (2 * h)
    np.testing.assert_allclose(g, fd, atol=1e-7 * np.abs(fd).max())
    assert np.all(g[:, [0, 3, 4, 5]] == 0.0)


def test_vjp_zero_for_hard_summary():
    mags = synth.make_mags(20, seed=9).astype(np.float64)
    g = summary.histogram_vjp(mags, A, B, CUT, 0.0, M, np.linspace(-24, -16, 5), 0.0, np.ones(4))
    assert np.all(g == 0.0)

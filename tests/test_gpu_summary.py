"""GPU parity of the Section 4.1 population summary (dsps_pop_summary and its
adjoint) against the FP64 oracle, on seeded synthetic magnitudes and end to
end at z = 0 (magnitudes -> summary -> gradients of every galaxy's
parameters through both adjoints)."""

import sys

import numpy as np
import pytest

import oracle
from oracle import summary as osum
import synth
from gpu_common import FP32_TOL_MAG, filters6, oracle_inputs, ssp_small

pytestmark = pytest.mark.gpu

A, B, M = 1, 2, 2
CUT = 0.55


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_06830_amd as P
    return P


def _spec(dev, edges, cw, mw, band_a=A, band_b=B, band_m=M):
    import torch
    return dev.SummarySpec(band_a=band_a, band_b=band_b, colour_cut=CUT, colour_width=cw,
                           band_m=band_m, edges=torch.tensor(edges, dtype=torch.float64, device="cuda"),
                           mag_width=mw)


@pytest.mark.parametrize("n_gal,cw,mw", [(4100, 0.0, 0.0), (4100, 0.06, 0.15), (9000, 0.02, 0.4),
                                         (1, 0.05, 0.1)])
def test_summary_matches_oracle(dev, n_gal, cw, mw):
    import torch
    mags = synth.make_mags(n_gal, seed=n_gal)
    edges = np.linspace(-23.5, -16.5, 29)
    if n_gal > 10:
        mags[3, M] = edges[5]            # on an interior edge
        mags[4, M] = edges[-1]           # on the last edge
    _say(f"summary n_gal={n_gal} widths=({cw}, {mw})")
    h = dev.pop_summary(torch.tensor(mags, device="cuda"), _spec(dev, edges, cw, mw)).cpu().numpy()
    ref = osum.histogram(mags, A, B, CUT, cw, M, edges, mw)
    if cw == 0.0 and mw == 0.0:
        np.testing.assert_array_equal(h, ref)
    else:
        np.testing.assert_allclose(h, ref, rtol=1e-12, atol=1e-12 * max(ref.max(), 1.0))


@pytest.mark.parametrize("band_m", [M, 3])
def test_summary_vjp_matches_oracle(dev, band_m):
    import torch
    mags = synth.make_mags(5000, seed=12)
    edges = np.linspace(-24.0, -16.0, 33)
    hb = np.random.default_rng(3).normal(size=32)
    _say(f"summary vjp band_m={band_m}")
    spec = _spec(dev, edges, 0.05, 0.2, band_m=band_m)
    g = dev.pop_summary_vjp(torch.tensor(mags, device="cuda"), spec, torch.tensor(hb)).cpu().numpy()
    ref = osum.histogram_vjp(mags, A, B, CUT, 0.05, band_m, edges, 0.2, hb)
    np.testing.assert_allclose(g, ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())
    assert np.all(g[:, [0, 4, 5]] == 0.0)


def test_summary_edge_cases_and_determinism(dev):
    import torch
    edges = np.linspace(-24.0, -16.0, 9)
    spec = _spec(dev, edges, 0.05, 0.2)
    _say("summary edge cases")
    empty = dev.pop_summary(torch.empty((0, 6), device="cuda"), spec).cpu().numpy()
    assert np.all(empty == 0.0)
    mags = synth.make_mags(3000, seed=21)
    bad = mags.copy()
    bad[:7, A] = np.nan
    bad[7:9, M] = np.inf
    h = dev.pop_summary(torch.tensor(bad, device="cuda"), spec).cpu().numpy()
    np.testing.assert_allclose(h, osum.histogram(mags[9:], A, B, CUT, 0.05, M, edges, 0.2),
                               rtol=1e-12)
    g = dev.pop_summary_vjp(torch.tensor(bad, device="cuda"), spec, torch.ones(8)).cpu().numpy()
    assert np.all(g[:9] == 0.0)
    one = _spec(dev, np.array([-30.0, -10.0]), 0.05, 0.2)
    h1 = dev.pop_summary(torch.tensor(mags, device="cuda"), one).cpu().numpy()
    np.testing.assert_allclose(h1, osum.histogram(mags, A, B, CUT, 0.05, M, [-30.0, -10.0], 0.2),
                               rtol=1e-12)
    t = torch.tensor(synth.make_mags(20000, seed=22), device="cuda")
    h_a = dev.pop_summary(t, spec)
    h_b = dev.pop_summary(t, spec)
    assert torch.equal(h_a, h_b)
    from paper_2112_06830_amd import DspsError
    with pytest.raises(DspsError):
        dev.pop_summary(t, _spec(dev, edges, -1.0, 0.2))
    with pytest.raises(DspsError):
        dev.pop_summary(t, _spec(dev, edges, 0.05, 0.2, band_a=6))


def test_forward_model_at_z0_and_population_gradient(dev):
    """Section 4.1 at z = 0 on 64 galaxies: absolute magnitudes, the summary,
    and the gradient of sum_k (H_k - target_k)^2 w.r.t. every galaxy's
    parameters through PopSummary and DspsMags, against the oracle's chain."""
    import torch
    from test_gpu_vjp import KEYS, grad_close
    ssp = ssp_small()
    ssp_h, flt_h = dev.SspBlock.from_synth(ssp), dev.FilterBank.from_synth(filters6())
    pop = synth.make_population(64, n_t=100, z_range=(0.1, 1.0), seed=33)
    pop.z[:] = 0.0
    inp = oracle_inputs(ssp, pop)
    _say("forward model at z = 0, 64 galaxies, population gradient")
    dp = dev.DevicePopulation.from_synth(pop, use_params=True)
    m_ref = oracle.mags(inp)
    par = dp.sfh_params.clone().requires_grad_(True)
    leaves = {k: getattr(dp, k).clone().requires_grad_(True) for k in KEYS}
    m = dev.dsps_mags(ssp_h, flt_h, dev.Cosmology(), dp, sfh_params=par, **leaves)
    assert np.max(np.abs(m.detach().cpu().numpy() - m_ref)) < FP32_TOL_MAG
    colour = m_ref[:, A] - m_ref[:, B]
    cut = float(np.median(colour))
    edges = np.linspace(m_ref[:, M].min() - 1.0, m_ref[:, M].max() + 1.0, 9)
    spec = dev.SummarySpec(band_a=A, band_b=B, colour_cut=cut, colour_width=0.05, band_m=M,
                           edges=torch.tensor(edges, device="cuda"), mag_width=0.3)
    h = dev.PopSummary.apply(m, spec)
    target = torch.full_like(h, 4.0)
    loss = ((h - target) ** 2).sum()
    loss.backward()
    h_ref = osum.histogram(m_ref, A, B, cut, 0.05, M, edges, 0.3)
    np.testing.assert_allclose(h.detach().cpu().numpy(), h_ref, rtol=1e-3, atol=1e-3)
    hbar = 2.0 * (h_ref - 4.0)
    mbar = osum.histogram_vjp(m_ref, A, B, cut, 0.05, M, edges, 0.3, hbar)
    ref = oracle.mags_vjp(inp, mbar)
    for k, rk in KEYS.items():
        ok, info = grad_close(leaves[k].grad.cpu().numpy(), ref[rk])
        assert ok, (k, info)
    for j in range(5):
        ok, info = grad_close(par.grad.cpu().numpy()[j], ref["sfh_params_bar"][j])
        assert ok, (j, info)

"""GPU parity of the forward hot path against the FP64 oracle, through the
C ABI: SFH table (a0), weights (a1-a4), SED (a5, a6), fused magnitudes
(a1-a7) in FP32 and BF16 (a8), edge cases, determinism and batch
independence."""

import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_common import (BF16_TOL_MAG, FP32_TOL_MAG, filters6, max_abs, oracle_inputs, ssp_large,
                        ssp_small)

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def small(dev):
    ssp = ssp_small()
    return dev.SspBlock.from_synth(ssp), dev.FilterBank.from_synth(filters6()), ssp


@pytest.fixture(scope="module")
def large(dev):
    ssp = ssp_large()
    return dev.SspBlock.from_synth(ssp), dev.FilterBank.from_synth(filters6()), ssp


def _pop(n, seed, z_range=(0.1, 1.0), n_t=100):
    return synth.make_population(n, n_t=n_t, z_range=z_range, seed=seed)


def test_sfh_table_matches_oracle(dev):
    import torch
    pop = _pop(333, seed=5, n_t=1000)
    _say("sfh_table n_gal=333 n_t=1000")
    t = torch.tensor(pop.t_table, device="cuda")
    par = torch.tensor(pop.sfh_params, device="cuda")
    got = dev.sfh_table(t, par).cpu().numpy()
    ref = oracle.sfh.sfr_from_params(pop.t_table, pop.sfh_params)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-300)


# time grids of one scan round (100), one full round plus its closing node
# (257), a second round of one segment (258) and four rounds, the last partial
# (1000), for the table and the parametric history
@pytest.mark.parametrize("n_t", [100, 257, 258, 1000])
@pytest.mark.parametrize("use_params", [False, True])
def test_weights_match_oracle(dev, small, use_params, n_t):
    ssp_h, _, ssp = small
    pop = _pop(131, seed=7, n_t=n_t)
    inp = oracle_inputs(ssp, pop)
    _say(f"weights n_gal=131 n_t={n_t} use_params={use_params}")
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr, use_params=use_params)
    w, ms = dev.weights(ssp_h, dev.Cosmology(), dp, with_mstar=True)
    w = w.cpu().numpy().astype(np.float64)
    ref, m_age, _, t_obs = oracle.weights(inp, return_parts=True)
    scale = ref.reshape(ref.shape[0], -1).max(axis=1)[:, None, None]
    assert np.all(np.abs(w - ref) <= 1e-6 * np.abs(ref) + 1e-9 * scale)
    # exact zeros where the triweight clips or ages exceed t_obs
    assert np.all(w[ref == 0] == 0)
    mstar = oracle.sfh.total_mass_formed(t_obs, inp.t_table, inp.sfr)
    np.testing.assert_allclose(ms.cpu().numpy(), mstar, rtol=1e-12)


@pytest.mark.parametrize("precision,apply_dust", [("fp32", False), ("fp32", True), ("bf16", True)])
def test_sed_matches_oracle(dev, small, precision, apply_dust):
    ssp_h, _, ssp = small
    pop = _pop(70, seed=9)
    inp = oracle_inputs(ssp, pop)
    _say(f"sed n_gal=70 precision={precision} dust={apply_dust}")
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    got = dev.sed(ssp_h, dev.Cosmology(), dp, apply_dust=apply_dust, precision=precision).cpu().numpy()
    ref = oracle.sed(inp, apply_dust=apply_dust)
    rel = np.abs(got - ref) / ref
    tol = 2e-5 if precision == "fp32" else 1.2e-2
    assert rel.max() < tol, rel.max()


def test_mags_fp32_small_workload(dev, small):
    """The 100-galaxy workload: SSP 12x94x1000, z ~ U[0.1, 1]."""
    ssp_h, flt_h, ssp = small
    pop = _pop(100, seed=2)
    inp = oracle_inputs(ssp, pop)
    _say("mags fp32 small workload n_gal=100")
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    m, bands = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp, precision="fp32", with_bands=True)
    ref, num, den = oracle.mags(inp, return_sums=True)
    assert max_abs(m.cpu().numpy(), ref) < FP32_TOL_MAG
    b = bands.cpu().numpy().astype(np.float64)
    # the trapezoid sums over lambda_obs themselves ((1+z) cancels between
    # d lambda_obs and 1/lambda_obs)
    np.testing.assert_allclose(b[:, 0, :], num, rtol=2e-5)
    np.testing.assert_allclose(b[:, 1, :], den, rtol=2e-5)


@pytest.mark.parametrize("n_t", [100, 300])
def test_mags_params_path_matches_table_path(dev, small, n_t):
    ssp_h, flt_h, ssp = small
    pop = _pop(100, seed=2, n_t=n_t)
    inp = oracle_inputs(ssp, pop)
    _say(f"mags fp32 params path n_gal=100 n_t={n_t}")
    dp = dev.DevicePopulation.from_synth(pop, use_params=True)
    m = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp).cpu().numpy()
    assert max_abs(m, oracle.mags(inp)) < FP32_TOL_MAG


def test_mags_bf16_small_workload(dev, small):
    ssp_h, flt_h, ssp = small
    pop = _pop(100, seed=2)
    inp = oracle_inputs(ssp, pop)
    _say("mags bf16 small workload n_gal=100")
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    m = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp, precision="bf16").cpu().numpy()
    assert max_abs(m, oracle.mags(inp)) < BF16_TOL_MAG


@pytest.mark.parametrize("n_gal", [1, 127, 129, 300])
def test_mags_ragged_sizes_large_grid(dev, large, n_gal):
    """Tile boundaries (128 galaxies) and the 5994-point grid, z ~ U[0.1, 3]."""
    ssp_h, flt_h, ssp = large
    pop = _pop(n_gal, seed=100 + n_gal, z_range=(0.1, 3.0))
    inp = oracle_inputs(ssp, pop)
    _say(f"mags fp32 large grid n_gal={n_gal}")
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    m = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp).cpu().numpy()
    assert max_abs(m, oracle.mags(inp)) < FP32_TOL_MAG


def test_mags_empty_population_is_noop(dev, small):
    import torch
    ssp_h, flt_h, ssp = small
    pop = _pop(4, seed=1)
    dp = dev.DevicePopulation.from_synth(pop, use_params=True)
    empty = dev.DevicePopulation(dp.t_table, None, dp.sfh_params[:, :0].contiguous(), dp.z[:0],
                                 dp.lgmet[:0], dp.sigma_z[:0], dp.av[:0], dp.delta[:0], dp.bump[:0])
    _say("mags n_gal=0")
    m = dev.mags(ssp_h, flt_h, dev.Cosmology(), empty)
    assert m.shape == (0, 6)
    torch.cuda.synchronize()


def test_mags_edge_parameters(dev, large):
    """A_V = 0 (identity), the narrowest MDF, q = 1 quenching, the extreme
    redshifts of the workload and a galaxy whose bluest band leaves the grid."""
    ssp_h, flt_h, ssp = large
    pop = _pop(8, seed=77, z_range=(0.1, 3.0))
    pop.av[0] = 0.0
    pop.sigma_z[1] = np.float32(0.1)
    pop.sfh_params[3, 2] = 1.0
    pop.sfh_params[4, 2] = 2.0
    pop.z[3] = np.float32(0.1)
    pop.z[4] = np.float32(3.0)
    pop.z[5] = np.float32(5.5)       # u-band support falls below 900 A rest
    inp = oracle_inputs(ssp, pop)
    _say("mags fp32 edge parameters")
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    m = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp).cpu().numpy()
    assert max_abs(m, oracle.mags(inp)) < FP32_TOL_MAG


def test_mags_deterministic_and_batch_independent(dev, large):
    """Run-to-run bitwise identical, and each galaxy's result is bitwise the
    same alone as inside a larger, differently ordered batch."""
    import torch
    ssp_h, flt_h, ssp = large
    pop = _pop(700, seed=31, z_range=(0.1, 3.0))
    inp = oracle_inputs(ssp, pop)
    _say("mags determinism n_gal=700")
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    m1 = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp).cpu().numpy()
    m2 = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp).cpu().numpy()
    assert np.array_equal(m1, m2)
    idx = np.array([5, 250, 251, 699, 17])
    sub = pop.subset(idx)
    dsub = dev.DevicePopulation.from_synth(sub, sfr=inp.sfr[idx])
    ms = dev.mags(ssp_h, flt_h, dev.Cosmology(), dsub).cpu().numpy()
    assert np.array_equal(ms, m1[idx])
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mags_each_galaxy_alone_equals_batch(dev, large, precision):
    """Each of a few galaxies across the redshift range, computed on its own
    (its tile's window is then its own, starting at an odd or an even chunk),
    is bitwise the same as inside the 700-galaxy batch, where its tile's
    window is its z-sorted mates' union."""
    ssp_h, flt_h, ssp = large
    pop = _pop(700, seed=31, z_range=(0.1, 3.0))
    inp = oracle_inputs(ssp, pop)
    _say(f"mags each galaxy alone vs batch, {precision}")
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    m_all = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp, precision=precision).cpu().numpy()
    order = np.argsort(pop.z)
    for i in order[np.linspace(0, pop.n_gal - 1, 9).astype(int)]:
        sub = pop.subset(np.array([i]))
        d1 = dev.DevicePopulation.from_synth(sub, sfr=inp.sfr[[i]])
        m1 = dev.mags(ssp_h, flt_h, dev.Cosmology(), d1, precision=precision).cpu().numpy()
        assert np.array_equal(m1[0], m_all[i]), (int(i), float(pop.z[i]))


@pytest.mark.parametrize("n_gal", [77, 129])
def test_mags_five_bands_unaligned_partial_slots(dev, n_gal):
    """Five bands (10 partial components per galaxy, 25 with the dust
    moments) and galaxy counts that leave a ragged last tile: FP32
    magnitudes without and with the moments against the FP64 oracle, and the
    moment instantiation's magnitudes equal to the plain ones bit for bit."""
    ssp = ssp_large()
    flt = synth.make_filters(n_band=5)
    pop = synth.make_population(n_gal, n_t=100, z_range=(0.1, 3.0), seed=61, n_band=5)
    inp = oracle.prepare_inputs(ssp, flt, pop)
    _say(f"mags five bands n_gal={n_gal}")
    ssp_h = dev.SspBlock.from_synth(ssp, precisions=("fp32",))
    flt_h = dev.FilterBank.from_synth(flt)
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    ref = oracle.mags(inp)
    m = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp).cpu().numpy()
    assert max_abs(m, ref) < FP32_TOL_MAG
    m2, _, _ = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp, with_moments=True)
    assert np.array_equal(m2.cpu().numpy(), m)


def test_mags_fp32_full_size_sampled(dev, large):
    """1e5 galaxies, 12x94x5994, z ~ U[0.1, 3] in one call (the FP32 bench
    configuration); 48 sampled galaxies against the oracle."""
    import torch
    ssp_h, flt_h, ssp = large
    pop = synth.make_population(100_000, n_t=100, z_range=(0.1, 3.0), seed=3)
    _say("mags fp32 full size n_gal=100000")
    dp = dev.DevicePopulation.from_synth(pop, use_params=True)
    m = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp).cpu().numpy()
    assert np.all(np.isfinite(m))
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(pop.n_gal, 48, replace=False))
    ref = oracle.mags(oracle_inputs(ssp, pop.subset(idx)))
    assert max_abs(m[idx], ref) < FP32_TOL_MAG
    torch.cuda.synchronize()


def test_quantize_bf16_bit_exact(dev):
    import torch
    ssp = ssp_large()
    rows = ssp.lum.reshape(-1, ssp.lum.shape[-1])
    _say("quantize_bf16 1128x5994")
    q, s = dev.quantize_bf16(torch.tensor(rows, device="cuda"))
    q_ref, s_ref = oracle.quantize_bf16_rne(rows)
    assert np.array_equal(s.cpu().numpy(), s_ref)
    assert np.array_equal(q.cpu().numpy().view(np.uint16), q_ref)


def test_mags_bf16_error_report_1e4_subset(dev, large):
    """The BF16 workload's error subset: the first 1e4 galaxies of the 1e6
    population (n_t = 1000, z ~ U[0.1, 3]); per-band max and RMS |dm| against
    the FP64 oracle, max within the BF16 target."""
    ssp_h, flt_h, ssp = large
    pop = synth.make_population(1_000_000, n_t=1000, z_range=(0.1, 3.0), seed=4).subset(np.arange(10_000))
    _say("mags bf16 error report, 1e4 galaxies of the 1e6 workload, n_t=1000")
    dp = dev.DevicePopulation.from_synth(pop, use_params=True)
    sfr = dev.sfh_table(dp.t_table, dp.sfh_params)
    m = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp.with_sfr(sfr), precision="bf16").cpu().numpy()
    ref = np.concatenate([oracle.mags(oracle_inputs(ssp, pop.subset(np.arange(s, min(s + 1000, pop.n_gal)))))
                          for s in range(0, pop.n_gal, 1000)])
    d = np.abs(m.astype(np.float64) - ref)
    _say("bf16 per-band max |dm| " + " ".join(f"{v:.2e}" for v in d.max(axis=0)) +
         "; rms " + " ".join(f"{v:.2e}" for v in np.sqrt((d ** 2).mean(axis=0))))
    assert d.max() < BF16_TOL_MAG

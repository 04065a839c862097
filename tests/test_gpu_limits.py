"""GPU parity at the build's size limits, through the C ABI: the largest SSP
grid (16 metallicities x 96 ages), the longest SFH table (2048 points), the
largest filter set (8 bands x 1024 points = DSPS_MAX_FILTER_FLOATS), and the
degenerate smallest grids (one metallicity, one age), each against the FP64
oracle on the same seeded inputs."""

import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_common import BF16_TOL_MAG, FP32_TOL_MAG, max_abs

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


def _check(dev, ssp, flt, pop, precisions=("fp32", "bf16")):
    ssp_h = dev.SspBlock.from_synth(ssp, precisions=precisions)
    flt_h = dev.FilterBank.from_synth(flt)
    inp = oracle.prepare_inputs(ssp, flt, pop)
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    w = dev.weights(ssp_h, dev.Cosmology(), dp).cpu().numpy().astype(np.float64)
    ref_w = oracle.weights(inp)
    scale = ref_w.reshape(ref_w.shape[0], -1).max(axis=1)[:, None, None]
    assert np.all(np.abs(w - ref_w) <= 1e-6 * np.abs(ref_w) + 1e-9 * scale)
    ref_m = oracle.mags(inp)
    for prec in precisions:
        m = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp, precision=prec).cpu().numpy()
        tol = FP32_TOL_MAG if prec == "fp32" else BF16_TOL_MAG
        assert max_abs(m, ref_m) < tol, prec


def test_largest_grids_and_tables(dev):
    ssp = synth.make_ssp(n_wave=2000, wave_lo=9.0e2, wave_hi=2.5e4, n_met=16, n_age=96,
                         lg_age_range=(5.3, 10.15))
    flt = synth.make_filters(n_band=8, n_pts=1024, centre_range=(3600.0, 11000.0))
    pop = synth.make_population(200, n_t=2048, z_range=(0.1, 3.0), seed=81, n_band=8)
    _say("limits: 16 x 96 x 2000 SSP, n_t=2048, 8 x 1024 filters, n_gal=200")
    _check(dev, ssp, flt, pop)


def test_age_dependent_dust_on_largest_grid(dev):
    """The age-dependent attenuation (age-major table and stage lists, per-group
    folds) on the 16 x 96 grid: all 16 metallicity slots of an age are real,
    so both halves of every age carry weight; forward magnitudes and the
    reverse pass against the oracle."""
    import torch
    from test_gpu_age_dust import AGED_KEYS, grad_close
    ssp = synth.make_ssp(n_wave=2000, wave_lo=9.0e2, wave_hi=2.5e4, n_met=16, n_age=96,
                         lg_age_range=(5.3, 10.15))
    flt = synth.make_filters(n_band=8, n_pts=1024, centre_range=(3600.0, 11000.0))
    pop = synth.make_population(160, n_t=100, z_range=(0.1, 3.0), seed=82, n_band=8,
                                age_dust=True, dust_pivot=7.0, dust_width=0.25)
    _say("limits: age-dependent attenuation on 16 x 96 x 2000, 8 bands, n_gal=160")
    ssp_h = dev.SspBlock.from_synth(ssp, precisions=("fp32",), age_major=True)
    flt_h = dev.FilterBank.from_synth(flt)
    inp = oracle.prepare_inputs(ssp, flt, pop)
    dp = dev.DevicePopulation.from_synth(pop, sfr=inp.sfr)
    ref_m = oracle.mags(inp)
    m = dev.mags(ssp_h, flt_h, dev.Cosmology(), dp, precision="fp32").cpu().numpy()
    assert max_abs(m, ref_m) < FP32_TOL_MAG
    bar = 2.0 * (ref_m - pop.targets)
    g = dev.mags_vjp(ssp_h, flt_h, dev.Cosmology(), dp, torch.tensor(bar, dtype=torch.float32))
    ref = oracle.mags_vjp(inp, bar)
    for k, rk in AGED_KEYS.items():
        ok, info = grad_close(g[k].cpu().numpy(), ref[rk])
        assert ok, (k, info)


def test_one_metallicity_one_age(dev):
    ssp = synth.make_ssp(n_wave=600, wave_lo=1.0e3, wave_hi=2.0e4, n_met=1, n_age=1,
                         lgz_range=(-2.0, -1.0), lg_age_range=(9.0, 10.0))
    flt = synth.make_filters()
    pop = synth.make_population(64, n_t=100, z_range=(0.1, 1.0), seed=83)
    _say("limits: 1 x 1 SSP grid, n_gal=64")
    _check(dev, ssp, flt, pop)


def test_two_point_time_grid(dev):
    ssp = synth.make_ssp(n_wave=600, wave_lo=1.0e3, wave_hi=2.0e4)
    flt = synth.make_filters()
    pop = synth.make_population(64, n_t=2, z_range=(0.1, 1.0), seed=85)
    _say("limits: n_t=2, n_gal=64")
    _check(dev, ssp, flt, pop, precisions=("fp32",))

"""dsps_mags_noalloc, the fused magnitudes on the library's fixed per-device
scratch (for callers that cannot allocate), against dsps_mags with a caller
workspace: consecutive calls, each later one on a smaller population, equal
bit for bit; and the host-side refusal of a population too large for the
scratch."""

import sys

import numpy as np
import pytest

import synth
from gpu_common import FP32_TOL_MAG, filters6, ssp_large

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


def test_noalloc_equals_workspace_call_on_consecutive_calls(dev):
    import torch
    P = dev
    ssp_h = P.SspBlock.from_synth(ssp_large(), precisions=("fp32", "bf16"))
    flt_h = P.FilterBank.from_synth(filters6())
    # 30000 galaxies on the 5994-wavelength grid run in several batches of the
    # scratch; the later calls are smaller (one batch) and leave the scratch
    # holding the earlier calls' larger contents
    cases = ((30000, 51, "fp32", False), (3000, 52, "fp32", True), (1500, 53, "bf16", False))
    for n, seed, prec, moments in cases:
        _say(f"noalloc vs workspace call: n_gal={n} precision={prec} moments={moments}")
        pop = synth.make_population(n, n_t=100, z_range=(0.1, 3.0), seed=seed)
        dp = P.DevicePopulation.from_synth(pop, use_params=True)
        if moments:
            ref, ref_b, ref_m = P.mags(ssp_h, flt_h, P.Cosmology(), dp, precision=prec,
                                       with_moments=True)
        else:
            ref, ref_b = P.mags(ssp_h, flt_h, P.Cosmology(), dp, precision=prec, with_bands=True)
        out = torch.full((n, 6), float("nan"), dtype=torch.float32, device="cuda")
        bands = torch.full((n, 2, 6), float("nan"), dtype=torch.float32, device="cuda")
        mom = (torch.full((n, 3, 6), float("nan"), dtype=torch.float32, device="cuda")
               if moments else None)
        P.mags_noalloc(ssp_h, flt_h, P.Cosmology(), dp, out, precision=prec, bands_out=bands,
                       moments_out=mom)
        torch.cuda.synchronize()
        # the tiling is exact, so the batch size cannot change any result
        d = float((out.double() - ref.double()).abs().max())
        assert d <= FP32_TOL_MAG, d
        assert torch.equal(out, ref), d
        assert torch.equal(bands, ref_b)
        if moments:
            assert torch.equal(mom, ref_m)


def test_noalloc_refuses_population_beyond_scratch(dev):
    import torch
    P = dev
    from paper_2112_06830_amd import DspsError
    ssp_h = P.SspBlock.from_synth(ssp_large(), precisions=("fp32",))
    flt_h = P.FilterBank.from_synth(filters6())
    # 3e6 galaxies need > 128 MiB for the per-galaxy arrays alone: refused on
    # the host before any launch (the inputs are valid all the same)
    n = 3_000_000
    _say(f"noalloc refusal: n_gal={n}")
    t = torch.linspace(0.01, 13.8, 100, dtype=torch.float64, device="cuda")
    par = torch.tensor([10.0, 3.0, 1.5, 0.5, 8.0], dtype=torch.float64,
                       device="cuda")[:, None].repeat(1, n).contiguous()
    f = lambda v: torch.full((n,), v, dtype=torch.float32, device="cuda")
    dp = P.DevicePopulation(t_table=t, sfr=None, sfh_params=par, z=f(0.5), lgmet=f(-2.0),
                            sigma_z=f(0.2), av=f(0.5), delta=f(-0.2), bump=f(1.0))
    out = torch.zeros((n, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(DspsError) as e:
        P.mags_noalloc(ssp_h, flt_h, P.Cosmology(), dp, out)
    assert e.value.status == -2 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 0).all())
    # and the next call in range still works
    pop = synth.make_population(700, n_t=100, z_range=(0.1, 3.0), seed=54)
    dp = P.DevicePopulation.from_synth(pop, use_params=True)
    ref = P.mags(ssp_h, flt_h, P.Cosmology(), dp)
    got = torch.empty_like(ref)
    P.mags_noalloc(ssp_h, flt_h, P.Cosmology(), dp, got)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert np.isfinite(got.cpu().numpy()).all()

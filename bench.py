#!/usr/bin/env python
"""Throughput benchmark of the fused DSPS magnitude path on one MI355X.

One step = one dsps_mags call over the whole population (redshift ordering,
age-bin masses and MDF weights, the fused W.SSP contraction with attenuation
and filter integrals, and the magnitude finalisation), inputs resident in HBM.
Default workload: 1e5 galaxies, SSP 12 x 94 x 5994 (9e2-2.5e4 A) in float32,
tabulated SFH on 100 times, z ~ U[0.1, 3], six Gaussian bands.

Prints ONE JSON line.  `roofline` describes the dominant kernel
(k_mags_gemm), timed with HIP events on its launch stream during the timed
region.  `cpu_baseline` times the FP64 oracle on a bounded sample of the
same workload on the host cores; the same leg reports the per-band error of
the GPU magnitudes against the oracle on that sample (FP32) and on the first
1e4 galaxies of the BF16 workload (`extra.error_vs_oracle`).
"""

from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "galaxies/sec 6-band mags, fwd & fwd+grad, plain FP32 vs BF16; p50/p99 latency"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}     # MI355X dense MFMA
HBM_PEAK_GBS = 8000.0
CALIBRATION_BYTES = 512 << 20
GEMM_SOURCES = ("paper_2112_06830_amd/csrc/k_mags.hip", "paper_2112_06830_amd/csrc/gemm_core.hpp",
                "paper_2112_06830_amd/csrc/dsps_internal.hpp")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """C++ source without comments and blank lines: edits to comments do not
    change the kernel the counters were taken on."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def gemm_source_hash() -> str:
    h = hashlib.sha256()
    for rel in GEMM_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def read_traffic(precision: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"k_mags_gemm_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.lstrip().startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != gemm_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def effective_wavelengths(wave, z, obs_lo, obs_hi):
    """Rest-grid points whose redshifted wavelength lies inside the union of
    the filter supports (the bands here overlap into one interval)."""
    lo = np.searchsorted(wave, obs_lo / (1.0 + z), side="left")
    hi = np.searchsorted(wave, obs_hi / (1.0 + z), side="right")
    return np.maximum(hi - lo, 0)


def algorithmic_flops(P, ssp_h, dpop, ssp, flt, z, per_galaxy=False):
    """2 * nnz(W_g) * n_lambda_eff(z_g) summed over galaxies: the multiply-adds
    the contraction must do for the wavelengths any filter sees (per galaxy
    with per_galaxy)."""
    import torch
    nnz = torch.zeros(dpop.n_gal, dtype=torch.int64, device="cuda")
    step = 16384
    for s in range(0, dpop.n_gal, step):
        e = min(s + step, dpop.n_gal)
        sub = P.DevicePopulation(dpop.t_table, dpop.sfr[s:e] if dpop.sfr is not None else None,
                                 dpop.sfh_params[:, s:e].contiguous() if dpop.sfh_params is not None else None,
                                 dpop.z[s:e], dpop.lgmet[s:e], dpop.sigma_z[s:e], dpop.av[s:e],
                                 dpop.delta[s:e], dpop.bump[s:e], dpop.lgmet_slope, dpop.lg_age_pivot)
        w = P.weights(ssp_h, P.Cosmology(), sub)
        nnz[s:e] = (w.view(e - s, -1) != 0).sum(dim=1)
    nnz = nnz.cpu().numpy().astype(np.float64)
    neff = effective_wavelengths(ssp.wave, z, flt.wave[:, 0].min(), flt.wave[:, -1].max())
    if per_galaxy:
        return 2.0 * nnz * neff
    return float(np.sum(2.0 * nnz * neff)), float(nnz.mean()), float(neff.mean())


def band_errors(got, ref):
    """Per-band max and RMS of |m_gpu - m_oracle| in mag."""
    d = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    return {"max_mag": [float(v) for v in d.max(axis=0)],
            "rms_mag": [float(v) for v in np.sqrt((d ** 2).mean(axis=0))]}


def cpu_baseline(ssp, flt, pop, m32, pop16=None, m16=None, min_seconds=10.0, block=512,
                 max_gal=24576, n16=10_000):
    """The FP64 oracle timed on the host on a bounded sample of the FP32
    workload (it tabulates its own SFR from the parametric history); the GPU
    magnitudes of the same galaxies are compared with it per band, and the
    BF16 workload's first n16 galaxies likewise."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    done = 0
    ref = []
    t0 = time.perf_counter()
    while done < min(max_gal, pop.n_gal):
        idx = np.arange(done, min(done + block, pop.n_gal))
        inp = oracle.prepare_inputs(ssp, flt, pop.subset(idx))
        ref.append(oracle.mags(inp))
        done += idx.size
        if time.perf_counter() - t0 >= min_seconds:
            break
    dt = time.perf_counter() - t0
    cpu = {"value": done / dt, "unit": "galaxies/s", "cores": int(threads), "kind": "oracle",
           "sample": f"first {done} galaxies of the same population (FP64 numpy oracle, "
                     f"{dt:.1f} s, BLAS threads={threads}, host cpus={os.cpu_count()})"}
    errors = {"fp32_fwd_1e5": dict(band_errors(m32[:done], np.concatenate(ref)), n_gal=done)}
    if pop16 is not None:
        idx = np.arange(min(n16, pop16.n_gal))
        ref16 = []
        for s0 in range(0, idx.size, block):
            inp = oracle.prepare_inputs(ssp, flt, pop16.subset(idx[s0:s0 + block]))
            ref16.append(oracle.mags(inp))
        errors["bf16_fwd_1e6"] = dict(band_errors(m16[:idx.size], np.concatenate(ref16)),
                                      n_gal=int(idx.size))
    return cpu, errors


def cpu_baseline_single_thread(ssp, flt, pop, min_seconds=10.0, block=256, max_gal=8192):
    """The same oracle timing with the BLAS thread pools held to one thread."""
    import oracle
    from threadpoolctl import threadpool_limits
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while done < min(max_gal, pop.n_gal):
            idx = np.arange(done, min(done + block, pop.n_gal))
            oracle.mags(oracle.prepare_inputs(ssp, flt, pop.subset(idx)))
            done += idx.size
            if time.perf_counter() - t0 >= min_seconds:
                break
        dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "galaxies/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} galaxies of the same population (FP64 numpy oracle, "
                      f"{dt:.1f} s, BLAS threads=1)"}


def run_workload(P, name, n_gal, n_t, precision, steps, warmup, seed, want_roofline=True):
    import torch
    import synth
    ssp = synth.make_ssp(n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4)
    flt = synth.make_filters()
    pop = synth.make_population(n_gal, n_t=n_t, z_range=(0.1, 3.0), seed=seed)
    log(f"{name}: uploading {n_gal} galaxies, n_t={n_t}, precision={precision}")
    ssp_h = P.SspBlock.from_synth(ssp, precisions=(precision,))
    flt_h = P.FilterBank.from_synth(flt)
    dpar = P.DevicePopulation.from_synth(pop, use_params=True)
    sfr = P.sfh_table(dpar.t_table, dpar.sfh_params)          # a0 on the GPU, untimed
    dpop = dpar.with_sfr(sfr)
    ws = P.Workspace(P.workspace_size(2, ssp_h, flt_h, n_gal, n_t, precision), dpop.device)
    out = torch.empty((n_gal, 6), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        P.mags(ssp_h, flt_h, P.Cosmology(), dpop, precision=precision, workspace=ws, out=out)
    torch.cuda.synchronize()
    P.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        P.mags(ssp_h, flt_h, P.Cosmology(), dpop, precision=precision, workspace=ws, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gemm_ms, gemm_n = P.profile_read("mags_gemm")
    w_ms, w_n = P.profile_read("weights")
    P.profile_enable(False)
    ms_step = (t1 - t0) * 1e3 / steps
    res = {"ms_per_step": ms_step, "galaxies_per_s": n_gal / (ms_step * 1e-3),
           "gemm_ms_per_launch": gemm_ms / max(gemm_n, 1), "gemm_launches_per_step": gemm_n / steps,
           "weights_ms_per_step": w_ms / steps, "gemm_ms_per_step": gemm_ms / steps,
           "finite": bool(torch.isfinite(out).all().item())}
    if want_roofline:
        flops, nnz_mean, neff_mean = algorithmic_flops(P, ssp_h, dpop, ssp, flt, pop.z)
        achieved = flops / (gemm_ms / steps * 1e-3) / 1e12
        res.update(alg_flops_per_step=flops, nnz_mean=nnz_mean, n_lambda_eff_mean=neff_mean,
                   achieved_tflops=achieved)
    return res, (ssp, flt, pop, out.cpu().numpy())


def run_grad(P, steps, warmup, n_gal=200_000, seed=5):
    """Forward plus adjoint of sum (m - target)^2 on the gradient workload:
    2e5 galaxies, parametric SFH (gradients w.r.t. A, tau, alpha, q, t_q,
    lgmet, sigma_Z, A_V, delta, bump), FP32, as one fused residual call (one
    sort, one weights pass); the two-call sequence (dsps_mags, the cotangent,
    dsps_mags_vjp) is timed beside it."""
    import torch
    import synth
    ssp = synth.make_ssp(n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4)
    flt = synth.make_filters()
    pop = synth.make_population(n_gal, n_t=100, z_range=(0.1, 3.0), seed=seed)
    log(f"grad_fp32_2e5: uploading {n_gal} galaxies")
    ssp_h = P.SspBlock.from_synth(ssp, precisions=("fp32",))
    flt_h = P.FilterBank.from_synth(flt)
    dpop = P.DevicePopulation.from_synth(pop, use_params=True)
    tgt = torch.tensor(pop.targets, dtype=torch.float32, device="cuda")
    ws_f = P.Workspace(P.workspace_size(2, ssp_h, flt_h, n_gal, 100, "fp32"), dpop.device)
    ws_b = P.Workspace(P.workspace_size(3, ssp_h, flt_h, n_gal, 100, "fp32"), dpop.device)
    m = torch.empty((n_gal, 6), dtype=torch.float32, device="cuda")
    bands = torch.empty((n_gal, 2, 6), dtype=torch.float32, device="cuda")
    mom = torch.empty((n_gal, 3, 6), dtype=torch.float32, device="cuda")
    outs = {"sfh_params": torch.empty((5, n_gal), dtype=torch.float64, device="cuda")}
    for k in ("lgmet", "sigma_z", "av", "delta", "bump"):
        outs[k] = torch.empty(n_gal, dtype=torch.float32, device="cuda")
    bar = torch.empty_like(m)

    def two_calls():
        P.mags(ssp_h, flt_h, P.Cosmology(), dpop, with_moments=True, workspace=ws_f, out=m,
               bands_out=bands, moments_out=mom)
        torch.sub(m, tgt, out=bar)
        bar.mul_(2.0)
        P.mags_vjp(ssp_h, flt_h, P.Cosmology(), dpop, bar, bands=bands, moments=mom, workspace=ws_b,
                   outs=outs)

    def step():
        P.mags_residual_vjp(ssp_h, flt_h, P.Cosmology(), dpop, tgt, workspace=ws_b, out=m,
                            outs=outs)

    for _ in range(warmup):
        two_calls()
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(steps // 2, 1)):
        two_calls()
    torch.cuda.synchronize()
    two_ms = (time.perf_counter() - t0) * 1e3 / max(steps // 2, 1)
    P.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = {"ms_per_step": (t1 - t0) * 1e3 / steps, "two_call_ms_per_step": two_ms}
    res["galaxies_per_s"] = n_gal / (res["ms_per_step"] * 1e-3)
    for k in ("mags_gemm", "vjp_lbar", "vjp_wbar", "vjp_weights", "weights"):
        ms, n = P.profile_read(k)
        res[f"{k}_ms_per_step"] = ms / steps
    P.profile_enable(False)
    res["finite"] = bool(all(torch.isfinite(v).all().item() for v in outs.values()))
    # algorithmic work: the forward contraction and the transposed one (W-bar)
    # each do 2 nnz(W_g) n_lambda_eff(z_g) flops per galaxy
    flops, _, _ = algorithmic_flops(P, ssp_h, dpop, ssp, flt, pop.z)
    peak = PEAK_TFLOPS["fp32"]
    roof = {"bound": "mfma", "peak": peak, "unit": "TFLOP/s", "alg_flops_per_contraction": flops}
    for k in ("mags_gemm", "vjp_wbar"):
        t = res[f"{k}_ms_per_step"] * 1e-3
        roof[k] = {"achieved": flops / t / 1e12, "frac": flops / t / 1e12 / peak}
    step_s = res["ms_per_step"] * 1e-3
    roof["step"] = {"alg_flops": 2.0 * flops, "achieved": 2.0 * flops / step_s / 1e12,
                    "frac": 2.0 * flops / step_s / 1e12 / peak}
    res["roofline"] = roof
    return res


def run_variants(P, steps, warmup, n_gal=100_000, seed=8, w0=-0.9, width=0.4):
    """The MDF and cosmology variants on the FP32 forward and forward +
    gradient of the 1e5-galaxy workload: the T_erf transition of the MDF
    centre with age (old-age centre per galaxy, width 0.4 dex) in a flat wCDM
    cosmology (w0 = -0.9).  Returns the timings and, for the oracle check of
    the CPU-baseline leg, the magnitudes of the first 128 galaxies."""
    import torch
    import synth
    ssp = synth.make_ssp(n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4)
    flt = synth.make_filters()
    pop = synth.make_population(n_gal, n_t=100, z_range=(0.1, 3.0), seed=seed, mdf="transition",
                                mdf_width=width)
    log(f"variants_fp32_1e5: transition MDF (width {width}), wCDM w0={w0}")
    ssp_h = P.SspBlock.from_synth(ssp, precisions=("fp32",))
    flt_h = P.FilterBank.from_synth(flt)
    cos = P.Cosmology(w0=w0)
    dpop = P.DevicePopulation.from_synth(pop, use_params=True)
    tgt = torch.tensor(pop.targets, dtype=torch.float32, device="cuda")
    ws_f = P.Workspace(P.workspace_size(2, ssp_h, flt_h, n_gal, 100, "fp32"), dpop.device)
    ws_b = P.Workspace(P.workspace_size(3, ssp_h, flt_h, n_gal, 100, "fp32"), dpop.device)
    m = torch.empty((n_gal, 6), dtype=torch.float32, device="cuda")
    bands = torch.empty((n_gal, 2, 6), dtype=torch.float32, device="cuda")
    mom = torch.empty((n_gal, 3, 6), dtype=torch.float32, device="cuda")
    outs = {"sfh_params": torch.empty((5, n_gal), dtype=torch.float64, device="cuda")}
    for k in ("lgmet", "lgmet_old", "sigma_z", "av", "delta", "bump"):
        outs[k] = torch.empty(n_gal, dtype=torch.float32, device="cuda")
    bar = torch.empty_like(m)

    def forward():
        P.mags(ssp_h, flt_h, cos, dpop, workspace=ws_f, out=m)

    def gradient():
        P.mags(ssp_h, flt_h, cos, dpop, with_moments=True, workspace=ws_f, out=m,
               bands_out=bands, moments_out=mom)
        torch.sub(m, tgt, out=bar)
        bar.mul_(2.0)
        P.mags_vjp(ssp_h, flt_h, cos, dpop, bar, bands=bands, moments=mom, workspace=ws_b,
                   outs=outs)

    res = {}
    for name, fn in (("forward", forward), ("forward_grad", gradient)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[name] = {"ms_per_step": ms, "galaxies_per_s": n_gal / (ms * 1e-3)}
    res["finite"] = bool(all(torch.isfinite(v).all().item() for v in outs.values()))
    forward()
    return res, (ssp, flt, pop.subset(np.arange(128)), m[:128].cpu().numpy(), w0)


def run_age_dust(P, steps, warmup, n_gal=100_000, seed=9, pivot=7.0, width=0.25):
    """Age-dependent attenuation (Section 3.4.1) on the FP32 forward of the
    1e5-galaxy workload: young-star and old-star A_V and delta joined by the
    cumulative triweight of log10 age (centre 10 Myr, width 0.25 dex).
    Returns the timings and the magnitudes of the first 128 galaxies for the
    oracle check of the CPU-baseline leg."""
    import torch
    import synth
    ssp = synth.make_ssp(n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4)
    flt = synth.make_filters()
    pop = synth.make_population(n_gal, n_t=100, z_range=(0.1, 3.0), seed=seed, age_dust=True,
                                dust_pivot=pivot, dust_width=width)
    log(f"age_dust_fp32_1e5: transition at log10 age {pivot}, width {width}")
    ssp_h = P.SspBlock.from_synth(ssp, precisions=("fp32",), age_major=True)
    flt_h = P.FilterBank.from_synth(flt)
    dpar = P.DevicePopulation.from_synth(pop, use_params=True)
    dpop = dpar.with_sfr(P.sfh_table(dpar.t_table, dpar.sfh_params))
    ws = P.Workspace(P.workspace_size(2, ssp_h, flt_h, n_gal, 100, "fp32"), dpop.device)
    m = torch.empty((n_gal, 6), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        P.mags(ssp_h, flt_h, P.Cosmology(), dpop, workspace=ws, out=m)
    torch.cuda.synchronize()
    P.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        P.mags(ssp_h, flt_h, P.Cosmology(), dpop, workspace=ws, out=m)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    gemm_ms, _ = P.profile_read("mags_gemm")
    w_ms, _ = P.profile_read("weights")
    P.profile_enable(False)
    res = {"ms_per_step": ms, "galaxies_per_s": n_gal / (ms * 1e-3),
           "gemm_ms_per_step": gemm_ms / steps, "weights_ms_per_step": w_ms / steps,
           "finite": bool(torch.isfinite(m).all().item())}
    # forward + adjoint of the squared error to target magnitudes, the
    # old-star cotangents included
    targets = torch.tensor(pop.targets, dtype=torch.float32, device="cuda")
    ws_v = P.Workspace(P.workspace_size(3, ssp_h, flt_h, n_gal, 100, "fp32"), dpop.device)

    def fwd_grad():
        mm, bands = P.mags(ssp_h, flt_h, P.Cosmology(), dpar, with_bands=True, workspace=ws)
        return P.mags_vjp(ssp_h, flt_h, P.Cosmology(), dpar, 2.0 * (mm - targets), bands=bands,
                          workspace=ws_v)
    for _ in range(warmup):
        fwd_grad()
    torch.cuda.synchronize()
    P.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        grads = fwd_grad()
    torch.cuda.synchronize()
    ms_grad = (time.perf_counter() - t0) * 1e3 / steps
    wbar_ms, _ = P.profile_read("vjp_wbar")
    P.profile_enable(False)
    # the per-age transposed contraction: four contractions (G F and its three
    # dust factors) of n_met rows per age over the wavelengths any filter sees
    neff = effective_wavelengths(ssp.wave, pop.z, flt.wave[:, 0].min(), flt.wave[:, -1].max())
    alg = 8.0 * ssp.lum.shape[0] * ssp.lum.shape[1] * float(np.sum(neff))
    wbar_s = wbar_ms / steps * 1e-3
    res["mags_and_gradient"] = {
        "ms_per_step": ms_grad, "galaxies_per_s": n_gal / (ms_grad * 1e-3),
        "wbar_ms_per_step": wbar_ms / steps, "wbar_alg_flops": alg,
        "wbar_achieved_tflops": alg / wbar_s / 1e12,
        "wbar_mfma_frac_fp32": alg / wbar_s / 1e12 / PEAK_TFLOPS["fp32"],
        "finite": bool(all(torch.isfinite(v).all().item() for v in grads.values()))}
    return res, (ssp, flt, pop.subset(np.arange(128)), m[:128].cpu().numpy())


# [OII], Hbeta, [OIII] 5007, Halpha: (centre, half-width, fit half-width), Angstrom
NEB_LINES = ((3727.42, 40.0, 150.0), (4862.68, 40.0, 150.0), (5008.24, 40.0, 150.0),
             (6564.61, 50.0, 180.0))


def run_nebular(P, steps, warmup, n_gal=100_000, seed=10, n_u=7):
    """Nebular ionization axis (Section 3.3, Eq. nebsed) on the FP32 forward
    of the 1e5-galaxy workload: the 12 x 94 x 5994 block with n_u = 7
    ionization points (log10 U_s -4..-1), log10 U_s ~ U[-3.5, -1.5] and
    sigma_u ~ U[0.1, 0.4] per galaxy.  Times the fused magnitudes, and the
    attenuated SED plus four equivalent widths (Section 2.2.2, Eq. eqw) of
    every galaxy.  Returns the timings and samples for the oracle check of the
    CPU-baseline leg."""
    import torch
    import synth
    ssp = synth.make_ssp_nebular(n_u=n_u, n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4)
    flt = synth.make_filters()
    pop = synth.make_population(n_gal, n_t=100, z_range=(0.1, 3.0), seed=seed, nebular=True)
    log(f"nebular_fp32_1e5: n_u={n_u}")
    ssp_h = P.SspBlock.from_synth(ssp)
    flt_h = P.FilterBank.from_synth(flt)
    dpar = P.DevicePopulation.from_synth(pop, use_params=True)
    dpop = dpar.with_sfr(P.sfh_table(dpar.t_table, dpar.sfh_params))
    ws = P.Workspace(P.workspace_size(2, ssp_h, flt_h, n_gal, 100, "fp32"), dpop.device)
    m = torch.empty((n_gal, 6), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        P.mags(ssp_h, flt_h, P.Cosmology(), dpop, workspace=ws, out=m)
    torch.cuda.synchronize()
    P.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        P.mags(ssp_h, flt_h, P.Cosmology(), dpop, workspace=ws, out=m)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    gemm_ms, _ = P.profile_read("mags_gemm")
    P.profile_enable(False)
    ew = None
    for _ in range(warmup):
        sed = P.sed(ssp_h, P.Cosmology(), dpop, apply_dust=True)
        ew = P.eqw(ssp_h, sed, NEB_LINES)
    torch.cuda.synchronize()
    P.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        sed = P.sed(ssp_h, P.Cosmology(), dpop, apply_dust=True)
        ew = P.eqw(ssp_h, sed, NEB_LINES)
    torch.cuda.synchronize()
    ms_ew = (time.perf_counter() - t0) * 1e3 / steps
    eqw_ms, _ = P.profile_read("eqw")
    P.profile_enable(False)
    # the same widths, and their derivative in log10 U_s, straight from the
    # population (the SED is computed only on the chunks near the lines)
    for _ in range(warmup):
        P.eqw_pop(ssp_h, P.Cosmology(), dpop, NEB_LINES)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ew_pop = P.eqw_pop(ssp_h, P.Cosmology(), dpop, NEB_LINES)
    torch.cuda.synchronize()
    ms_ew_pop = (time.perf_counter() - t0) * 1e3 / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        _, dew = P.eqw_pop(ssp_h, P.Cosmology(), dpop, NEB_LINES, wrt="lgu")
    torch.cuda.synchronize()
    ms_ew_pop_d = (time.perf_counter() - t0) * 1e3 / steps
    same = bool(torch.equal(ew_pop, ew))
    # forward + adjoint of the squared error to target magnitudes, every
    # cotangent including the ionization centre and width
    targets = torch.tensor(pop.targets, dtype=torch.float32, device="cuda")
    ws_v = P.Workspace(P.workspace_size(3, ssp_h, flt_h, n_gal, 100, "fp32"), dpop.device)

    def fwd_grad():
        mm, bands, mom = P.mags(ssp_h, flt_h, P.Cosmology(), dpar, with_moments=True, workspace=ws)
        return P.mags_vjp(ssp_h, flt_h, P.Cosmology(), dpar, 2.0 * (mm - targets), bands=bands,
                          moments=mom, workspace=ws_v)
    for _ in range(warmup):
        fwd_grad()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        grads = fwd_grad()
    torch.cuda.synchronize()
    ms_grad = (time.perf_counter() - t0) * 1e3 / steps
    # algorithmic work of the fused GEMM: 2 nnz(W_g) n_u,nz(g) n_lambda_eff(z_g),
    # n_u,nz the ionization points inside the galaxy's +-3 sigma support
    per_g = algorithmic_flops(P, ssp_h, dpar, ssp, flt, pop.z, per_galaxy=True)
    edges = np.concatenate([[-np.inf], 0.5 * (ssp.lgu[1:] + ssp.lgu[:-1]), [np.inf]])
    lo, hi = pop.lgu - 3.0 * pop.sigma_u, pop.lgu + 3.0 * pop.sigma_u
    n_unz = ((edges[None, :-1] < hi[:, None]) & (edges[None, 1:] > lo[:, None])).sum(axis=1)
    alg = float(np.sum(n_unz * per_g))
    gemm_s = gemm_ms / steps * 1e-3
    res = {"mags": {"ms_per_step": ms, "galaxies_per_s": n_gal / (ms * 1e-3),
                    "gemm_ms_per_step": gemm_ms / steps,
                    "alg_flops_per_step": alg, "achieved_tflops": alg / gemm_s / 1e12,
                    "mfma_frac_fp32": alg / gemm_s / 1e12 / PEAK_TFLOPS["fp32"],
                    "mean_ion_points": float(n_unz.mean())},
           "sed_and_eqw": {"ms_per_step": ms_ew, "galaxies_per_s": n_gal / (ms_ew * 1e-3),
                           "eqw_ms_per_step": eqw_ms / steps, "n_lines": len(NEB_LINES)},
           "eqw_from_population": {"ms_per_step": ms_ew_pop,
                                   "galaxies_per_s": n_gal / (ms_ew_pop * 1e-3),
                                   "with_dW_dlgu_ms_per_step": ms_ew_pop_d,
                                   "equal_to_sed_then_eqw": same},
           "mags_and_gradient": {"ms_per_step": ms_grad, "galaxies_per_s": n_gal / (ms_grad * 1e-3),
                                 "finite": bool(all(torch.isfinite(v).all().item()
                                                    for v in grads.values()))},
           "finite": bool(torch.isfinite(m).all().item() and torch.isfinite(ew).all().item())}
    idx = np.arange(64)
    return res, (ssp, flt, pop.subset(idx), m[:64].cpu().numpy(), ew[:64].cpu().numpy())


def run_forward_model(P, steps, warmup, n_gal=100_000, seed=7):
    """The Section 4.1 forward model at z = 0: parametric SFH -> SFR table ->
    six-band absolute magnitudes (FP32) -> red colour cut (g - r above the
    population median, triweight width 0.05) -> histogram of M_r (40 bins,
    width 0.1); and the same step plus the population gradient of
    sum_k (H_k - target_k)^2 w.r.t. every galaxy's parameters."""
    import torch
    import synth
    ssp = synth.make_ssp(n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4)
    flt = synth.make_filters()
    pop = synth.make_population(n_gal, n_t=100, z_range=(0.1, 1.0), seed=seed)
    pop.z[:] = 0.0
    log(f"forward_model_z0: {n_gal} galaxies at z = 0")
    ssp_h = P.SspBlock.from_synth(ssp, precisions=("fp32",))
    flt_h = P.FilterBank.from_synth(flt)
    dpar = P.DevicePopulation.from_synth(pop, use_params=True)
    ws_f = P.Workspace(P.workspace_size(2, ssp_h, flt_h, n_gal, 100, "fp32"), dpar.device)
    ws_b = P.Workspace(P.workspace_size(3, ssp_h, flt_h, n_gal, 100, "fp32"), dpar.device)
    m = torch.empty((n_gal, 6), dtype=torch.float32, device="cuda")
    bands = torch.empty((n_gal, 2, 6), dtype=torch.float32, device="cuda")
    mom = torch.empty((n_gal, 3, 6), dtype=torch.float32, device="cuda")
    P.mags(ssp_h, flt_h, P.Cosmology(), dpar, workspace=ws_f, out=m)
    colour = (m[:, 1] - m[:, 2]).float()
    spec = P.SummarySpec(band_a=1, band_b=2, colour_cut=float(colour.median()), colour_width=0.05,
                         band_m=2, edges=torch.linspace(float(m[:, 2].min()) - 0.5,
                                                        float(m[:, 2].max()) + 0.5, 41,
                                                        dtype=torch.float64, device="cuda"),
                         mag_width=0.1)
    hist = torch.empty(40, dtype=torch.float64, device="cuda")
    target = torch.full_like(hist, n_gal / 80.0)
    outs = {"sfh_params": torch.empty((5, n_gal), dtype=torch.float64, device="cuda")}
    for k in ("lgmet", "sigma_z", "av", "delta", "bump"):
        outs[k] = torch.empty(n_gal, dtype=torch.float32, device="cuda")

    def forward():
        # SFH generation (the SFR table), photometry, colour cut and histogram
        sfr = P.sfh_table(dpar.t_table, dpar.sfh_params)
        P.mags(ssp_h, flt_h, P.Cosmology(), dpar.with_sfr(sfr), workspace=ws_f, out=m)
        P.pop_summary(m, spec, out=hist)

    def gradient():
        # the parametric history is evaluated inside the weights kernels
        P.mags(ssp_h, flt_h, P.Cosmology(), dpar, with_moments=True, workspace=ws_f, out=m,
               bands_out=bands, moments_out=mom)
        P.pop_summary(m, spec, out=hist)
        mbar = P.pop_summary_vjp(m, spec, 2.0 * (hist - target))
        P.mags_vjp(ssp_h, flt_h, P.Cosmology(), dpar, mbar, bands=bands, moments=mom,
                   workspace=ws_b, outs=outs)

    res = {}
    for name, fn in (("forward", forward), ("forward_grad", gradient)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[name] = {"ms_per_step": ms, "galaxies_per_s": n_gal / (ms * 1e-3)}
    res["red_fraction"] = float(P.pop_summary(m, spec).sum().item()) / n_gal
    res["finite"] = bool(all(torch.isfinite(v).all().item() for v in outs.values()))
    return res


def run_serve(seconds=30.0, rate_hz=200.0):
    """Serving workload: Poisson arrivals at 200 req/s, N ~ logU[1e3, 1e5]
    galaxies per request with a per-request redshift range, 30% asking for
    gradients of the squared residual (FP32), the rest forward on the BF16
    table; then the same trace served request by request through the plain
    calls with the same arithmetic."""
    import torch
    import synth
    import paper_2112_06830_amd as P
    import paper_2112_06830_amd.serve as S
    ssp = P.SspBlock.from_synth(synth.make_ssp(n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4),
                                precisions=("fp32", "bf16"))
    flt = P.FilterBank.from_synth(synth.make_filters())
    t_table = synth.population.make_time_grid(100)
    n_req = int(seconds * rate_hz)
    arrivals, reqs = S.make_trace(n_req, rate_hz=rate_hz, seed=6)
    eng = S.ServeEngine(ssp, flt, t_table, hbm_budget_bytes=48 << 30)
    log("serve: capturing slot graphs")
    eng.warm()
    log(f"serve: {eng.stats['captures_in_warm']} slots captured in {eng.stats['warm_s']:.1f} s; "
        f"replaying {n_req} requests over {seconds:.0f} s")
    eng.start()
    wall = S.replay_trace(eng, arrivals, reqs, timeout_s=300)
    eng.stop()
    res = S.latency_summary(reqs, wall)
    st = eng.stats
    res["engine"] = {
        "slots": st["captures_in_warm"], "warm_s": st["warm_s"],
        "captures_in_loop": st["captures_in_loop"], "evictions": st["evictions"],
        "batches": dict(st["batches"]),
        "mean_batch_galaxies": {k: st["galaxies"][k] / max(st["batches"][k], 1) for k in S.KINDS},
        "slot_fill": {k: st["galaxies"][k] / max(st["slot_galaxies"][k], 1) for k in S.KINDS},
        "grad_batch_galaxies": eng.planner.batch_galaxies.get(S.KIND_GRAD)}
    log(f"serve: p50 {res['p50_ms']:.1f} ms p99 {res['p99_ms']:.1f} ms "
        f"(fwd p99 {res['fwd']['p99_ms']:.1f}, grad p99 {res['grad']['p99_ms']:.1f}), "
        f"{res['throughput_galaxies_per_s']:.3e} gal/s")
    _, reqs2 = S.make_trace(n_req, rate_hz=rate_hz, seed=6)
    log("serve: the same trace request by request")
    base = S.serial_baseline(ssp, flt, eng.cosmo, t_table, arrivals, reqs2)
    log(f"request by request: p50 {base['p50_ms']:.1f} ms p99 {base['p99_ms']:.1f} ms "
        f"(fwd p99 {base['fwd']['p99_ms']:.1f}, grad p99 {base['grad']['p99_ms']:.1f})")
    res["request_by_request"] = base
    torch.cuda.synchronize()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the BF16 1e6, forward+gradient and serving legs")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--pmc-pass", nargs="?", const="fp32_1e5", default=None,
                    choices=("fp32_1e5", "bf16_1e6", "grad_2e5"),
                    help="short run of one leg (default the FP32 forward) plus a calibration "
                         "copy, for rocprofv3 --pmc")
    args = ap.parse_args()

    if args.pmc_pass:
        # A short run for hardware-counter collection: one leg's workload for
        # enough steps that the first (cold) launch weighs little in the
        # trace average, then a device copy of known size whose FETCH_SIZE and
        # WRITE_SIZE calibrate the counters (bytes read = bytes written =
        # CALIBRATION_BYTES).
        import torch
        import paper_2112_06830_amd as P
        if args.pmc_pass == "fp32_1e5":
            run_workload(P, "fwd_fp32_1e5", 100_000, 100, "fp32", 12, 2, seed=3, want_roofline=False)
        elif args.pmc_pass == "bf16_1e6":
            run_workload(P, "fwd_bf16_1e6", 1_000_000, 1000, "bf16", 5, 1, seed=4, want_roofline=False)
        else:
            run_grad(P, 6, 1)
        n = CALIBRATION_BYTES // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"pmc pass done; calibration copy of {CALIBRATION_BYTES} bytes")
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(galaxies shard with no exchange; see the design notes). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    import paper_2112_06830_amd as P

    main_res, (ssp, flt, pop, m32) = run_workload(
        P, "fwd_fp32_1e5", 100_000, 100, "fp32", args.steps, args.warmup, seed=3)
    log(f"fp32 1e5: {main_res['ms_per_step']:.3f} ms/step, gemm {main_res['gemm_ms_per_step']:.3f} ms/step")

    pop16 = m16 = None
    extra = {"fp32_fwd_1e5": {k: main_res[k] for k in ("ms_per_step", "galaxies_per_s",
                                                         "gemm_ms_per_step", "weights_ms_per_step",
                                                         "nnz_mean", "n_lambda_eff_mean")}}
    if not args.no_extra:
        bf, (_, _, pop16, m16) = run_workload(P, "fwd_bf16_1e6", 1_000_000, 1000, "bf16", max(3, args.steps // 4),
                             1, seed=4, want_roofline=True)
        extra["bf16_fwd_1e6"] = {
            "ms_per_step": bf["ms_per_step"], "galaxies_per_s": bf["galaxies_per_s"],
            "gemm_ms_per_step": bf["gemm_ms_per_step"], "weights_ms_per_step": bf["weights_ms_per_step"],
            "mfma_frac_bf16": bf["achieved_tflops"] / PEAK_TFLOPS["bf16"],
            "sfh_read_hbm_frac": (1_000_000 * 1000 * 8 / (bf["weights_ms_per_step"] * 1e-3)) / 1e9 / HBM_PEAK_GBS}
        log(f"bf16 1e6: {bf['ms_per_step']:.3f} ms/step")
        gr = run_grad(P, max(3, args.steps // 4), 1)
        extra["fp32_fwd_grad_2e5"] = gr
        fm = run_forward_model(P, max(3, args.steps // 4), 1)
        extra["forward_model_z0_1e5"] = fm
        log(f"forward model z=0 1e5: {fm['forward']['ms_per_step']:.3f} ms/step, "
            f"with population gradient {fm['forward_grad']['ms_per_step']:.3f} ms/step")
        log(f"fp32 fwd+grad 2e5: {gr['ms_per_step']:.3f} ms/step")
        ad, ad_sample = run_age_dust(P, max(3, args.steps // 4), 1)
        extra["age_dust_fp32_1e5"] = ad
        log(f"age-dependent dust 1e5: {ad['ms_per_step']:.3f} ms/step, gemm {ad['gemm_ms_per_step']:.3f}")
        nb, nb_sample = run_nebular(P, max(3, args.steps // 4), 1)
        extra["nebular_fp32_1e5"] = nb
        log(f"nebular 1e5: mags {nb['mags']['ms_per_step']:.3f} ms/step, "
            f"sed + widths {nb['sed_and_eqw']['ms_per_step']:.3f} ms/step, "
            f"widths from the population {nb['eqw_from_population']['ms_per_step']:.3f} ms/step, "
            f"mags + gradient {nb['mags_and_gradient']['ms_per_step']:.3f} ms/step")
        va, va_sample = run_variants(P, max(3, args.steps // 4), 1)
        extra["variants_transition_mdf_wcdm_1e5"] = va
        log(f"variants 1e5: forward {va['forward']['ms_per_step']:.3f} ms/step, "
            f"with gradient {va['forward_grad']['ms_per_step']:.3f} ms/step")
        extra["serve_poisson_200hz"] = run_serve(seconds=args.serve_seconds)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle on a bounded sample")
        cpu, errors = cpu_baseline(ssp, flt, pop, m32, pop16, m16)
        extra["cpu_baseline_single_thread"] = cpu_baseline_single_thread(ssp, flt, pop)
        if not args.no_extra:
            import oracle
            v_ssp, v_flt, v_pop, v_m, v_w0 = va_sample
            v_ref = oracle.mags(oracle.prepare_inputs(v_ssp, v_flt, v_pop, w0=v_w0))
            errors["variants_transition_mdf_wcdm_1e5"] = band_errors(v_m, v_ref)
            a_ssp, a_flt, a_pop, a_m = ad_sample
            errors["age_dust_fp32_1e5"] = band_errors(
                a_m, oracle.mags(oracle.prepare_inputs(a_ssp, a_flt, a_pop)))
            n_ssp, n_flt, n_pop, n_m, n_ew = nb_sample
            n_inp = oracle.prepare_inputs(n_ssp, n_flt, n_pop)
            errors["nebular_fp32_1e5"] = band_errors(n_m, oracle.mags(n_inp))
            n_sed = oracle.sed(n_inp, apply_dust=True)
            n_ref = np.stack([oracle.nebular.equivalent_width(n_ssp.wave, n_sed, c, h, f)
                              for c, h, f in NEB_LINES], axis=1)
            errors["nebular_eqw_1e5"] = {"max_abs_angstrom": float(np.max(np.abs(n_ew - n_ref))),
                                         "max_rel": float(np.max(np.abs(n_ew - n_ref)
                                                                 / np.maximum(np.abs(n_ref), 1.0)))}
        extra["error_vs_oracle"] = errors

    traffic = read_traffic("fp32", "fp32_1e5")
    achieved = main_res["achieved_tflops"]
    line = {
        "metric": METRIC,
        "value": main_res["galaxies_per_s"],
        "unit": "galaxies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fwd_fp32_1e5: 1e5 galaxies, SSP 12x94x5994 float32 (9e2-2.5e4 A), "
                               "tabulated SFH n_t=100, z~U[0.1,3], 6 Gaussian bands, forward magnitudes",
                   "n_gal": 100_000, "n_t": 100, "n_wave": 5994, "n_met": 12, "n_age": 94,
                   "n_band": 6, "precision": "fp32"},
        "roofline": {"bound": "mfma", "kernel": "k_mags_gemm<fp32>", "achieved": achieved,
                     "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["fp32"],
                     "traffic": traffic,
                     "avg_launch_ms": main_res["gemm_ms_per_launch"],
                     "launches_per_step": main_res["gemm_launches_per_step"],
                     "alg_flops_per_step": main_res["alg_flops_per_step"]},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Shared set-up for the GPU parity tests: seeded synthetic inputs, the oracle
on the same inputs, and device-resident handles.  The GPU side is reached
only through the C ABI (via the thin ctypes binding)."""

from __future__ import annotations

import functools

import numpy as np

import synth

FP32_TOL_MAG = 1e-4     # FP32 path vs the FP64 oracle (workload target)
BF16_TOL_MAG = 5e-3     # BF16 path vs the FP64 oracle (workload target)


@functools.lru_cache(maxsize=None)
def ssp_small():
    return synth.make_ssp(n_wave=1000, wave_lo=1.0e3, wave_hi=2.0e4)


@functools.lru_cache(maxsize=None)
def ssp_large():
    return synth.make_ssp(n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4)


@functools.lru_cache(maxsize=None)
def filters6():
    return synth.make_filters()


def oracle_inputs(ssp, pop, sfr=None):
    import oracle
    return oracle.prepare_inputs(ssp, filters6(), pop, sfr=sfr)


def max_abs(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    both_nan = np.isnan(a) & np.isnan(b)
    d = np.abs(a - b)
    d[both_nan] = 0.0
    return float(np.nanmax(np.where(np.isnan(d), np.inf, d))) if d.size else 0.0

"""Seeded synthetic magnitude tables for the population-summary kernels.

Absolute magnitudes of a z = 0 population in six bands: the r band (index
2) ~ N(-20, 1.5), and adjacent-band colours drawn so that g - r is bimodal
(a blue cloud near 0.35 and a red sequence near 0.75, widths 0.1).  Float32,
like the magnitudes the library returns.
"""

from __future__ import annotations

import numpy as np


def make_mags(n_gal: int, seed: int = 7, n_band: int = 6) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(n_gal)
    r = rng.normal(-20.0, 1.5, n)
    red = rng.uniform(size=n) < 0.45
    gr = np.where(red, rng.normal(0.75, 0.1, n), rng.normal(0.35, 0.1, n))
    out = np.empty((n, n_band))
    out[:, 2] = r
    out[:, 1] = r + gr
    out[:, 0] = out[:, 1] + np.where(red, 1.6, 1.0) + rng.normal(0.0, 0.15, n)
    for b in range(3, n_band):
        out[:, b] = out[:, b - 1] - (0.25 + rng.normal(0.0, 0.05, n)) * np.where(red, 1.2, 0.8)
    return out.astype(np.float32)

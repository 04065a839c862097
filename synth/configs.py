"""The five workloads, named by what they are and sized as stated.

Each entry fixes the grid sizes, population size, redshift range and seeds that
the synthetic generators use.  Sizes follow the published problem statement of
the method; all data are synthetic stand-ins (see the package docstring).
"""

from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class Workload:
    name: str
    n_gal: int
    n_t: int
    n_wave: int
    wave_lo: float
    wave_hi: float
    z_range: tuple
    precision: str           # "fp64" (oracle only), "fp32", "bf16"
    grad: bool
    ssp_seed: int = 1
    pop_seed: int = 2
    description: str = ""


WORKLOADS = {
    "small_fp64": Workload(
        name="small_fp64", n_gal=100, n_t=100, n_wave=1000, wave_lo=1.0e3, wave_hi=2.0e4,
        z_range=(0.1, 1.0), precision="fp64", grad=False, pop_seed=2,
        description="100 galaxies, SSP 12x94x1000 (1e3-2e4 A), n_t=100, z~U[0.1,1]"),
    "fwd_fp32_1e5": Workload(
        name="fwd_fp32_1e5", n_gal=100_000, n_t=100, n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4,
        z_range=(0.1, 3.0), precision="fp32", grad=False, pop_seed=3,
        description="1e5 galaxies, SSP 12x94x5994 fp32 (9e2-2.5e4 A), n_t=100, z~U[0.1,3]"),
    "fwd_bf16_1e6": Workload(
        name="fwd_bf16_1e6", n_gal=1_000_000, n_t=1000, n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4,
        z_range=(0.1, 3.0), precision="bf16", grad=False, pop_seed=4,
        description="1e6 galaxies, BF16 SSP with per-row scales, n_t=1000, z~U[0.1,3]"),
    "grad_fp32_2e5": Workload(
        name="grad_fp32_2e5", n_gal=200_000, n_t=100, n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4,
        z_range=(0.1, 3.0), precision="fp32", grad=True, pop_seed=5,
        description="2e5 galaxies, fp32 forward + adjoint of sum (m - target)^2"),
    "serve_poisson": Workload(
        name="serve_poisson", n_gal=0, n_t=100, n_wave=5994, wave_lo=9.0e2, wave_hi=2.5e4,
        z_range=(0.1, 3.0), precision="mixed", grad=False, pop_seed=6,
        description="Poisson 200 req/s, N~logU[1e3,1e5], per-request z range, 30% with gradients"),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]

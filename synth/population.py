"""Seeded synthetic galaxy populations.

Each galaxy carries the parameters of a parametric star-formation history
(A, tau, alpha, q, t_q) that stands in for the paper's Diffstar model
(Section 3.1), a metallicity-distribution centre and width (Section 3.2), dust
attenuation parameters (Section 3.4) and an observed redshift.  Only random
draws happen here; turning the parameters into a tabulated history is part of
the method and is done by each consumer.

Per-galaxy float parameters are rounded to float32 precision at the source so
that a float32 consumer and a float64 consumer see identical values.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# The shared cosmic-time grid runs from 0.01 Gyr to 13.8 Gyr, which lies past
# the age of a flat LCDM universe with Om0 = 0.3 and h = 0.7 (13.47 Gyr), so
# every observation time falls inside it.
TIME_GRID_START_GYR = 0.01
TIME_GRID_END_GYR = 13.8


def _f32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float64)


@dataclass
class Population:
    """Structure-of-arrays population.

    t_table:    [n_t] shared cosmic-time grid in Gyr (float64)
    sfh_params: [5, n_gal] float64 rows (A [M_sun/yr], tau [Gyr], alpha,
                q, t_q [Gyr])
    z, lgmet, sigma_z, av, delta, bump: [n_gal] float32-representable float64
    targets:    [n_gal, n_band] target magnitudes for the squared-error loss
    lgmet_slope, lg_age_pivot: age dependence of the metallicity centre
    lgmet_old:  [n_gal] old-age metallicity centre of the transition MDF, or
                None for the linear model; mdf_width its width in dex
    """

    t_table: np.ndarray
    sfh_params: np.ndarray
    z: np.ndarray
    lgmet: np.ndarray
    sigma_z: np.ndarray
    av: np.ndarray
    delta: np.ndarray
    bump: np.ndarray
    targets: np.ndarray
    lgmet_slope: float = 0.1
    lg_age_pivot: float = 9.0
    lgmet_old: np.ndarray | None = None
    mdf_width: float = 0.5
    av_old: np.ndarray | None = None
    delta_old: np.ndarray | None = None
    dust_pivot: float = 7.0
    dust_width: float = 0.25
    lgu: np.ndarray | None = None       # ionization distribution centre log10 U_s
    sigma_u: np.ndarray | None = None   # and width in dex
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_gal(self) -> int:
        return int(self.z.shape[0])

    @property
    def n_t(self) -> int:
        return int(self.t_table.shape[0])

    def subset(self, idx) -> "Population":
        idx = np.asarray(idx)
        return Population(
            t_table=self.t_table, sfh_params=self.sfh_params[:, idx].copy(),
            z=self.z[idx].copy(), lgmet=self.lgmet[idx].copy(),
            sigma_z=self.sigma_z[idx].copy(), av=self.av[idx].copy(),
            delta=self.delta[idx].copy(), bump=self.bump[idx].copy(),
            targets=self.targets[idx].copy(), lgmet_slope=self.lgmet_slope,
            lg_age_pivot=self.lg_age_pivot,
            lgmet_old=None if self.lgmet_old is None else self.lgmet_old[idx].copy(),
            mdf_width=self.mdf_width,
            av_old=None if self.av_old is None else self.av_old[idx].copy(),
            delta_old=None if self.delta_old is None else self.delta_old[idx].copy(),
            dust_pivot=self.dust_pivot, dust_width=self.dust_width,
            lgu=None if self.lgu is None else self.lgu[idx].copy(),
            sigma_u=None if self.sigma_u is None else self.sigma_u[idx].copy(),
            seed=self.seed, meta=dict(self.meta))


def make_time_grid(n_t: int) -> np.ndarray:
    return np.linspace(TIME_GRID_START_GYR, TIME_GRID_END_GYR, n_t)


def make_population(n_gal: int, n_t: int = 100, z_range=(0.1, 1.0), seed: int = 2,
                    n_band: int = 6, lgmet_slope: float = 0.1,
                    lg_age_pivot: float = 9.0, mdf: str = "linear",
                    mdf_width: float = 0.5, age_dust: bool = False,
                    dust_pivot: float = 7.0, dust_width: float = 0.25,
                    nebular: bool = False) -> Population:
    """Draw a population with the parameter distributions of the workloads.

    log10 A ~ U[0, 2], tau ~ U[1, 5] Gyr, alpha ~ U[0.5, 3], q ~ U[0, 1],
    t_q ~ U[2, 13] Gyr; lgmet ~ U[-3, -1.7], sigma_Z ~ U[0.1, 0.5];
    A_V ~ U[0, 2], delta ~ U[-0.7, 0.3], bump ~ U[0, 3]; z ~ U[z_range];
    targets ~ N(22, 1) mag per galaxy and band.  mdf="transition" adds an
    old-age centre lgmet_old = lgmet - U[0, 0.6] (older stars more metal-poor)
    for the T_erf transition model, drawn from its own stream so the other
    parameters are those of the linear model with the same seed.
    age_dust=True adds old-star attenuation parameters for the age-dependent
    dust model: A_V,old = A_V * U[0.2, 0.6] (young stars sit behind more dust)
    and delta_old = U[-0.7, 0.3], from their own stream.
    nebular=True adds the ionization distribution of Section 3.3: centre
    log10 U_s ~ U[-3.5, -1.5] and width sigma_u ~ U[0.1, 0.4] dex (the
    paper's example uses 0.25), from their own stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(n_gal)
    log_a = rng.uniform(0.0, 2.0, n)
    tau = rng.uniform(1.0, 5.0, n)
    alpha = rng.uniform(0.5, 3.0, n)
    q = rng.uniform(0.0, 1.0, n)
    t_q = rng.uniform(2.0, 13.0, n)
    sfh_params = np.stack([10.0 ** log_a, tau, alpha, q, t_q]).astype(np.float64)
    lgmet = _f32(rng.uniform(-3.0, -1.7, n))
    sigma_z = _f32(rng.uniform(0.1, 0.5, n))
    av = _f32(rng.uniform(0.0, 2.0, n))
    delta = _f32(rng.uniform(-0.7, 0.3, n))
    bump = _f32(rng.uniform(0.0, 3.0, n))
    z = _f32(rng.uniform(z_range[0], z_range[1], n))
    trng = np.random.Generator(np.random.PCG64(seed + 1000003))
    targets = _f32(trng.normal(22.0, 1.0, (n, n_band)))
    lgmet_old = None
    if mdf == "transition":
        mrng = np.random.Generator(np.random.PCG64(seed + 2000003))
        lgmet_old = _f32(lgmet - mrng.uniform(0.0, 0.6, n))
    elif mdf != "linear":
        raise ValueError(f"unknown mdf model {mdf!r}")
    av_old = delta_old = None
    if age_dust:
        drng = np.random.Generator(np.random.PCG64(seed + 3000003))
        av_old = _f32(av * drng.uniform(0.2, 0.6, n))
        delta_old = _f32(drng.uniform(-0.7, 0.3, n))
    lgu = sigma_u = None
    if nebular:
        urng = np.random.Generator(np.random.PCG64(seed + 4000003))
        lgu = _f32(urng.uniform(-3.5, -1.5, n))
        sigma_u = _f32(urng.uniform(0.1, 0.4, n))
    return Population(t_table=make_time_grid(n_t), sfh_params=np.ascontiguousarray(sfh_params),
                      z=z, lgmet=lgmet, sigma_z=sigma_z, av=av, delta=delta, bump=bump,
                      targets=targets, lgmet_slope=lgmet_slope, lg_age_pivot=lg_age_pivot,
                      lgmet_old=lgmet_old, mdf_width=float(mdf_width), av_old=av_old,
                      delta_old=delta_old, dust_pivot=float(dust_pivot),
                      dust_width=float(dust_width), lgu=lgu, sigma_u=sigma_u, seed=seed)

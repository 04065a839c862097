"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package only draws random numbers and lays out input arrays: the SSP
spectral block, the per-galaxy parameter population, the observed-frame filter
curves and the shared cosmic-time grid.  It contains none of the arithmetic of
the population-synthesis method itself (no star-formation history, no weights,
no attenuation, no photometry); every consumer computes those on its own side.

The paper's workloads use FSPS/MILES SSP tables, Diffstar histories and
LSST-like filters (Section 4.1), none of which ship with this repository, so the
generators below produce stand-ins with the same shapes, units and structure.
"""

from .ssp import make_ssp, make_ssp_nebular, make_line_spectra, SspTable, NEBULAR_LINES
from .population import make_population, Population, TIME_GRID_END_GYR
from .filters import make_filters, FilterSet
from .configs import WORKLOADS, Workload, workload
from .mags import make_mags

__all__ = [
    "make_mags",
    "make_ssp", "make_ssp_nebular", "make_line_spectra", "SspTable", "NEBULAR_LINES",
    "make_population", "Population", "TIME_GRID_END_GYR",
    "make_filters", "FilterSet",
    "WORKLOADS", "Workload", "workload",
]

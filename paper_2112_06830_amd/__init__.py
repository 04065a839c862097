"""MI355X-native hot path of differentiable stellar population synthesis.

The compute lives in libdsps.so (HIP for gfx950, C ABI in include/dsps.h);
this package only marshals arguments.  Importing it loads the library and
raises if it has not been built.
"""

from . import _native
from ._native import DspsError, load as load_library

load_library()

from .api import (Cosmology, DevicePopulation, FilterBank, SspBlock, SummarySpec,  # noqa: E402
                  Workspace, eqw, eqw_pop, mags, mags_ion_tangent, mags_noalloc,
                  mags_residual_vjp, mags_vjp, pop_summary, pop_summary_vjp, profile_enable,
                  profile_read, quantize_bf16, sed, sed_ion_tangent, sfh_table, weights,
                  workspace_size)
from .autograd import DspsMags, PopSummary, dsps_mags  # noqa: E402

__all__ = [
    "Cosmology", "DevicePopulation", "FilterBank", "SspBlock", "Workspace", "DspsError",
    "mags", "quantize_bf16", "sed", "sfh_table", "weights", "workspace_size", "load_library",
    "profile_enable", "profile_read", "mags_vjp", "DspsMags", "dsps_mags",
    "SummarySpec", "pop_summary", "pop_summary_vjp", "PopSummary", "eqw", "sed_ion_tangent",
    "mags_ion_tangent", "eqw_pop", "mags_noalloc", "mags_residual_vjp",
]

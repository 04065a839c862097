"""FP64 CPU oracle for the DSPS hot path (arxiv 2112.06830).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU path is checked against.  Only the test suite, the
smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code, constants or tables with the GPU library and
never imports it; the only code both sides use is the seeded input generator
package ``synth``, which holds none of the method's arithmetic.

Everything is float64 numpy/scipy, dense (no wavelength windowing, no skipping
of zero weights), written step by step in the paper's order:

  cosmology   t(z) and the distance modulus (Section 2.2.1)
  sfh         parametric SFR table, cumulative mass formed and age-bin masses
              (Section 3.1, Eqs. cspsum and mstartot)
  kernels     triweight kernel and its cumulative T_erf (Appendix B)
  mdf         age-dependent metallicity weights (Section 3.2.2, Eq. agedep_mdf)
  dust        Salim-type attenuation with a Drude bump (Section 3.4,
              Eqs. attenuation, salim, kzero, uvbump), and its age-dependent
              form (Section 3.4.1, Eq. agedep_dust_csp)
  photometry  redshifted filter integrals and AB magnitudes (Section 2.2.1,
              Eq. restmag)
  nebular     the ionization axis of the SSP block and emission-line
              equivalent widths (Section 3.3, Eq. nebsed; Section 2.2.2,
              Eq. eqw)
  pipeline    weights, SEDs, magnitudes and BF16 quantisation of the SSP block
  adjoint     hand-written reverse-mode gradient of the magnitudes
  summary     the population summary of the Section 4.1 forward model: a
              red-colour cut and an r-band magnitude histogram, triweight-
              smoothed (Appendix B), and its gradient

Readings of passages that are silent, ambiguous or garbled are stated in the
docstring of the function that takes them.  Parity status: every function here
is pinned by a CPU test against closed forms, invariants, brute force on tiny
inputs or finite differences; none is "parity unpinned".
"""

from . import (constants, cosmology, kernels, sfh, mdf, dust, nebular, photometry, pipeline,
               adjoint)
from .pipeline import (weights, sed, band_sums, mags, quantize_bf16_rne, bf16_to_f32,
                       OracleInputs, prepare_inputs)
from .adjoint import mags_vjp

__all__ = [
    "constants", "cosmology", "kernels", "sfh", "mdf", "dust", "nebular", "photometry", "pipeline",
    "adjoint", "weights", "sed", "band_sums", "mags", "mags_vjp", "quantize_bf16_rne",
    "bf16_to_f32", "OracleInputs", "prepare_inputs",
]

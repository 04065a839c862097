"""ctypes declarations of the libdsps C ABI (include/dsps.h).

Loading fails loudly: there is no fallback implementation of any entry point.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DSPS_LIB", os.path.join(HERE, "libdsps.so"))

DSPS_OK = 0
STATUS_NAMES = {0: "DSPS_OK", -1: "DSPS_ERR_ARG", -2: "DSPS_ERR_SHAPE", -3: "DSPS_ERR_DEVICE",
                -4: "DSPS_ERR_WORKSPACE", -5: "DSPS_ERR_UNSUPPORTED", -6: "DSPS_ERR_ALLOC"}
FP32, BF16 = 0, 1
K0_SALIM, K0_PRINTED = 0, 1
OP_WEIGHTS, OP_SED, OP_MAGS, OP_MAGS_VJP = 0, 1, 2, 3

# Every symbol include/dsps.h declares.
EXPORTS = (
    "dsps_abi_version", "dsps_last_error", "dsps_ssp_create", "dsps_ssp_destroy",
    "dsps_ssp_info", "dsps_filters_create", "dsps_filters_destroy", "dsps_filters_info",
    "dsps_workspace_size", "dsps_sfh_table", "dsps_weights", "dsps_sed", "dsps_mags",
    "dsps_mags_vjp", "dsps_quantize_bf16", "dsps_profile_enable", "dsps_profile_read",
    "dsps_pop_summary_workspace", "dsps_pop_summary", "dsps_pop_summary_vjp",
    "dsps_ssp_create_neb", "dsps_ssp_ion_info", "dsps_eqw", "dsps_eqw_jvp",
    "dsps_sed_ion_tangent", "dsps_mags_ion_tangent", "dsps_eqw_pop", "dsps_eqw_pop_workspace",
    "dsps_mags_noalloc", "dsps_mags_residual_vjp",
)
MAX_ION, MAX_LINES = 16, 16

KERNEL_IDS = {"weights": 0, "mags_gemm": 1, "mags_finalize": 2, "zsort": 3, "sed_gemm": 4,
              "vjp_lbar": 5, "vjp_wbar": 6, "vjp_weights": 7, "summary": 8, "eqw": 9}


class DspsError(RuntimeError):
    def __init__(self, status: int, fn: str, message: str):
        self.status = status
        super().__init__(f"{fn} failed with {STATUS_NAMES.get(status, status)}: {message}")


class Cosmo(ctypes.Structure):
    _fields_ = [("om0", ctypes.c_double), ("w0", ctypes.c_double), ("h", ctypes.c_double)]


class Pop(ctypes.Structure):
    _fields_ = [
        ("n_gal", ctypes.c_int), ("n_t", ctypes.c_int),
        ("t_table", ctypes.c_void_p), ("sfr", ctypes.c_void_p), ("sfh_params", ctypes.c_void_p),
        ("z", ctypes.c_void_p), ("lgmet", ctypes.c_void_p), ("sigma_z", ctypes.c_void_p),
        ("av", ctypes.c_void_p), ("delta", ctypes.c_void_p), ("bump", ctypes.c_void_p),
        ("lgmet_slope", ctypes.c_double), ("lg_age_pivot", ctypes.c_double),
        ("lgmet_old", ctypes.c_void_p), ("mdf_width", ctypes.c_double),
        ("av_old", ctypes.c_void_p), ("delta_old", ctypes.c_void_p),
        ("dust_pivot", ctypes.c_double), ("dust_width", ctypes.c_double),
        ("lgu", ctypes.c_void_p), ("sigma_u", ctypes.c_void_p),
        ("n_live", ctypes.c_void_p),
    ]


class Line(ctypes.Structure):
    _fields_ = [("centre", ctypes.c_double), ("half_width", ctypes.c_double),
                ("fit_half_width", ctypes.c_double)]


SSP_AGE_MAJOR = 4   # dsps_ssp_create: also the age-major float32 table


_LIB = None


def _declare(lib):
    P, I, S, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    IP = ctypes.POINTER(ctypes.c_int)
    sig = {
        "dsps_abi_version": (I, []),
        "dsps_last_error": (ctypes.c_char_p, []),
        "dsps_ssp_create": (I, [I, I, I, P, P, P, P, I, I, PP]),
        "dsps_ssp_create_neb": (I, [I, I, I, I, P, P, P, P, P, I, I, PP]),
        "dsps_ssp_ion_info": (I, [P, IP]),
        "dsps_eqw": (I, [P, P, I, ctypes.POINTER(Line), I, P, P]),
        "dsps_eqw_jvp": (I, [P, P, P, I, ctypes.POINTER(Line), I, P, P, P]),
        "dsps_eqw_pop_workspace": (I, [P, I, ctypes.POINTER(Line), I, I, ctypes.POINTER(S)]),
        "dsps_eqw_pop": (I, [P, ctypes.POINTER(Cosmo), ctypes.POINTER(Pop), I, ctypes.POINTER(Line), I,
                             I, P, P, P, S, P]),
        "dsps_sed_ion_tangent": (I, [P, ctypes.POINTER(Cosmo), ctypes.POINTER(Pop), I, I, P, P, S,
                                     P]),
        "dsps_mags_ion_tangent": (I, [P, P, ctypes.POINTER(Cosmo), ctypes.POINTER(Pop), I, P, P, P,
                                      S, P]),
        "dsps_ssp_destroy": (None, [P]),
        "dsps_ssp_info": (I, [P, IP, IP, IP, IP, IP]),
        "dsps_filters_create": (I, [I, I, P, P, PP]),
        "dsps_filters_destroy": (None, [P]),
        "dsps_filters_info": (I, [P, IP, IP]),
        "dsps_workspace_size": (I, [I, P, P, I, I, I, ctypes.POINTER(S)]),
        "dsps_sfh_table": (I, [P, I, P, I, P, P]),
        "dsps_weights": (I, [P, ctypes.POINTER(Cosmo), ctypes.POINTER(Pop), P, P, P, S, P]),
        "dsps_sed": (I, [P, ctypes.POINTER(Cosmo), ctypes.POINTER(Pop), I, I, P, P, S, P]),
        "dsps_mags": (I, [P, P, ctypes.POINTER(Cosmo), ctypes.POINTER(Pop), I, P, P, P, P, S, P]),
        "dsps_mags_noalloc": (I, [P, P, ctypes.POINTER(Cosmo), ctypes.POINTER(Pop), I, P, P, P, P]),
        "dsps_mags_vjp": (I, [P, P, ctypes.POINTER(Cosmo), ctypes.POINTER(Pop), I, P, P, P,
                              P, P, P, P, P, P, P, P, P, P, P, P, P, S, P]),
        "dsps_mags_residual_vjp": (I, [P, P, ctypes.POINTER(Cosmo), ctypes.POINTER(Pop), P, P, P,
                                       P, P, P, P, P, P, P, P, P, P, P, P, P, S, P]),
        "dsps_quantize_bf16": (I, [P, I, I, P, P, P]),
        "dsps_pop_summary_workspace": (I, [I, I, ctypes.POINTER(S)]),
        "dsps_pop_summary": (I, [P, I, I, I, I, D, D, I, P, I, D, P, P, S, P]),
        "dsps_pop_summary_vjp": (I, [P, I, I, I, I, D, D, I, P, I, D, P, P, P]),
        "dsps_profile_enable": (I, [I]),
        "dsps_profile_read": (I, [I, ctypes.POINTER(ctypes.c_double), IP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args


def _hip_runtimes() -> set:
    """Distinct HIP runtime libraries mapped into this process (Linux)."""
    try:
        with open("/proc/self/maps") as f:
            return {ln.split()[-1] for ln in f if "libamdhip64" in ln and "/" in ln}
    except OSError:
        return set()


def load(path: str | None = None):
    """Load libdsps.so (once).  Raises if the library is missing.

    The library must bind to the HIP runtime that PyTorch already uses: the
    binding hands it PyTorch's device pointers and stream handles, which only
    that runtime instance understands.  torch is therefore imported first, so
    that the library's libamdhip64.so.7 dependency resolves to the copy torch
    has loaded; a second runtime in the process is refused.
    """
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(
            f"libdsps.so not found at {p}; build it with "
            "`python paper_2112_06830_amd/build.py` (hipcc, gfx950). There is no fallback.")
    import torch  # noqa: F401  (loads torch's HIP runtime before ours binds)
    lib = ctypes.CDLL(p, mode=ctypes.RTLD_LOCAL)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError(
            "two HIP runtimes are loaded in this process (" + ", ".join(sorted(runtimes)) + "); "
            "libdsps must share torch's. Import torch before any other HIP library.")
    _declare(lib)
    if path is None:
        _LIB = lib
    return lib


def check(status: int, fn: str):
    if status != DSPS_OK:
        msg = load().dsps_last_error()
        raise DspsError(status, fn, msg.decode() if msg else "")

"""Thin Python binding over the libdsps C ABI.

Argument marshalling only: torch provides device memory and the current
stream, every step of the computation runs in the HIP library.  Function
names follow the C entry points (dsps_weights -> weights, ...).
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N

_PREC = {"fp32": N.FP32, "bf16": N.BF16, N.FP32: N.FP32, N.BF16: N.BF16}
_K0 = {"salim": N.K0_SALIM, "printed": N.K0_PRINTED}


def _lib():
    return N.load()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(x, dtype, device):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)


def _workspace(nbytes: int, device) -> tuple[torch.Tensor | None, int]:
    if nbytes == 0:
        return None, 0
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, off


class SspBlock:
    """Resident SSP block (dsps_ssp_create, or dsps_ssp_create_neb with an
    ionization grid lgu and lum [n_met, n_age, n_u, n_wave])."""

    def __init__(self, lgz, lg_age, wave, lum, precisions=("fp32", "bf16"), k0_reading="salim",
                 age_major=False, lgu=None):
        """age_major also prepares the age-major float32 table that the
        age-dependent attenuation needs (dsps_pop.av_old)."""
        lgz = np.ascontiguousarray(lgz, dtype=np.float64)
        lg_age = np.ascontiguousarray(lg_age, dtype=np.float64)
        wave = np.ascontiguousarray(wave, dtype=np.float64)
        lum = np.ascontiguousarray(lum, dtype=np.float32)
        n_met, n_age, n_wave = lgz.size, lg_age.size, wave.size
        n_u = 1 if lgu is None else int(np.size(lgu))
        if lum.size != n_met * n_age * n_u * n_wave:
            raise ValueError("lum has the wrong size")
        mask = N.SSP_AGE_MAJOR if age_major else 0
        for p in precisions:
            mask |= 1 << _PREC[p]
        torch.cuda.init()
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        if lgu is None:
            rc = _lib().dsps_ssp_create(n_met, n_age, n_wave, lgz.ctypes.data, lg_age.ctypes.data,
                                        wave.ctypes.data, lum.ctypes.data, mask, _K0[k0_reading],
                                        ctypes.byref(h))
            N.check(rc, "dsps_ssp_create")
        else:
            lgu = np.ascontiguousarray(lgu, dtype=np.float64)
            rc = _lib().dsps_ssp_create_neb(n_met, n_age, n_u, n_wave, lgz.ctypes.data,
                                            lg_age.ctypes.data, lgu.ctypes.data, wave.ctypes.data,
                                            lum.ctypes.data, mask, _K0[k0_reading], ctypes.byref(h))
            N.check(rc, "dsps_ssp_create_neb")
        self.handle = h
        self.n_met, self.n_age, self.n_wave, self.n_u = n_met, n_age, n_wave, n_u
        self.wave = wave

    @classmethod
    def from_synth(cls, ssp, **kw):
        lgu = getattr(ssp, "lgu", None)
        if lgu is not None and "precisions" not in kw:
            kw["precisions"] = ("fp32",)
        return cls(ssp.lgz, ssp.lg_age, ssp.wave, ssp.lum, lgu=lgu, **kw)

    def close(self):
        if getattr(self, "handle", None):
            _lib().dsps_ssp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FilterBank:
    """Resident filter set (dsps_filters_create)."""

    def __init__(self, wave, trans):
        wave = np.ascontiguousarray(wave, dtype=np.float64)
        trans = np.ascontiguousarray(trans, dtype=np.float64)
        n_band, n_pts = wave.shape
        h = ctypes.c_void_p()
        rc = _lib().dsps_filters_create(n_band, n_pts, wave.ctypes.data, trans.ctypes.data,
                                        ctypes.byref(h))
        N.check(rc, "dsps_filters_create")
        self.handle = h
        self.n_band, self.n_pts = n_band, n_pts

    @classmethod
    def from_synth(cls, f):
        return cls(f.wave, f.trans)

    def close(self):
        if getattr(self, "handle", None):
            _lib().dsps_filters_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Cosmology:
    om0: float = 0.3
    h: float = 0.7
    w0: float = -1.0

    def c(self):
        return N.Cosmo(self.om0, self.w0, self.h)


@dataclass
class DevicePopulation:
    """Device-resident population (structure of arrays)."""

    t_table: torch.Tensor
    sfr: torch.Tensor | None
    sfh_params: torch.Tensor | None
    z: torch.Tensor
    lgmet: torch.Tensor
    sigma_z: torch.Tensor
    av: torch.Tensor
    delta: torch.Tensor
    bump: torch.Tensor
    lgmet_slope: float = 0.1
    lg_age_pivot: float = 9.0
    lgmet_old: torch.Tensor | None = None   # transition MDF: old-age centre, float32
    mdf_width: float = 0.5
    av_old: torch.Tensor | None = None      # age-dependent attenuation: old-star A_V, delta
    delta_old: torch.Tensor | None = None
    dust_pivot: float = 7.0
    dust_width: float = 0.25
    lgu: torch.Tensor | None = None         # ionization distribution: centre, width
    sigma_u: torch.Tensor | None = None
    # int32 [1] on the device, or None: galaxies at and past it are padding
    # (not read, their output rows left as they were)
    n_live: torch.Tensor | None = None

    @property
    def n_gal(self):
        return int(self.z.shape[0])

    @property
    def n_t(self):
        return int(self.t_table.shape[0])

    @property
    def device(self):
        return self.z.device

    def c(self):
        return N.Pop(self.n_gal, self.n_t, _ptr(self.t_table), _ptr(self.sfr), _ptr(self.sfh_params),
                     _ptr(self.z), _ptr(self.lgmet), _ptr(self.sigma_z), _ptr(self.av),
                     _ptr(self.delta), _ptr(self.bump), self.lgmet_slope, self.lg_age_pivot,
                     _ptr(self.lgmet_old), self.mdf_width, _ptr(self.av_old), _ptr(self.delta_old),
                     self.dust_pivot, self.dust_width, _ptr(self.lgu), _ptr(self.sigma_u),
                     _ptr(self.n_live))

    @classmethod
    def from_synth(cls, pop, device="cuda", sfr=None, use_params=False):
        """Upload a synth.Population.  With use_params the library evaluates
        the parametric history itself; otherwise `sfr` (host or device table)
        is used."""
        d = torch.device(device)
        f32 = lambda a: _dev(a, torch.float32, d)
        if use_params:
            sfr_t, par = None, _dev(pop.sfh_params, torch.float64, d)
        else:
            if sfr is None:
                raise ValueError("give an SFR table or use_params=True")
            sfr_t, par = _dev(sfr, torch.float64, d), None
        return cls(t_table=_dev(pop.t_table, torch.float64, d), sfr=sfr_t, sfh_params=par,
                   z=f32(pop.z), lgmet=f32(pop.lgmet), sigma_z=f32(pop.sigma_z), av=f32(pop.av),
                   delta=f32(pop.delta), bump=f32(pop.bump), lgmet_slope=float(pop.lgmet_slope),
                   lg_age_pivot=float(pop.lg_age_pivot),
                   lgmet_old=(None if getattr(pop, "lgmet_old", None) is None
                              else f32(pop.lgmet_old)),
                   mdf_width=float(getattr(pop, "mdf_width", 0.5)),
                   av_old=(None if getattr(pop, "av_old", None) is None else f32(pop.av_old)),
                   delta_old=(None if getattr(pop, "delta_old", None) is None
                              else f32(pop.delta_old)),
                   dust_pivot=float(getattr(pop, "dust_pivot", 7.0)),
                   dust_width=float(getattr(pop, "dust_width", 0.25)),
                   lgu=(None if getattr(pop, "lgu", None) is None else f32(pop.lgu)),
                   sigma_u=(None if getattr(pop, "sigma_u", None) is None else f32(pop.sigma_u)))

    def with_sfr(self, sfr):
        return DevicePopulation(self.t_table, sfr, None, self.z, self.lgmet, self.sigma_z, self.av,
                                self.delta, self.bump, self.lgmet_slope, self.lg_age_pivot,
                                self.lgmet_old, self.mdf_width, self.av_old, self.delta_old,
                                self.dust_pivot, self.dust_width, self.lgu, self.sigma_u,
                                self.n_live)


def workspace_size(op: int, ssp: SspBlock, filters: FilterBank | None, n_gal: int, n_t: int,
                   precision="fp32") -> int:
    out = ctypes.c_size_t()
    rc = _lib().dsps_workspace_size(op, ssp.handle, filters.handle if filters else None, n_gal, n_t,
                                    _PREC[precision], ctypes.byref(out))
    N.check(rc, "dsps_workspace_size")
    return int(out.value)


def sfh_table(t_table: torch.Tensor, sfh_params: torch.Tensor, stream=None) -> torch.Tensor:
    """dsps_sfh_table: float64 [n_gal, n_t] from params [5, n_gal]."""
    t_table = t_table.contiguous()
    sfh_params = sfh_params.contiguous()
    n_t, n_gal = t_table.shape[0], sfh_params.shape[1]
    out = torch.empty((n_gal, n_t), dtype=torch.float64, device=t_table.device)
    rc = _lib().dsps_sfh_table(_ptr(t_table), n_t, _ptr(sfh_params), n_gal, _ptr(out), _stream(stream))
    N.check(rc, "dsps_sfh_table")
    return out


def weights(ssp: SspBlock, cosmo: Cosmology, pop: DevicePopulation, with_mstar=False, out=None,
            mstar_out=None, stream=None):
    """dsps_weights: W [n_gal, n_met, n_age] float32 (and M_star float64);
    `out` and `mstar_out` may supply the output tensors."""
    w = out if out is not None else torch.empty((pop.n_gal, ssp.n_met, ssp.n_age),
                                                dtype=torch.float32, device=pop.device)
    ms = None
    if with_mstar:
        ms = mstar_out if mstar_out is not None else torch.empty(pop.n_gal, dtype=torch.float64,
                                                                 device=pop.device)
    nbytes = workspace_size(N.OP_WEIGHTS, ssp, None, pop.n_gal, pop.n_t, "fp32")
    buf, off = _workspace(nbytes, pop.device)
    ws = ctypes.c_void_p(buf.data_ptr() + off) if buf is not None else None
    c, p = cosmo.c(), pop.c()
    rc = _lib().dsps_weights(ssp.handle, ctypes.byref(c), ctypes.byref(p), _ptr(w), _ptr(ms), ws, nbytes,
                             _stream(stream))
    N.check(rc, "dsps_weights")
    return (w, ms) if with_mstar else w


def sed(ssp: SspBlock, cosmo: Cosmology, pop: DevicePopulation, apply_dust=True, precision="fp32",
        out=None, stream=None):
    """dsps_sed: rest-frame SED [n_gal, n_wave] float32 (into `out` if given)."""
    if out is None:
        out = torch.empty((pop.n_gal, ssp.n_wave), dtype=torch.float32, device=pop.device)
    nbytes = workspace_size(N.OP_SED, ssp, None, pop.n_gal, pop.n_t, precision)
    buf, off = _workspace(nbytes, pop.device)
    c, p = cosmo.c(), pop.c()
    ws = ctypes.c_void_p(buf.data_ptr() + off) if buf is not None else None
    rc = _lib().dsps_sed(ssp.handle, ctypes.byref(c), ctypes.byref(p), int(bool(apply_dust)),
                         _PREC[precision], _ptr(out), ws, nbytes, _stream(stream))
    N.check(rc, "dsps_sed")
    return out


def sed_ion_tangent(ssp: SspBlock, cosmo: Cosmology, pop: DevicePopulation, wrt="lgu",
                    apply_dust=True, stream=None):
    """dsps_sed_ion_tangent: dSED/d(lgu) or dSED/d(sigma_u) [n_gal, n_wave]."""
    out = torch.empty((pop.n_gal, ssp.n_wave), dtype=torch.float32, device=pop.device)
    nbytes = workspace_size(N.OP_SED, ssp, None, pop.n_gal, pop.n_t, "fp32")
    buf, off = _workspace(nbytes, pop.device)
    c, p = cosmo.c(), pop.c()
    ws = ctypes.c_void_p(buf.data_ptr() + off) if buf is not None else None
    rc = _lib().dsps_sed_ion_tangent(ssp.handle, ctypes.byref(c), ctypes.byref(p),
                                     int(bool(apply_dust)), {"lgu": 0, "sigma_u": 1}[wrt], _ptr(out),
                                     ws, nbytes, _stream(stream))
    N.check(rc, "dsps_sed_ion_tangent")
    return out


def mags_ion_tangent(ssp: SspBlock, filters: FilterBank, cosmo: Cosmology, pop: DevicePopulation,
                     wrt="lgu", bands: torch.Tensor | None = None,
                     workspace: Workspace | None = None, stream=None) -> torch.Tensor:
    """dsps_mags_ion_tangent: dm/d(lgu) or dm/d(sigma_u) [n_gal, n_band]
    float32, per galaxy.  bands: the forward band sums (mags(...,
    with_bands=True)), or None to run the forward pass inside."""
    out = torch.empty((pop.n_gal, filters.n_band), dtype=torch.float32, device=pop.device)
    if workspace is None:
        workspace = Workspace(workspace_size(N.OP_MAGS, ssp, filters, pop.n_gal, pop.n_t, "fp32"),
                              pop.device)
    b = None if bands is None else bands.to(torch.float32).contiguous()
    c, p = cosmo.c(), pop.c()
    rc = _lib().dsps_mags_ion_tangent(ssp.handle, filters.handle, ctypes.byref(c), ctypes.byref(p),
                                      {"lgu": 0, "sigma_u": 1}[wrt], _ptr(b), _ptr(out),
                                      workspace.ptr(), workspace.nbytes, _stream(stream))
    N.check(rc, "dsps_mags_ion_tangent")
    return out


def _lines(lines):
    lines = list(lines)
    return (N.Line * len(lines))(*[N.Line(float(c), float(h), float(f)) for c, h, f in lines]), len(lines)


def eqw(ssp: SspBlock, sed: torch.Tensor, lines, dsed: torch.Tensor | None = None, stream=None):
    """dsps_eqw: equivalent widths [n_gal, n_line] float32 (rest-frame
    Angstrom) of SEDs [n_gal, n_wave] on the block's grid, for lines given as
    (centre, half_width, fit_half_width) triples.  With an SED tangent dsed
    (dsps_eqw_jvp) returns (widths, their tangent)."""
    sed = sed.to(torch.float32).contiguous()
    arr, n_line = _lines(lines)
    out = torch.empty((sed.shape[0], n_line), dtype=torch.float32, device=sed.device)
    if dsed is None:
        rc = _lib().dsps_eqw(ssp.handle, _ptr(sed), int(sed.shape[0]), arr, n_line, _ptr(out),
                             _stream(stream))
        N.check(rc, "dsps_eqw")
        return out
    dsed = dsed.to(torch.float32).contiguous()
    dout = torch.empty_like(out)
    rc = _lib().dsps_eqw_jvp(ssp.handle, _ptr(sed), _ptr(dsed), int(sed.shape[0]), arr, n_line,
                             _ptr(out), _ptr(dout), _stream(stream))
    N.check(rc, "dsps_eqw_jvp")
    return out, dout


def eqw_pop(ssp: SspBlock, cosmo: Cosmology, pop: DevicePopulation, lines, apply_dust=True,
            wrt: str | None = None, stream=None):
    """dsps_eqw_pop: equivalent widths [n_gal, n_line] straight from the
    population (the SED is computed only near the lines); with wrt ("lgu" or
    "sigma_u") returns (widths, their derivative)."""
    arr, n_line = _lines(lines)
    w = -1 if wrt is None else {"lgu": 0, "sigma_u": 1}[wrt]
    nbytes = ctypes.c_size_t()
    N.check(_lib().dsps_eqw_pop_workspace(ssp.handle, pop.n_gal, arr, n_line, w, ctypes.byref(nbytes)),
            "dsps_eqw_pop_workspace")
    buf, off = _workspace(int(nbytes.value), pop.device)
    ws = ctypes.c_void_p(buf.data_ptr() + off) if buf is not None else None
    out = torch.empty((pop.n_gal, n_line), dtype=torch.float32, device=pop.device)
    dout = torch.empty_like(out) if w >= 0 else None
    c, p = cosmo.c(), pop.c()
    rc = _lib().dsps_eqw_pop(ssp.handle, ctypes.byref(c), ctypes.byref(p), int(bool(apply_dust)), arr,
                             n_line, w, _ptr(out), _ptr(dout), ws, int(nbytes.value), _stream(stream))
    N.check(rc, "dsps_eqw_pop")
    return out if w < 0 else (out, dout)


class Workspace:
    """Reusable workspace for repeated calls of one shape."""

    def __init__(self, nbytes: int, device):
        self.nbytes = nbytes
        self.buf, self.off = _workspace(nbytes, device)

    def ptr(self):
        return None if self.buf is None else ctypes.c_void_p(self.buf.data_ptr() + self.off)


def mags(ssp: SspBlock, filters: FilterBank, cosmo: Cosmology, pop: DevicePopulation,
         precision="fp32", with_bands=False, with_moments=False, workspace: Workspace | None = None,
         out=None, bands_out=None, moments_out=None, stream=None):
    """dsps_mags: apparent AB magnitudes [n_gal, n_band] float32.

    with_bands also returns the band sums [n_gal, 2, n_band]; with_moments
    (float32 only) returns (mags, bands, moments) with the dust moments
    [n_gal, 3, n_band], which is what mags_vjp needs to skip its forward pass.
    """
    nb = filters.n_band
    m = out if out is not None else torch.empty((pop.n_gal, nb), dtype=torch.float32, device=pop.device)
    bands = mom = None
    if with_bands or with_moments:
        bands = bands_out if bands_out is not None else torch.empty(
            (pop.n_gal, 2, nb), dtype=torch.float32, device=pop.device)
    if with_moments:
        mom = moments_out if moments_out is not None else torch.empty(
            (pop.n_gal, 3, nb), dtype=torch.float32, device=pop.device)
    if workspace is None:
        workspace = Workspace(workspace_size(N.OP_MAGS, ssp, filters, pop.n_gal, pop.n_t, precision),
                              pop.device)
    c, p = cosmo.c(), pop.c()
    rc = _lib().dsps_mags(ssp.handle, filters.handle, ctypes.byref(c), ctypes.byref(p),
                          _PREC[precision], _ptr(m), _ptr(bands), _ptr(mom), workspace.ptr(),
                          workspace.nbytes, _stream(stream))
    N.check(rc, "dsps_mags")
    if with_moments:
        return m, bands, mom
    return (m, bands) if with_bands else m


def mags_noalloc(ssp: SspBlock, filters: FilterBank, cosmo: Cosmology, pop: DevicePopulation,
                 out: torch.Tensor, precision="fp32", bands_out: torch.Tensor | None = None,
                 moments_out: torch.Tensor | None = None, stream=None):
    """dsps_mags_noalloc: dsps_mags on the library's fixed per-device scratch,
    allocating nothing; the caller passes the outputs (out [n_gal, n_band],
    optionally bands_out [n_gal, 2, n_band] and moments_out [n_gal, 3,
    n_band], float32).  Calls that overlap on one device race."""
    c, p = cosmo.c(), pop.c()
    rc = _lib().dsps_mags_noalloc(ssp.handle, filters.handle, ctypes.byref(c), ctypes.byref(p),
                                  _PREC[precision], _ptr(out), _ptr(bands_out), _ptr(moments_out),
                                  _stream(stream))
    N.check(rc, "dsps_mags_noalloc")
    return out


def quantize_bf16(x: torch.Tensor, stream=None):
    """dsps_quantize_bf16: (bf16 bits as int16 [rows, cols], scale float32 [rows])."""
    x = x.to(torch.float32).contiguous()
    rows, cols = x.shape
    q = torch.empty((rows, cols), dtype=torch.int16, device=x.device)
    s = torch.empty(rows, dtype=torch.float32, device=x.device)
    rc = _lib().dsps_quantize_bf16(_ptr(x), rows, cols, _ptr(q), _ptr(s), _stream(stream))
    N.check(rc, "dsps_quantize_bf16")
    return q, s


def profile_enable(on: bool = True):
    """Start (clearing earlier records) or stop kernel-level event timing."""
    N.check(_lib().dsps_profile_enable(int(bool(on))), "dsps_profile_enable")


def profile_read(kernel: str):
    """(total milliseconds, launches) recorded for one kernel since enabling."""
    ms = ctypes.c_double()
    n = ctypes.c_int()
    N.check(_lib().dsps_profile_read(N.KERNEL_IDS[kernel], ctypes.byref(ms), ctypes.byref(n)),
            "dsps_profile_read")
    return float(ms.value), int(n.value)


def mags_vjp(ssp: SspBlock, filters: FilterBank, cosmo: Cosmology, pop: DevicePopulation,
             mags_bar: torch.Tensor, bands: torch.Tensor | None = None,
             moments: torch.Tensor | None = None,
             want=("sfr", "sfh_params", "lgmet", "lgmet_old", "sigma_z", "av", "delta", "bump",
                   "av_old", "delta_old", "lgu", "sigma_u"),
             workspace: Workspace | None = None, outs: dict | None = None, stream=None) -> dict:
    """dsps_mags_vjp: cotangents of the population inputs for a magnitude
    cotangent mags_bar [n_gal, n_band] (float32 path).  bands and moments come
    from mags(..., with_moments=True) on the same inputs, or are both None
    (the forward pass then runs inside).  With the age-dependent attenuation
    there are no moments: bands alone (from mags) or nothing.  `outs` may
    supply preallocated output tensors (then `want` is ignored)."""
    n, d = pop.n_gal, pop.device
    aged = pop.av_old is not None
    if aged and moments is not None:
        raise ValueError("the age-dependent attenuation takes no moments")
    if not aged and (bands is None) != (moments is None):
        raise ValueError("bands and moments are given together or not at all")
    mags_bar = mags_bar.to(device=d, dtype=torch.float32).contiguous()
    if bands is not None:
        bands = bands.to(device=d, dtype=torch.float32).contiguous()
    if moments is not None:
        moments = moments.to(device=d, dtype=torch.float32).contiguous()
    out = _grad_outputs(ssp, pop, want, outs)
    if workspace is None:
        workspace = Workspace(workspace_size(N.OP_MAGS_VJP, ssp, filters, n, pop.n_t, "fp32"), d)
    c, p = cosmo.c(), pop.c()
    rc = _lib().dsps_mags_vjp(ssp.handle, filters.handle, ctypes.byref(c), ctypes.byref(p), N.FP32,
                              _ptr(mags_bar), _ptr(bands), _ptr(moments), *_grad_ptrs(out),
                              workspace.ptr(), workspace.nbytes, _stream(stream))
    N.check(rc, "dsps_mags_vjp")
    return out


_GRAD_ORDER = ("sfr", "sfh_params", "lgmet", "lgmet_old", "sigma_z", "av", "delta", "bump",
               "av_old", "delta_old", "lgu", "sigma_u")


def _grad_ptrs(out):
    return [_ptr(out.get(k)) for k in _GRAD_ORDER]


def _grad_outputs(ssp, pop, want, outs):
    """Gradient tensors by input name: `outs` as given, else fresh ones for
    the names in `want` the population carries."""
    n, d = pop.n_gal, pop.device
    aged = pop.av_old is not None
    out = {}
    if outs is not None:
        out = dict(outs)
        want = ()
    if "sfr" in want:
        out["sfr"] = torch.empty((n, pop.n_t), dtype=torch.float64, device=d)
    if "sfh_params" in want and pop.sfh_params is not None:
        out["sfh_params"] = torch.empty((5, n), dtype=torch.float64, device=d)
    for k in ("lgmet", "sigma_z", "av", "delta", "bump"):
        if k in want:
            out[k] = torch.empty(n, dtype=torch.float32, device=d)
    if "lgmet_old" in want and pop.lgmet_old is not None:
        out["lgmet_old"] = torch.empty(n, dtype=torch.float32, device=d)
    for k in ("av_old", "delta_old"):
        if k in want and aged:
            out[k] = torch.empty(n, dtype=torch.float32, device=d)
    for k in ("lgu", "sigma_u"):
        if k in want and getattr(ssp, "n_u", 1) > 1:
            out[k] = torch.empty(n, dtype=torch.float32, device=d)
    return out


def mags_residual_vjp(ssp: SspBlock, filters: FilterBank, cosmo: Cosmology, pop: DevicePopulation,
                      target: torch.Tensor, wt: torch.Tensor | None = None,
                      want=_GRAD_ORDER, workspace: Workspace | None = None, out=None,
                      outs: dict | None = None, stream=None):
    """dsps_mags_residual_vjp: float32 magnitudes [n_gal, n_band] and the
    gradients of sum wt (m - target)^2 (wt None: all 1) in one call that
    sorts and computes the weights once.  Returns (mags, gradients by
    input name); `out` and `outs` may supply the output tensors."""
    n, d = pop.n_gal, pop.device
    target = target.to(device=d, dtype=torch.float32).contiguous()
    if wt is not None:
        wt = wt.to(device=d, dtype=torch.float32).contiguous()
    m = out if out is not None else torch.empty((n, filters.n_band), dtype=torch.float32, device=d)
    grads = _grad_outputs(ssp, pop, want, outs)
    if workspace is None:
        workspace = Workspace(workspace_size(N.OP_MAGS_VJP, ssp, filters, n, pop.n_t, "fp32"), d)
    c, p = cosmo.c(), pop.c()
    rc = _lib().dsps_mags_residual_vjp(ssp.handle, filters.handle, ctypes.byref(c), ctypes.byref(p),
                                       _ptr(target), _ptr(wt), _ptr(m), *_grad_ptrs(grads),
                                       workspace.ptr(), workspace.nbytes, _stream(stream))
    N.check(rc, "dsps_mags_residual_vjp")
    return m, grads


@dataclass
class SummarySpec:
    """Population summary of the Section 4.1 forward model: colour
    m[band_a] - m[band_b] cut at colour_cut (triweight-smoothed over
    colour_width), histogram of m[band_m] over `edges` (smoothed over
    mag_width).  Zero widths give the hard cut and the plain histogram."""
    band_a: int = 1
    band_b: int = 2
    colour_cut: float = 0.55
    colour_width: float = 0.05
    band_m: int = 2
    edges: torch.Tensor | None = None      # [n_bins + 1] float64, device
    mag_width: float = 0.1

    def args(self, mags):
        e = self.edges.to(device=mags.device, dtype=torch.float64).contiguous()
        return e, (int(mags.shape[1]), int(self.band_a), int(self.band_b), float(self.colour_cut),
                   float(self.colour_width), int(self.band_m))


def pop_summary(mags: torch.Tensor, spec: SummarySpec, out=None, workspace=None, stream=None):
    """dsps_pop_summary: the summary histogram [n_bins] float64."""
    mags = mags.to(dtype=torch.float32).contiguous()
    edges, (nb, a, b, cut, cw, bm) = spec.args(mags)
    n, n_bins = int(mags.shape[0]), int(edges.numel()) - 1
    hist = out if out is not None else torch.empty(n_bins, dtype=torch.float64, device=mags.device)
    if workspace is None:
        size = ctypes.c_size_t()
        N.check(_lib().dsps_pop_summary_workspace(n, n_bins, ctypes.byref(size)),
                "dsps_pop_summary_workspace")
        workspace = Workspace(size.value, mags.device)
    rc = _lib().dsps_pop_summary(_ptr(mags), n, nb, a, b, cut, cw, bm, _ptr(edges), n_bins,
                                 float(spec.mag_width), _ptr(hist), workspace.ptr(),
                                 workspace.nbytes, _stream(stream))
    N.check(rc, "dsps_pop_summary")
    return hist


def pop_summary_vjp(mags: torch.Tensor, spec: SummarySpec, hist_bar: torch.Tensor, out=None,
                    stream=None):
    """dsps_pop_summary_vjp: d(sum_k hist_bar_k hist_k)/d mags [n_gal, n_band]."""
    mags = mags.to(dtype=torch.float32).contiguous()
    edges, (nb, a, b, cut, cw, bm) = spec.args(mags)
    n, n_bins = int(mags.shape[0]), int(edges.numel()) - 1
    hb = hist_bar.to(device=mags.device, dtype=torch.float64).contiguous()
    g = out if out is not None else torch.empty_like(mags)
    rc = _lib().dsps_pop_summary_vjp(_ptr(mags), n, nb, a, b, cut, cw, bm, _ptr(edges), n_bins,
                                     float(spec.mag_width), _ptr(hb), _ptr(g), _stream(stream))
    N.check(rc, "dsps_pop_summary_vjp")
    return g

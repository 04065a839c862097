"""The C-ABI library loads and exports every symbol include/dsps.h declares.
Host-side argument checks are exercised without touching a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsps.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dsps_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2112_06830_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.fail("libdsps.so is not built: run `python paper_2112_06830_amd/build.py`")
    return _native.load()


def test_header_declares_the_hot_path():
    names = _declared_functions()
    for fn in ("dsps_weights", "dsps_sed", "dsps_mags", "dsps_mags_vjp", "dsps_sfh_table",
               "dsps_quantize_bf16", "dsps_workspace_size"):
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2112_06830_amd import _native
    names = _declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_native.EXPORTS)


def test_abi_version_and_error_string(lib):
    assert lib.dsps_abi_version() == 9
    assert isinstance(lib.dsps_last_error(), bytes)


def test_host_side_argument_checks_fail_before_any_launch(lib):
    from paper_2112_06830_amd import _native as N
    h = ctypes.c_void_p()
    dummy = (ctypes.c_double * 4)(1.0, 2.0, 3.0, 4.0)
    lum = (ctypes.c_float * 4)(1.0, 1.0, 1.0, 1.0)
    # n_met = 0 is a shape error
    rc = lib.dsps_ssp_create(0, 2, 2, dummy, dummy, dummy, lum, 1, 0, ctypes.byref(h))
    assert rc == -2 and b"n_met" in lib.dsps_last_error()
    # bad precision mask
    rc = lib.dsps_ssp_create(1, 2, 2, dummy, dummy, dummy, lum, 0, 0, ctypes.byref(h))
    assert rc == -1
    # descending wavelengths
    desc = (ctypes.c_double * 2)(2.0, 1.0)
    rc = lib.dsps_ssp_create(1, 2, 2, dummy, dummy, desc, lum, 1, 0, ctypes.byref(h))
    assert rc == -1 and b"ascending" in lib.dsps_last_error()
    # non-uniform filter grid is unsupported; too many bands is a shape error
    fw = (ctypes.c_double * 3)(1000.0, 1100.0, 1300.0)
    ft = (ctypes.c_double * 3)(0.1, 0.2, 0.3)
    rc = lib.dsps_filters_create(1, 3, fw, ft, ctypes.byref(h))
    assert rc == -5
    rc = lib.dsps_filters_create(9, 3, fw, ft, ctypes.byref(h))
    assert rc == -2
    # NULL handles
    size = ctypes.c_size_t()
    assert lib.dsps_workspace_size(2, None, None, 10, 10, 0, ctypes.byref(size)) == -1
    c = N.Cosmo(0.3, -1.0, 0.7)
    p = N.Pop()
    assert lib.dsps_mags(None, None, ctypes.byref(c), ctypes.byref(p), 0, None, None, None, None, 0,
                         None) == -1
    # zero-size requests are no-ops
    assert lib.dsps_sfh_table(None, 10, None, 0, None, None) == 0
    assert lib.dsps_quantize_bf16(None, 0, 5, None, None, None) == 0


def test_library_binds_to_torch_hip_runtime():
    """Importing the package first (before torch) must still leave a single
    HIP runtime in the process: the library shares torch's."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2112_06830_amd as P\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l and '/' in l}\n"
            "print(len(libs))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_pop_summary_host_checks(lib):
    size = ctypes.c_size_t()
    assert lib.dsps_pop_summary_workspace(10000, 32, ctypes.byref(size)) == 0
    assert size.value >= 8 * 32 * 5                     # 5 partial blocks of 2048 galaxies
    assert lib.dsps_pop_summary_workspace(10, 0, ctypes.byref(size)) == -2
    assert lib.dsps_pop_summary_workspace(10, 4097, ctypes.byref(size)) == -2
    d = ctypes.c_double
    dummy = ctypes.c_void_p(1)
    # band index out of range, negative width, n_bins 0: rejected before any launch
    assert lib.dsps_pop_summary(dummy, 10, 6, 6, 2, d(0.5), d(0.1), 2, dummy, 8, d(0.1), dummy,
                                dummy, 1 << 20, None) == -1
    assert lib.dsps_pop_summary(dummy, 10, 6, 1, 2, d(0.5), d(-0.1), 2, dummy, 8, d(0.1), dummy,
                                dummy, 1 << 20, None) == -1
    assert lib.dsps_pop_summary(dummy, 10, 6, 1, 2, d(0.5), d(0.1), 2, dummy, 0, d(0.1), dummy,
                                dummy, 1 << 20, None) == -2
    assert lib.dsps_pop_summary_vjp(dummy, 0, 6, 1, 2, d(0.5), d(0.1), 2, dummy, 8, d(0.1), None,
                                    None, None) == 0


def test_host_side_checks_of_the_ionization_axis_and_line_widths(lib):
    from paper_2112_06830_amd import _native as N
    h = ctypes.c_void_p()
    d = (ctypes.c_double * 4)(1.0, 2.0, 3.0, 4.0)
    lum = (ctypes.c_float * 16)(*([1.0] * 16))
    # too many ionization points
    rc = lib.dsps_ssp_create_neb(1, 1, 17, 2, d, d, d, d, lum, 1, 0, ctypes.byref(h))
    assert rc == -2 and b"n_u" in lib.dsps_last_error()
    # the axis is float32 only
    rc = lib.dsps_ssp_create_neb(1, 1, 2, 2, d, d, d, d, lum, 3, 0, ctypes.byref(h))
    assert rc == -5
    # descending ionization grid; missing grid
    desc = (ctypes.c_double * 2)(-1.0, -2.0)
    rc = lib.dsps_ssp_create_neb(1, 1, 2, 2, d, d, desc, d, lum, 1, 0, ctypes.byref(h))
    assert rc == -1 and b"lgu" in lib.dsps_last_error()
    rc = lib.dsps_ssp_create_neb(1, 1, 2, 2, d, d, None, d, lum, 1, 0, ctypes.byref(h))
    assert rc == -1
    # equivalent widths: NULL handle, bad line counts
    line = (N.Line * 1)(N.Line(5000.0, 20.0, 100.0))
    assert lib.dsps_eqw(None, None, 4, line, 1, None, None) == -1
    n_u = ctypes.c_int()
    assert lib.dsps_ssp_ion_info(None, ctypes.byref(n_u)) == -1

"""The host code of the library (handle creation, workspace sizing, planning,
argument checks, every compute entry point's host side) under the address and
undefined-behaviour sanitizers: tests/host_check.cpp, built with the sanitizers
on the host compilation only by `python paper_2112_06830_amd/build.py
--host-check` (also part of the build entry point), runs end to end on the
GPU."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BINARY = os.path.join(ROOT, "paper_2112_06830_amd", "dsps_host_check")


def test_host_code_under_address_and_ub_sanitizers():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(BINARY), \
        "build it with `python paper_2112_06830_amd/build.py --host-check`"
    print("[gpu] host check under ASan/UBSan", flush=True)
    sys.stdout.flush()
    env = dict(os.environ)
    # leaks of the HIP runtime's own host allocations at exit are not ours
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    res = subprocess.run([BINARY], env=env, capture_output=True, text=True, timeout=150)
    assert res.returncode == 0, (res.stdout[-2000:], res.stderr[-4000:])
    assert "host check passed" in res.stdout

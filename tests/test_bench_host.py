"""Host-side pieces of bench.py that decide what its JSON line reports: the
count of rest wavelengths the filter set can see (the n_lambda,eff in the
roofline's algorithmic flops, 2 nnz(W_g) n_lambda,eff(z_g) per galaxy), the
gate that reports HBM traffic only for the kernel source its counters were
taken on, and the refusal of more than one GPU.  No GPU is touched."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_effective_wavelengths_count_points_inside_the_redshifted_window():
    # a rest grid point lambda is seen when obs_lo <= lambda (1 + z) <= obs_hi,
    # both ends included; counted point by point against the binary searches
    rng = np.random.default_rng(11)
    wave = np.sort(rng.uniform(900.0, 25000.0, 400))
    z = np.concatenate([[0.0, 1.0, 40.0], rng.uniform(0.0, 3.0, 60)])
    obs_lo, obs_hi = 3600.0, 9700.0
    got = bench.effective_wavelengths(wave, z, obs_lo, obs_hi)
    for k, zk in enumerate(z):
        lo, hi = obs_lo / (1.0 + zk), obs_hi / (1.0 + zk)
        want = sum(1 for w in wave if lo <= w <= hi)
        assert got[k] == want, (k, zk)
    assert got[2] == 0   # at z = 40 the window lies below the grid


def test_effective_wavelengths_include_grid_points_on_the_window_edges():
    wave = np.array([1000.0, 2000.0, 3000.0, 4000.0, 5000.0])
    n = bench.effective_wavelengths(wave, np.array([0.0, 1.0]), 2000.0, 4000.0)
    assert list(n) == [3, 2]   # z = 0: 2000, 3000, 4000; z = 1: 1000, 2000


def test_code_hash_ignores_comments_but_not_code():
    src = "int f(int x) {\n  return x + 1;  // one\n}\n/* block\n comment */\n"
    same = "// header\nint f(int x) {\n\n  return x + 1;  // another\n}\n"
    other = "int f(int x) {\n  return x + 2;\n}\n"
    assert bench._code_only(src) == bench._code_only(same)
    assert bench._code_only(src) != bench._code_only(other)


def test_traffic_is_reported_only_for_the_profiled_source(monkeypatch):
    assert bench.read_traffic("fp32", "no_such_workload") is None
    monkeypatch.setattr(bench, "gemm_source_hash", lambda: "0" * 16)
    assert bench.read_traffic("fp32", "fp32_1e5") is None


def test_committed_counter_summary_matches_the_committed_kernels():
    # the HBM traffic in the bench line comes from this summary; it must have
    # been taken on the GEMM sources as they stand
    t = bench.read_traffic("fp32", "fp32_1e5")
    assert t is not None and t > 1e9


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""

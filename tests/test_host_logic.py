"""Host-side logic of the benchmark driver (CPU only): the algorithmic byte
counts the roofline divides by, the mixed-vs-FP64 agreement summary, the
source-hash gate on stored counter traffic, and the one-GPU refusal."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_sweep_bytes_per_launch():
    """16 B per complex128 element read once, the basis vector once, and
    41 B per column (nrm, acc read and write, mask, coefficient); 8 B per
    complex64 element in the mixed sweep."""
    N, M = 10000, 409600
    assert bench.sweep_bytes(N, M) == 65552953600
    assert bench.sweep32_bytes(N, M) == 32784873600
    assert bench.sweep_bytes(1, 1) == 16 + 16 + 41
    assert bench.sweep32_bytes(2, 3) == 8 * 6 + 16 + 41 * 3


def test_agreement_summary():
    piv0 = np.array([3, 1, 4, 0, 5])
    err0 = np.array([1.0, 0.5, 0.25, 0.125, 0.0625, 0.03])
    a = bench.agreement(piv0, err0, piv0.copy(), err0 * (1 + 1e-12))
    assert a["pivot_agreement"] == 1.0 and a["first_divergence"] is None
    assert a["err_rel_deviation_max"] < 2e-12
    b = bench.agreement(piv0, err0, np.array([3, 1, 9, 0]), err0[:5] * np.array([1, 1, 1.5, 1, 1]))
    assert b["first_divergence"] == 2 and abs(b["pivot_agreement"] - 0.75) < 1e-15
    assert abs(b["err_rel_deviation_max"] - 0.5) < 1e-15 and b["k"] == 4 and b["k_ref"] == 5
    assert abs(b["common_pivots"] - 3 / 5) < 1e-15 and b["err_rel_deviation_median"] < 1e-15


def test_measured_traffic_is_gated_by_source_hash():
    """Stored counter traffic is reported only for the kernel source it was
    measured on, for launches with the number of vectors it was measured at
    (and never for an unknown kernel)."""
    assert bench.measured_traffic("k_unknown", "chirp_10k_409600_c128") is None
    key = ("k_sweep_z", "chirp_10k_409600_c128")
    src, h, vec, value = bench.MEASURED_TRAFFIC[key]
    assert bench.measured_traffic(*key, vec) == value
    saved = bench.MEASURED_TRAFFIC[key]
    try:
        bench.MEASURED_TRAFFIC[key] = (src, "0" * 16, vec, value)
        assert bench.measured_traffic(*key, vec) is None
    finally:
        bench.MEASURED_TRAFFIC[key] = saved
    lk = ("k_sweep_c_look", "chirp_10k_409600_c64")
    v = bench.MEASURED_TRAFFIC[lk][2]
    assert bench.measured_traffic(*lk, v) is not None
    assert bench.measured_traffic(*lk, v + 1) is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_run_spread():
    """Median and interquartile range of the timed runs (numpy's linear
    percentiles): for 1, 2, 3, 4 s the quartiles are 1.75 and 3.25."""
    import bench
    r = bench.run_spread([(t, None) for t in (4.0, 1.0, 3.0, 2.0)])
    assert r["run_times_s"] == [4.0, 1.0, 3.0, 2.0]
    assert r["median_s"] == 2.5 and r["iqr_s"] == 1.5

"""bench.py's host-side arithmetic: the FLOPs of counted tests, fractions of
peak, and the committed rocprofv3 figures it reports only while the kernel
source they were measured on is unchanged."""

import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402  (module object only: its helper names start with test_)

COUNTS = {"sphere_tests": 1000, "plane_tests": 10, "exec_sphere_tests": 40,
          "exec_plane_tests": 10}


def test_test_flops_counts_sixteen_per_sphere_and_twelve_per_plane():
    assert bench.test_flops(COUNTS, executed=False) == 16 * 1000 + 12 * 10
    assert bench.test_flops(COUNTS, executed=True) == 16 * 40 + 12 * 10


def test_fraction_of_peak():
    # 157.3e9 FLOPs in 1 ms is exactly the 157.3 TFLOP/s peak
    assert bench.frac_of_peak(157.3e9, 1.0) == pytest.approx(1.0, rel=1e-12)
    assert bench.frac_of_peak(157.3e9, 4.0) == pytest.approx(0.25, rel=1e-12)


def test_executed_fp32_rate_and_absence():
    assert bench.executed_fp32({}, 0.07) is None
    r = bench.executed_fp32({"executed_fp32_flops_per_launch": 1.4e9}, 0.07)
    assert r["tflops"] == pytest.approx(20.0, abs=1e-3)
    assert r["frac"] == pytest.approx(20.0 / 157.3, abs=1e-4)


def _write(path, **kw):
    with open(path, "w") as f:
        json.dump(kw, f)
    return str(path)


def test_measured_profile_only_for_the_same_source_and_workload(tmp_path):
    digest = bench.source_digest(bench.KERNEL_SOURCES)
    good = _write(tmp_path / "p.json", workload="w", kernel_digest=digest, bytes_per_launch=7)
    assert bench.measured_profile(good, bench.KERNEL_SOURCES, "w")["bytes_per_launch"] == 7
    # another workload, another source, no file, no JSON: nothing is reported
    assert bench.measured_profile(good, bench.KERNEL_SOURCES, "other") == {}
    stale = _write(tmp_path / "s.json", workload="w", kernel_digest="0" * 16, bytes_per_launch=7)
    assert bench.measured_profile(stale, bench.KERNEL_SOURCES, "w") == {}
    assert bench.measured_profile(str(tmp_path / "none.json"), bench.KERNEL_SOURCES, "w") == {}
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert bench.measured_profile(str(bad), bench.KERNEL_SOURCES, "w") == {}


def test_source_digest_follows_every_byte(tmp_path):
    a = tmp_path / "a.txt"
    a.write_bytes(b"kernel source")
    rel = os.path.relpath(str(a), bench.ROOT)
    d0 = bench.source_digest([rel])
    a.write_bytes(b"kernel sourcf")
    assert bench.source_digest([rel]) != d0
    assert len(d0) == 16

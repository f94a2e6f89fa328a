"""Host logic of bench.py: the algorithmic operation count behind the
roofline, the hash that ties stored counter data to the kernel sources they
were measured on, the stored counter summary itself, and the refusal of more
than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("m,ops", [(0, 6), (1, 10), (8, 38), (32, 134)])
def test_algorithmic_ops_is_4m_plus_6(m, ops):
    # 2m window terms, 2m+1 row sums, 5 for the update and projection
    assert bench.algorithmic_ops(m, 0) == ops
    assert bench.algorithmic_ops(m, 1) == ops


@pytest.mark.parametrize("m", [0, 1, 8, 32])
def test_algorithmic_flops(m):
    # constant kernel: adds only, plus mul, fma (2), add in the update
    assert bench.algorithmic_flops(m, 0) == 4 * m + 5
    # Gaussian: m of the window terms and the 2m+1 row sums are fmas
    assert bench.algorithmic_flops(m, 1) == 7 * m + 6


@pytest.mark.parametrize("R2,ops", [(9, 16.0), (16, 19.5), (25, 22.0), (64, 31.5)])
def test_split_window_ops(R2, ops):
    """Lane-ops per site-step of the four-column kernel's shared running
    sums: at m = 8 the disc uses the half-widths 0, 3, 5, 6, 7, 8, so a
    lane's row costs 2m + 2 = 18 running-sum additions plus 4 x 5 window
    additions for its 4 columns (4.5 + 5 per site), then 2m + 1 = 17 row
    additions and 5 for the update: 31.5 against the outward sums' 38."""
    m = int(R2 ** 0.5)
    assert bench.split_window_ops(R2) == ops
    assert bench.split_window_ops(R2) < bench.algorithmic_ops(m, 0)


def test_roofline_labels_in_source():
    """The roofline object names its unit in lane-operations, carries the
    FLOP-based fraction against the published 157.3 TFLOP/s, the LDS
    fractions against both measured read rates and the binding pipe."""
    src = open(os.path.join(ROOT, "bench.py")).read()
    for key in ('"unit": "T lane-ops/s"', '"frac_flops"', '"peak_tflops": peak_tf',
                '"frac_measured_8B"', '"frac_measured_16B"', '"binding_pipe"',
                '"us_per_time_step"', '"arithmetic"'):
        assert key in src, key
    assert bench.FP32_PEAK_TFLOPS == 157.3
    assert bench.FP64_PEAK_TFLOPS == 78.6
    assert abs(bench.VALU_PEAK_TOPS - 78.6432) < 1e-3


def test_source_hash_tracks_the_kernel_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash("k_resident4h")
    assert len(h) == 16 and int(h, 16) >= 0
    assert bench.kernel_source_hash("k_resident4h") == h
    # copies of the sources: comments and blank lines added keep the hash,
    # one changed token changes it
    csrc = os.path.join(ROOT, "paper_2310_10750_amd", "csrc")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    fake = tmp_path / "paper_2310_10750_amd" / "csrc"
    fake.mkdir(parents=True)

    def copy(extra):
        for f in bench.KERNEL_SOURCES["k_resident4h"]:
            data = open(os.path.join(csrc, f), "rb").read()
            if f == "kern_rowrun_impl.h":
                data += extra
            (fake / f).write_bytes(data)
        return bench.kernel_source_hash("k_resident4h")

    assert copy(b"\n// a note\n/* and\n   another */\n\n") == h
    assert copy(b"\nstatic_assert(true);\n") != h


def test_stored_counters_are_consistent():
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    e = d["k_resident4h"]
    assert e["bytes_per_launch"] == pytest.approx(e["fetch_bytes"] + e["write_bytes"], abs=2)
    assert e["algorithmic_bytes"] == 2 * 4096 * 128 * 128 * 4
    # HBM: within a few percent of reading and writing each state once
    assert 0.99 < e["bytes_per_launch"] / e["algorithmic_bytes"] < 1.05
    if "lds_bytes_per_launch" in e:
        assert e["lds_bytes_per_launch"] == e["lds_load_bytes"] + e["lds_store_bytes"]


def test_stored_counters_only_for_their_workload_and_sources(monkeypatch):
    e = bench.stored_counters("k_resident4h", "C3")
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["k_resident4h"]
    if d["source_hash"] == bench.kernel_source_hash("k_resident4h"):
        assert e is not None and e["bytes_per_launch"] == d["bytes_per_launch"]
        assert bench.stored_traffic("k_resident4h", "C3") == d["bytes_per_launch"]
    else:
        assert e is None
    assert bench.stored_counters("k_resident4h", "V3") is None
    assert bench.stored_counters("k_rowrun", "C3") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k="k_resident4h": "0" * 16)
    assert bench.stored_counters("k_resident4h", "C3") is None
    assert bench.stored_traffic("k_resident4h", "C3") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_host_info_names_the_cpu():
    h = bench.host_info()
    assert h["logical_cpus"] == os.cpu_count()
    assert h["usable_cpus"] is None or 1 <= h["usable_cpus"] <= h["logical_cpus"]

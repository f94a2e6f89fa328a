"""The peak-measurement program built beside the library runs on the GPU and
reports rates that are positive and within the chip's published peaks (a
measurement above a published peak would mean a mis-counted kernel)."""
import json
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PEAKS = os.path.join(ROOT, "paper_2310_10750_amd", "peaks", "nlch_peaks")


@pytest.mark.skipif(not os.path.exists(PEAKS), reason="peaks program not built")
def test_measured_peaks_are_within_published_ones():
    print("running %s" % PEAKS, flush=True)
    r = subprocess.run([PEAKS], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    d = json.loads(r.stdout.strip().splitlines()[-1])
    cus = d["cus"]
    assert cus > 0
    clock = 2.4e9
    # published: HBM 8 TB/s; FP32 157.3 TFLOP/s = 78.6 T lane-ops/s (FMA as one);
    # FP64 78.6 TFLOP/s = 39.3 T FMA lane-ops/s
    assert 0.5 < d["hbm_copy_tbs"] <= 8.0 * 1.02
    assert 0.0 < d["fp32_add_tops"] <= cus * 128 * clock / 1e12 * 1.05
    assert 0.0 < d["fp32_fma_tops"] <= cus * 128 * clock / 1e12 * 1.05
    assert 0.0 < d["fp64_fma_tops"] <= cus * 64 * clock / 1e12 * 1.05
    # wider LDS reads are not slower than narrower ones
    assert 0.0 < d["lds_read_b64_tbs"] <= d["lds_read_b128_tbs"] * 1.05

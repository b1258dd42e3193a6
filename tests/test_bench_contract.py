"""Host-side checks of bench.py's contract (no GPU): the one-GPU refusal, and
the HBM traffic figure tied to the kernel source it was measured on and to the
committed rocprofv3 summary it comes from."""
import os
import re
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_matches_profile_and_source():
    t = bench.measured_traffic()
    if t is None:
        # bench.py then reports roofline.traffic as null, as it must
        pytest.skip("the X-engine source changed since its FETCH/WRITE counters were taken")
    with open(os.path.join(ROOT, "profiles", "xeng_mfma_128_i8_c3.md")) as fh:
        prof = fh.read()
    assert bench.TRAFFIC_SHA1 in prof
    # the counter readings (KiB per dispatch) and the calibration factors of the summary
    row = re.search(r"\| xeng_mfma_128_kernel<0> \(mean of 4\) \| ([\d ]+) \| ([\d ]+) \|", prof)
    fetch_kib, write_kib = (float(g.replace(" ", "")) for g in row.groups())
    assert "FETCH x 2.000" in prof and "WRITE x 1.000" in prof
    want = 2.0 * fetch_kib * 1024 + 1.0 * write_kib * 1024
    assert abs(t - want) / want < 1e-5
    total = re.search(r"total ([\d.]+) GB \(bench `roofline.traffic`\)", prof)
    assert abs(t / 1e9 - float(total.group(1))) < 0.01


def test_traffic_is_withheld_for_another_source(monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_SHA1", "0" * 40)
    assert bench.measured_traffic() is None

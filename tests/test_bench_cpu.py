"""Host-side checks of bench.py's reporting (no GPU): the one-GPU limit, the
roofline and HBM arithmetic, and that stale counter figures are not used."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1910_02639_amd import profiling  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_roofline_arithmetic():
    # 1e9 tests of 8 lane-ops in 1 ms: 8e12 lane-ops/s against the
    # non-packed VALU issue rate of 256 CU x 4 SIMD x 16 lanes x 2.4 GHz.
    r = bench.roofline(1.0, 1e9, 8, "k_sweep<fp32>", "no-such-workload")
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9
    assert abs(r["achieved"] - 8.0) < 1e-9
    assert abs(r["frac"] - 8.0 / 39.3216) < 1e-12
    assert r["bound"] == "alu" and r["traffic"] is None


def test_search_hbm_bytes():
    # 44 compulsory bytes per particle plus 4 per list entry.
    r = bench.search_hbm(1000, 5000, 1.0)
    assert r["algorithmic_bytes"] == 1000 * 44 + 4 * 5000
    assert abs(r["achieved_GBs"] - 64000 / 1e-3 / 1e9) < 1e-9


def test_stored_traffic_matches_the_sources_or_is_ignored():
    """Counter bytes are used only when they were taken on the current search
    sources; a stale hash makes bench.py report null."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    d = json.load(open(p))
    e = d["sweep_kernel"]["Batch64"]
    t = bench.load_traffic("sweep_kernel", "Batch64")
    if e["source_hash"] == profiling.source_hash():
        assert t == e["bytes_per_launch"]
        m = bench.hbm_measured({"sweep_kernel": 2.0, "place_kernel": 1.0}, "Batch64")
        assert abs(m["k_sweep"]["GB_s"] - t / 2e-3 / 1e9) < 1e-6
    else:
        assert t is None
    assert bench.load_traffic("sweep_kernel", "no-such-workload") is None

"""Host-side logic of bench.py that runs without a GPU: the one-GPU guard
and the rule that measured HBM traffic is reported only while the kernel
and layout sources are those the counters were taken with."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout.strip() == ""


def test_traffic_follows_the_source_digest(monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    entry = rec["k_gs_vel_s/interface"]
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: rec["sources_sha256"])
    assert bench.measured_traffic("k_gs_vel_s", "interface") == entry["bytes_per_launch"]
    assert bench.measured_traffic("k_gs_vel_s", "no_such_form") is None
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: "0" * 64)
    assert bench.measured_traffic("k_gs_vel_s", "interface") is None


def test_traffic_record_is_consistent():
    """Every kernel entry carries fetched + written bytes that add up, at a
    plausible share of the algorithmic bytes of the roofline kernel."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert len(rec["sources_sha256"]) == 64
    kernels = {k: v for k, v in rec.items() if isinstance(v, dict)}
    assert "k_gs_vel_s/interface" in kernels
    for k, v in kernels.items():
        assert v["bytes_per_launch"] == pytest.approx(v["fetch_bytes"] + v["write_bytes"], rel=1e-9), k
        assert v["avg_us"] > 0, k
    # 81/4 B per interior vertex of the 257^3 lattice per colour-phase launch
    alg = 81 / 4 * 255 ** 3
    assert 1.0 <= kernels["k_gs_vel_s/interface"]["bytes_per_launch"] / alg < 2.0

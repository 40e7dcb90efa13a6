"""Host logic of the benchmark (no GPU): the roofline arithmetic of a kernel's event
timings, the guard that drops counter traffic once a kernel's sources have changed since
the counters were taken, the committed counter summary, and the one-GPU refusal."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_hop_roofline_arithmetic():
    # 4 launches, 10 ms and 40 GB in total: 2.5 ms and 10 GB per launch, 4000 GB/s
    r = bench.hop_roofline({"kernel": "no_such_kernel", "ms": 10.0, "launches": 4, "bytes": 4e10})
    assert r["avg_launch_ms"] == 2.5
    assert r["algorithmic_bytes_per_launch"] == 1e10
    assert r["achieved"] == pytest.approx(4000.0)
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert r["frac"] == pytest.approx(0.5)
    assert r["traffic"] is None and r["traffic_rate_frac"] is None


def _summary(path, kernel, src, digest, nbytes=7.5e9):
    with open(path, "w") as f:
        json.dump({kernel: {"bytes_per_launch": nbytes, "sources": [src], "sources_sha256": digest,
                            "profile": "a_profile.md"}}, f)


def test_traffic_follows_the_sources(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "traffic.json"
    _summary(summary, "k<f16,inv,R32>", str(src), digest)
    monkeypatch.setattr(bench, "TRAFFIC", str(summary))  # absolute: os.path.join keeps it
    t = bench.measured_traffic("k<f16,inv,R32>")
    assert t["bytes_per_launch"] == 7.5e9 and "a_profile.md" in t["source"]
    assert bench.measured_traffic("k<f16,plain,R32>") is None
    r = bench.hop_roofline({"kernel": "k<f16,inv,R32>", "ms": 3.0, "launches": 2, "bytes": 8e9})
    assert r["traffic"] == 7.5e9
    assert r["traffic_rate_frac"] == pytest.approx(7.5e9 / 1.5e-3 / 1e9 / 8000.0, rel=1e-3)
    # an edited kernel: the counters no longer describe it
    src.write_text("// kernel source, edited\n")
    assert bench.measured_traffic("k<f16,inv,R32>") is None
    assert bench.hop_roofline({"kernel": "k<f16,inv,R32>", "ms": 3.0, "launches": 2, "bytes": 8e9})["traffic"] is None


def test_committed_traffic_summary_is_well_formed():
    path = os.path.join(ROOT, bench.TRAFFIC)
    with open(path) as f:
        rec = json.load(f)
    assert rec
    for kernel, e in rec.items():
        assert e["bytes_per_launch"] > 0, kernel
        assert len(e["sources_sha256"]) == 64, kernel
        for s in e["sources"]:
            assert os.path.exists(os.path.join(ROOT, s)), (kernel, s)
        assert os.path.exists(os.path.join(ROOT, "profiles", e["profile"])), (kernel, e["profile"])


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""

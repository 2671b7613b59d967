"""CPU: the host-side logic of bench.py -- the algorithmic byte count the
roofline divides by, the traffic record lookup (reported only while the
kernel sources hash as they did when the counters were taken), and the
one-GPU refusal."""

import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_stage_bytes_by_hand():
    # N = 3, nq1 = 5: per element and slice 3 fields x 16 nodes x 8 B x
    # (read Q_in, write Q_out, write res, read res in 4 of 5 stages) = 1459.2 B;
    # per element geometry (6 x 25 + 12 x 5) x 8 B + 8 int32 = 1712 B
    # per element and slice: Q read and written every stage, the residual
    # read in 4 and written in 4 of the 5 stages: 3 * 16 * 8 * 3.6 B
    assert bench.stage_bytes(1, 1, 3, 5) == pytest.approx(1382.4 + 1712)
    assert bench.stage_bytes(4096, 64, 3, 5) == pytest.approx(4096 * (64 * 1382.4 + 1712))
    # FP32-bulk: values are 4 bytes, the int32 offsets stay 32 B
    assert bench.stage_bytes(1, 1, 3, 5, word=4) == pytest.approx(691.2 + 840 + 32)


def test_traffic_record_follows_the_sources(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("x = a * b;  // kernel v1\n")
    (tmp_path / "profiles").mkdir()
    rec = {"kernel": "k<double>", "workload": "w", "fetch_bytes_per_launch": 300,
           "write_bytes_per_launch": 200, "sources": ["k.hip"],
           "sources_sha1": hashlib.sha1(b"x=a*b;").hexdigest()}   # code, no comments or blanks
    (tmp_path / "profiles" / "hbm_traffic.json").write_text(json.dumps({"records": [rec]}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k<double>", "w") == 500
    assert bench.measured_traffic("k<double>", "other") is None
    assert bench.measured_traffic("other", "w") is None
    src.write_text("/* the product */\nx = a * b;   // reworded comment\n")
    assert bench.measured_traffic("k<double>", "w") == 500      # comments only: still valid
    src.write_text("x = a * c;  // kernel v1\n")    # the code changed since the counters
    assert bench.measured_traffic("k<double>", "w") is None


def test_four_array_count_by_hand():
    # the scope table's count for the 128x128 workload: 4 x 48 values x 8 B per
    # element and slice, (6 x 25 + 12 x 5) x 8 B of geometry per element
    assert bench.stage_bytes_4(16384, 256, 3, 5) == 16384 * (256 * 1536 + 1680)
    assert bench.stage_bytes_4(16384, 256, 3, 5) == pytest.approx(6.47e9, rel=1e-3)
    r = bench.roofline("k", 8e9, 1.0, bytes_4=4e9)
    assert r["frac_4_state_arrays"] == pytest.approx(0.5)
    assert "frac_4_state_arrays" not in bench.roofline("k", 8e9, 1.0)


def test_alu_roofline_by_hand():
    # the scope table's flop count at N = 3, nq1 = 5: volume 3,180 + mass
    # inverse 2,235 + surface 2,224 + update 192; the volume part by hand:
    # per column and field group 4 (N+1)^2 + nq1 (4 (N+1) + 2) FMAs and 2 nq1
    # products, 5 columns, 2 groups
    vol = 2 * 5 * (2 * (4 * 16 + 5 * (4 * 4 + 2)) + 2 * 5)
    inv = 3 * (2 * (2 * 5 * 16 + 2 * 25 * 4) + 25)
    assert (vol, inv) == (3180, 2235)
    assert bench.FLOPS_PER_ELEMENT_STAGE[(3, 5)] == vol + inv + 2224 + 192
    r = bench.roofline_alu(157.3e9, 1.0, 157.3)
    assert r["bound"] == "alu" and r["frac"] == pytest.approx(1.0)
    assert r["frac_of_unpacked_rate"] == pytest.approx(2.0)


def test_roofline_fields():
    r = bench.roofline("k", 8e9, 1.0, traffic=4e9)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(8000.0) and r["frac"] == pytest.approx(1.0)
    assert r["traffic_frac"] == pytest.approx(0.5)
    assert bench.roofline("k", 8e9, 2.0)["traffic_frac"] is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_cpu_baseline_all_cores_reports_its_sample():
    """The all-cores oracle baseline runs whole slices in worker processes
    and states its core count, host and sample."""
    import bench
    b = bench.cpu_baseline_all_cores("wadg4", slices_per_worker=1)
    assert b["kind"] == "oracle" and b["unit"] == "grid-point-steps/s"
    assert 1 <= b["cores"] <= 16 and b["value"] > 0
    assert "wadg4" in b["sample"] and b["nproc"] >= 1 and b["host_cpu"]

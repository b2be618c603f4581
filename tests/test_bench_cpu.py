"""Host logic of bench.py (no GPU): the algorithmic bytes behind the
roofline, the rule that counter traffic is reported only for the kernel
sources it was measured on, and the one-GPU guard."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_of_the_headline_products():
    """100k terms x 200k documents, 20 M nonzeros, k = 50, float32, steady
    state nnz(U) = 50 000 and nnz(V) = 100 000, written out term by term."""
    # V half: A by documents (value + index per nonzero, 8-byte offsets), U's
    # entries (value + topic byte, 4-byte offsets), V_pre written once
    v = (20_000_000 * 8 + 200_001 * 8) + (50_000 * 5 + 100_001 * 4) + 200_000 * 50 * 4
    # U half: A by terms, V's entries, U_pre and the kept raw product A V
    u = (20_000_000 * 8 + 100_001 * 8) + (100_000 * 5 + 200_001 * 4) + 2 * 100_000 * 50 * 4
    assert bench.spmm_algorithmic_bytes(200_000, 100_000, 20_000_000, 50_000, 50, 4, False) == v
    assert bench.spmm_algorithmic_bytes(100_000, 200_000, 20_000_000, 100_000, 50, 4, True) == u
    assert round(v / 1e6, 2) == 202.25 and round(u / 1e6, 2) == 202.10


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    rec = {"kernel_sha": bench.kernels_sha(),
           "stages": {"spmm_v": {"fetch_bytes": 300.0, "write_bytes": 40.0}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.read_traffic("spmm_v") == 340.0
    assert bench.read_traffic("spmm_u") is None  # stage not measured
    rec["kernel_sha"] = "0" * 16  # counters of other kernel sources
    f.write_text(json.dumps(rec))
    assert bench.read_traffic("spmm_v") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.read_traffic("spmm_v") is None


def test_committed_traffic_record_has_the_read_fields():
    with open(os.path.join(ROOT, "profiles", "spmm_traffic_100kx200k.json")) as fh:
        rec = json.load(fh)
    assert len(rec["kernel_sha"]) == 16
    for stage in ("spmm_v", "spmm_u"):
        s = rec["stages"][stage]
        assert s["fetch_bytes"] > 0 and s["write_bytes"] > 0
    cal = rec["copy_calibration"]
    assert cal["fetch_scale"] > 0 and cal["write_scale"] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""

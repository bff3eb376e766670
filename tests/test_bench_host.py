"""Host-side checks of bench.py (no GPU): it refuses more than one GPU with a
message, and it reports the counted HBM traffic only for the kernel sources
the counters were taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "8"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_is_consistent():
    # the committed counter record: reported only while it matches the
    # kernel sources, and then self-consistent
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    if rec["source_sha256_16"] != bench.kernel_source_hash():
        assert bench.measured_traffic("32") is None
        return
    for key in ("32", "64"):
        r = rec[key]
        assert bench.measured_traffic(key) == r["bytes_per_launch"] == r["fetch_bytes"] + r["write_bytes"]
        alg = bench.STEP_IMPL_BYTES[int(key)] * 16384 * 16384 // 2
        assert r["algorithmic_read_bytes"] == r["algorithmic_write_bytes"] == alg
    assert bench.measured_traffic("two_kernel_32") == rec["two_kernel_32"]["bytes_per_step"]
    # two steps per launch: one read and one write of the state per launch
    for key in ("two_step_32", "two_step_32_mrt"):
        r = rec[key]
        assert bench.measured_traffic(key) == r["bytes_per_launch"] == r["fetch_bytes"] + r["write_bytes"]
        alg = bench.TWO_STEP_IMPL_BYTES[32] * 16384 * 16384
        assert r["algorithmic_read_bytes"] == r["algorithmic_write_bytes"] == alg


def test_traffic_withheld_for_other_sources(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    rec["source_sha256_16"] = "0" * 16
    other = tmp_path / "traffic.json"
    other.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(other))
    assert bench.measured_traffic("32") is None
    assert bench.measured_traffic("64") is None

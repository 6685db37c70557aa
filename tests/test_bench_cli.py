"""bench.py's command-line contract on the host, without a GPU.

- More than one GPU is refused with a message and exit status 2.
- The committed HBM-traffic record has its calibration fields, and the
  bench takes it only while the stage kernel's sources hash to the recorded
  value.
"""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_is_keyed_to_the_stage_sources():
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    ent = rec["rain-3d-q3-64x64x32-fp32"]["stage"]
    for k in ("csrc_hash", "bytes_per_launch", "fetch_kib", "write_kib", "fetch_scale", "write_scale"):
        assert k in ent
    want = ent["fetch_kib"] * 1024 * ent["fetch_scale"] + ent["write_kib"] * 1024 * ent["write_scale"]
    assert abs(ent["bytes_per_launch"] - want) < 1e-6 * want
    got = bench.traffic_for("stage", "rain-3d-q3-64x64x32-fp32")
    assert got == (ent["bytes_per_launch"] if ent["csrc_hash"] == bench.csrc_hash() else None)

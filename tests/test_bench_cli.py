"""bench.py on the CPU: the one-GPU contract and the traffic record lookup
(no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_traffic_record_lookup(monkeypatch):
    """The recorded HBM traffic is reported only for the kernel source, cell
    count and unknowns per cell it was measured on."""
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    monkeypatch.setattr(bench, "layer_source_hash", lambda: rec["source_sha256"])
    assert bench.recorded_traffic(rec["cells"], 3) == rec["bytes_per_launch"]
    assert bench.recorded_traffic(rec["cells"], 4) is None       # measured on nv = 3
    assert bench.recorded_traffic(rec["cells"] + 1, 3) is None   # another grid
    monkeypatch.setattr(bench, "layer_source_hash", lambda: "0" * 64)
    assert bench.recorded_traffic(rec["cells"], 3) is None       # the kernel changed since
    # the per-launch figure is the scaled fetch plus the scaled write
    assert rec["bytes_per_launch"] == rec["fetch_bytes"] + rec["write_bytes"]
    assert rec["algorithmic_bytes"] == rec["cells"] * (2 * 64 * 2 + 6 * 16 * 2)

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


def test_traffic_record_lookup(monkeypatch, tmp_path):
    """The recorded HBM traffic of a learned layer is reported only for the
    kernel source, cell count and unknowns per cell it was measured on."""
    rec = {"kernels": [dict(layer=1, cells=1048576, nv=3, source_sha256="a" * 64, bytes_per_launch=123,
                            fetch_bytes=100, write_bytes=23)]}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    monkeypatch.setattr(bench, "layer_source_hash", lambda: "a" * 64)
    assert bench.recorded_traffic(1, 1048576, 3) == 123
    assert bench.recorded_traffic(2, 1048576, 3) is None         # another layer
    assert bench.recorded_traffic(1, 1048576, 4) is None         # measured on nv = 3
    assert bench.recorded_traffic(1, 1048577, 3) is None         # another grid
    monkeypatch.setattr(bench, "layer_source_hash", lambda: "0" * 64)
    assert bench.recorded_traffic(1, 1048576, 3) is None         # the kernel changed since


def test_layer_method_bytes():
    """The method's bytes per cell of the three learned layers: nv x nv BF16
    edge blocks (no padding), BF16 activations, FP32 r, FP64 z2."""
    assert bench.layer_method_bytes(1, 3) == 128 + 6 * 9 * 2 + 128
    assert bench.layer_method_bytes(0, 3) == 12 + 108 + 128
    assert bench.layer_method_bytes(2, 3) == 128 + 108 + 12 + 24
    assert bench.layer_method_bytes(1, 4) == 128 + 6 * 16 * 2 + 128

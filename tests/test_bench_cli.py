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


def test_spmv_traffic_record_follows_its_own_source(monkeypatch, tmp_path):
    """The FP64 BSR product's record is keyed to the source file of its
    kernel, not to that of the learned layers."""
    rec = {"kernels": [dict(layer="spmv", cells=1048576, nv=3, source_sha256="b" * 64, bytes_per_launch=77)]}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    monkeypatch.setattr(bench, "layer_source_hash", lambda: "a" * 64)
    monkeypatch.setattr(bench, "spmv_source_hash", lambda: "b" * 64)
    assert bench.recorded_traffic("spmv", 1048576, 3) == 77
    monkeypatch.setattr(bench, "spmv_source_hash", lambda: "a" * 64)
    assert bench.recorded_traffic("spmv", 1048576, 3) is None


def test_copy_reference_uses_the_largest_dispatches(tmp_path):
    """The scale of a counter comes from the large reference copy alone,
    not from small device copies of the same kernel elsewhere in the run."""
    import sqlite3
    for name, counter, big in (("f.db", "FETCH_SIZE", 524288.0), ("w.db", "WRITE_SIZE", 1048576.0)):
        c = sqlite3.connect(tmp_path / name)
        c.execute("create table counters_collection (kernel_name text, grid_size int, counter_name text, value real)")
        rows = [("__amd_rocclr_copyBuffer", 512, counter, 3.0)] * 5 + [("__amd_rocclr_copyBuffer", 131072, counter, big)] * 3
        for key, k in ((0, "void cptr::k_lrn_layer_first<3, true, false, short, float, float>(int)"),
                       (1, "void cptr::k_lrn_layer_col<3, false, false, short, float, float>(int)"),
                       (2, "void cptr::k_lrn_layer_col<3, false, true, short, float, float>(int)"),
                       (3, "void cptr::k_bsr_spmv_sliced<3, float, false>(int)")):
            rows.append((k, 4096, counter, 1024.0 * (key + 1)))
        c.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
        c.commit()
        c.close()
    old = bench.TRAFFIC_FILE
    bench.TRAFFIC_FILE = str(tmp_path / "out.json")
    try:
        rec = bench.record_traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"), 1048576, 3)
    finally:
        bench.TRAFFIC_FILE = old
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    by = {k["layer"]: k for k in rec["kernels"]}
    assert by["spmv"]["fetch_bytes"] == 4096 * 1024 * 2 and by["spmv"]["write_bytes"] == 4096 * 1024
    assert by[0]["bytes_per_launch"] == 1024 * 1024 * 3


def test_layer_method_bytes():
    """The method's bytes per cell of the three learned layers inside a solve:
    nv x nv BF16 edge blocks (no padding), BF16 activations, FP32 r, the FP32
    p and T components of x1 and the FP32 output z; and of the Krylov product."""
    assert bench.layer_method_bytes(1, 3) == 128 + 6 * 9 * 2 + 128
    assert bench.layer_method_bytes(0, 3) == 12 + 108 + 128
    assert bench.layer_method_bytes(2, 3) == 128 + 108 + 12 + 8 + 12
    assert bench.layer_method_bytes(1, 4) == 128 + 6 * 16 * 2 + 128
    assert bench.product_method_bytes(10, 40, 3) == 40 * 76 + 44 + 10 * 3 * 12


def test_in_solve_rooflines_skip_kernels_that_did_not_run(monkeypatch):
    """Once the learned stage has fallen back to BILU(0) no layer runs inside
    the timed solves: only the Krylov product gets a roofline row."""
    from types import SimpleNamespace
    from paper_1907_04229_amd import cptr
    monkeypatch.setattr(cptr, "cptr_kernel_timing", lambda h, on: None)
    monkeypatch.setattr(cptr, "cptr_get_kernel_times", lambda h: ([116.0, 0.0, 0.0, 0.0], [60, 0, 0, 0]))
    monkeypatch.setattr(bench, "recorded_traffic", lambda key, n, nv: None)
    solver = SimpleNamespace(problem=SimpleNamespace(n=1000, nv=4, nnzb=7000), h=None,
                             solve=lambda *a, **k: None)
    rows = bench.in_solve_rooflines(solver, None, 30)
    assert [r["layer"] for r in rows] == [None]
    assert rows[0]["launches"] == 60 and rows[0]["achieved"] > 0

"""Host-side logic of bench.py (no device): the one-GPU rule and the
traffic figure taken from the committed counter summaries."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "--gpus" in r.stderr and r.stdout.strip() == ""


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path, monkeypatch):
    import bench
    for kernel in ("k_tile_fp64", "k_tile_mixed"):
        t = bench._measured_traffic(kernel, "c3")
        # the committed summary was taken on the current source
        assert t is not None and 1e9 < t < 1e10
    # a different source hash (the kernel changed since) gives no figure
    monkeypatch.setattr(bench, "_source_hash", lambda: "0" * 64)
    assert bench._measured_traffic("k_tile_fp64", "c3") is None
    # no summary for a workload gives no figure
    assert bench._measured_traffic("k_tile_fp64", "no_such_workload") is None

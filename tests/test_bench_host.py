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
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    h = bench._source_hash()
    (tmp_path / "k_tile_fp64_c3_traffic.md").write_text(
        "hbm_bytes_per_launch: 4.5e+09\nsource_sha256: %s\n" % h)
    assert bench._measured_traffic("k_tile_fp64", "c3") == 4.5e9
    # a different source hash (the kernel changed since) gives no figure
    monkeypatch.setattr(bench, "_source_hash", lambda: "0" * 64)
    assert bench._measured_traffic("k_tile_fp64", "c3") is None
    # no summary for a workload gives no figure
    assert bench._measured_traffic("k_tile_fp64", "no_such_workload") is None

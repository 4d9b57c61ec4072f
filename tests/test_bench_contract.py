"""Host-side checks of bench.py (CPU only): more than one GPU is refused with
a message, and the committed HBM counter summaries are used only while the
render sources still hash to the value recorded in them."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_summary_is_tied_to_the_render_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    good = tmp_path / "bwd.txt"
    good.write_text(f"# header\nkernel_source_sha256_16: {bench.kernel_source_hash()}\nhbm_bytes_per_launch: 1234\n")
    stale = tmp_path / "fwd.txt"
    stale.write_text("kernel_source_sha256_16: 0000000000000000\nhbm_bytes_per_launch: 99\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"bwd": str(good), "fwd": str(stale)})
    assert bench.measured_traffic("bwd") == 1234.0
    assert bench.measured_traffic("fwd") is None

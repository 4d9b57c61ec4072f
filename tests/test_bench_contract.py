"""Host-side checks of bench.py (CPU only): more than one GPU is refused with
a message, and the committed HBM counter summaries are used only while the
render sources still hash to the value recorded in them and for the same
timed steps."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_summary_is_tied_to_the_render_sources_and_steps(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import argparse
    import bench
    args = argparse.Namespace(steps=20, start_ite=0, views=1, tile=(16, 16), pending=6, force_rounds=False)
    key = bench.traffic_key(args)
    assert key == "--steps 20 --start-ite 0 --views 1 --tile 16 16 --pending 6"
    good = tmp_path / "bwd.txt"
    good.write_text(f"# header\nkernel_source_sha256_16: {bench.kernel_source_hash()}\nbench_args: {key}\n"
                    "hbm_bytes_per_launch: 1234\n")
    stale = tmp_path / "fwd.txt"
    stale.write_text(f"kernel_source_sha256_16: 0000000000000000\nbench_args: {key}\nhbm_bytes_per_launch: 99\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"bwd": str(good), "fwd": str(stale)})
    assert bench.measured_traffic("bwd", key) == 1234.0
    assert bench.measured_traffic("fwd", key) is None
    # counters taken over other steps (another trajectory) are not used either
    args.steps = 5000
    assert bench.measured_traffic("bwd", bench.traffic_key(args)) is None

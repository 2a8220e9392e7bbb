"""CPU checks of bench.py's command line: a multi-GPU request is refused with
a message (the product runs on one GPU), and the stored HBM traffic figure is
read only for the sources it was measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "--gpus 2 is not supported" in (r.stdout + r.stderr)


def test_stored_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 64
    (tmp_path / "traffic_step_cx.md").write_text(
        f"source_sha256: {h}\ntraffic_bytes_per_launch: 1234\n")
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    assert bench.stored_traffic("step", "cx") == 1234.0
    (tmp_path / "traffic_step_cx.md").write_text(
        f"source_sha256: {'0' * 64}\ntraffic_bytes_per_launch: 1234\n")
    assert bench.stored_traffic("step", "cx") is None

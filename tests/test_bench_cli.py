"""Host-side checks of the benchmark script (no GPU)."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_for_the_profiled_kernel_source(tmp_path, monkeypatch):
    src_dir = tmp_path / "paper_1304_5966_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = src_dir / "engine.hip"
    src.write_bytes(b"// kernel v1\n")
    sha = hashlib.sha256(b"// kernel v1\n").hexdigest()[:16]
    (tmp_path / "profiles" / "engine_kernel_5Mx4M_counters.md").write_text(
        f"# counters\n\nengine_hip_sha256_prefix: {sha}\ntraffic_bytes: 123456\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic() == 123456
    src.write_bytes(b"// kernel v2\n")  # source changed since the counters were taken
    assert bench.profiled_traffic() is None


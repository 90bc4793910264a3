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


def test_counters_only_for_the_profiled_kernel_source(tmp_path, monkeypatch):
    src_dir = tmp_path / "paper_1304_5966_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = src_dir / "engine.hip"
    src.write_bytes(b"// kernel v1\n")
    sha = hashlib.sha256(b"// kernel v1\n").hexdigest()[:16]
    (tmp_path / "profiles" / "engine_kernel_5Mx4M_counters.md").write_text(
        f"# counters\n\nengine_hip_sha256_prefix: {sha}\ntraffic_bytes: 123456\n"
        f"sq_insts_valu: 2.5e11\ncells: 2.0e12\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    c = bench.profiled_counters()
    assert c == {"match": True, "traffic": 123456, "valu_per_cell": 8.0}
    r = bench.roofline(2.0e12, 1.0, c)
    # 2.5e11 wave instructions x 64 lanes / 2e12 cells = 8 lane-instructions per cell; 8 x 2e12 in 1 s
    assert r["achieved"] == 16.0 and r["frac"] == round(16e12 / bench.VALU_PEAK, 4)
    assert r["traffic"] == 123456 and r["valu_per_cell"] == 8.0
    assert r["algorithmic_tops"] == 20.0  # 10 operations per cell
    src.write_bytes(b"// kernel v2\n")  # source changed since the counters were taken
    c = bench.profiled_counters()
    assert c["match"] is False
    r = bench.roofline(2.0e12, 1.0, c)
    # neither the traffic nor an instruction count of another source is reported
    assert r["traffic"] is None and r["frac"] is None and r["achieved"] is None and r["valu_per_cell"] is None
    assert r["algorithmic_tops"] == 20.0


def test_committed_counters_match_the_kernel_source():
    c = bench.profiled_counters()
    assert c is not None and c["match"], "profiles/engine_kernel_5Mx4M_counters.md is stale: re-take the counters"


def test_extra_leg_skipped_when_the_time_budget_is_spent():
    import time
    ran = []
    t0 = time.perf_counter()
    out = bench.run_leg("genome_scale", lambda: ran.append(1) or {"ok": 1}, t0, budget=100.0)
    assert ran == [] and "time budget" in out["skipped"]
    out = bench.run_leg("alignment", lambda: ran.append(1) or {"ok": 1}, t0, budget=1000.0)
    assert ran == [1] and out == {"ok": 1}
    # every leg of the default run has an estimate, and together they fit the default budget
    # when the genome leg is left out of it
    assert set(bench.LEG_SECONDS) == {"alignment", "batched", "learned_pruned", "protein", "genome_scale"}
    assert sum(v for k, v in bench.LEG_SECONDS.items() if k != "genome_scale") < 540

"""bench.py's command line on the CPU: the one-GPU contract (a request for more GPUs ends with a message,
before any device work)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1", "--warmup", "0"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")   # no bench line


def test_cpu_baseline_leg_runs_on_the_cpu():
    """The oracle leg of the bench line (run before any device work): a dry-run count of one group's
    operations times their measured cost, plus the plaintext forest walk, on the one-query workload."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2104_09583_amd import synth
    w = synth.WORKLOADS["c2_forest16_d5"]
    text, queries, seed = synth.workload_inputs(w)
    out = bench.cpu_baseline(w, text, queries, seed, all_cores=False)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "queries/s"
    assert 0 < out["value"] < 10 and out["seconds_per_group"] > 0.1
    assert out["plain_forest"]["value"] > out["value"]

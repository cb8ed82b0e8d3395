"""The benchmark's command line, on the CPU: one GPU only (a multi-GPU request exits with
status 2 and a message, before anything touches a device), and the defaults a plain
`python bench.py` runs with (one GPU, the N = 200 dense workload, 5 untimed and 20 timed
batched RK4 steps, FP64)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_multi_gpu_request_exits(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=60, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "--gpus %d" % n in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_defaults(monkeypatch):
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.remove(ROOT)
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.gpus, a.steps, a.warmup, a.precision, a.config) == (1, 20, 5, "fp64", "c4")
    assert not a.full_job and not a.no_cpu_baseline

"""bench.py's command line on the host: it measures one GPU and refuses any other count
before touching a device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=120)


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], None), (["--gpus", "8"], None),
                                      (["--gpus", "0"], None), ([], {"WORLD_SIZE": "2"})])
def test_bench_refuses_other_gpu_counts(args, env):
    r = run_bench(args, env)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_rejects_unknown_workload():
    r = run_bench(["--workload", "nope"])
    assert r.returncode == 2 and "invalid choice" in r.stderr

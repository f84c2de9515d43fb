"""Command-line guards of bench.py that act before any device work (CPU):
runs on more than one GPU are refused with a message, and so are
domain-decomposition grids beyond the sizes whose factorisation is
parity-checked."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=e,
                          capture_output=True, text=True, timeout=120)


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], None), (["--gpus", "8"], None),
                                      ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_refused(args, env):
    r = _run(args, env)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_large_dd_grid_refused():
    r = _run(["--cluster", "dd", "--side", "256"])
    assert r.returncode == 2
    assert "domain-decomposition" in r.stderr and r.stdout == ""

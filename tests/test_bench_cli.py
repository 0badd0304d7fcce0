"""bench.py's command line on the host: it refuses more than one GPU before touching
any device, and its solve options map the mode names onto the C-ABI's options."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("mode,expect", [
    ("mixed-rb", dict(mode=1, reduce=1, precond=0)),
    ("fp64", dict(mode=0, reduce=0, precond=0)),
    ("fp64-line", dict(mode=0, reduce=0, precond=1)),
    ("gmres", dict(mode=3, reduce=0, precond=0)),
    ("learned-rb", dict(mode=2, reduce=1, precond=0)),
])
def test_bench_mode_options(mode, expect):
    sys.path.insert(0, ROOT)
    import bench
    from paper_1001_3301_amd import rt
    o = bench.mode_opts(rt, mode, 1e-8, 1000, 1e-4, net=None, budget=5)
    for k, v in expect.items():
        assert getattr(o, k) == v, (mode, k)
    assert o.tol == 1e-8 and o.max_iter == 1000 and o.launch == 0

"""Host-side contracts without a GPU: the seeded structure-search draws are
valid for every target, and the benchmark refuses more than one GPU before it
touches any device."""
import os
import subprocess
import sys

import numpy as np

from workloads.search import de_draws, uniforms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_de_draws_are_valid_and_seeded():
    d = de_draws(7, 5, seed=3)
    r = d["r"]
    assert r.shape == (7, 5, 3)
    for i in range(7):
        for a in range(5):
            assert len(set(r[i, a].tolist())) == 3 and i not in r[i, a]
            assert np.all((r[i, a] >= 0) & (r[i, a] < 7))
    assert np.all(d["radius"] >= 1.5) and np.all(d["radius"] <= 3.0)
    e = de_draws(7, 5, seed=3)
    assert all(np.array_equal(d[k], e[k]) for k in d)
    u = uniforms(100, 4)
    assert np.all((u >= 0) & (u < 1)) and np.array_equal(u, uniforms(100, 4))


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr

"""The benchmark's command line on the CPU: it runs on exactly one GPU and says so for any
other count, and its workload recipe draws the stated size mix."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_workload_recipe():
    from bench import workload
    L, beta, m0 = workload(1512, 512)
    assert len(L) == len(beta) == len(m0) == 512
    counts = {l: L.count(l) for l in (16, 32, 64, 128)}
    assert counts == {16: 197, 32: 139, 64: 123, 128: 53}
    assert sum(l * l for l in L) == 1564928
    assert 1.0 <= min(beta) and max(beta) <= 4.0 and 0.02 <= min(m0) and max(m0) <= 0.2
    # deterministic in the seed
    assert workload(1512, 512) == (L, beta, m0) and workload(7, 512)[0] != L
    assert np.isclose(np.mean([l == 16 for l in L]), 0.4, atol=0.05)

"""Host checks of the benchmark's command line (no GPU): the one-GPU build
refuses several GPUs with a JSON message, and the batched configuration's
problem sizes are the seeded log-uniform draw in [2^14, 2^18]."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    line = json.loads(res.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_batched_sizes_are_log_uniform_in_range():
    rng = np.random.default_rng(3)
    sizes = np.exp(rng.uniform(np.log(16384), np.log(262144), 48)).astype(int)
    assert sizes.min() >= 16384 and sizes.max() <= 262144
    assert int(sizes.sum()) == 4199708          # the batch measured in the design notes
    # log-uniform: about half of the problems below the geometric mean 65536
    assert 16 <= int((sizes < 65536).sum()) <= 32

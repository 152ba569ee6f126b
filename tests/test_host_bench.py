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


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_default_run_asks_for_no_extra_part():
    """The benchmark's standard command (--gpus 1 --steps 20 --warmup 5) requests none of
    the opt-in parts, and the extra runners then do nothing at all (they get
    None for every handle, so any work they started would fail)."""
    bench = _bench()
    args = bench.parse(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert bench.extras_requested(args) == []
    assert bench.run_extras(args, [], None, None, None, None, None, None, 0.0) == {}
    assert bench.run_extras_alone(args, [], None, None, None) == {}
    # every flag maps to its part
    every = bench.parse(["--c1", "--diff", "--bem", "--batched-first", "3", "--part-a",
                         "--cg-smoother", "--sixteen-rhs"])
    assert bench.extras_requested(every) == list(bench.EXTRAS)


def test_extra_parts_are_called_only_from_the_extra_runners():
    """Static check of bench.py: the long opt-in parts are called from the
    runners of the extras (or from their own exclusive modes), never from the
    default path in main()."""
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    long_parts = {"c1_latency", "differentiation", "boundary_elements", "batched", "part_a",
                  "many_rhs_solve"}
    allowed = {"run_extras", "run_extras_alone"}
    callers = {}
    for fn in tree.body:
        if not isinstance(fn, ast.FunctionDef):
            continue
        for node in ast.walk(fn):
            if isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and node.func.id in long_parts:
                callers.setdefault(node.func.id, set()).add(fn.name)
    for part, fns in callers.items():
        extra = fns - allowed
        # main() may call batched() only in its exclusive --batched mode
        if part == "batched":
            extra -= {"main"}
        assert not extra, (part, extra)
    main = next(f for f in tree.body if isinstance(f, ast.FunctionDef) and f.name == "main")
    batched_calls = [n for n in ast.walk(main) if isinstance(n, ast.Call)
                     and isinstance(n.func, ast.Name) and n.func.id == "batched"]
    assert len(batched_calls) == 1            # the --batched mode, which returns right after


def test_timed_solves_respect_the_budget():
    """Warmup and timed steps stop early when the next solve would pass the
    deadline, after at least one of each; the counts reported are the ones run."""
    bench = _bench()

    class FakeTorch:
        class cuda:
            @staticmethod
            def synchronize():
                pass

    class FakeG:
        calls = 0

        def solve(self, b, **kw):
            FakeG.calls += 1
            return "x", {"cycles": 3, "status": "OK", "rel_residual": 1e-9, "converged": True}

    import time as _t
    args = bench.parse(["--steps", "20", "--warmup", "5"])
    # deadline already passed: one warmup and one timed solve still run
    warm, times, infos, x = bench.timed_solves(args, FakeTorch, FakeG(), None, _t.perf_counter() - 1)
    assert warm == 1 and len(times) == 1 and FakeG.calls == 2
    # generous deadline: everything requested runs
    FakeG.calls = 0
    warm, times, infos, x = bench.timed_solves(args, FakeTorch, FakeG(), None, _t.perf_counter() + 3600)
    assert warm == 5 and len(times) == 20 and FakeG.calls == 25


def test_galerkin_flop_count_matches_the_oracle_partition():
    """The setup profile's flop counts (bench.galerkin_flops, from the
    library's plan) against the same formulas over the oracle's own tree and
    partition: 4 r^3 per far pair, 2 r n_s n_t + 2 r^2 n_s per close leaf
    pair, 12 r^3 per close pair above the leaves, upper triangles only."""
    sys.path.insert(0, ROOT)
    import bench
    import synth
    from oracle.partition import build_partition
    from oracle.tree import build_tree
    P = synth.uniform_points(6000, 3, 5)
    leaf, eta, m = 64, 0.7, 3
    r = m ** 3
    got = bench.galerkin_flops(P, leaf, eta, m, 3)
    tree = build_tree(P, leaf)
    part = build_partition(tree, eta)
    L = tree.L
    far = sum(int(np.sum(np.asarray(part.far[d])[:, 0] < np.asarray(part.far[d])[:, 1]))
              for d in range(L + 1) if len(part.far[d]))
    near_l = np.asarray(part.near[L])
    near_l = near_l[near_l[:, 0] <= near_l[:, 1]]
    sizes = np.diff(np.asarray(tree.offsets[L])).astype(np.float64)
    ns, nt = sizes[near_l[:, 0]], sizes[near_l[:, 1]]
    upper = sum(int(np.sum(np.asarray(part.near[d])[:, 0] <= np.asarray(part.near[d])[:, 1]))
                for d in range(part.d_top, L))
    assert got["far_blocks"] == far and got["coupling"] == far * 4.0 * r ** 3
    assert got["leaf_blocks"] == len(near_l)
    assert got["pi_leaf"] == float(np.sum(2.0 * r * ns * nt + 2.0 * r * r * ns))
    assert got["upper_blocks"] == upper and got["pi_upper"] == upper * 12.0 * r ** 3


def test_profiled_traffic_is_tied_to_the_profiled_kernel_source(tmp_path, monkeypatch):
    """The roofline's traffic comes from a counter profile only while the
    block-GEMV sources hash to the profiled ones: it scales the profile's
    HBM / algorithmic ratio to the run's bytes, and is None for another
    source or a kernel kind the profile does not list."""
    import hashlib
    import shutil
    bench = _bench()
    csrc = tmp_path / "paper_2501_17656_amd" / "csrc"
    csrc.mkdir(parents=True)
    h = hashlib.sha256()
    for f in ("kernels_apply.hip", "device_common.h"):
        shutil.copy(os.path.join(ROOT, "paper_2501_17656_amd", "csrc", f), csrc / f)
        h.update((csrc / f).read_bytes())
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "gemv_counters_test.md").write_text(
        "    traffic gemv_fp32 src=%s per_launch_bytes=1.020000e+10 alg_per_launch_bytes=1.000000e+10\n"
        % h.hexdigest()[:16])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("gemv_fp32", 5.0e9) == round(5.0e9 * 1.02)
    assert bench.profiled_traffic("gemv_fp64", 5.0e9) is None
    with open(csrc / "kernels_apply.hip", "a") as f:
        f.write("\n// changed\n")
    assert bench.profiled_traffic("gemv_fp32", 5.0e9) is None

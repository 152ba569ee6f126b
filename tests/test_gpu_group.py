"""Independent problems solved in one sequence of launches (h2mg_solve_group):
every tile product of a cycle step is one kernel launch over the task lists
of all active problems.

Each problem's arithmetic is that of its own 16-column solve, in the same
order (the group kernel runs every problem's blocks exactly as a launch of
its own would), so the solutions must equal the per-problem block solves
bit for bit, with the same cycle counts.  Covered: uneven sizes and depths
(problems whose coarse levels end at different steps), ranks 16, 27 and 64
in one group (three tile widths, so three launches per step), near-field
tiles stored for some problems and evaluated for others, FP64 and FP32 /
BF16 cycles, V- and W-cycles, graphs on and off, more problems than one
launch takes (the 16-member limit), and a failing problem that leaves the
others running.
"""
import numpy as np
import pytest

import synth

from test_gpu_h2 import SHAPES, _points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# (n, dim, kernel, length, shift, leaf, m, points seed, stored near field)
MIXED = [
    (1500, 3, "gauss", 0.1, 1.0, 64, 3, 40, True),        # rank 27, few levels
    (6000, 3, "gauss", 0.1, 1.0, 64, 3, 41, False),       # rank 27, one level more
    (4096, 2, "exp", 0.1, 1e-2, 64, 4, 42, True),         # rank 16
    (9000, 3, "exp", 0.2, 1e-1, 128, 4, 43, False),       # rank 64, ragged leaves
    (2500, 2, "matern32", 0.1, 1e-2, 40, 3, 44, False),   # rank 9, ragged leaves
]


def _problems(spec, nrhs_of=lambda i: 16 if i % 2 == 0 else 5):
    from paper_2501_17656_amd import H2Matrix
    probs = []
    for i, (n, dim, ker, ell, shift, leaf, m, seed, stored) in enumerate(spec):
        P = (synth.gaussian_mixture_points(n, dim, seed=seed) if ker == "gauss"
             else synth.uniform_points(n, dim, seed))
        g = H2Matrix(_dev(P), ker, ell, shift, leaf, 0.7, m)
        if stored:
            g.store_near(True)
        B = synth.normal_vector(n, 70 + i, nrhs=nrhs_of(i)).reshape(n, -1)
        probs.append((g, _dev(B)))
        print(f"[gpu] group member {i}: n={n} rank {m ** dim} levels {g.levels} stored {stored}", flush=True)
    return probs


@pytest.mark.parametrize("precision,method,graphs", [("fp64", "v", False), ("fp32", "v", True),
                                                     ("bf16", "w", True), ("fp64", "w", True)])
def test_group_equals_per_problem_block_solves(precision, method, graphs):
    from paper_2501_17656_amd import solve_batch
    spec = MIXED if precision != "bf16" else [s for s in MIXED if s[2] != "gauss"]
    probs = _problems(spec)
    kw = dict(rtol=1e-8, precision=precision, smoother="bj", method=method, raise_on_error=False)
    ref = [g.solve_multi(B, **kw) for g, B in probs]
    for g, _ in probs:
        g.set_graphs(graphs)
    xs, infos = solve_batch(probs, mode="group", **kw)
    assert len({g.levels for g, _ in probs}) >= 2
    assert sum(i["converged"] for _, i in ref) >= len(probs) - 1
    for i, ((g, B), (xr, ir), x, inf) in enumerate(zip(probs, ref, xs, infos)):
        print(f"[gpu] {precision} {method} graphs={graphs} member {i}: n={g.n} cycles {inf['cycles']} "
              f"(own solve {ir['cycles']}) residual {inf['rel_residual']:.2e} {inf['status']}")
        assert inf["status"] == ir["status"] and inf["cycles"] == ir["cycles"]
        assert inf["history"] == ir["history"]
        np.testing.assert_array_equal(_host(x), _host(xr))
    for g, _ in probs:
        g.close()


def test_group_larger_than_one_launch():
    """18 problems: each step's tile products need two launches (16 + 2)."""
    from paper_2501_17656_amd import solve_batch
    spec = [(800 + 150 * i, 2, "exp", 0.1, 1e-2, 32, 3, 100 + i, i % 3 == 0) for i in range(18)]
    probs = _problems(spec, nrhs_of=lambda i: 1 + i % 16)
    kw = dict(rtol=1e-8, precision="fp32", smoother="bj")
    ref = [g.solve_multi(B, **kw) for g, B in probs]
    xs, infos = solve_batch(probs, mode="group", **kw)
    for (g, B), (xr, ir), x, inf in zip(probs, ref, xs, infos):
        assert inf["converged"] and inf["cycles"] == ir["cycles"]
        np.testing.assert_array_equal(_host(x), _host(xr))
    for g, _ in probs:
        g.close()


def test_group_reports_a_failing_problem_and_finishes_the_others():
    from paper_2501_17656_amd import H2Matrix, H2MGError, solve_batch
    kind, n, dim, ker, ell, shift, leaf, eta, m = SHAPES["gauss3d_gmm_r27"]
    bad = H2Matrix(_dev(_points(kind, n, dim)), ker, ell, shift, leaf, eta, m)
    P = synth.gaussian_mixture_points(3000, 3, seed=41)
    good = H2Matrix(_dev(P), "gauss", 0.1, 1.0, 64, 0.7, 3)
    probs = [(bad, _dev(synth.normal_vector(n, 60, nrhs=4))), (good, _dev(synth.normal_vector(3000, 61, nrhs=4)))]
    with pytest.raises(H2MGError, match="NOT_SPD"):
        solve_batch(probs, rtol=1e-8, smoother="bj", mode="group")
    xs, infos = solve_batch(probs, rtol=1e-8, smoother="bj", mode="group", raise_on_error=False)
    assert infos[0]["status"] == "NOT_SPD" and not infos[0]["converged"]
    assert infos[1]["converged"] and infos[1]["rel_residual"] < 1e-8
    ref, _ = good.solve_multi(probs[1][1], rtol=1e-8, smoother="bj")
    np.testing.assert_array_equal(_host(xs[1]), _host(ref))
    with pytest.raises(H2MGError):
        solve_batch([probs[1], probs[1]], mode="group")        # a handle twice
    bad.close()
    good.close()

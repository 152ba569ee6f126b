"""Captured cycle graphs (h2mg_set_graphs) against direct launches.

A solve with graphs launches the cycle captured on its first iteration once
per cycle, with the FP64 residual, its norm read-back and the stopping test
done by direct launches and a host synchronisation between the replays.  The
arithmetic is the same launch for launch, so the solution and the residual
history after every replay must equal those of the direct-launch solve bit
for bit, for every cycle kind, smoother and precision.
"""
import time

import numpy as np
import pytest

import synth

from test_gpu_h2 import SHAPES, _dev, _host, _points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fresh(name):
    from paper_2501_17656_amd import H2Matrix
    kind, n, dim, ker, ell, shift, leaf, eta, m = SHAPES[name]
    P = _points(kind, n, dim)
    print(f"[gpu] build {name} n={n}", flush=True)
    return P, H2Matrix(_dev(P), ker, ell, shift, leaf, eta, m)


CASES = [("v", "cg", "fp64"), ("v", "bj", "fp32"), ("v", "cg", "bf16"), ("w", "cg", "fp64"),
         ("f", "bj", "fp64")]


@pytest.mark.parametrize("name", ["exp2d_4k", "exp3d_r8"])
def test_graph_solve_equals_direct_launches(name):
    P, g = _fresh(name)
    b = _dev(synth.normal_vector(len(P), 1))
    for method, smoother, prec in CASES:
        kw = dict(rtol=1e-8, method=method, smoother=smoother, precision=prec)
        g.set_graphs(False)
        g.solve(b, **kw)                                   # warm-up (setup, inverses)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x0, i0 = g.solve(b, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.set_graphs(True)
        x1, i1 = g.solve(b, **kw)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        x2, i2 = g.solve(b, **kw)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        print(f"[gpu] {name} {method}/{smoother}/{prec}: {i0['cycles']} cycles, direct "
              f"{t1 - t0:.3f} s, graph {t2 - t1:.3f} s (again {t3 - t2:.3f} s)")
        assert i0["converged"] and i1["converged"]
        assert i1["cycles"] == i0["cycles"] and i2["cycles"] == i0["cycles"]
        assert i1["history"] == i0["history"] and i2["history"] == i0["history"]
        np.testing.assert_array_equal(_host(x1), _host(x0))
        np.testing.assert_array_equal(_host(x2), _host(x0))
    g.close()


def test_graphs_are_skipped_while_timing():
    """With kernel timing on, cycles run launch by launch (events sit between
    the launches), and the result is still the same."""
    P, g = _fresh("exp2d_4k")
    b = _dev(synth.normal_vector(len(P), 1))
    x0, i0 = g.solve(b, smoother="bj")
    g.set_graphs(True)
    g.set_timing(True)
    x1, i1 = g.solve(b, smoother="bj")
    st = g.kernel_stats("gemv_fp64")
    assert st["launches"] > 0
    g.set_timing(False)
    np.testing.assert_array_equal(_host(x1), _host(x0))
    assert i1["history"] == i0["history"]
    g.close()

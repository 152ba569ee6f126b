"""The solve that allocates nothing (h2mg_solve_noalloc) against h2mg_solve.

Both entry points run the same kernels in the same order (fixed-order
reductions, no atomics), so on the same handle, right-hand side and options
the no-allocation solve must return the same iterate bit for bit, with the
same cycle count and residual history; its residual recomputed by the
oracle's matvec must be below the 1e-8 target.  Two calls in a row share the
GPU's fixed scratch region, the second on a smaller problem, so the second
sees the first one's leftovers.  Also checked: the STATE error before the
hierarchy exists, and that a solve which needs more than the fixed region is
refused before any launch.
"""
import numpy as np
import pytest

import synth
from oracle.h2 import H2 as OracleH2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (n, dim, kernel, length, shift, leaf, eta, m): the first is the larger problem
PROBLEMS = [(4096, 2, "exp", 0.1, 1e-2, 64, 0.7, 4), (1200, 2, "exp", 0.1, 1e-2, 32, 0.7, 3)]
CASES = [("fp64", "cg", "v"), ("fp32", "bj", "v"), ("bf16", "bj", "v"), ("fp64", "bj", "w")]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_noalloc_solve_equals_solve_on_two_calls_in_a_row():
    from paper_2501_17656_amd import H2Matrix
    for idx, (n, dim, ker, ell, shift, leaf, eta, m) in enumerate(PROBLEMS):
        P = synth.uniform_points(n, dim, 30 + idx)
        print(f"[gpu] no-alloc problem {idx}: n={n} leaf={leaf} rank {m ** dim}", flush=True)
        g = H2Matrix(_dev(P), ker, ell, shift, leaf, eta, m)
        o = OracleH2(P, ker, shift, leaf, eta, m, ell)
        b = synth.normal_vector(n, 31 + idx)
        bd = _dev(b)
        g.setup(("fp64", "fp32", "bf16"))
        for prec, smoother, method in CASES:
            kw = dict(rtol=1e-8, precision=prec, smoother=smoother, method=method, max_cycles=400)
            x_ref, i_ref = g.solve(bd, **kw)                        # builds what the smoother needs
            h_ref = list(i_ref["history"])
            out = torch.full_like(bd, float("nan"))
            x_na, i_na = g.solve(bd, noalloc=True, out=out, **kw)
            xr, xn = _host(x_ref), _host(x_na)
            res = np.linalg.norm(b - o.matvec(xn)) / np.linalg.norm(b)
            print(f"[gpu] problem {idx} {prec} {smoother} {method}: cycles {i_na['cycles']} "
                  f"(solve {i_ref['cycles']}), bitwise equal {np.array_equal(xr, xn)}, "
                  f"oracle residual {res:.2e}", flush=True)
            assert i_na["status"] == "OK" and i_na["cycles"] == i_ref["cycles"]
            assert i_na["history"] == h_ref
            assert np.array_equal(xr, xn)
            assert res < 1e-8
        g.close()


def test_noalloc_solve_needs_the_hierarchy_first():
    from paper_2501_17656_amd import H2Matrix
    from paper_2501_17656_amd._lib import H2MGError
    n, dim, ker, ell, shift, leaf, eta, m = PROBLEMS[1]
    P = synth.uniform_points(n, dim, 40)
    g = H2Matrix(_dev(P), ker, ell, shift, leaf, eta, m)
    bd = _dev(synth.normal_vector(n, 41))
    with pytest.raises(H2MGError) as e:
        g.solve(bd, noalloc=True)
    assert e.value.status_name == "STATE"
    g.setup(("fp64",))
    with pytest.raises(H2MGError) as e:                  # FP32 operators not prepared
        g.solve(bd, noalloc=True, precision="fp32")
    assert e.value.status_name == "STATE"
    with pytest.raises(H2MGError) as e:                  # block-smoother inverses not built
        g.solve(bd, noalloc=True, smoother="bj")
    assert e.value.status_name == "STATE"
    x, info = g.solve(bd, noalloc=True)
    assert info["converged"]
    g.close()


def test_noalloc_solve_refuses_a_problem_larger_than_the_region():
    """N = 2^22 in FP64 needs about 8 (2 sum_k N_k + 7 n) > 300 MB of vectors,
    more than the 256 MiB region: the call fails with INVALID_ARG and the
    bytes it needs, before any launch."""
    from paper_2501_17656_amd import H2Matrix
    from paper_2501_17656_amd._lib import H2MGError
    n = 1 << 22
    P = synth.uniform_points(n, 2, 42)
    g = H2Matrix(_dev(P), "exp", 0.2, 1.0, 256, 0.7, 2)
    g.setup(("fp64",))
    bd = _dev(synth.normal_vector(n, 43))
    with pytest.raises(H2MGError) as e:
        g.solve(bd, noalloc=True)
    assert e.value.status_name == "INVALID_ARG" and "bytes of scratch" in str(e.value)
    g.close()

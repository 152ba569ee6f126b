"""GPU parity of the cycles and solves on blocks of right-hand sides
(h2mg_solve_multi) and of the batched solve of independent problems
(h2mg_solve_batch) against the CPU oracle.

* two cycles on 16 columns with 2 coarse CG steps (where the iterate is a
  well-conditioned function of its inputs): every column against two oracle
  cycles of its own, for the CG and the block-Jacobi smoothers, V- and
  W-cycles, ranks 9 (padded tiles, chunk-padded near field), 16 and 27.
  The bar is 1e-10 relative, 5e-10 for the Gaussian-mixture shape, whose
  two oracle cycles move by 1.2e-11 (V) and 2.3e-11 (W) when b is perturbed
  by 1e-15 relative (kappa ~ 1e5): rounding alone moves it that far;
* solves to 1e-8: each column's FP64 residual recomputed by the oracle's
  matvec, and each column against the oracle's dense solution (kappa times
  the residual), in FP64 and in FP32 / BF16 cycles inside FP64 refinement
  (BF16 only where the operator stays positive definite after rounding its
  blocks to 2^-9 relative: not on the Gaussian-mixture shape, whose
  lambda_min / lambda_max is 1e-5, where a run reported NOT_SPD);
* the batched solve of uneven problems equals the per-problem block solve
  bit for bit (same kernels in the same order, only the streams differ);
* the near-field tiles evaluated inside the products (no stored near
  field) give the stored-tile results up to rounding;
* the tile-run tuner keeps the results (up to summation order);
* error paths: nrhs, method, rank, shared handles.
"""
import numpy as np
import pytest

import synth
from oracle.galerkin import Hierarchy
from oracle.vcycle import mg_cycle

from test_gpu_h2 import SHAPES, _points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_cache = {}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make(name):
    """GPU handle with the near field stored, oracle H2 and its hierarchy."""
    if name not in _cache:
        from paper_2501_17656_amd import H2Matrix
        from oracle.h2 import H2 as OracleH2
        kind, n, dim, ker, ell, shift, leaf, eta, m = SHAPES[name]
        P = _points(kind, n, dim)
        print(f"[gpu] block: build {name} n={len(P)} leaf={leaf} m={m}", flush=True)
        g = H2Matrix(_dev(P), ker, ell, shift, leaf, eta, m)
        g.store_near(True)
        o = OracleH2(P, ker, shift, leaf, eta, m, ell)
        _cache[name] = (P, g, o, Hierarchy(o))
    return _cache[name]


CYCLE_TOL = {"exp2d_ragged_r9": 1e-10, "exp2d_4k": 1e-10, "gauss3d_gmm4k_r27": 5e-10}


@pytest.mark.parametrize("name", ["exp2d_ragged_r9", "exp2d_4k", "gauss3d_gmm4k_r27"])
@pytest.mark.parametrize("smoother,kind", [("cg", "v"), ("bj", "v"), ("cg", "w")])
def test_two_block_cycles_match_oracle(name, smoother, kind):
    P, g, o, H = make(name)
    n = len(P)
    B = synth.normal_vector(n, 31, nrhs=16)
    X, info = g.solve_multi(_dev(B), rtol=1e-300, n_coarse=2, max_cycles=2, smoother=smoother,
                            method=kind, raise_on_error=False)
    assert info["status"] == "NOT_CONVERGED" and info["cycles"] == 2
    X = _host(X)
    perm = o.tree.perm
    worst = 0.0
    for k in range(16):
        xt = np.zeros(n)
        for _ in range(2):
            xt = mg_cycle(H, xt, B[perm, k], kind.upper(), 1, 2, smoother=smoother)
        xo = np.empty(n)
        xo[perm] = xt
        worst = max(worst, np.linalg.norm(X[:, k] - xo) / np.linalg.norm(xo))
    print(f"[gpu] {name} {smoother}/{kind}: two block cycles, worst column rel diff {worst:.2e}")
    assert worst <= CYCLE_TOL[name]


@pytest.mark.parametrize("name,nrhs,prec,smoother", [
    ("exp2d_4k", 16, "fp64", "cg"), ("exp2d_4k", 16, "fp64", "bj"), ("exp2d_4k", 16, "fp32", "bj"),
    ("exp2d_4k", 16, "bf16", "bj"), ("gauss3d_gmm4k_r27", 5, "fp64", "cg"),
    ("gauss3d_gmm4k_r27", 5, "fp64", "bj"), ("gauss3d_gmm4k_r27", 5, "fp32", "bj")])
def test_block_solve_reaches_oracle_solution(name, nrhs, prec, smoother):
    P, g, o, H = make(name)
    n = len(P)
    B = synth.normal_vector(n, 32, nrhs=nrhs)
    X, info = g.solve_multi(_dev(B), rtol=1e-8, precision=prec, smoother=smoother)
    X = _host(X)
    A = o.dense()
    kappa = np.linalg.cond(A)
    for k in range(nrhs):
        res = np.linalg.norm(B[:, k] - o.matvec(X[:, k])) / np.linalg.norm(B[:, k])
        xd = np.linalg.solve(A, B[:, k])
        err = np.linalg.norm(X[:, k] - xd) / np.linalg.norm(xd)
        assert res < 1.5e-8, (k, res)
        assert abs(res - info["column_residuals"][k]) <= 1e-9
        assert err <= kappa * 1.5e-8, (k, err)
    print(f"[gpu] {name} {prec}/{smoother} nrhs={nrhs}: {info['cycles']} cycles, "
          f"max residual {info['rel_residual']:.2e}")
    assert info["converged"] and info["rel_residual"] < 1e-8


def test_block_single_level_direct_solve():
    """No far blocks: one level, solved directly by the dense Cholesky factor
    on all 16 columns in one cycle."""
    P, g, o, H = make("no_far")
    n = len(P)
    B = synth.normal_vector(n, 38, nrhs=16)
    X, info = g.solve_multi(_dev(B), rtol=1e-8)
    X = _host(X)
    assert g.levels == 1 and info["cycles"] == 1
    for k in range(16):
        res = np.linalg.norm(B[:, k] - o.matvec(X[:, k])) / np.linalg.norm(B[:, k])
        assert res < 1e-12, (k, res)


def test_block_columns_are_independent():
    """A column's iterate does not depend on the other columns: solving a
    single column reproduces that column of the 16-column cycles (the per
    column CG scalars are computed from that column alone)."""
    P, g, o, H = make("exp2d_4k")
    n = len(P)
    B = synth.normal_vector(n, 33, nrhs=16)
    X16, _ = g.solve_multi(_dev(B), rtol=1e-300, n_coarse=5, max_cycles=2, raise_on_error=False)
    X1, _ = g.solve_multi(_dev(np.ascontiguousarray(B[:, 7:8])), rtol=1e-300, n_coarse=5, max_cycles=2,
                          raise_on_error=False)
    np.testing.assert_array_equal(_host(X16)[:, 7], _host(X1)[:, 0])


def test_block_solve_zero_and_graphs():
    P, g, o, H = make("exp2d_4k")
    n = len(P)
    B = synth.normal_vector(n, 34, nrhs=4)
    B[:, 2] = 0.0
    X, info = g.solve_multi(_dev(B), rtol=1e-8, smoother="bj")
    X = _host(X)
    assert np.all(X[:, 2] == 0.0) and info["column_residuals"][2] == 0.0
    g.set_graphs(True)
    try:
        Xg, infog = g.solve_multi(_dev(B), rtol=1e-8, smoother="bj")
    finally:
        g.set_graphs(False)
    np.testing.assert_array_equal(_host(Xg), X)       # graph replay = direct launches
    assert infog["cycles"] == info["cycles"]


def test_batch_of_uneven_problems_equals_block_solves():
    from paper_2501_17656_amd import H2Matrix, solve_batch
    probs = []
    for i, n in enumerate((1500, 3000, 5000)):
        Pi = synth.gaussian_mixture_points(n, 3, seed=40 + i)
        gi = H2Matrix(_dev(Pi), "gauss", 0.1, 1.0, 64, 0.7, 3)
        gi.store_near(True)
        probs.append((gi, _dev(synth.normal_vector(n, 50 + i, nrhs=16 if i != 1 else 3))))
    ref = [g.solve_multi(B, rtol=1e-8, precision="fp32", smoother="bj") for g, B in probs]
    for g, _ in probs:
        g.set_graphs(True)
    xs, infos = solve_batch(probs, rtol=1e-8, precision="fp32", smoother="bj", nstreams=2)
    for i, ((g, B), (xr, ir), x, inf) in enumerate(zip(probs, ref, xs, infos)):
        print(f"[gpu] batch problem {i}: n={g.n} cycles {inf['cycles']} residual {inf['rel_residual']:.2e}")
        assert inf["converged"] and inf["cycles"] == ir["cycles"]
        np.testing.assert_array_equal(_host(x), _host(xr))
    for g, _ in probs:
        g.close()


def test_autotuned_runs_keep_results():
    """With tuning on, every task set is rebuilt with the fastest run length
    among {2, 4, 8, 16, 32}; only the summation order of the partials
    changes, so two cycles agree with the untuned ones to the rounding
    sensitivity of this shape."""
    P, g, o, H = make("gauss3d_gmm4k_r27")
    n = len(P)
    B = synth.normal_vector(n, 37, nrhs=16)
    kw = dict(rtol=1e-300, n_coarse=2, max_cycles=2, smoother="bj", raise_on_error=False)
    X0, _ = g.solve_multi(_dev(B), **kw)
    g.set_autotune(True)
    try:
        X1, _ = g.solve_multi(_dev(B), **kw)
        tun = g.block_tuning()
    finally:
        g.set_autotune(False)
    print(f"[gpu] tuned runs: {tun}")
    assert "fine" in tun and "near" in tun and any(isinstance(k, int) for k in tun)
    assert all(v["run"] in (2, 4, 8, 16, 32) and v["ms"] > 0 for v in tun.values())
    rel = np.linalg.norm(_host(X1) - _host(X0)) / np.linalg.norm(_host(X0))
    print(f"[gpu] tuned vs untuned two cycles: rel diff {rel:.2e}")
    assert rel <= CYCLE_TOL["gauss3d_gmm4k_r27"]


def test_batch_reports_a_failing_problem_and_finishes_the_others():
    """One problem of the batch is indefinite after compression (the rank-27
    Gaussian-mixture shape of the single-vector error tests): the batch
    returns its NOT_SPD status while the other problem still converges."""
    from paper_2501_17656_amd import H2Matrix, H2MGError, solve_batch
    kind, n, dim, ker, ell, shift, leaf, eta, m = SHAPES["gauss3d_gmm_r27"]
    bad = H2Matrix(_dev(_points(kind, n, dim)), ker, ell, shift, leaf, eta, m)
    P = synth.gaussian_mixture_points(3000, 3, seed=41)
    good = H2Matrix(_dev(P), "gauss", 0.1, 1.0, 64, 0.7, 3)
    probs = [(bad, _dev(synth.normal_vector(n, 60, nrhs=4))), (good, _dev(synth.normal_vector(3000, 61, nrhs=4)))]
    with pytest.raises(H2MGError, match="NOT_SPD"):
        solve_batch(probs, rtol=1e-8, smoother="bj")
    xs, infos = solve_batch(probs, rtol=1e-8, smoother="bj", raise_on_error=False)
    assert infos[0]["status"] == "NOT_SPD" and not infos[0]["converged"]
    assert infos[1]["converged"] and infos[1]["rel_residual"] < 1e-8
    bad.close()
    good.close()


def test_block_error_paths():
    from paper_2501_17656_amd import H2Matrix, H2MGError, solve_batch
    P, g, o, H = make("exp2d_4k")
    n = len(P)
    with pytest.raises(H2MGError):
        g.solve_multi(_dev(np.zeros((n, 17))))
    with pytest.raises(H2MGError):
        g.solve_multi(_dev(np.ones((n, 2))), method="cg")
    bad = np.ones((n, 2))
    bad[3, 1] = np.nan
    with pytest.raises(H2MGError):
        g.solve_multi(_dev(bad))
    with pytest.raises(H2MGError):
        solve_batch([(g, _dev(np.ones((n, 2)))), (g, _dev(np.ones((n, 2))))])
    P2 = synth.uniform_points(2048, 2, 5)
    g2 = H2Matrix(_dev(P2), "exp", 0.1, 1e-2, 64, 0.7, 2)             # rank 4: tiles too small
    with pytest.raises(H2MGError):
        g2.solve_multi(_dev(np.ones((2048, 2))))
    g2.close()


def test_block_solve_with_evaluated_near_field():
    """Without stored tiles every near-field tile product evaluates its tile
    from the points; two cycles match the stored-tile cycles up to rounding
    and the solve reaches the oracle's residual bar."""
    from paper_2501_17656_amd import H2Matrix
    kind, n, dim, ker, ell, shift, leaf, eta, m = SHAPES["exp2d_ragged_r9"]
    P = _points(kind, n, dim)
    g = H2Matrix(_dev(P), ker, ell, shift, leaf, eta, m)
    o = make("exp2d_ragged_r9")[2]
    B = synth.normal_vector(n, 36, nrhs=6)
    Xe, _ = g.solve_multi(_dev(B), rtol=1e-300, n_coarse=2, max_cycles=2, smoother="bj", raise_on_error=False)
    g.store_near(True)
    Xs, _ = g.solve_multi(_dev(B), rtol=1e-300, n_coarse=2, max_cycles=2, smoother="bj", raise_on_error=False)
    g.store_near(False)
    assert np.linalg.norm(_host(Xe) - _host(Xs)) <= 1e-12 * np.linalg.norm(_host(Xs))
    for prec in ("fp64", "fp32"):
        X, info = g.solve_multi(_dev(B), rtol=1e-8, precision=prec, smoother="bj")
        X = _host(X)
        for k in range(6):
            res = np.linalg.norm(B[:, k] - o.matvec(X[:, k])) / np.linalg.norm(B[:, k])
            assert res < 1.5e-8, (prec, k, res)
    g.close()

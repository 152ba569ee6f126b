"""GPU parity of the low-precision cycles (FP32 and BF16 operators inside
FP64 iterative refinement) against the oracle's refinement on a lowered
hierarchy, one cycle at a time.

A refinement solve stopped after one step from x0 = 0 returns
x_1 = V_lp(b): one V-cycle of Algorithm 1 on the low-precision operators
with the FP64 right-hand side.  The oracle computes the same cycle on its
dense hierarchy with the library's precision policy (`oracle.ir.lowered`:
far parts, coarse operators and transfers rounded to the precision, the
close leaf blocks of the fine operator to FP32), in FP64 arithmetic, and
once more with FP32 vectors (`oracle.ir.vcycle_fp32`), as the library runs
it.  With n_c = 2 the cycle is a well-conditioned map, so the library's
result differs from the oracle's only by rounding:

* delta_p is how far rounding moves the cycle: the largest distance to the
  FP64 cycle among the oracle's lowered cycle (operators rounded) and its
  FP32-arithmetic cycle in two summation orders (A v and v A of the same
  symmetric operator), relative to ||V_fp64(b)||; these realisations of
  FP32 rounding scatter by a factor of up to about 4 among themselves;
* the library's cycle is another FP32-arithmetic realisation of the same
  computation (other factorisations rounded, other summation orders), so it
  must lie within 6 delta_p of the FP64 cycle and of the oracle's lowered
  cycle.

A tile read with a wrong layout gives an O(1) error in the products it
touches, orders of magnitude above these bars.  Ranks 16, 27 and 64 run the
tile widths T = 2, 4 and 8 of the single-vector kernels and of the
16-column matrix-core products.  Refinement-step counts to 1e-8 are
compared with the oracle's `ir_solve` on the same policy, and every level
product is checked against its rounding bound.
"""
import numpy as np
import pytest

import synth
from oracle.galerkin import Hierarchy
from oracle.h2 import H2 as OracleH2
from oracle.ir import ir_solve, lowered, vcycle_fp32
from oracle.vcycle import coarsest_factor, smoothers, vcycle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = {
    # name: (n, dim, kernel, length, shift, leaf, eta, m)   rank m^dim -> tile width T
    "exp2d_r16": (4096, 2, "exp", 0.1, 1e-2, 64, 0.7, 4),     # T = 2
    "exp3d_r27": (4096, 3, "exp", 0.2, 1e-1, 32, 0.7, 3),     # T = 4 (padded tiles)
    "exp3d_r64": (8192, 3, "exp", 0.2, 1e-1, 64, 0.7, 4),     # T = 8
}
NC = 2


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


_cache = {}


def make(name):
    if name not in _cache:
        from paper_2501_17656_amd import H2Matrix
        n, dim, ker, ell, shift, leaf, eta, m = SHAPES[name]
        P = synth.uniform_points(n, dim, 0)
        print(f"[gpu] build {name} n={n} dim={dim} leaf={leaf} rank {m ** dim}", flush=True)
        g = H2Matrix(_dev(P), ker, ell, shift, leaf, eta, m)
        g.setup(("fp64", "fp32", "bf16"))
        o = OracleH2(P, ker, shift, leaf, eta, m, ell)
        H = Hierarchy(o)
        assert H.levels >= 3, "the shape must have a coarse level between the fine and the dense one"
        _cache[name] = (P, o, H, g)
    return _cache[name]


_ref = {}


def _oracle_cycles(H, o, b_user, smoother, key):
    """One cycle from zero (user order): FP64, lowered in FP32 and BF16 (FP64
    arithmetic), and with FP32 vectors on the FP32 and BF16 operators."""
    if key in _ref:
        return _ref[key]
    perm = o.tree.perm
    bt = b_user[perm]
    factor = coarsest_factor(H.ops[-1])
    precs = smoothers(H, smoother)
    out = {}
    for prec in ("fp64", "fp32", "bf16"):
        Hl = H if prec == "fp64" else lowered(H, prec)
        out[prec] = vcycle(Hl, np.zeros_like(bt), bt, 1, NC, factor, r1=bt, precs=precs)
        if prec != "fp64":
            out[prec + "_arith"] = vcycle_fp32(H, bt, prec, 1, NC, smoother)
            out[prec + "_arith_t"] = vcycle_fp32(H, bt, prec, 1, NC, smoother, transposed=True)
    res = {}
    for k, d in out.items():
        x = np.empty_like(d)
        x[perm] = d
        res[k] = x
    _ref[key] = res
    return res


def _check(name, prec, xg, ref, label):
    d64 = ref["fp64"]
    nrm = np.linalg.norm(d64)
    delta = max(np.linalg.norm(ref[k] - d64) / nrm for k in (prec, prec + "_arith", prec + "_arith_t"))
    to64 = np.linalg.norm(xg - d64) / nrm
    tolow = np.linalg.norm(xg - ref[prec]) / nrm
    print(f"[gpu] {name} {label} {prec}: |x - oracle_{prec}| {tolow:.2e}, |x - oracle_fp64| {to64:.2e}, "
          f"delta_{prec} {delta:.2e}")
    assert delta > 0
    assert to64 <= 6 * delta
    assert tolow <= 6 * delta


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("smoother", ["cg", "bj"])
def test_one_low_precision_cycle_matches_lowered_oracle(name, prec, smoother):
    P, o, H, g = make(name)
    b = synth.normal_vector(len(P), 1)
    x, info = g.solve(_dev(b), rtol=1e-30, max_cycles=1, n_coarse=NC, precision=prec,
                      smoother=smoother, raise_on_error=False)
    assert info["status"] == "NOT_CONVERGED" and info["cycles"] == 1, info
    ref = _oracle_cycles(H, o, b, smoother, (name, smoother, 1))
    _check(name, prec, _host(x), ref, f"single-vector {smoother}")


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_one_low_precision_block_cycle_matches_lowered_oracle(name, prec):
    """The 16-column cycle (matrix-core tile products, near field evaluated
    inside the products): every compared column as in the single-vector
    test."""
    P, o, H, g = make(name)
    B = synth.normal_vector(len(P), 23, nrhs=16)
    X, info = g.solve_multi(_dev(B), rtol=1e-30, max_cycles=1, n_coarse=NC, precision=prec,
                            smoother="bj", raise_on_error=False)
    assert info["cycles"] == 1, info
    Xh = _host(X)
    for k in (0, 9, 15):
        ref = _oracle_cycles(H, o, np.ascontiguousarray(B[:, k]), "bj", (name, "bj", 23, k))
        _check(name, prec, Xh[:, k], ref, f"16-column col {k}")


@pytest.mark.parametrize("name", ["exp2d_r16", "exp3d_r27"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_refinement_steps_match_oracle_ir(name, prec):
    """Refinement steps to a 1e-8 FP64 residual: the library's count is
    within two steps (and 20%) of the oracle's on the lowered hierarchy."""
    P, o, H, g = make(name)
    b = synth.normal_vector(len(P), 1)
    x, info = g.solve(_dev(b), rtol=1e-8, n_coarse=5, precision=prec, smoother="bj",
                      max_cycles=200, raise_on_error=False)
    perm = o.tree.perm
    ref = ir_solve(H, b[perm], prec, rtol=1e-8, max_outer=200, n_c=5, smoother="bj")
    res = np.linalg.norm(b - o.matvec(_host(x))) / np.linalg.norm(b)
    print(f"[gpu] {name} {prec} refinement steps gpu {info['cycles']} oracle {ref.cycles}, "
          f"oracle residual of gpu x {res:.2e}")
    assert info["converged"] and ref.converged and res < 1e-8
    assert abs(info["cycles"] - ref.cycles) <= max(2, 0.2 * ref.cycles)


# unit roundoff of FP32 (24 significant bits) and BF16 (8 significant bits)
U = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8}


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_low_precision_level_products(name, prec):
    """y = A_k x on every level with the operators of the mixed cycles, against
    the oracle's FP64 level operator.  The library rounds each stored factor
    (bases, transfers, couplings, projected blocks) once to the precision
    and accumulates in FP32; a coupling of depth d passes through at most
    2 (L - d) + 3 rounded factors, and FP32 partial sums add their own
    rounding, so the bar is c u ||(|A_k|) |x|||, u the precision's unit
    roundoff, with c = 4 (2 L + 3): the longest chain of rounded factors,
    times 4 for the FP32 sums and the FP32 near-field evaluation.  A tile
    element read from a wrong position is an O(1) error in its block row."""
    P, o, H, g = make(name)
    c = 4 * (2 * o.L + 3)
    for k in range(1, H.levels + 1):
        nk = H.ops[k - 1].shape[0]
        x = synth.normal_vector(nk, 40 + k)
        if k == 1:
            A = H.ops[0]
            perm = o.tree.perm
            yref = np.empty(nk)
            yref[perm] = A @ x[perm]
            bound_vec = np.empty(nk)
            bound_vec[perm] = np.abs(A) @ np.abs(x[perm])
        else:
            A = H.ops[k - 1]
            yref = A @ x
            bound_vec = np.abs(A) @ np.abs(x)
        y = _host(g.level_apply(k, _dev(x), precision=prec))
        err = np.linalg.norm(y - yref)
        bound = c * U[prec] * np.linalg.norm(bound_vec)
        print(f"[gpu] {name} level {k} {prec}: |y - A x| / |A x| {err / np.linalg.norm(yref):.2e}, "
              f"err / bound {err / bound:.3f}")
        assert err <= bound

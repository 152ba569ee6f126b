"""The H2-MG V-cycle (Algorithm 1) and repeated cycles (oracle).

Paper: Section 3.3, Algorithm 1:
    r_1 = b - A_1 x_0
    for i = 1 .. l-1:  e~_i = Iter(A_i, r_i, 0);  r_{i+1} = U_i^T (r_i - A_i e~_i)
    e_l = dir_sol(A_l, r_l)                      (Cholesky)
    for i = l-1 .. 1:  e~_i = e~_i + V_i^T e_{i+1};  e_i = Iter(A_i, r_i, e~_i)
    x* = x_0 + e_1
and successive V-cycles restart from x*.  Iter uses n_f CG steps on the
finest level and n_c on the others (Remark on fine and coarse iterations).

Readings:
* restriction U_i^T and prolongation V_i^T = U_i (symmetric case), i.e. the
  transposed and plain level transfers P_i of galerkin.py;
* the residual r_i - A_i e~_i is formed explicitly (one product);
* both pre- and post-smoothing use n_f steps on level 1 and n_c elsewhere;
* outer loop: x_0 = 0; before each cycle the FP64 residual b - A_H2 x is
  measured and the loop stops when ||b - A_H2 x|| / ||b|| < rtol
  (rtol = 1e-8) or after max_cycles cycles;
* smoother "bj": preconditioned CG with M = the diagonal blocks of each
  level's operator (leaf blocks of A_H2 on level 1, one r x r block per
  cluster on coarser levels): a block smoother on the diagonal blocks.

Other cycles (the text after Algorithm 1 names W- and F-cycles without
defining them; the textbook recursive forms are used).  Written as a
recursion MG(i, r_i) returning e_i: pre-smooth from zero, restrict the
residual, coarse correction, prolongate, post-smooth, with the coarsest
level solved directly.  The coarse correction of level i is
  V: e_{i+1} = V(i+1, r_{i+1});
  W: e_{i+1} = W(i+1, r_{i+1}), then e_{i+1} += W(i+1, r_{i+1} - A_{i+1} e_{i+1});
  F: e_{i+1} = F(i+1, r_{i+1}), then e_{i+1} += V(i+1, r_{i+1} - A_{i+1} e_{i+1});
the second call is skipped when level i+1 is the coarsest (its solve is
exact).  The V form is exactly Algorithm 1.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from .cg import block_jacobi, cg, pcg


@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    cycles: int
    converged: bool
    history: list          # relative residual before each cycle, and at exit


def coarsest_factor(A: np.ndarray):
    return scipy.linalg.cho_factor(A, lower=True)


def level_offsets(H, i):
    """Row blocks of level i+1 (0-based i): leaves on level 1, clusters of r
    coefficients on coarser levels."""
    h2 = H.h2
    if i == 0:
        return h2.tree.offsets[h2.L]
    nb = H.ops[i].shape[0] // h2.r
    return np.arange(nb + 1) * h2.r


def smoothers(H, smoother):
    if smoother == "cg":
        return None
    if smoother == "bj":
        return [block_jacobi(H.ops[i], level_offsets(H, i)) for i in range(len(H.ops) - 1)]
    raise ValueError(smoother)


def vcycle(H, x0: np.ndarray, b: np.ndarray, n_f: int = 1, n_c: int = 40,
           factor=None, r1=None, smoother="cg", precs=None) -> np.ndarray:
    """One V-cycle of Algorithm 1 on the dense hierarchy H (tree order)."""
    ops, P = H.ops, H.prolong
    l = len(ops)
    if factor is None:
        factor = coarsest_factor(ops[-1])
    if precs is None:
        precs = smoothers(H, smoother)

    def iterate(i, rhs, e0, n):
        if precs is None:
            return cg(ops[i].__matmul__, rhs, e0, n)
        return pcg(ops[i].__matmul__, precs[i], rhs, e0, n)
    r = [None] * l
    et = [None] * l
    r[0] = b - ops[0] @ x0 if r1 is None else r1
    for i in range(l - 1):
        n = n_f if i == 0 else n_c
        et[i] = iterate(i, r[i], None, n)
        r[i + 1] = P[i].T @ (r[i] - ops[i] @ et[i])
    e = scipy.linalg.cho_solve(factor, r[l - 1])
    for i in range(l - 2, -1, -1):
        n = n_f if i == 0 else n_c
        et[i] = et[i] + P[i] @ e
        e = iterate(i, r[i], et[i], n)
    return x0 + e


def mg_cycle(H, x0: np.ndarray, b: np.ndarray, kind: str = "V", n_f: int = 1, n_c: int = 40,
             factor=None, r1=None, smoother="cg", precs=None) -> np.ndarray:
    """One V-, W- or F-cycle on the dense hierarchy H (tree order)."""
    ops, P = H.ops, H.prolong
    l = len(ops)
    if factor is None:
        factor = coarsest_factor(ops[-1])
    if precs is None:
        precs = smoothers(H, smoother)

    def iterate(i, rhs, e0, n):
        if precs is None:
            return cg(ops[i].__matmul__, rhs, e0, n)
        return pcg(ops[i].__matmul__, precs[i], rhs, e0, n)

    def mg(i, rhs, kd):
        if i == l - 1:
            return scipy.linalg.cho_solve(factor, rhs)
        n = n_f if i == 0 else n_c
        e = iterate(i, rhs, None, n)
        rc = P[i].T @ (rhs - ops[i] @ e)
        ec = mg(i + 1, rc, kd)
        if kd != "V" and i + 1 < l - 1:
            ec = ec + mg(i + 1, rc - ops[i + 1] @ ec, "V" if kd == "F" else "W")
        e = e + P[i] @ ec
        return iterate(i, rhs, e, n)

    if kind not in ("V", "W", "F"):
        raise ValueError(kind)
    r = b - ops[0] @ x0 if r1 is None else r1
    return x0 + mg(0, r, kind)


def solve(H, b: np.ndarray, rtol: float = 1e-8, max_cycles: int = 500,
          n_f: int = 1, n_c: int = 40, x0=None, smoother="cg", kind="V") -> SolveResult:
    """Repeated V-cycles on A_H2 x = b (b and x in tree order)."""
    A = H.ops[0]
    factor = coarsest_factor(H.ops[-1])
    precs = smoothers(H, smoother)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    hist = []
    if nb == 0.0:
        return SolveResult(np.zeros_like(b), 0, True, [0.0])
    for cyc in range(max_cycles + 1):
        res = b - A @ x
        rel = float(np.linalg.norm(res)) / nb
        hist.append(rel)
        if rel < rtol:
            return SolveResult(x, cyc, True, hist)
        if cyc == max_cycles:
            break
        if kind == "V":
            x = vcycle(H, x, b, n_f, n_c, factor, r1=res, precs=precs)
        else:
            x = mg_cycle(H, x, b, kind, n_f, n_c, factor, r1=res, precs=precs)
    return SolveResult(x, max_cycles, False, hist)


def solve_user(h2, H, b_user: np.ndarray, **kw) -> SolveResult:
    """solve() with b and x in user order."""
    perm = h2.tree.perm
    res = solve(H, np.asarray(b_user, dtype=np.float64)[perm], **kw)
    x = np.empty_like(res.x)
    x[perm] = res.x
    return dataclasses.replace(res, x=x)


def smoothing_error_components(H, x_true: np.ndarray, n_f: int = 1, n_c: int = 40,
                               cycles: int = 2, smoother="cg"):
    """The error analysis of the experiments (tree order): with b = A x_true
    and x_0 = 0, the error e = x_k + e~_1 - x_true right after the first
    fine-level smoothing of cycle k+1, split into its part in the range of
    U_1 (the restricted error U_1^T e) and its part in the complement,
    ||Q_1^T e|| = sqrt(||e||^2 - ||U_1^T e||^2) for orthonormal [U_1 Q_1].
    Returns one (U_1^T e, ||Q_1^T e||) pair per cycle."""
    A, P = H.ops[0], H.prolong[0]
    precs = smoothers(H, smoother)
    factor = coarsest_factor(H.ops[-1])
    b = A @ x_true
    x = np.zeros_like(b)
    out = []
    for _ in range(cycles):
        r = b - A @ x
        e1 = cg(A.__matmul__, r, None, n_f) if precs is None else pcg(A.__matmul__, precs[0], r, None, n_f)
        err = x + e1 - x_true
        ue = P.T @ err
        qn = float(np.sqrt(max(float(err @ err) - float(ue @ ue), 0.0)))
        out.append((ue, qn))
        x = vcycle(H, x, b, n_f, n_c, factor, precs=precs)
    return out

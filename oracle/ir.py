"""FP64 iterative refinement around a low-precision V-cycle (oracle).

Not in the paper (its experiments use one precision).  The mixed-precision
form keeps the outer residual, the update, the norms and the coarsest
Cholesky factor in FP64 and runs the V-cycle on operators stored in FP32 or
BF16:

    x = 0;  loop:  r = b - A_H2 x (FP64);  stop when ||r|| / ||b|| < rtol;
                   d = V-cycle(low-precision hierarchy, x_0 = 0, rhs r);
                   x = x + d.

Emulation: every stored operator of the hierarchy except the coarsest one
(whose FP64 Cholesky factor is kept) and every level transfer is rounded
entrywise to the low precision, except the close leaf blocks of the fine
operator, which stay FP32 in both low-precision forms (the near field is
FP32 there); the block-smoother inverses come from the FP64 operators; the
V-cycle arithmetic stays FP64.  `vcycle_fp32` also rounds the vectors to
FP32, for bounding the effect of FP32 arithmetic on one cycle.  BF16
rounding is FP64 -> FP32 (round to nearest even) followed by
round-to-nearest-even to 8 significant bits on the FP32 bit pattern.

Parity unpinned for the convergence rate of the low-precision forms: only
the fixed point (FP64 residual below rtol) and the FP64 special case
(refinement with an FP64 inner cycle is exactly the plain V-cycle iteration)
are pinned.
"""
from __future__ import annotations

import copy

import numpy as np

from .cg import cg, pcg
from .vcycle import SolveResult, coarsest_factor, smoothers, vcycle


def round_fp32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(a: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


ROUNDING = {"fp64": lambda a: np.array(a, dtype=np.float64),
            "fp32": round_fp32, "bf16": round_bf16}


def near_mask(H) -> np.ndarray:
    """Entries of the fine operator (tree order) that belong to close leaf
    pairs (the near field)."""
    h2 = H.h2
    L = h2.L
    mask = np.zeros((h2.n, h2.n), dtype=bool)
    for s, t in h2.part.near[L]:
        mask[h2.rows(L, s), h2.rows(L, t)] = True
    return mask


def lowered(H, precision: str):
    """A copy of the hierarchy with stored operators and transfers rounded
    (the coarsest operator stays FP64).  The close leaf blocks of the fine
    operator are rounded to FP32 whatever the precision: the low-precision
    forms keep the near field in FP32 (its blocks hold the diagonal, which
    BF16 rounding can push below the smallest eigenvalue)."""
    rnd = ROUNDING[precision]
    Hl = copy.copy(H)
    A1 = H.ops[0]
    if precision == "fp64" or len(H.ops) == 1:
        ops = [rnd(A) for A in H.ops[:-1]]
    else:
        ops = [np.where(near_mask(H), round_fp32(A1), rnd(A1))] + [rnd(A) for A in H.ops[1:-1]]
    Hl.ops = ops + [H.ops[-1]]
    Hl.prolong = [rnd(P) for P in H.prolong]
    return Hl


def vcycle_fp32(H, b: np.ndarray, precision: str = "fp32", n_f: int = 1, n_c: int = 40,
                smoother: str = "cg", transposed: bool = False) -> np.ndarray:
    """One cycle of Algorithm 1 from zero for A e = b as the low-precision
    forms run it: operators of `lowered(H, precision)` (BF16 values held in
    FP32), FP32 vectors, the CG scalars from FP32 dot products, the coarsest
    level solved by the FP64 Cholesky factor, and the block-smoother inverses
    from the FP64 operators.  Returns e (FP64).  Used to measure how far the
    rounding of FP32 arithmetic moves one cycle; `transposed` applies the
    (symmetric) operators as row vector times matrix, another summation
    order, i.e. another rounding realisation of the same cycle."""
    import scipy.linalg

    Hl = lowered(H, precision)
    ops = [A.astype(np.float32) for A in Hl.ops[:-1]]
    P = [Pk.astype(np.float32) for Pk in Hl.prolong]
    factor = coarsest_factor(H.ops[-1])
    pre = smoothers(H, smoother)
    l = len(H.ops)

    def iterate(i, rhs, e0, n):
        # transposed: the same symmetric product summed in the other order
        apply = ops[i].__rmatmul__ if transposed else ops[i].__matmul__
        if pre is None:
            return cg(apply, rhs, e0, n)
        prec = pre[i]
        return pcg(apply, lambda v: prec(v.astype(np.float64)).astype(np.float32), rhs, e0, n)

    if l == 1:
        return scipy.linalg.cho_solve(factor, b)
    r = [None] * l
    et = [None] * l
    r[0] = b.astype(np.float32)
    for i in range(l - 1):
        n = n_f if i == 0 else n_c
        et[i] = iterate(i, r[i], None, n)
        r[i + 1] = P[i].T @ (r[i] - ops[i] @ et[i])
    e = scipy.linalg.cho_solve(factor, r[l - 1].astype(np.float64)).astype(np.float32)
    for i in range(l - 2, -1, -1):
        n = n_f if i == 0 else n_c
        et[i] = et[i] + P[i] @ e
        e = iterate(i, r[i], et[i], n)
    return e.astype(np.float64)


def ir_solve(H, b: np.ndarray, precision: str = "fp32", rtol: float = 1e-8,
             max_outer: int = 500, n_f: int = 1, n_c: int = 40,
             smoother: str = "cg") -> SolveResult:
    A = H.ops[0]
    Hl = lowered(H, precision)
    factor = coarsest_factor(H.ops[-1])
    # the block-smoother inverses come from the FP64 operators
    precs = smoothers(H, smoother)
    x = np.zeros_like(b)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return SolveResult(x, 0, True, [0.0])
    hist = []
    for it in range(max_outer + 1):
        res = b - A @ x
        rel = float(np.linalg.norm(res)) / nb
        hist.append(rel)
        if rel < rtol:
            return SolveResult(x, it, True, hist)
        if it == max_outer:
            break
        x = x + vcycle(Hl, np.zeros_like(b), res, n_f, n_c, factor, r1=res, precs=precs)
    return SolveResult(x, max_outer, False, hist)

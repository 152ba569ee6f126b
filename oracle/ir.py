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
entrywise to the low precision; the V-cycle arithmetic stays FP64.  BF16
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

from .vcycle import SolveResult, coarsest_factor, vcycle


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


def lowered(H, precision: str):
    """A copy of the hierarchy with stored operators and transfers rounded
    (the coarsest operator stays FP64)."""
    rnd = ROUNDING[precision]
    Hl = copy.copy(H)
    Hl.ops = [rnd(A) for A in H.ops[:-1]] + [H.ops[-1]]
    Hl.prolong = [rnd(P) for P in H.prolong]
    return Hl


def ir_solve(H, b: np.ndarray, precision: str = "fp32", rtol: float = 1e-8,
             max_outer: int = 500, n_f: int = 1, n_c: int = 40,
             smoother: str = "cg") -> SolveResult:
    A = H.ops[0]
    Hl = lowered(H, precision)
    factor = coarsest_factor(H.ops[-1])
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
        x = x + vcycle(Hl, np.zeros_like(b), res, n_f, n_c, factor, r1=res,
                       smoother=smoother)
    return SolveResult(x, max_outer, False, hist)

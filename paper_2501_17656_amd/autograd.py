"""Differentiable loss L = b^T A^{-1} b, A = K(p; l) + s I in H2 form.

Forward: one H2-MG solve A x = b and L = b^T x.  Backward (hand-written
adjoint; A is symmetric, so the adjoint solve is the forward solve and x is
reused): the library builds the H2 matrices of dk/dl and of g = k'(r)/r on
the same tree and returns
    dL/dl = -x^T (dA/dl) x,  dL/ds = -x^T x,
    dL/dp_ia = -2 x_i [p_ia (G x)_i - (G (x * p_.a))_i],  dL/db = 2 x,
each multiplied by the incoming gradient.  Every product and reduction runs
in libh2mg.so; this module only passes tensors through the C ABI.
"""
from __future__ import annotations

import torch

from .h2mg import H2Matrix


class _QuadraticLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, points, length_scale, shift, b, cfg):
        g = H2Matrix(points.detach().contiguous(), cfg["kernel"], float(length_scale), float(shift),
                     cfg["leaf"], cfg["eta"], cfg["m"])
        bd = b.detach().contiguous()
        x, info = g.solve(bd, rtol=cfg["rtol"], smoother=cfg["smoother"], method=cfg["method"],
                          max_cycles=cfg["max_cycles"], precision=cfg["precision"])
        loss, _, _, _, _ = g.quadratic_gradient(None, None, bd, x)
        ctx.g, ctx.x, ctx.b, ctx.info = g, x, bd, info
        ctx.dtypes = (length_scale, shift)
        return torch.tensor(loss, dtype=torch.float64, device=points.device)

    @staticmethod
    def backward(ctx, grad_out):
        g, x, b = ctx.g, ctx.x, ctx.b
        need_p, need_l, need_s, need_b = ctx.needs_input_grad[:4]
        scale = float(grad_out)
        h_dl = g.derivative("dl") if need_l else None
        h_g = g.derivative("g") if need_p else None
        try:
            _, dl, ds, gp, gb = g.quadratic_gradient(h_dl, h_g, b, x, scale, b_grad=need_b)
        finally:
            for d in (h_dl, h_g):
                if d is not None:
                    d.close()
        ell, s = ctx.dtypes

        def like(v, ref):
            if not torch.is_tensor(ref):
                return None
            return torch.tensor(v, dtype=ref.dtype, device=ref.device)
        return (gp if need_p else None, like(dl, ell) if need_l else None,
                like(ds, s) if need_s else None, gb if need_b else None, None)


def quadratic_loss(points, length_scale, shift, b, kernel: str = "exp", leaf: int = 64,
                   eta: float = 0.7, m: int = 4, rtol: float = 1e-10, smoother: str = "bj",
                   method: str = "v", max_cycles: int = 500, precision: str = "fp64"):
    """L = b^T A^{-1} b with A the H2 approximation of K(points; length_scale)
    + shift I, differentiable in points (n x dim), length_scale, shift (0-d
    tensors or floats) and b (device float64 tensors).  The solve stops at
    relative residual rtol, which bounds the accuracy of L and its gradient;
    precision "fp32" / "bf16" runs its cycles in that precision inside FP64
    refinement (same fixed point)."""
    cfg = dict(kernel=kernel, leaf=int(leaf), eta=float(eta), m=int(m), rtol=float(rtol),
               smoother=smoother, method=method, max_cycles=int(max_cycles), precision=precision)
    return _QuadraticLoss.apply(points, length_scale, shift, b, cfg)

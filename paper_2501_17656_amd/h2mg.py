"""Thin Python layer over the C ABI (argument marshalling only).

Device buffers are torch tensors on the current HIP device; work is queued
on torch's current stream.  No numerical step happens here.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import check, lib

KERNELS = {"exp": 0, "gauss": 1, "matern32": 2, "laplace": 3}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
SMOOTHERS = {"cg": 0, "bj": 1}
METHODS = {"v": 0, "w": 1, "f": 2, "cg": 3}
DERIVATIVES = {"value": 0, "dl": 1, "g": 2}


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements (got {t.numel()})")
    return ctypes.c_void_p(t.data_ptr())


def _info_dict(h, info, st, message=""):
    hist = (ctypes.c_double * max(info.history_len, 1))()
    lib().h2mg_solve_history(h._h, hist, info.history_len)
    return {"cycles": info.cycles, "converged": bool(info.converged),
            "rel_residual": info.rel_residual, "solve_seconds": info.solve_seconds,
            "history": list(hist)[:info.history_len], "status": _lib.STATUS.get(st, st),
            "message": message}


class Plan:
    """Host-side cluster tree and block partition of a point set."""

    def __init__(self, points: np.ndarray, leaf: int, eta: float, m: int):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        n, dim = pts.shape
        opts = _lib.BuildOpts(int(leaf), float(eta), int(m))
        h = ctypes.c_void_p()
        check(lib().h2mg_plan_create(pts.ctypes.data_as(ctypes.c_void_p), n, dim,
                                     ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        info = _lib.PlanInfo()
        check(lib().h2mg_plan_query(h, ctypes.byref(info)))
        self.n, self.dim, self.depth = info.n, info.dim, info.depth
        self.d_top = None if info.d_top < 0 else info.d_top
        self.rank, self.leaf_min, self.leaf_max = info.rank, info.leaf_min, info.leaf_max

    def perm(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        check(lib().h2mg_plan_perm(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def offsets(self, depth: int) -> np.ndarray:
        out = np.empty((1 << depth) + 1, dtype=np.int64)
        check(lib().h2mg_plan_offsets(self._h, depth, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def pairs(self, depth: int, far: bool) -> np.ndarray:
        cnt = ctypes.c_int64()
        check(lib().h2mg_plan_pair_count(self._h, depth, int(far), ctypes.byref(cnt)))
        out = np.empty((cnt.value, 2), dtype=np.int64)
        if cnt.value:
            check(lib().h2mg_plan_pairs(self._h, depth, int(far), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            lib().h2mg_plan_destroy(self._h)
            self._h = None


class H2Matrix:
    """H2 approximation of a kernel matrix, built and applied on the GPU."""

    def __init__(self, points, kernel: str = "matern32", length_scale: float = 0.2,
                 shift: float = 1e-3, leaf: int = 128, eta: float = 0.7, m: int = 4,
                 derivative: str = "value", scale=None, diag=None):
        """scale, diag: optional per-point s and d (float64 device tensors,
        user order) of the scaled form diag(s) K diag(s) + diag(d)."""
        if points is None:                 # wrapped handle (see derivative())
            return
        pts = points if points.is_contiguous() else points.contiguous()
        n, dim = pts.shape
        _dev_f64(pts, name="points")
        self.n, self.dim = int(n), int(dim)
        ker = _lib.Kernel(KERNELS[kernel], float(length_scale), float(shift), DERIVATIVES[derivative])
        opts = _lib.BuildOpts(int(leaf), float(eta), int(m))
        h = ctypes.c_void_p()
        if scale is None and diag is None:
            check(lib().h2mg_build(ctypes.c_void_p(pts.data_ptr()), self.n, self.dim, ctypes.byref(ker),
                                   ctypes.byref(opts), _stream(), ctypes.byref(h)))
        else:
            check(lib().h2mg_build_scaled(
                ctypes.c_void_p(pts.data_ptr()), self.n, self.dim, ctypes.byref(ker), ctypes.byref(opts),
                _dev_f64(scale, self.n, "scale") if scale is not None else None,
                _dev_f64(diag, self.n, "diag") if diag is not None else None, _stream(), ctypes.byref(h)))
        self._h = h

    # ------------------------------------------------------------ derivatives
    def derivative(self, which: str) -> "H2Matrix":
        """H2 matrix of dk/dl ("dl") or g = k'(r)/r ("g") on the same points
        and tree (shift 0)."""
        h = ctypes.c_void_p()
        check(lib().h2mg_build_derivative(self._h, DERIVATIVES[which], _stream(), ctypes.byref(h)))
        d = H2Matrix(None)
        d.n, d.dim, d._h = self.n, self.dim, h
        return d

    def quadratic_gradient(self, h_dl, h_g, b, x, scale: float = 1.0, b_grad: bool = False):
        """L = b^T x and scale * (dL/dl, dL/ds, dL/dp, dL/db) for x = A^{-1} b.
        dL/dl needs h_dl = derivative("dl"), dL/dp needs h_g = derivative("g");
        pass None to skip them.  Returns (L, dl or None, ds, grad_points or
        None, grad_b or None)."""
        import torch
        loss, gl, gs = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        gp = (torch.empty((self.n, self.dim), dtype=torch.float64, device=x.device)
              if h_g is not None else None)
        gb = torch.empty_like(x) if b_grad else None
        check(lib().h2mg_quadratic_gradient(
            self._h, h_dl._h if h_dl is not None else None, h_g._h if h_g is not None else None,
            _dev_f64(b, self.n, "b"), _dev_f64(x, self.n, "x"), float(scale), ctypes.byref(loss),
            ctypes.byref(gl) if h_dl is not None else None, ctypes.byref(gs),
            _dev_f64(gp) if gp is not None else None, _dev_f64(gb) if gb is not None else None,
            _stream()))
        return loss.value, (gl.value if h_dl is not None else None), gs.value, gp, gb

    # ------------------------------------------------------------ products
    def matvec(self, x, out=None):
        import torch
        y = torch.empty_like(x) if out is None else out
        check(lib().h2mg_matvec(self._h, _dev_f64(x, self.n, "x"), _dev_f64(y, self.n, "y"), _stream()))
        return y

    def matvec_multi(self, X, out=None):
        """Y = A_H2 X for X of shape (n, nrhs), nrhs <= 16 (FP64; needs a rank
        of 9 to 64; the close blocks are the stored tiles after store_near(),
        else they are evaluated from the points inside the product)."""
        import torch
        if X.dim() != 2 or X.shape[0] != self.n:
            raise ValueError("X must have shape (n, nrhs)")
        nrhs = int(X.shape[1])
        xp = _dev_f64(X, name="X")
        Y = torch.empty_like(X) if out is None else out
        yp = _dev_f64(Y, name="out")
        if tuple(Y.shape) != tuple(X.shape):
            raise ValueError(f"out must have the shape of X {tuple(X.shape)} (got {tuple(Y.shape)})")
        check(lib().h2mg_matvec_multi(self._h, nrhs, xp, nrhs, yp, nrhs, _stream()))
        return Y

    def set_near_quadrature(self, qy, qu) -> None:
        """Close entries by quadrature: qy (n, nq, dim) sub-points and qu (n, nq)
        weights per point (float64, GPU, user order); stores the near field."""
        if qy.dim() != 3 or qy.shape[0] != self.n or qy.shape[2] != self.dim:
            raise ValueError("qy must have shape (n, nq, dim)")
        nq = int(qy.shape[1])
        if tuple(qu.shape) != (self.n, nq):
            raise ValueError(f"qu must have shape ({self.n}, {nq})")
        check(lib().h2mg_set_near_quadrature(self._h, _dev_f64(qy, name="qy"), _dev_f64(qu, name="qu"), nq,
                                             _stream()))

    def store_near(self, enable: bool = True) -> None:
        """Store the close leaf blocks as FP64 tiles (enable) or release them;
        FP64 fine-level products then stream the tiles."""
        check(lib().h2mg_store_near(self._h, int(bool(enable)), _stream()))

    def setup(self, precisions=("fp64",)) -> None:
        mask = 0
        for p in precisions:
            mask |= 1 << PRECISIONS[p]
        check(lib().h2mg_setup_mg(self._h, mask, _stream()))

    @property
    def levels(self) -> int:
        v = ctypes.c_int32()
        check(lib().h2mg_level_count(self._h, ctypes.byref(v)))
        return v.value

    def level_size(self, level: int) -> int:
        v = ctypes.c_int64()
        check(lib().h2mg_level_size(self._h, level, ctypes.byref(v)))
        return v.value

    def level_apply(self, level: int, x, out=None, precision: str = "fp64"):
        """y = A_k x on level k (FP64 vectors; precision "fp32" / "bf16" applies
        the low-precision operators of the mixed cycles, prepared by setup)."""
        import torch
        y = torch.empty_like(x) if out is None else out
        nk = self.level_size(level)
        xp, yp = _dev_f64(x, nk, "x"), _dev_f64(y, nk, "y")
        if precision == "fp64":
            check(lib().h2mg_level_apply(self._h, level, xp, yp, _stream()))
        else:
            check(lib().h2mg_level_apply_precision(self._h, level, PRECISIONS[precision], xp, yp,
                                                   _stream()))
        return y

    def restrict(self, level: int, r):
        import torch
        out = torch.empty(self.level_size(level + 1), dtype=torch.float64, device=r.device)
        check(lib().h2mg_restrict(self._h, level, _dev_f64(r, self.level_size(level), "r"),
                                  _dev_f64(out), _stream()))
        return out

    def prolong(self, level: int, e_next):
        import torch
        out = torch.empty(self.level_size(level), dtype=torch.float64, device=e_next.device)
        check(lib().h2mg_prolong(self._h, level, _dev_f64(e_next, self.level_size(level + 1), "e"),
                                 _dev_f64(out), _stream()))
        return out

    def smooth(self, level: int, r, nsteps: int, e0=None, smoother: str = "cg"):
        """e = Iter(A_level, r, e0): nsteps of the smoother in FP64."""
        import torch
        nk = self.level_size(level)
        e = torch.zeros_like(r) if e0 is None else e0.clone()
        check(lib().h2mg_smooth(self._h, level, _dev_f64(r, nk, "r"), _dev_f64(e, nk, "e"), int(nsteps),
                                SMOOTHERS[smoother], int(e0 is not None), _stream()))
        return e

    # ------------------------------------------------------------ solves
    @staticmethod
    def _opts(rtol, n_fine, n_coarse, max_cycles, precision, use_x0, smoother="cg", method="v"):
        return _lib.SolveOpts(int(n_fine), int(n_coarse), float(rtol), int(max_cycles),
                              PRECISIONS[precision], int(use_x0), SMOOTHERS[smoother],
                              METHODS[method])

    def vcycle(self, x0, b, n_fine: int = 1, n_coarse: int = 40, out=None, smoother: str = "cg",
               method: str = "v"):
        """One cycle (V, W or F) from x0."""
        import torch
        x = torch.empty_like(b) if out is None else out
        o = self._opts(1e-8, n_fine, n_coarse, 1, "fp64", 1, smoother, method)
        check(lib().h2mg_vcycle(self._h, _dev_f64(x0, self.n, "x0"), _dev_f64(b, self.n, "b"),
                                _dev_f64(x, self.n, "x"), ctypes.byref(o), _stream()))
        return x

    def solve(self, b, rtol: float = 1e-8, n_fine: int = 1, n_coarse: int = 40,
              max_cycles: int = 500, precision: str = "fp64", x0=None, raise_on_error: bool = True,
              smoother: str = "cg", method: str = "v", noalloc: bool = False, out=None):
        """Solve A_H2 x = b by V-, W- or F-cycles, or by CG alone (method
        "cg"; max_cycles then counts CG iterations).  Returns (x, info).
        noalloc: h2mg_solve_noalloc, which allocates no device memory (its
        vectors live in the library's fixed scratch region; the hierarchy in
        this precision, and the block smoother's inverses, must exist).
        out: write x there (with x0, out holds the initial guess on entry)."""
        import torch
        if out is None:
            x = torch.zeros_like(b) if x0 is None else x0.clone()
        else:
            x = out
            if x0 is not None and x0.data_ptr() != out.data_ptr():
                x.copy_(x0)
        o = self._opts(rtol, n_fine, n_coarse, max_cycles, precision, x0 is not None, smoother,
                       method)
        info = _lib.SolveInfo()
        fn = lib().h2mg_solve_noalloc if noalloc else lib().h2mg_solve
        st = fn(self._h, _dev_f64(b, self.n, "b"), _dev_f64(x, self.n, "x"),
                ctypes.byref(o), ctypes.byref(info), _stream())
        msg = _lib.last_error() if st != 0 else ""
        out = _info_dict(self, info, st, msg)
        if st != 0 and raise_on_error:
            check(st, msg)
        return x, out

    def solve_multi(self, B, rtol: float = 1e-8, n_fine: int = 1, n_coarse: int = 40,
                    max_cycles: int = 500, precision: str = "fp64", X0=None, raise_on_error: bool = True,
                    smoother: str = "cg", method: str = "v"):
        """Solve A_H2 X = B for B of shape (n, nrhs), nrhs <= 16, all columns
        per cycle (needs a rank of 9 to 64; the close blocks are the stored
        tiles after store_near(), else evaluated inside the products).
        Returns (X, info); info["column_residuals"] holds each column's final
        relative residual."""
        import torch
        if B.dim() != 2 or B.shape[0] != self.n:
            raise ValueError("B must have shape (n, nrhs)")
        nrhs = int(B.shape[1])
        bp = _dev_f64(B, name="B")
        if X0 is not None:
            _dev_f64(X0, name="X0")
            if tuple(X0.shape) != tuple(B.shape):
                raise ValueError(f"X0 must have the shape of B {tuple(B.shape)} (got {tuple(X0.shape)})")
        X = torch.zeros_like(B) if X0 is None else X0.clone()
        o = self._opts(rtol, n_fine, n_coarse, max_cycles, precision, X0 is not None, smoother, method)
        info = _lib.SolveInfo()
        cr = (ctypes.c_double * nrhs)()
        st = lib().h2mg_solve_multi(self._h, nrhs, bp, nrhs, _dev_f64(X, name="X"), nrhs,
                                    ctypes.byref(o), ctypes.byref(info), cr, _stream())
        msg = _lib.last_error() if st != 0 else ""
        out = _info_dict(self, info, st, msg)
        out["column_residuals"] = list(cr)
        if st != 0 and raise_on_error:
            check(st, msg)
        return X, out

    KERNEL_KINDS = {"gemv_fp64": 0, "gemv_fp32": 1, "gemv_bf16": 2, "near_fp64": 3, "near_fp32": 4,
                    "near_gemv_fp64": 5, "near_gemm16_fp64": 6}

    def set_graphs(self, enabled: bool) -> None:
        """Launch each solver cycle as one captured HIP graph."""
        check(lib().h2mg_set_graphs(self._h, int(bool(enabled))))

    def set_autotune(self, enabled: bool) -> None:
        """Choose the tile-run length of every 16-column task set by timing
        the candidates on this device (applies from the next 16-column call)."""
        check(lib().h2mg_set_autotune(self._h, int(bool(enabled))))

    def block_tuning(self) -> dict:
        """Run length, measured ms (product + reduce) and tiles read per
        product of every built 16-column task set: keys "near", "fine" and
        the depths of the restricted operators."""
        out = {}
        for which in [-2, -1] + list(range(0, 64)):
            run, ms, tiles = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int64()
            st = lib().h2mg_block_tuning(self._h, which, ctypes.byref(run), ctypes.byref(ms), ctypes.byref(tiles))
            if st != 0:
                break
            if run.value:
                key = {-2: "near", -1: "fine"}.get(which, which)
                out[key] = {"run": run.value, "ms": round(ms.value, 4), "tiles_read": tiles.value}
        return out

    def set_timing(self, enabled: bool) -> None:
        check(lib().h2mg_set_timing(self._h, int(bool(enabled))))

    def kernel_stats(self, kind: str) -> dict:
        n, ms, work = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        check(lib().h2mg_kernel_stats(self._h, self.KERNEL_KINDS[kind], ctypes.byref(n),
                                      ctypes.byref(ms), ctypes.byref(work)))
        return {"launches": n.value, "ms": ms.value, "work": work.value}

    def gemv_launch_info(self, level: int) -> dict:
        """Waves and stored blocks of the block-GEMV launch of level `level`'s
        product (1: the fine couplings)."""
        t, b = ctypes.c_int64(), ctypes.c_int64()
        check(lib().h2mg_gemv_launch_info(self._h, level, ctypes.byref(t), ctypes.byref(b)))
        return {"tasks": t.value, "blocks": b.value, "grid": (t.value + 3) // 4}

    def memory_bytes(self) -> int:
        v = ctypes.c_int64()
        check(lib().h2mg_memory_bytes(self._h, ctypes.byref(v)))
        return v.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            check(lib().h2mg_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(problems, rtol: float = 1e-8, n_fine: int = 1, n_coarse: int = 40, max_cycles: int = 500,
                precision: str = "fp64", smoother: str = "cg", method: str = "v", nstreams: int = 0,
                raise_on_error: bool = True, mode: str = "streams"):
    """Solve independent problems together: `problems` is a list of
    (H2Matrix, B) with B of shape (n_i, nrhs_i), nrhs_i <= 16 (distinct
    matrices).  mode "streams": each problem on one of `nstreams` streams
    (h2mg_solve_batch); "group": all problems cycle together and every tile
    product step is one launch over all of them (h2mg_solve_group).
    Returns (list of X, list of info dicts)."""
    if mode not in ("streams", "group"):
        raise ValueError(f"unknown mode {mode!r}")
    import torch
    k = len(problems)
    hs = (ctypes.c_void_p * k)()
    nr = (ctypes.c_int32 * k)()
    bp = (ctypes.c_void_p * k)()
    xp = (ctypes.c_void_p * k)()
    xs = []
    for i, (g, B) in enumerate(problems):
        if B.dim() != 2 or B.shape[0] != g.n:
            raise ValueError(f"problem {i}: B must have shape (n, nrhs)")
        X = torch.zeros_like(B)
        xs.append(X)
        hs[i] = g._h
        nr[i] = int(B.shape[1])
        bp[i] = _dev_f64(B, name="B").value
        xp[i] = _dev_f64(X, name="X").value
    o = H2Matrix._opts(rtol, n_fine, n_coarse, max_cycles, precision, 0, smoother, method)
    infos = (_lib.SolveInfo * k)()
    stats = (ctypes.c_int32 * k)()
    if mode == "group":
        st = lib().h2mg_solve_group(k, hs, nr, bp, nr, xp, nr, ctypes.byref(o), infos, stats, _stream())
    else:
        st = lib().h2mg_solve_batch(k, hs, nr, bp, nr, xp, nr, ctypes.byref(o), infos, stats, int(nstreams),
                                    _stream())
    msg = _lib.last_error() if st != 0 else ""
    out = [_info_dict(g, infos[i], stats[i], msg if stats[i] else "") for i, (g, _) in enumerate(problems)]
    if st != 0 and raise_on_error:
        check(st, msg)
    return xs, out


# ---------------------------------------------------------------- boundary elements
def bem_quadrature7(vertices, triangles):
    """Radon's seven-point rule per triangle: points (nt, 7, 3) and weights
    times sqrt(area) (nt, 7), for H2Matrix.set_near_quadrature."""
    import torch
    nt = int(triangles.shape[0])
    if triangles.dtype != torch.int64 or not triangles.is_cuda or not triangles.is_contiguous():
        raise TypeError("triangles must be a contiguous int64 tensor on the GPU")
    qy = torch.empty((nt, 7, 3), dtype=torch.float64, device=vertices.device)
    qu = torch.empty((nt, 7), dtype=torch.float64, device=vertices.device)
    check(lib().h2mg_bem_quadrature7(_dev_f64(vertices), int(vertices.shape[0]),
                                     ctypes.c_void_p(triangles.data_ptr()), nt, _dev_f64(qy), _dev_f64(qu),
                                     _stream()))
    return qy, qu


def bem_panels(vertices, triangles):
    """Centroids (nt x 3), scale sqrt(area) and diagonal I_i / (4 pi) of a
    triangle mesh (device float64 vertices nv x 3, int64 triangles nt x 3)."""
    import torch
    nt = int(triangles.shape[0])
    if triangles.dtype != torch.int64 or not triangles.is_cuda or not triangles.is_contiguous():
        raise TypeError("triangles must be a contiguous int64 tensor on the GPU")
    y = torch.empty((nt, 3), dtype=torch.float64, device=vertices.device)
    s = torch.empty(nt, dtype=torch.float64, device=vertices.device)
    d = torch.empty(nt, dtype=torch.float64, device=vertices.device)
    check(lib().h2mg_bem_panels(_dev_f64(vertices), int(vertices.shape[0]),
                                ctypes.c_void_p(triangles.data_ptr()), nt, _dev_f64(y), _dev_f64(s),
                                _dev_f64(d), _stream()))
    return y, s, d


def bem_point_source_rhs(centroids, scale, x0):
    """W^(1/2) f for the point source x0 (three floats)."""
    import torch
    n = int(scale.numel())
    f = torch.empty(n, dtype=torch.float64, device=scale.device)
    x = (ctypes.c_double * 3)(*[float(v) for v in x0])
    check(lib().h2mg_bem_point_source_rhs(_dev_f64(centroids), _dev_f64(scale, n, "scale"), n, x,
                                          _dev_f64(f), _stream()))
    return f


def bem_harmonic_rhs(centroids, scale, coeffs):
    """W^(1/2) f for f = sum_k c_k h_k, the harmonic basis 1, x, y, z, xy, yz,
    zx, x^2 - y^2, x^2 + y^2 - 2 z^2 (nine floats)."""
    import torch
    n = int(scale.numel())
    c = [float(v) for v in coeffs]
    if len(c) != 9:
        raise ValueError("coeffs must hold 9 values")
    f = torch.empty(n, dtype=torch.float64, device=scale.device)
    check(lib().h2mg_bem_harmonic_rhs(_dev_f64(centroids), _dev_f64(scale, n, "scale"), n,
                                      (ctypes.c_double * 9)(*c), _dev_f64(f), _stream()))
    return f


def bem_density(y, scale):
    """sigma = y / s."""
    import torch
    n = int(scale.numel())
    out = torch.empty_like(y)
    check(lib().h2mg_bem_density(_dev_f64(y, n, "y"), _dev_f64(scale, n, "scale"), n, _dev_f64(out),
                                 _stream()))
    return out

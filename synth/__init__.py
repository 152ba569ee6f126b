"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and names workloads. It holds none of
the method's arithmetic (no kernel, tree, basis or solver code), so the oracle
and the HIP path can both consume its output without sharing any numerics.

All generators use numpy's PCG64 (`numpy.random.default_rng(seed)`) and return
float64 arrays in *user order*.  Points are row-major (n, dim).

The workloads mirror the shapes of the paper's experiments (kernel matrices
on point clouds in the unit square/cube, Section 4) with the parameters the
benchmarks are quoted on.  There is no public dataset involved.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "uniform_points", "gaussian_mixture_points", "tensor_grid_points",
    "normal_vector", "bumpy_torus_mesh", "Workload", "WORKLOADS", "workload",
]


def uniform_points(n: int, dim: int, seed: int = 0) -> np.ndarray:
    """n points i.i.d. uniform in [0, 1)^dim."""
    rng = np.random.default_rng(seed)
    return rng.random((int(n), int(dim)), dtype=np.float64)


def gaussian_mixture_points(n: int, dim: int, components: int = 8,
                            sigma: float = 0.05, seed: int = 0) -> np.ndarray:
    """n points from an isotropic Gaussian mixture.

    Component centres are uniform in [0.2, 0.8)^dim, weights are equal, and
    every component has standard deviation `sigma` per axis.
    """
    rng = np.random.default_rng(seed)
    centres = 0.2 + 0.6 * rng.random((components, dim))
    which = rng.integers(0, components, size=int(n))
    return centres[which] + sigma * rng.standard_normal((int(n), int(dim)))


def tensor_grid_points(n: int, dim: int = 2) -> np.ndarray:
    """Cell-centred uniform tensor grid on the unit square/cube.

    round(n ** (1/dim)) points per side (the paper's grids are not always
    perfect squares, so the count is rounded per side).
    """
    side = max(1, int(round(n ** (1.0 / dim))))
    g = (np.arange(side, dtype=np.float64) + 0.5) / side
    mesh = np.meshgrid(*([g] * dim), indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def bumpy_torus_mesh(n_major: int, n_minor: int, bumps: int = 40, amplitude: float = 0.05,
                     width: float = 0.1, major: float = 1.0, minor: float = 0.35,
                     seed: int = 0):
    """Closed triangulated surface: a torus (major radius `major`, tube radius
    `minor`) whose tube radius carries `bumps` Gaussian bumps of height
    `amplitude` and width `width` (measured along the surface) at seeded
    random positions.  Parameter grid n_major x n_minor, each cell split
    into two triangles, so there are 2 * n_major * n_minor triangles.
    Returns (vertices (nv, 3) float64, triangles (nt, 3) int64), triangles
    oriented outwards."""
    rng = np.random.default_rng(seed)
    th_c = 2 * np.pi * rng.random(bumps)
    ph_c = 2 * np.pi * rng.random(bumps)
    th = 2 * np.pi * np.arange(n_major) / n_major
    ph = 2 * np.pi * np.arange(n_minor) / n_minor
    T, F = np.meshgrid(th, ph, indexing="ij")
    rad = np.full(T.shape, float(minor))
    for k in range(bumps):
        dth = np.angle(np.exp(1j * (T - th_c[k]))) * major
        dph = np.angle(np.exp(1j * (F - ph_c[k]))) * minor
        rad += amplitude * np.exp(-(dth ** 2 + dph ** 2) / (2 * width ** 2))
    ring = major + rad * np.cos(F)
    V = np.stack([ring * np.cos(T), ring * np.sin(T), rad * np.sin(F)], axis=-1).reshape(-1, 3)
    i = np.arange(n_major)[:, None]
    j = np.arange(n_minor)[None, :]
    a = i * n_minor + j
    b = ((i + 1) % n_major) * n_minor + j
    c = ((i + 1) % n_major) * n_minor + (j + 1) % n_minor
    d = i * n_minor + (j + 1) % n_minor
    tris = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3),
                           np.stack([a, c, d], -1).reshape(-1, 3)])
    return V, tris.astype(np.int64)


def harmonic_coefficients(seed: int = 7) -> np.ndarray:
    """Nine N(0,1) coefficients for the degree-2 harmonic polynomial basis
    (1, x, y, z, xy, yz, zx, x^2 - y^2, x^2 + y^2 - 2 z^2) of a random
    boundary-element right-hand side."""
    return np.random.default_rng(seed).standard_normal(9)


def normal_vector(n: int, seed: int = 1, nrhs: int = 1) -> np.ndarray:
    """Standard normal vector (n,) or matrix (n, nrhs)."""
    rng = np.random.default_rng(seed)
    if nrhs == 1:
        return rng.standard_normal(int(n))
    return rng.standard_normal((int(n), int(nrhs)))


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named synthetic problem: points, kernel and H2 build parameters."""
    name: str
    n: int
    dim: int
    kernel: str            # "exp" | "gauss" | "matern32"
    length_scale: float
    shift: float
    leaf: int
    eta: float
    cheb_m: int            # Chebyshev nodes per axis; rank r = cheb_m ** dim
    points: str = "uniform"
    point_seed: int = 0
    rhs_seed: int = 1
    x_seed: int = 2

    @property
    def rank(self) -> int:
        return self.cheb_m ** self.dim

    def make_points(self) -> np.ndarray:
        if self.points == "uniform":
            return uniform_points(self.n, self.dim, self.point_seed)
        if self.points == "gmm":
            return gaussian_mixture_points(self.n, self.dim, 8, 0.05,
                                           self.point_seed)
        if self.points == "grid":
            return tensor_grid_points(self.n, self.dim)
        raise ValueError(self.points)

    def make_rhs(self, nrhs: int = 1) -> np.ndarray:
        return normal_vector(self.n, self.rhs_seed, nrhs)

    def make_x(self) -> np.ndarray:
        return normal_vector(self.n, self.x_seed)

    def scaled(self, n: int) -> "Workload":
        """The same workload shape at another size."""
        return dataclasses.replace(self, n=int(n), name=f"{self.name}@{n}")


WORKLOADS = {
    # small 2D exponential-kernel problem (N = 4096, leaf 64, rank 16)
    "exp2d_4k": Workload("exp2d_4k", 4096, 2, "exp", 0.1, 1e-2, 64, 0.7, 4),
    # headline 3D Matern-3/2 problem (N = 2^20, leaf 128, rank 64)
    "matern3d_1m": Workload("matern3d_1m", 1 << 20, 3, "matern32", 0.2, 1e-3,
                            128, 0.7, 4),
    # the same points, kernel and H2 parameters with the diagonal shift raised
    # to 0.3: the rank-64 Chebyshev approximation of the 1e-3-shift matrix has
    # eigenvalues down to -0.0936 at this size, so every shift below 0.095 is
    # indefinite; at 0.1 (smallest eigenvalue about 0.005) the V-cycle needs
    # hundreds of cycles, at 0.3 it converges in about 25
    "matern3d_1m_spd": Workload("matern3d_1m_spd", 1 << 20, 3, "matern32", 0.2, 0.3,
                                128, 0.7, 4),
    # the same with the shift raised to 1 (solver growth and smoothing sweeps)
    "matern3d_1m_shift1": Workload("matern3d_1m_shift1", 1 << 20, 3, "matern32", 0.2, 1.0,
                                   128, 0.7, 4),
    # Gaussian-kernel problem on Gaussian-mixture clouds (rank 27, leaf 64)
    "gauss3d_gmm": Workload("gauss3d_gmm", 65536, 3, "gauss", 0.1, 1e-2, 64,
                            0.7, 3, points="gmm"),
    # exponential kernel in 3D (rank 64, leaf 128)
    "exp3d_256k": Workload("exp3d_256k", 262144, 3, "exp", 0.15, 1e-2, 128,
                           0.7, 4),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]

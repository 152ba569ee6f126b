"""MI355X-native H2 matrix and H2-MG solver (HIP kernels behind a C ABI).

`H2Matrix` builds the H2 approximation of a kernel matrix from points on the
GPU, multiplies by it and solves with the H2-MG V-cycle, one right-hand side
at a time (`matvec`, `solve`) or 16 at a time (`matvec_multi`,
`solve_multi`); `solve_batch` solves many independent problems together;
`Plan` exposes the host-side cluster tree and block partition;
`quadratic_loss` is L = b^T A^{-1} b as a differentiable torch function.  Every numerical step runs in
libh2mg.so; this package only marshals arguments.
"""
from .h2mg import H2Matrix, Plan, KERNELS, PRECISIONS  # noqa: F401
from .h2mg import (bem_density, bem_harmonic_rhs, bem_panels, bem_point_source_rhs, bem_quadrature7,  # noqa: F401
                   solve_batch)
from ._lib import H2MGError  # noqa: F401
from .autograd import quadratic_loss  # noqa: F401

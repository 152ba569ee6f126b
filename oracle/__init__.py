"""Plain, slow CPU FP64 oracle for the H2 matvec and the H2-MG V-cycle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
(its own tree, partition, Chebyshev bases, orthogonalisation, Galerkin
operators, CG and V-cycle), and it reads inputs only from `synth`.

Paper sections followed (Sushnikova, Turkiyyah, Chow, Keyes, "H2-MG: A
multigrid method for hierarchical rank structured matrices"):

* kernels.py   -- kernel matrices (Section 4, eq. a_gau and eq. a_exp)
* tree.py      -- block partition by recursive bisection (Section 3.1)
* partition.py -- close/far block classification (Section 3.1, eq. f)
* cheb.py      -- nested cluster bases, transfers and couplings (Section 3.1,
                  eq. f, eq. s1, eq. h2), realised by tensor Chebyshev
                  interpolation
* h2.py        -- the H2 matrix and its matvec (Section 3.1, eq. h2 and the
                  matvec recursion that follows it)
* ortho.py     -- orthonormal bases assumed by the restriction (Section 3.3)
* galerkin.py  -- restricted operators A_k (Section 3.3, eq. a2_str)
* cg.py        -- the CG smoother Iter(A, r, e0) (Section 3.3)
* vcycle.py    -- Algorithm 1 and repeated V-cycles (Section 3.3)
* ir.py        -- FP64 iterative refinement around a low-precision V-cycle
                  (not in the paper; emulated by rounding stored operators)

Readings taken where the paper is silent are listed in each module header.

Parity status: every function here is pinned by a `-m "not gpu"` test
against closed forms, library routines, invariants or brute force, except
those whose header says "parity unpinned".
"""

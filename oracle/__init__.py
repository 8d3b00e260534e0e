"""FP64 CPU oracle for the epsilon-circulant RBD-preconditioned GMRES solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP implementation: every
function here is written from the paper with plain NumPy/SciPy (sparse
matrices, dense Fourier matrices, sparse LU), in float64.

Modules:
  discretize -- grid, K = -L_h (or the Q1 finite-element M and K), B_n,
                C_eps, the KKT matrices and the RHS
                (Section 1: eq. main_system_before, eq. matrix_A_before,
                eq. main_system, eq. matrix_A, eq. matrix_T)
  precond    -- P_eps^{-1} by the four steps of Section 2.1, the dense
                P_eps and P (eq. matrix_P_eps, eq. matrix_P), ideal RBD apply
  krylov     -- GMRES (left, right, flexible), MGS Arnoldi + Givens
  multigrid  -- one complex-shifted V-cycle (Section 3, Example 2)
  adjoint    -- A^{-T} solves, gradient maps, the reduced cost J_h
  examples   -- post-solve of y^N, p^0 and the error e_h (Section 3)

Parity status: every function above is pinned by a test under tests/
against a fact fixed by the paper or by mathematics (see the test names);
the multigrid V-cycle's detailed choices (smoother ordering, transfer
operators) are this project's reading, pinned by textbook properties but
not by a number printed in the paper.
"""
from . import discretize, precond, krylov, multigrid, adjoint, examples  # noqa: F401
from .discretize import Problem, make_problem  # noqa: F401

"""Oracle: one geometric-multigrid V-cycle for the complex-shifted spatial
systems (sigma I + tau K_a) z = r of Step 2 in Section 2.1 (test
infrastructure only).

Section 3 (Example 2) fixes only: one V-cycle, a Gauss-Seidel pre-smoother,
no post-smoother.  The remaining choices are this project's reading, stated
once here and implemented identically on the GPU:
  * zero initial guess; one Gauss-Seidel sweep per level, by default
    red-black (red = even index sum points first, then black); optionally
    ``smoother="lex"``, one sweep in the natural (lexicographic, x1 fastest)
    order, or ``smoother="sym"``, that sweep followed by one in the reverse
    order (symmetric Gauss-Seidel);
  * vertex-centred coarsening nx -> (nx-1)/2 (nx = 2^p - 1) down to a single
    point, which is solved exactly;
  * coarse operators re-discretised: sigma I + tau K_a with the coarse mesh
    width and a evaluated at the coarse face midpoints;
  * full-weighting restriction (tensor product of [1/4, 1/2, 1/4]) and
    multilinear prolongation; the coarse correction is added last.
"""
from __future__ import annotations

from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretize import stiffness


def prolongation_1d(nxc: int) -> sp.csr_matrix:
    """Linear interpolation from nxc coarse to 2*nxc+1 fine points."""
    nxf = 2 * nxc + 1
    rows, cols, vals = [], [], []
    for I in range(nxc):
        f = 2 * I + 1
        rows += [f - 1, f, f + 1]
        cols += [I, I, I]
        vals += [0.5, 1.0, 0.5]
    return sp.coo_matrix((vals, (rows, cols)), shape=(nxf, nxc)).tocsr()


def prolongation(dim: int, nxc: int) -> sp.csr_matrix:
    P1 = prolongation_1d(nxc)
    P = P1
    for _ in range(dim - 1):
        P = sp.kron(P1, P, format="csr")
    return P


def restriction(dim: int, nxc: int) -> sp.csr_matrix:
    """Full weighting: the transpose of the prolongation scaled by 2^-d."""
    return (prolongation(dim, nxc).T / 2 ** dim).tocsr()


def red_mask(dim: int, nx: int) -> np.ndarray:
    idx = np.arange(nx ** dim)
    s = np.zeros_like(idx)
    for axis in range(dim):
        s += (idx // nx ** axis) % nx
    return (s % 2) == 0


class ShiftedVCycle:
    """Hierarchy for sigma I + tau K_a; ``apply(r)`` is one V-cycle from z = 0."""

    def __init__(self, dim: int, nx: int, tau: float, coeff: Optional[Callable] = None, smoother: str = "rb"):
        if nx < 1 or (nx + 1) & nx:
            raise ValueError("multigrid needs nx = 2^p - 1")
        if smoother not in ("rb", "lex", "sym"):
            raise ValueError(smoother)
        self.dim = dim
        self.tau = tau
        self.smoother = smoother
        self.levels: List[dict] = []
        n = nx
        while True:
            K = stiffness(dim, n, coeff)
            lev = {"nx": n, "K": K, "red": red_mask(dim, n)}
            if n > 1:
                nc = (n - 1) // 2
                lev["P"] = prolongation(dim, nc)
                lev["R"] = restriction(dim, nc)
            self.levels.append(lev)
            if n == 1:
                break
            n = (n - 1) // 2

    def _matrix(self, lev: dict, sigma: complex) -> sp.csr_matrix:
        m = lev["nx"] ** self.dim
        return (sigma * sp.identity(m, format="csr", dtype=np.complex128)
                + self.tau * lev["K"].astype(np.complex128)).tocsr()

    def smooth(self, l: int, r: np.ndarray, sigma: complex) -> np.ndarray:
        """The pre-smoothing sweep(s) on level l from z = 0."""
        lev = self.levels[l]
        A = self._matrix(lev, sigma)
        if self.smoother == "rb":
            d = A.diagonal()
            off = A - sp.diags(d)
            red = lev["red"]
            z = np.zeros_like(r)
            # one red-black Gauss-Seidel sweep: red points, then black points
            z[red] = ((r - off @ z) / d)[red]
            z[~red] = ((r - off @ z) / d)[~red]
            return z
        # a Gauss-Seidel sweep in the natural order from z = 0 solves with the
        # lower triangle D + L of A; the reverse sweep corrects with D + U
        z = spla.spsolve_triangular(sp.tril(A, format="csr"), r, lower=True)
        if self.smoother == "sym":
            z = z + spla.spsolve_triangular(sp.triu(A, format="csr"), r - A @ z, lower=False)
        return z

    def _cycle(self, l: int, r: np.ndarray, sigma: complex) -> np.ndarray:
        lev = self.levels[l]
        A = self._matrix(lev, sigma)
        if lev["nx"] == 1:
            return r / A.diagonal()
        z = self.smooth(l, r, sigma)
        res = r - A @ z
        ec = self._cycle(l + 1, lev["R"] @ res, sigma)
        return z + lev["P"] @ ec

    def apply(self, r: np.ndarray, sigma: complex) -> np.ndarray:
        return self._cycle(0, np.asarray(r, dtype=np.complex128), sigma)

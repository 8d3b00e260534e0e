"""Oracle: post-processing of the discrete solution and the error measure
of Section 3 (test infrastructure only).

After the all-at-once solve, the two end levels y^N and p^0 follow from one
elliptic solve each with M + tau K (Section 1, the two formulas after
eq. Toeplitz_Mat_B); e_h is the discrete L^inf-in-time, L^2-in-space error of
Section 3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretize import Problem


def post_solve(pb: Problem, y: np.ndarray, p: np.ndarray, fN: np.ndarray, g0: np.ndarray,
               y0: np.ndarray, pN=None):
    """y^N and p^0 from (M + tau K) y^N = M y^{N-1} + tau M f^N + (tau/gamma) M p^N
    and (M + tau K) p^0 = M p^1 + tau M g^0 - tau M y^0 (M = I for finite
    differences)."""
    if pN is None:
        pN = np.zeros(pb.m)
    Mm = pb.Mm.tocsc()
    lu = spla.splu((Mm + pb.tau * pb.K.tocsc()).tocsc())
    yN = lu.solve(Mm @ (y[-1] + pb.tau * fN + (pb.tau / pb.gamma) * pN))
    p0 = lu.solve(Mm @ (p[0] + pb.tau * g0 - pb.tau * y0))
    return yN, p0


def error_eh(pb: Problem, y_full: np.ndarray, p_full: np.ndarray, y_exact, p_exact) -> float:
    """e_h = h^{d/2} max_{1<=j<=N} max(||y^j - y(t_j)||_2, ||p^{j-1} - p(t_{j-1})||_2).

    ``y_full``/``p_full`` hold levels 0..N ([N+1][m]); ``y_exact(t)`` and
    ``p_exact(t)`` evaluate the analytic solution on the grid."""
    N = pb.nt
    err = 0.0
    for j in range(1, N + 1):
        ey = np.linalg.norm(y_full[j] - y_exact(j * pb.tau))
        ep = np.linalg.norm(p_full[j - 1] - p_exact((j - 1) * pb.tau))
        err = max(err, ey, ep)
    return pb.h ** (pb.dim / 2.0) * err

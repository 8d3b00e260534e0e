"""Oracle: the adjoint (transposed) KKT solve and the gradients it yields
(test infrastructure only).

For a loss L(y, p) of the solution of A x = b (eq. main_system) with
y = x_1/sqrt(gamma), p = x_2, the chain rule gives dL/db = A^{-T} dL/dx with
dL/dx = [dL/dy / sqrt(gamma); dL/dp].  The right-hand side b depends on the
data through b_1^j = tau M g^j and b_2^j = -sqrt(gamma) M (tau f^j + [j = 1] y0)
(eq. main_system_before; M symmetric), so
    dL/dg^j = tau M lam_1^j,  dL/df^j = -sqrt(gamma) tau M lam_2^j,
    dL/dy0  = -sqrt(gamma) M lam_2^1,       lam = A^{-T} dL/dx.

The discrete cost whose optimality system is eq. main_system_before is
J_h = tau/2 sum_{j=1}^{n} ||y^j - g^j||_M^2 + gamma tau/2 sum_{j=1}^{n} ||u^j||_M^2
under (M + tau K) y^j - M y^{j-1} = tau M (f^j + u^j) (||v||_M^2 = v^T M v);
at the optimum u = p/gamma and its derivatives with respect to the data are
    dJ*/dg^j = -tau M (y^j - g^j),  dJ*/df^j = -tau M p^j,  dJ*/dy0 = -M p^1.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretize import Problem, kkt_scaled


def adjoint_solve(pb: Problem, r: np.ndarray) -> np.ndarray:
    """lam = A^{-T} r by a direct sparse solve."""
    return spla.spsolve(kkt_scaled(pb).T.tocsc(), r)


def data_gradients(pb: Problem, lam: np.ndarray):
    """Map lam = A^{-T} dL/dx to (dL/dg [n][m], dL/df [n][m], dL/dy0 [m])."""
    nm = pb.n * pb.m
    Mm = pb.Mm
    l1 = (Mm @ lam[:nm].reshape(pb.n, pb.m).T).T
    l2 = (Mm @ lam[nm:].reshape(pb.n, pb.m).T).T
    sg = math.sqrt(pb.gamma)
    return pb.tau * l1, -sg * pb.tau * l2, -sg * l2[0]


def loss_to_x_grad(pb: Problem, dLdy: np.ndarray, dLdp: np.ndarray) -> np.ndarray:
    """dL/dx from dL/dy and dL/dp (y = x_1/sqrt(gamma), p = x_2)."""
    return np.concatenate([np.ravel(dLdy) / math.sqrt(pb.gamma), np.ravel(dLdp)])


def state_from_control(pb: Problem, u: np.ndarray, f: np.ndarray, y0: np.ndarray) -> np.ndarray:
    """Backward-Euler states y^1..y^n for a control u (levels 1..n)."""
    Mm = pb.Mm.tocsc()
    lu = spla.splu((Mm + pb.tau * pb.K.tocsc()).tocsc())
    y = np.zeros((pb.n, pb.m))
    prev = np.asarray(y0, dtype=np.float64)
    for j in range(pb.n):
        y[j] = lu.solve(Mm @ (prev + pb.tau * (f[j] + u[j])))
        prev = y[j]
    return y


def cost(pb: Problem, y: np.ndarray, u: np.ndarray, g: np.ndarray) -> float:
    """J_h(y, u) = tau/2 sum ||y^j - g^j||_M^2 + gamma tau / 2 sum ||u^j||_M^2."""
    Mm = pb.Mm
    e = np.asarray(y - g).reshape(pb.n, pb.m)
    uu = np.asarray(u).reshape(pb.n, pb.m)
    return 0.5 * pb.tau * float(np.sum(e * (Mm @ e.T).T)) + 0.5 * pb.gamma * pb.tau * float(np.sum(uu * (Mm @ uu.T).T))


def envelope_gradients(pb: Problem, y: np.ndarray, p: np.ndarray, g: np.ndarray):
    """dJ*/dg, dJ*/df, dJ*/dy0 at the optimum (closed forms above)."""
    Mm = pb.Mm
    return -pb.tau * (Mm @ (y - g).T).T, -pb.tau * (Mm @ p.T).T, -(Mm @ p[0])

"""Oracle: the adjoint (transposed) KKT solve and the gradients it yields
(test infrastructure only).

For a loss L(y, p) of the solution of A x = b (eq. main_system) with
y = x_1/sqrt(gamma), p = x_2, the chain rule gives dL/db = A^{-T} dL/dx with
dL/dx = [dL/dy / sqrt(gamma); dL/dp].  The right-hand side b depends on the
data through b_1^j = tau g^j and b_2^j = -sqrt(gamma)(tau f^j + [j = 1] y0)
(eq. main_system_before, M = I), so
    dL/dg^j = tau lam_1^j,  dL/df^j = -sqrt(gamma) tau lam_2^j,
    dL/dy0  = -sqrt(gamma) lam_2^1,       lam = A^{-T} dL/dx.

The discrete cost whose optimality system is eq. main_system_before is
J_h = tau/2 sum_{j=1}^{n} ||y^j - g^j||^2 + gamma tau/2 sum_{j=1}^{n} ||u^j||^2
under (I + tau K) y^j - y^{j-1} = tau (f^j + u^j); at the optimum u = p/gamma
and its derivatives with respect to the data are
    dJ*/dg^j = -tau (y^j - g^j),  dJ*/df^j = -tau p^j,  dJ*/dy0 = -p^1.
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
    l1 = lam[:nm].reshape(pb.n, pb.m)
    l2 = lam[nm:].reshape(pb.n, pb.m)
    sg = math.sqrt(pb.gamma)
    return pb.tau * l1, -sg * pb.tau * l2, -sg * l2[0]


def loss_to_x_grad(pb: Problem, dLdy: np.ndarray, dLdp: np.ndarray) -> np.ndarray:
    """dL/dx from dL/dy and dL/dp (y = x_1/sqrt(gamma), p = x_2)."""
    return np.concatenate([np.ravel(dLdy) / math.sqrt(pb.gamma), np.ravel(dLdp)])


def state_from_control(pb: Problem, u: np.ndarray, f: np.ndarray, y0: np.ndarray) -> np.ndarray:
    """Backward-Euler states y^1..y^n for a control u (levels 1..n)."""
    E = (sp.identity(pb.m, format="csc") + pb.tau * pb.K.tocsc()).tocsc()
    lu = spla.splu(E)
    y = np.zeros((pb.n, pb.m))
    prev = np.asarray(y0, dtype=np.float64)
    for j in range(pb.n):
        y[j] = lu.solve(prev + pb.tau * (f[j] + u[j]))
        prev = y[j]
    return y


def cost(pb: Problem, y: np.ndarray, u: np.ndarray, g: np.ndarray) -> float:
    """J_h(y, u) = tau/2 sum ||y^j - g^j||^2 + gamma tau / 2 sum ||u^j||^2."""
    return 0.5 * pb.tau * float(np.sum((y - g) ** 2)) + 0.5 * pb.gamma * pb.tau * float(np.sum(u ** 2))


def envelope_gradients(pb: Problem, y: np.ndarray, p: np.ndarray, g: np.ndarray):
    """dJ*/dg, dJ*/df, dJ*/dy0 at the optimum (closed forms above)."""
    return -pb.tau * (y - g), -pb.tau * p, -p[0]

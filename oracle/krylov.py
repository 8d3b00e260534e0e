"""Oracle: GMRES (Saad and Schultz) with modified Gram-Schmidt Arnoldi and
Givens rotations, for the preconditioned system of eq. preconditioned_system.

Test infrastructure only.  Three variants:
  * ``left``:     GMRES on P^{-1} A x = P^{-1} b; the residual that is
                  monitored is the preconditioned one, as in the experiments
                  of Section 3 (zero initial guess, tolerance 1e-8 on the
                  relative residual).
  * ``right``:    GMRES on A P^{-1} u = b, x = P^{-1} u; the monitored
                  residual is the true residual b - A x.
  * ``flexible``: right preconditioning that stores Z_j = P^{-1} v_j and
                  forms x = x0 + Z y (for a preconditioner that is not an
                  exact linear map, e.g. one evaluated in FP32).

The relative residual is measured against the initial residual norm
||r_0|| (with x0 = 0 this is ||P^{-1} b|| for left and ||b|| for right).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    converged: bool
    history: List[float] = field(default_factory=list)  # relative residual estimates, index 0 = 1
    hessenberg: Optional[np.ndarray] = None


def _givens(a: float, b: float):
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def gmres(apply_A: Callable, b: np.ndarray, apply_P: Optional[Callable] = None,
          side: str = "left", x0: Optional[np.ndarray] = None, rtol: float = 1e-8,
          restart: int = 30, maxit: int = 300, fixed_iters: Optional[int] = None) -> GmresResult:
    """Restarted GMRES.  ``fixed_iters`` (if given) runs exactly that many
    Arnoldi steps in the first cycle, ignoring the tolerance (used to compare
    iterates at a fixed k)."""
    P = apply_P if apply_P is not None else (lambda v: v)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)

    def residual(xc):
        r = b - apply_A(xc)
        return P(r) if side == "left" else r

    r = residual(x)
    beta0 = np.linalg.norm(r)
    history = [1.0]
    if beta0 == 0.0:
        return GmresResult(x, 0, True, history)
    total = 0
    H_last = None
    while True:
        beta = np.linalg.norm(r)
        kmax = restart if fixed_iters is None else fixed_iters
        V = np.zeros((kmax + 1, b.size))
        Z = np.zeros((kmax, b.size)) if side == "flexible" else None
        H = np.zeros((kmax + 1, kmax))
        cs = np.zeros(kmax)
        sn = np.zeros(kmax)
        s = np.zeros(kmax + 1)
        s[0] = beta
        V[0] = r / beta
        k_done = 0
        converged = False
        for j in range(kmax):
            if side == "left":
                w = P(apply_A(V[j]))
            elif side == "right":
                w = apply_A(P(V[j]))
            else:
                Z[j] = P(V[j])
                w = apply_A(Z[j])
            for i in range(j + 1):            # modified Gram-Schmidt
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            if hnext > 0.0:
                V[j + 1] = w / hnext
            for i in range(j):                # apply previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            s[j + 1] = -sn[j] * s[j]
            s[j] = cs[j] * s[j]
            k_done = j + 1
            total += 1
            rel = abs(s[j + 1]) / beta0
            history.append(rel)
            if fixed_iters is None and (rel <= rtol or total >= maxit):
                converged = rel <= rtol
                break
            if hnext == 0.0:
                converged = True                  # lucky breakdown: exact solution
                break
        k = k_done
        y = np.linalg.solve(np.triu(H[:k, :k]), s[:k]) if k > 0 else np.zeros(0)
        H_last = H
        if side == "left":
            x = x + V[:k].T @ y
        elif side == "right":
            x = x + P(V[:k].T @ y)
        else:
            x = x + Z[:k].T @ y
        if fixed_iters is not None:
            r = residual(x)
            return GmresResult(x, total, np.linalg.norm(r) <= rtol * beta0, history, H_last)
        if converged or total >= maxit:
            return GmresResult(x, total, converged, history, H_last)
        r = residual(x)
        if np.linalg.norm(r) <= rtol * beta0:
            return GmresResult(x, total, True, history, H_last)

"""Helpers shared by the oracle tests (they only call ``oracle`` and ``workloads``)."""
import math
import os

import numpy as np

import workloads as W
from oracle import discretize as D, examples as E, krylov as K, precond as P

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


def example1_solve(nx, nt, gamma, eps=None, side="left", rtol=1e-8, dim=2, precond="eps"):
    """Solve Example 1 with the oracle; returns (iters, e_h, result, problem).
    precond "eps": P_eps (Section 2.1), "ideal": P of eq. matrix_P."""
    tau = 1.0 / nt
    e = min(0.5, tau / 2) if eps is None else eps
    pb = D.make_problem(dim, nx, nt, gamma, eps=e)
    g, f, y0 = W.example_fields(1, dim, nx, nt)
    b = D.rhs_scaled(pb, g, f, y0)
    A = D.kkt_scaled(pb)
    pc = P.EpsCirculantRBD(pb) if precond == "eps" else P.IdealRBD(pb)
    res = K.gmres(lambda v: A @ v, b, pc.apply, side=side, rtol=rtol)
    y, p = D.unpack_solution(pb, res.x)
    fN, _ = W.example1_source(dim, nx, 1.0)
    _, g0 = W.example1_source(dim, nx, 0.0)
    yN, p0 = E.post_solve(pb, y, p, fN, g0, y0)
    yf = np.vstack([y0[None], y, yN[None]])
    pf = np.vstack([p0[None], p, np.zeros((1, pb.m))])
    eh = E.error_eh(pb, yf, pf, lambda t: W.example1_exact(dim, nx, t)[0],
                    lambda t: W.example1_exact(dim, nx, t)[1])
    return res.iters, eh, res, pb


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))

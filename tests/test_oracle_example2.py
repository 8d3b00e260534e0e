"""Oracle pins for Example 2 (variable coefficient, multigrid spatial solves):
e_h as printed in Table 7 to 3 significant digits, and the iteration counts.
The counts depend on the V-cycle's smoother when the shift is small; with
the red-black Gauss-Seidel reading they equal the printed ones in these rows
for gamma <= 1e-4 and exceed them by a few iterations for gamma >= 1e-2
(exact spatial solves give the printed counts there, see the second test)."""
import numpy as np
import pytest

import workloads as W
from oracle import discretize as D, examples as E, krylov as K, precond as P
from oracle_helpers import read_rows

ROWS = [r for r in read_rows("paper_example2_rows.txt") if r[0] == "T7" and int(r[3]) <= 64]


def example2_solve(nx, nt, gamma, spatial="mg", precond="eps", smoother="rb"):
    tau = 1.0 / nt
    pb = D.make_problem(2, nx, nt, gamma, eps=min(0.5, tau / 2), coeff=W.coeff_example2)
    g, f, y0 = W.example_fields(2, 2, nx, nt, gamma=gamma)
    b = D.rhs_scaled(pb, g, f, y0)
    A = D.kkt_scaled(pb)
    if precond == "eps":
        pc = P.EpsCirculantRBD(pb, spatial=spatial, coeff=W.coeff_example2, smoother=smoother)
    else:
        pc = P.IdealRBD(pb, spatial=spatial, coeff=W.coeff_example2, smoother=smoother)
    res = K.gmres(lambda v: A @ v, b, pc.apply, side="left", rtol=1e-8)
    y, p = D.unpack_solution(pb, res.x)
    fN, _ = W.example2_source(nx, 1.0, gamma)
    _, g0 = W.example2_source(nx, 0.0, gamma)
    yN, p0 = E.post_solve(pb, y, p, fN, g0, y0)
    yf = np.vstack([y0[None], y, yN[None]])
    pf = np.vstack([p0[None], p, np.zeros((1, pb.m))])
    eh = E.error_eh(pb, yf, pf, lambda t: W.example2_exact(nx, t, gamma)[0],
                    lambda t: W.example2_exact(nx, t, gamma)[1])
    return res.iters, eh


@pytest.mark.parametrize("row", ROWS, ids=[" ".join(r[:4]) for r in ROWS])
def test_example2_table7_rows(row):
    _, gamma, nx, nt, dof, iters, eh = row[:7]
    gamma, nx, nt, iters = float(gamma), int(nx), int(nt), int(iters)
    it, e = example2_solve(nx, nt, gamma)
    assert float(f"{e:.2e}") == pytest.approx(float(eh), rel=1e-12)
    if gamma <= 1e-4:
        assert it == iters
    else:
        assert iters <= it <= iters + 3


@pytest.mark.parametrize("gamma,nt,iters", [(1.0, 32, 10), (1e-2, 32, 13)])
def test_example2_counts_with_exact_spatial_solves(gamma, nt, iters):
    """With exact (LU) spatial solves the printed counts of Table 7 appear for
    gamma >= 1e-2 as well."""
    it, _ = example2_solve(31, nt, gamma, spatial="lu")
    assert it == iters


# the rows whose counts depend on the smoother (gamma >= 1e-2; below it every
# reading gives the printed count)
SYM_ROWS = [r for r in read_rows("paper_example2_rows.txt")
            if r[0] == "T7" and int(r[3]) <= 64 and float(r[1]) >= 1e-2]


@pytest.mark.parametrize("row", SYM_ROWS, ids=[" ".join(r[:4]) for r in SYM_ROWS])
def test_example2_table7_counts_with_symmetric_gauss_seidel(row):
    """With a symmetric Gauss-Seidel pre-smoother (one sweep in the natural
    order, one in the reverse order) the printed iteration counts of Table 7
    appear for every gamma, including gamma >= 1e-2 where the red-black
    reading takes more (the printed e_h does not depend on the smoother)."""
    _, gamma, nx, nt, dof, iters, eh = row[:7]
    gamma, nx, nt, iters = float(gamma), int(nx), int(nt), int(iters)
    it, e = example2_solve(nx, nt, gamma, smoother="sym")
    assert it == iters
    assert float(f"{e:.2e}") == pytest.approx(float(eh), rel=1e-12)

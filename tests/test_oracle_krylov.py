"""Pins for oracle.krylov (GMRES) and the paper's printed iteration counts."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import discretize as D, krylov as K, precond as P
from oracle_helpers import example1_solve, read_rows, rel


def _system(gamma=1e-4, nx=7, nt=8, seed=5, eps=None):
    pb = D.make_problem(2, nx, nt, gamma, eps=eps)
    g, f, y0 = W.random_fields(2, nx, nt, seed)
    b = D.rhs_scaled(pb, g, f, y0)
    A = D.kkt_scaled(pb)
    return pb, A, b


@pytest.mark.parametrize("side", ["left", "right", "flexible"])
def test_gmres_converges_to_direct_solution(side):
    pb, A, b = _system()
    pc = P.EpsCirculantRBD(pb)
    res = K.gmres(lambda v: A @ v, b, pc.apply, side=side, rtol=1e-12)
    x_ref = spla.spsolve(A.tocsc(), b)
    assert res.converged
    assert rel(res.x, x_ref) < 1e-9


@pytest.mark.parametrize("side", ["left", "right"])
def test_gmres_iterate_is_krylov_minimiser(side):
    """Lemma krylov: the k-th iterate minimises the residual over x0 + K_k;
    checked by brute force (explicit Krylov basis + least squares)."""
    pb, A, b = _system(nx=3, nt=5)
    Pm = np.linalg.inv(P.eps_circulant_dense(pb))
    Ad = A.toarray()
    for k in (1, 2, 4):
        res = K.gmres(lambda v: Ad @ v, b, lambda v: Pm @ v, side=side, fixed_iters=k)
        if side == "left":
            Op, r0 = Pm @ Ad, Pm @ b
            basis = [r0]
            for _ in range(k - 1):
                basis.append(Op @ basis[-1])
            Bm = np.array(basis).T
            c = np.linalg.lstsq(Op @ Bm, r0, rcond=None)[0]
            x_bf = Bm @ c
        else:
            Op = Ad @ Pm
            basis = [b]
            for _ in range(k - 1):
                basis.append(Op @ basis[-1])
            Bm = np.array(basis).T
            c = np.linalg.lstsq(Op @ Bm, b, rcond=None)[0]
            x_bf = Pm @ (Bm @ c)
        assert rel(res.x, x_bf) < 1e-8


def test_residual_history_monotone_and_matches_true_residual():
    pb, A, b = _system(gamma=1e-2)
    pc = P.EpsCirculantRBD(pb)
    res = K.gmres(lambda v: A @ v, b, pc.apply, side="right", rtol=1e-10)
    h = np.array(res.history)
    assert np.all(np.diff(h) <= 1e-15)
    true = np.linalg.norm(b - A @ res.x) / np.linalg.norm(b)
    assert true <= 1e-10 * 1.01


def test_restart_and_maxit():
    pb, A, b = _system(gamma=1e-2)
    pc = P.EpsCirculantRBD(pb)
    r1 = K.gmres(lambda v: A @ v, b, pc.apply, side="right", rtol=1e-10, restart=4)
    assert r1.converged
    assert rel(r1.x, spla.spsolve(A.tocsc(), b)) < 1e-8
    r2 = K.gmres(lambda v: A @ v, b, pc.apply, side="right", rtol=1e-14, maxit=3)
    assert not r2.converged and r2.iters == 3


def test_convergence_bound_theorem():
    """thm:gmres_conv with c_0 = 1 (M = I): for eps <= c_tau(delta) the
    preconditioned residuals satisfy ||r_k|| <= rho(delta)^k ||r_0||."""
    delta = 0.5
    rho = math.sqrt(-delta ** 2 + 8 * delta + 2) / (2 + delta)
    for gamma, nt in [(1e-6, 16), (1e-2, 8), (1.0, 12)]:
        tau = 1.0 / nt
        c_tau = delta * math.sqrt(tau) / (delta * math.sqrt(tau) + 2.0)
        pb, A, b = _system(gamma=gamma, nx=5, nt=nt, eps=c_tau)
        pc = P.EpsCirculantRBD(pb)
        res = K.gmres(lambda v: A @ v, b, pc.apply, side="left", rtol=1e-12)
        for k, r in enumerate(res.history):
            assert r <= rho ** k * (1 + 1e-9)


def test_iteration_counts_flat_in_n_and_gamma():
    """Iteration counts stay bounded (here <= 20) across grid sizes, time
    steps and gamma for eps = sqrt(tau) (abstract, Remark after thm:gmres_conv)."""
    counts = []
    for nx, nt in [(7, 8), (15, 16), (31, 32)]:
        for gamma in (1e-10, 1e-6, 1e-2, 1.0):
            it, _, _, _ = example1_solve(nx, nt, gamma, eps=math.sqrt(1.0 / nt), side="right")
            counts.append(it)
    assert max(counts) <= 20


ROWS = read_rows("paper_table_rows.txt")


@pytest.mark.parametrize("row", ROWS, ids=[" ".join(r[:4]) for r in ROWS])
def test_paper_table_rows(row):
    """Iteration count (exact) and e_h (3 significant digits) of GMRES-P_eps on
    Example 1 as printed in Tables 1-3."""
    table, gamma, nx, nt, dof, iters, eh = row[:7]
    if len(row) > 7:  # printed exponent off by one; same mantissa
        assert row[7].split("e")[0] == eh.split("e")[0]
        eh = row[7]
    nx, nt, dof, iters = int(nx), int(nt), int(dof), int(iters)
    assert dof == 2 * nx * nx * nt
    it, e, _, _ = example1_solve(nx, nt, float(gamma))
    assert it == iters
    assert float(f"{e:.2e}") == pytest.approx(float(eh), rel=1e-12)


ROWS4 = [r for r in read_rows("paper_table4_rows.txt") if int(r[3]) <= 128]


@pytest.mark.parametrize("row", ROWS4, ids=[" ".join(r[:4]) for r in ROWS4])
def test_paper_table4_rows_ideal(row):
    """Iteration count (exact) and e_h (3 significant digits) of GMRES-P with the
    ideal RBD preconditioner on Example 1 as printed in Table 4."""
    table, gamma, nx, nt, dof, iters, eh = row[:7]
    nx, nt, dof, iters = int(nx), int(nt), int(dof), int(iters)
    assert dof == 2 * nx * nx * nt
    it, e, _, _ = example1_solve(nx, nt, float(gamma), precond="ideal")
    assert it == iters
    assert float(f"{e:.2e}") == pytest.approx(float(eh), rel=1e-12)

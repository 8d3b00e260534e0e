"""Pins for oracle.adjoint: transposed solves and data gradients, checked
against finite differences and the closed-form derivatives of the optimal
cost (envelope theorem)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import adjoint as ADJ, discretize as D
from oracle_helpers import rel


def _solve(pb, g, f, y0):
    x = spla.spsolve(D.kkt_scaled(pb).tocsc(), D.rhs_scaled(pb, g, f, y0))
    return D.unpack_solution(pb, x)


@pytest.mark.parametrize("gamma", [1e-6, 1e-2])
def test_linear_loss_gradients_match_finite_differences(gamma):
    pb = D.make_problem(2, 5, 6, gamma)
    g, f, y0 = W.random_fields(2, 5, 6, seed=11)
    rng = np.random.default_rng(12)
    cy, cp = rng.standard_normal((pb.n, pb.m)), rng.standard_normal((pb.n, pb.m))
    L = lambda g_, f_, y0_: float(np.sum(cy * _solve(pb, g_, f_, y0_)[0]) + np.sum(cp * _solve(pb, g_, f_, y0_)[1]))
    lam = ADJ.adjoint_solve(pb, ADJ.loss_to_x_grad(pb, cy, cp))
    dg, df, dy0 = ADJ.data_gradients(pb, lam)
    h = 1.0  # the loss is linear in the data: central differences are exact up to rounding
    for (j, i) in [(0, 3), (2, 7), (pb.n - 1, 24)]:
        e = np.zeros_like(g)
        e[j, i] = h
        fd_g = (L(g + e, f, y0) - L(g - e, f, y0)) / (2 * h)
        fd_f = (L(g, f + e, y0) - L(g, f - e, y0)) / (2 * h)
        assert fd_g == pytest.approx(dg[j, i], rel=1e-7, abs=1e-12)
        assert fd_f == pytest.approx(df[j, i], rel=1e-7, abs=1e-12)
    e0 = np.zeros_like(y0)
    e0[5] = h
    fd_y0 = (L(g, f, y0 + e0) - L(g, f, y0 - e0)) / (2 * h)
    assert fd_y0 == pytest.approx(dy0[5], rel=1e-7, abs=1e-12)


def test_adjoint_solve_by_sign_flips():
    """A^{-T} r = J A^{-1} J r (A^T = J A J with M = I)."""
    pb = D.make_problem(2, 5, 7, 1e-4)
    r = np.random.default_rng(3).standard_normal(2 * pb.n * pb.m)
    J = np.r_[np.ones(pb.n * pb.m), -np.ones(pb.n * pb.m)]
    lam = ADJ.adjoint_solve(pb, r)
    lam2 = J * spla.spsolve(D.kkt_scaled(pb).tocsc(), J * r)
    assert rel(lam, lam2) < 1e-12


@pytest.mark.parametrize("gamma", [1e-4, 1e-1])
def test_kkt_solution_minimises_discrete_cost(gamma):
    """The KKT solution with u = p/gamma is the minimiser of the reduced cost
    J(u) = J_h(y(u), u): every directional derivative vanishes and random
    perturbations increase the cost."""
    pb = D.make_problem(2, 5, 6, gamma)
    g, f, y0 = W.random_fields(2, 5, 6, seed=7)
    y, p = _solve(pb, g, f, y0)
    u = p / gamma
    assert rel(ADJ.state_from_control(pb, u, f, y0), y) < 1e-10
    J0 = ADJ.cost(pb, y, u, g)
    rng = np.random.default_rng(8)
    for _ in range(3):
        d = rng.standard_normal(u.shape)
        s = 1e-4 * np.linalg.norm(u) / np.linalg.norm(d) + 1e-6
        Jp = ADJ.cost(pb, ADJ.state_from_control(pb, u + s * d, f, y0), u + s * d, g)
        Jm = ADJ.cost(pb, ADJ.state_from_control(pb, u - s * d, f, y0), u - s * d, g)
        # J is quadratic in u: at a stationary point J(u + sd) = J(u - sd)
        assert Jp > J0 and Jm > J0
        assert abs(Jp - Jm) <= 1e-6 * (Jp - J0) + 1e-13 * abs(J0)


def test_envelope_gradients_match_finite_differences():
    """dJ*/dg = -tau (y - g), dJ*/df = -tau p, dJ*/dy0 = -p^1 at the optimum."""
    gamma = 1e-3
    pb = D.make_problem(2, 5, 6, gamma)
    g, f, y0 = W.random_fields(2, 5, 6, seed=9)

    def Jstar(g_, f_, y0_):
        y_, p_ = _solve(pb, g_, f_, y0_)
        return ADJ.cost(pb, y_, p_ / gamma, g_)

    y, p = _solve(pb, g, f, y0)
    dg, df, dy0 = ADJ.envelope_gradients(pb, y, p, g)
    h = 1e-5
    for (j, i) in [(0, 0), (3, 12), (pb.n - 1, 20)]:
        e = np.zeros_like(g)
        e[j, i] = h
        assert (Jstar(g + e, f, y0) - Jstar(g - e, f, y0)) / (2 * h) == pytest.approx(dg[j, i], rel=1e-6, abs=1e-10)
        assert (Jstar(g, f + e, y0) - Jstar(g, f - e, y0)) / (2 * h) == pytest.approx(df[j, i], rel=1e-6, abs=1e-10)
    e0 = np.zeros_like(y0)
    e0[4] = h
    assert (Jstar(g, f, y0 + e0) - Jstar(g, f, y0 - e0)) / (2 * h) == pytest.approx(dy0[4], rel=1e-6, abs=1e-10)


def test_envelope_equals_adjoint_chain_rule():
    """The envelope derivative equals the total derivative obtained from the
    adjoint gradients of J* = J_h(y(g), p(g)/gamma; g) plus its explicit g term."""
    gamma = 1e-2
    pb = D.make_problem(2, 5, 6, gamma)
    g, f, y0 = W.random_fields(2, 5, 6, seed=10)
    y, p = _solve(pb, g, f, y0)
    dLdy = pb.tau * (y - g)
    dLdp = pb.tau * p / gamma
    lam = ADJ.adjoint_solve(pb, ADJ.loss_to_x_grad(pb, dLdy, dLdp))
    dg, df, dy0 = ADJ.data_gradients(pb, lam)
    dg_total = dg - pb.tau * (y - g)      # explicit dependence of J_h on g
    eg, ef, ey0 = ADJ.envelope_gradients(pb, y, p, g)
    assert rel(dg_total, eg) < 1e-9
    assert rel(df, ef) < 1e-9
    assert rel(dy0, ey0) < 1e-9

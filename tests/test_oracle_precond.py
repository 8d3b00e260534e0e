"""Pins for oracle.precond: the epsilon-circulant factorisation, the four-step
apply against the explicitly assembled preconditioner, and the spectral
statements of Section 2."""
import numpy as np
import pytest

import workloads as W
from oracle import discretize as D, precond as P
from oracle_helpers import rel


@pytest.mark.parametrize("n,eps", [(5, 0.3), (8, 0.01), (31, 0.125)])
def test_eps_circulant_factorisation(n, eps):
    """C_eps = D^{-1} F Lambda F^* D with D = diag(eps^{(i-1)/n}) (eq. decomposition_eps)."""
    F = P.fourier_matrix(n)
    d = P.d_eps(n, eps)
    lam = P.lambda_eps(n, eps)
    C = np.diag(1 / d) @ F @ np.diag(lam) @ F.conj().T @ np.diag(d)
    assert np.abs(C - D.eps_circulant(n, eps)).max() < 1e-13
    assert np.abs(F @ F.conj().T - np.eye(n)).max() < 1e-13


def test_factorisation_exponent_over_N_fails():
    """Reading check: with the exponent (i-1)/(n+1) the factorisation breaks."""
    n, eps = 8, 0.1
    F = P.fourier_matrix(n)
    d = eps ** (np.arange(n) / (n + 1))
    lam = P.lambda_eps(n, eps)
    C = np.diag(1 / d) @ F @ np.diag(lam) @ F.conj().T @ np.diag(d)
    assert np.abs(C - D.eps_circulant(n, eps)).max() > 1e-3


def test_transpose_factorisation():
    """C_eps^T = D F conj(Lambda) F^* D^{-1}; the transposed form printed in the
    Implementation subsection, (F^* D)^T conj(Lambda) ((F^* D)^T)^{-1}, is not."""
    n, eps = 9, 0.2
    F = P.fourier_matrix(n)
    d = P.d_eps(n, eps)
    lam = P.lambda_eps(n, eps)
    C = D.eps_circulant(n, eps)
    Ct = np.diag(d) @ F @ np.diag(lam.conj()) @ F.conj().T @ np.diag(1 / d)
    assert np.abs(Ct - C.T).max() < 1e-13
    U1 = (F.conj().T @ np.diag(d)).T
    printed = U1 @ np.diag(lam.conj()) @ np.linalg.inv(U1)
    assert np.abs(printed - C.T).max() > 1e-2


@pytest.mark.parametrize("dim,nx,nt,gamma,eps", [
    (2, 3, 6, 1e-4, None), (2, 4, 5, 1.0, 0.5), (1, 6, 8, 1e-8, 0.01), (3, 2, 4, 1e-2, 1.0)])
def test_four_step_apply_equals_dense_inverse(dim, nx, nt, gamma, eps):
    """The four steps of Section 2.1 compute P_eps^{-1} v for P_eps of eq. matrix_P_eps."""
    pb = D.make_problem(dim, nx, nt, gamma, eps=eps)
    v = np.random.default_rng(0).standard_normal(2 * pb.n * pb.m)
    w = P.EpsCirculantRBD(pb).apply(v)
    w_ref = np.linalg.solve(P.eps_circulant_dense(pb), v)
    assert rel(w, w_ref) < 1e-12


def test_ideal_rbd_apply_equals_dense_inverse():
    pb = D.make_problem(2, 3, 7, 1e-3)
    v = np.random.default_rng(1).standard_normal(2 * pb.n * pb.m)
    assert rel(P.IdealRBD(pb).apply(v), np.linalg.solve(P.ideal_rbd_dense(pb), v)) < 1e-12


def test_ideal_rbd_multigrid_single_point_is_exact():
    """On a one-point grid the V-cycle is the exact solve, so the multigrid
    variant of the ideal preconditioner equals the LU one."""
    pb = D.make_problem(2, 1, 9, 1e-3, coeff=W.coeff_sines3d)
    v = np.random.default_rng(2).standard_normal(2 * pb.n * pb.m)
    a = P.IdealRBD(pb, spatial="mg", coeff=W.coeff_sines3d).apply(v)
    assert rel(a, P.IdealRBD(pb).apply(v)) < 1e-14


def test_ideal_rbd_multigrid_power_series():
    """With M the (linear) V-cycle operator, forward substitution gives
    z_2^j = sum_{i <= j} M^{j-i+1} v_2^i and backward substitution
    z_1^j = sum_{i >= j} M^{i-j+1} v_1^i; w = [z_1 - z_2; z_1 + z_2]."""
    from oracle.multigrid import ShiftedVCycle
    pb = D.make_problem(2, 7, 6, 1e-2, coeff=W.coeff_sines3d)
    n, m = pb.n, pb.m
    mg = ShiftedVCycle(2, 7, pb.tau, W.coeff_sines3d)
    M = np.stack([mg.apply(e, complex(1.0 + pb.alpha, 0.0)).real for e in np.eye(m)], axis=1)
    pw = [np.eye(m)]
    for _ in range(n):
        pw.append(M @ pw[-1])
    v = np.random.default_rng(3).standard_normal((2, n, m))
    z2 = np.array([sum(pw[j - i + 1] @ v[1, i] for i in range(j + 1)) for j in range(n)])
    z1 = np.array([sum(pw[i - j + 1] @ v[0, i] for i in range(j, n)) for j in range(n)])
    w = P.IdealRBD(pb, spatial="mg", coeff=W.coeff_sines3d).apply(v.ravel())
    assert rel(w, np.concatenate([(z1 - z2).ravel(), (z1 + z2).ravel()])) < 1e-13


def test_ideal_rbd_spectrum():
    """sigma(P^{-1} A) lies on Re = 1 with |Im| <= 1 (thm:spectum_of_H_inv_B, M = I)."""
    for gamma in (1e-6, 1e-2, 1.0):
        pb = D.make_problem(2, 3, 8, gamma)
        A = D.kkt_scaled(pb).toarray()
        ev = np.linalg.eigvals(np.linalg.solve(P.ideal_rbd_dense(pb), A))
        assert np.abs(ev.real - 1).max() < 1e-10
        assert np.abs(ev.imag).max() <= 1 + 1e-10


@pytest.mark.parametrize("gamma,eps", [(1e-4, 0.3), (1e-8, 0.05), (1.0, 1.0)])
def test_H_eps_inverse_H_spectrum(gamma, eps):
    """thm:eigenvalue_P_eps_inv_A: rank(H_eps^{-1} H - I) = 2m, 2(n-1)m eigenvalues
    equal to 1, and the remaining ones are 1/(1 - eps (1 + alpha + tau mu_j)^{-n})
    (twice each), so that |lambda - 1| <= eps/(1 - eps)."""
    dim, nx, nt = 2, 3, 7
    pb = D.make_problem(dim, nx, nt, gamma, eps=eps)
    n, m = pb.n, pb.m
    Kd = pb.K.toarray()
    I = np.eye(n * m)
    Tm = np.kron(D.toeplitz_B(n).toarray(), np.eye(m)) + pb.tau * np.kron(np.eye(n), Kd)
    Cm = np.kron(D.eps_circulant(n, eps), np.eye(m)) + pb.tau * np.kron(np.eye(n), Kd)
    Z = np.zeros_like(I)
    H = np.block([[Tm.T + pb.alpha * I, Z], [Z, Tm + pb.alpha * I]])
    He = np.block([[Cm.T + pb.alpha * I, Z], [Z, Cm + pb.alpha * I]])
    X = np.linalg.solve(He, H)
    assert np.linalg.matrix_rank(X - np.eye(2 * n * m), tol=1e-9) == 2 * m
    mu = np.linalg.eigvalsh(Kd)
    expect = 1.0 / (1.0 - eps * (1 + pb.alpha + pb.tau * mu) ** (-n))
    # X - I has the eigenvalues expect - 1 (twice each) and otherwise only
    # zero (partly defective), so compare power sums via traces of powers
    Y = X - np.eye(2 * n * m)
    Yk = np.eye(2 * n * m)
    for k in (1, 2, 3):
        Yk = Yk @ Y
        got = np.trace(Yk)
        want = 2.0 * np.sum((expect - 1.0) ** k)
        assert abs(got - want) <= 1e-9 * abs(want) + 1e-14
    if eps < 1:
        assert np.max(np.abs(expect - 1)) <= eps / (1 - eps)
    ev = np.linalg.eigvals(X)
    assert np.abs(ev - 1).max() <= (eps / (1 - eps) if eps < 1 else 10.0) + 1e-6


def test_sherman_morrison_woodbury_identity():
    """lem:C_eps_invertible: (C_eps + a I)^{-1}(T + a I) = I + (T + a I)^{-1} E_1 Z^{-1} E_n^T,
    Z = eps^{-1}(I - eps T_0^{-n}), T_0 = (1 + alpha) I + tau K (M = I)."""
    pb = D.make_problem(2, 3, 6, 1e-3, eps=0.4)
    n, m, eps, a = pb.n, pb.m, pb.eps, pb.alpha
    Kd = pb.K.toarray()
    Tm = np.kron(D.toeplitz_B(n).toarray(), np.eye(m)) + pb.tau * np.kron(np.eye(n), Kd) + a * np.eye(n * m)
    Cm = np.kron(D.eps_circulant(n, eps), np.eye(m)) + pb.tau * np.kron(np.eye(n), Kd) + a * np.eye(n * m)
    T0 = (1 + a) * np.eye(m) + pb.tau * Kd
    Zm = (np.eye(m) - eps * np.linalg.matrix_power(np.linalg.inv(T0), n)) / eps
    E1 = np.kron(np.eye(n)[:, [0]], np.eye(m))
    En = np.kron(np.eye(n)[:, [n - 1]], np.eye(m))
    lhs = np.linalg.solve(Cm, Tm)
    rhs = np.eye(n * m) + np.linalg.solve(Tm, E1 @ np.linalg.solve(Zm, En.T))
    assert np.abs(lhs - rhs).max() < 1e-10


def test_multigrid_spatial_option_matches_lu_when_exact():
    """On the 1-point grid the V-cycle is an exact solve, so both spatial
    options of the oracle give the same P_eps^{-1} v."""
    pb = D.make_problem(2, 1, 9, 1e-4)
    v = np.random.default_rng(2).standard_normal(2 * pb.n * pb.m)
    a = P.EpsCirculantRBD(pb, spatial="lu").apply(v)
    b = P.EpsCirculantRBD(pb, spatial="mg").apply(v)
    assert rel(a, b) < 1e-13


@pytest.mark.parametrize("dim,nx,nt,eps", [(2, 3, 6, 0.3), (1, 5, 9, 1.0), (3, 2, 4, 0.05)])
def test_forward_preconditioner_equals_assembled(dim, nx, nt, eps):
    pb = D.make_problem(dim, nx, nt, 1e-4, eps=eps)
    w = np.random.default_rng(3).standard_normal(2 * pb.n * pb.m)
    assert rel(P.eps_circulant_apply(pb, w), P.eps_circulant_dense(pb) @ w) < 1e-14
    # and it inverts the four-step apply
    assert rel(P.eps_circulant_apply(pb, P.EpsCirculantRBD(pb).apply(w)), w) < 1e-12

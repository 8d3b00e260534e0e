"""Pins for oracle.discretize: the spatial operator, the KKT matrix and the
right-hand side, checked against facts the paper or mathematics fixes."""
import math

import numpy as np
import pytest
import scipy.fft as sfft
import scipy.sparse.linalg as spla

import workloads as W
from oracle import discretize as D
from oracle_helpers import rel


@pytest.mark.parametrize("dim,nx", [(1, 7), (2, 7), (3, 5)])
def test_dst_diagonalises_K(dim, nx):
    """The orthonormal DST-I diagonalises the constant-coefficient K with the
    textbook eigenvalues (the fast spatial solve of Example 1)."""
    K = D.stiffness(dim, nx).toarray()
    m = nx ** dim
    S = np.zeros((m, m))
    shape = (nx,) * dim
    for c in range(m):
        e = np.zeros(m)
        e[c] = 1.0
        S[:, c] = sfft.dstn(e.reshape(shape), type=1, norm="ortho").ravel()
    Dm = S @ K @ S
    mu = D.dst_eigenvalues(dim, nx)
    assert np.allclose(Dm, np.diag(mu), atol=1e-9 * mu.max())


def test_variable_coefficient_reduces_to_constant():
    for dim, nx in [(2, 7), (3, 3)]:
        Kc = D.stiffness(dim, nx)
        Kv = D.stiffness(dim, nx, W.coeff_one)
        assert abs(Kc - Kv).max() < 1e-9


def test_variable_coefficient_spd_and_consistent():
    """Flux form: symmetric positive definite, and second-order consistent with
    -div(a grad u) for a = 1 + x1, u = sin(pi x1) sin(pi x2)."""
    a = lambda x1, x2: 1.0 + x1
    errs = []
    for nx in (15, 31, 63):
        K = D.stiffness(2, nx, a)
        assert abs(K - K.T).max() < 1e-8
        x1, x2 = W.mesh(2, nx)
        u = np.sin(np.pi * x1) * np.sin(np.pi * x2)
        exact = -(np.pi * np.cos(np.pi * x1) * np.sin(np.pi * x2)) + 2 * np.pi ** 2 * (1 + x1) * u
        errs.append(np.max(np.abs(K @ u - exact)))
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5
    K = D.stiffness(2, 7, a).toarray()
    assert np.linalg.eigvalsh(K).min() > 0


def test_3d_sines_coefficient_symmetric_positive():
    K = D.stiffness(3, 7, W.coeff_sines3d)
    assert abs(K - K.T).max() < 1e-8
    ev = np.linalg.eigvalsh(K.toarray())
    assert ev.min() > 0


def _small(gamma=1e-3, nx=5, nt=7, dim=2):
    return D.make_problem(dim, nx, nt, gamma)


def test_scaled_matrix_block_structure():
    """A = [[alpha I, T^T], [-T, alpha I]], T = B (x) I + tau I (x) K (eq. matrix_A)."""
    pb = _small()
    A = D.kkt_scaled(pb).toarray()
    n, m = pb.n, pb.m
    Tm = np.kron(D.toeplitz_B(n).toarray(), np.eye(m)) + pb.tau * np.kron(np.eye(n), pb.K.toarray())
    I = np.eye(n * m)
    A2 = np.block([[pb.alpha * I, Tm.T], [-Tm, pb.alpha * I]])
    assert np.abs(A - A2).max() < 1e-12 * np.abs(A2).max()


def test_scaled_matrix_skew_part_and_adjoint_symmetry():
    """With M = I, A - alpha I is skew-symmetric, hence A^T = J A J, J = diag(I, -I)."""
    pb = _small()
    A = D.kkt_scaled(pb).toarray()
    S = A - pb.alpha * np.eye(A.shape[0])
    assert np.abs(S + S.T).max() < 1e-12 * np.abs(S).max()
    J = np.diag(np.r_[np.ones(pb.n * pb.m), -np.ones(pb.n * pb.m)])
    assert np.abs(A.T - J @ A @ J).max() < 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("gamma", [1e-6, 1e-2, 1.0])
def test_kkt_solution_satisfies_time_stepping(gamma):
    """The solution of the all-at-once system satisfies the backward-Euler
    state recursion with u = p/gamma and the adjoint recursion with p^N = 0
    (Section 1, the two difference equations before eq. main_system_before),
    checked step by step."""
    pb = D.make_problem(2, 7, 9, gamma)
    g, f, y0 = W.random_fields(2, 7, 9, seed=3)
    x = spla.spsolve(D.kkt_scaled(pb).tocsc(), D.rhs_scaled(pb, g, f, y0))
    y, p = D.unpack_solution(pb, x)
    K, tau = pb.K, pb.tau
    prev = y0
    for j in range(pb.n):
        lhs = (y[j] - prev) / tau + K @ y[j]
        rhs = f[j] + p[j] / gamma
        assert np.abs(lhs - rhs).max() < 1e-8 * (1 + np.abs(rhs).max())
        prev = y[j]
    for j in range(pb.n):
        nxt = p[j + 1] if j + 1 < pb.n else np.zeros(pb.m)
        lhs = -(nxt - p[j]) / tau + K @ p[j]
        rhs = g[j] - y[j]
        assert np.abs(lhs - rhs).max() < 1e-8 * (1 + np.abs(rhs).max())


def test_dof_column_matches_paper():
    """The DoF column of the tables is 2 m N: 61 504 at h = tau = 2^-5 and
    33 292 800 at h = tau = 2^-8."""
    assert 2 * 31 ** 2 * 32 == 61504
    assert 2 * 255 ** 2 * 256 == 33292800


@pytest.mark.parametrize("dim,nx,nt,coeff", [(2, 5, 7, None), (3, 3, 5, W.coeff_sines3d), (2, 4, 2, None)])
@pytest.mark.parametrize("transpose", [False, True])
def test_blockwise_matvec_equals_assembled(dim, nx, nt, coeff, transpose):
    pb = D.make_problem(dim, nx, nt, 1e-3, coeff=coeff)
    x = np.random.default_rng(5).standard_normal(2 * pb.n * pb.m)
    assert rel(D.kkt_apply_blocks(pb, x, transpose), D.kkt_apply(pb, x, transpose)) < 1e-14

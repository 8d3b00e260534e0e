"""Oracle pins for the finite-element form of the problem (Section 1: M_m and
K_m of a finite element discretisation, M_m != I), built from bilinear
(2-D) and trilinear (3-D) elements on the uniform grid with a = 1."""
import itertools
import math

import numpy as np
import pytest
import scipy.fft
import scipy.linalg
import scipy.sparse.linalg as spla

from oracle import adjoint as ADJ
from oracle import examples as EX
from oracle import discretize as D
from oracle import precond as P

import workloads as W


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _element_assembly(dim, nx):
    """Q1 mass and stiffness matrices assembled element by element with
    two-point Gauss quadrature per axis (exact for these polynomial degrees),
    keeping interior nodes only (zero Dirichlet data)."""
    h = 1.0 / (nx + 1)
    m = nx ** dim
    Mg = np.zeros((m, m))
    Kg = np.zeros((m, m))
    gp = [0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)]    # on [0, 1], weights 1/2
    corners = list(itertools.product((0, 1), repeat=dim))

    def node(c):
        # grid node index (0..nx+1 per axis) -> interior index or None
        if any(v < 1 or v > nx for v in c):
            return None
        return sum((c[a] - 1) * nx ** a for a in range(dim))

    for cell in itertools.product(range(nx + 1), repeat=dim):
        ids = [node(tuple(cell[a] + cr[a] for a in range(dim))) for cr in corners]
        for q in itertools.product(gp, repeat=dim):
            wq = (0.5 ** dim) * h ** dim
            phi = [np.prod([q[a] if cr[a] else 1 - q[a] for a in range(dim)]) for cr in corners]
            grad = []
            for cr in corners:
                gvec = []
                for a in range(dim):
                    d = (1.0 if cr[a] else -1.0) / h
                    gvec.append(d * np.prod([q[b] if cr[b] else 1 - q[b] for b in range(dim) if b != a]))
                grad.append(np.array(gvec))
            for s, t in itertools.product(range(len(corners)), repeat=2):
                if ids[s] is None or ids[t] is None:
                    continue
                Mg[ids[s], ids[t]] += wq * phi[s] * phi[t]
                Kg[ids[s], ids[t]] += wq * grad[s] @ grad[t]
    return Mg, Kg


@pytest.mark.parametrize("dim,nx", [(2, 3), (2, 4), (3, 2)])
def test_q1_matrices_match_element_quadrature(dim, nx):
    M, K = D.fem_q1(dim, nx)
    Mg, Kg = _element_assembly(dim, nx)
    assert np.abs(M.toarray() - Mg).max() < 1e-15
    assert np.abs(K.toarray() - Kg).max() < 1e-13


@pytest.mark.parametrize("dim,nx", [(2, 7), (3, 3)])
def test_q1_matrices_diagonalised_by_dst(dim, nx):
    """With S the orthonormal DST-I (scipy.fft.dstn, a library routine) in
    every axis, S M S = diag(prod_d m_{j_d}) and S K S =
    diag(sum_d k_{j_d} prod_{e != d} m_{j_e}), m_j = (h/3)(2 + cos(pi j h)),
    k_j = (4/h) sin^2(pi j h/2): the spatial solves of Step 2 stay divisions
    in the sine basis."""
    M, K = D.fem_q1(dim, nx)
    m = nx ** dim
    h = 1.0 / (nx + 1)
    E = np.eye(m).reshape((m,) + (nx,) * dim)
    axes = tuple(range(1, dim + 1))
    S = scipy.fft.dstn(E[..., ::1].transpose((0,) + tuple(range(dim, 0, -1))), type=1, norm="ortho", axes=axes)
    S = S.transpose((0,) + tuple(range(dim, 0, -1))).reshape(m, m)   # back to x1-fastest columns
    j = np.arange(1, nx + 1)
    m1 = (h / 3.0) * (2.0 + np.cos(np.pi * j * h))
    k1 = (4.0 / h) * np.sin(np.pi * j * h / 2.0) ** 2
    idx = np.arange(m)
    sub = [(idx // nx ** a) % nx for a in range(dim)]
    mdiag = np.prod([m1[s] for s in sub], axis=0)
    kdiag = sum(k1[sub[d]] * np.prod([m1[sub[e]] for e in range(dim) if e != d], axis=0) for d in range(dim))
    assert np.abs(S @ M.toarray() @ S.T - np.diag(mdiag)).max() < 1e-14
    assert np.abs(S @ K.toarray() @ S.T - np.diag(kdiag)).max() < 1e-12


@pytest.mark.parametrize("dim,nx,nt", [(2, 3, 6), (3, 2, 5)])
def test_fem_kkt_solution_satisfies_backward_euler(dim, nx, nt):
    """The solution of eq. main_system_before with M != I satisfies the two
    discrete recursions of Section 1 level by level:
    M (y^j - y^{j-1})/tau + K y^j = M (f^j + p^j/gamma) with y^0 = y0, and
    -M (p^{j+1} - p^j)/tau + K p^j = M (g^j - y^j) with p^N = 0."""
    gamma = 1e-3
    pb = D.make_problem(dim, nx, nt, gamma, mass="q1")
    g, f, y0 = W.random_fields(dim, nx, nt, seed=5)
    x = spla.spsolve(D.kkt_scaled(pb).tocsc(), D.rhs_scaled(pb, g, f, y0))
    y, p = D.unpack_solution(pb, x)
    M, K, tau, n = pb.Mm.toarray(), pb.K.toarray(), pb.tau, pb.n
    scale = np.abs(M @ g.T).max()
    for j in range(n):
        yprev = y0 if j == 0 else y[j - 1]
        r = M @ (y[j] - yprev) / tau + K @ y[j] - M @ (f[j] + p[j] / gamma)
        assert np.abs(r).max() < 1e-9 * (1 + scale / tau), j
        pnext = p[j + 1] if j + 1 < n else np.zeros(pb.m)
        r = -M @ (pnext - p[j]) / tau + K @ p[j] - M @ (g[j] - y[j])
        assert np.abs(r).max() < 1e-9 * (1 + scale / tau), j


@pytest.mark.parametrize("transpose", [False, True])
def test_fem_blocks_match_assembled(transpose):
    pb = D.make_problem(2, 5, 7, 1e-4, mass="q1")
    x = np.random.default_rng(3).standard_normal(2 * pb.n * pb.m)
    assert rel(D.kkt_apply_blocks(pb, x, transpose), D.kkt_apply(pb, x, transpose)) < 1e-14


@pytest.mark.parametrize("dim,nx,nt,eps", [(2, 3, 6, None), (2, 3, 5, 0.3), (3, 2, 4, None)])
def test_fem_four_step_apply_equals_dense_inverse(dim, nx, nt, eps):
    pb = D.make_problem(dim, nx, nt, 1e-4, eps=eps, mass="q1")
    v = np.random.default_rng(7).standard_normal(2 * pb.n * pb.m)
    w = P.EpsCirculantRBD(pb).apply(v)
    assert rel(w, np.linalg.solve(P.eps_circulant_dense(pb), v)) < 1e-12
    assert rel(P.eps_circulant_apply(pb, w), v) < 1e-12


def test_fem_ideal_rbd_spectrum():
    """sigma(P^{-1} A) lies on Re = 1 with |Im| <= 1 (thm:spectum_of_H_inv_B;
    the theorem covers any SPD M)."""
    for gamma in (1e-6, 1e-2, 1.0):
        pb = D.make_problem(2, 3, 6, gamma, mass="q1")
        A = D.kkt_scaled(pb).toarray()
        ev = np.linalg.eigvals(np.linalg.solve(P.ideal_rbd_dense(pb), A))
        assert np.abs(ev.real - 1).max() < 1e-10
        assert np.abs(ev.imag).max() <= 1 + 1e-10


@pytest.mark.parametrize("gamma,eps", [(1e-4, 0.3), (1e-8, 0.05)])
def test_fem_H_eps_inverse_H_spectrum(gamma, eps):
    """thm:eigenvalue_P_eps_inv_A with M != I: the non-unit eigenvalues of
    H_eps^{-1} H are 1/(1 - eps (1 + alpha + tau mu_j)^{-n}) with mu_j the
    generalised eigenvalues of (K, M) (twice each), compared through traces
    of powers of H_eps^{-1} H - I."""
    pb = D.make_problem(2, 3, 6, gamma, eps=eps, mass="q1")
    n, m = pb.n, pb.m
    Md, Kd = pb.Mm.toarray(), pb.K.toarray()
    Tm = np.kron(D.toeplitz_B(n).toarray(), Md) + pb.tau * np.kron(np.eye(n), Kd)
    Cm = np.kron(D.eps_circulant(n, eps), Md) + pb.tau * np.kron(np.eye(n), Kd)
    AM = pb.alpha * np.kron(np.eye(n), Md)
    Z = np.zeros_like(Tm)
    H = np.block([[Tm.T + AM, Z], [Z, Tm + AM]])
    He = np.block([[Cm.T + AM, Z], [Z, Cm + AM]])
    Y = np.linalg.solve(He, H) - np.eye(2 * n * m)
    mu = scipy.linalg.eigh(Kd, Md, eigvals_only=True)
    expect = 1.0 / (1.0 - eps * (1 + pb.alpha + pb.tau * mu) ** (-n))
    Yk = np.eye(2 * n * m)
    for k in (1, 2, 3):
        Yk = Yk @ Y
        want = 2.0 * np.sum((expect - 1.0) ** k)
        assert abs(np.trace(Yk) - want) <= 1e-9 * abs(want) + 1e-14


def test_fem_envelope_gradients_match_finite_differences():
    """The KKT solution minimises J_h with M-weighted norms; its derivatives
    with respect to g, f, y0 (closed forms) match central differences of the
    optimal cost."""
    pb = D.make_problem(2, 3, 5, 1e-2, mass="q1")
    g, f, y0 = W.random_fields(2, 3, 5, seed=11)
    A = D.kkt_scaled(pb).tocsc()

    def optimum(gg, ff, yy0):
        x = spla.spsolve(A, D.rhs_scaled(pb, gg, ff, yy0))
        y, p = D.unpack_solution(pb, x)
        return y, p, ADJ.cost(pb, y, p / pb.gamma, gg)

    y, p, _ = optimum(g, f, y0)
    dg, df, dy0 = ADJ.envelope_gradients(pb, y, p, g)
    rng = np.random.default_rng(2)
    for which, grad in (("g", dg), ("f", df), ("y0", dy0)):
        dirn = rng.standard_normal(grad.shape)
        h = 1e-6
        args_p = [g.copy(), f.copy(), y0.copy()]
        args_m = [g.copy(), f.copy(), y0.copy()]
        k = {"g": 0, "f": 1, "y0": 2}[which]
        args_p[k] = args_p[k] + h * dirn
        args_m[k] = args_m[k] - h * dirn
        fd = (optimum(*args_p)[2] - optimum(*args_m)[2]) / (2 * h)
        assert abs(fd - np.sum(grad * dirn)) <= 1e-6 * (abs(fd) + 1e-12), which


def test_fem_post_solve_completes_the_recursions():
    """The end levels y^N and p^0 of the post-solve satisfy the two discrete
    recursions of Section 1 at k1 = N - 1 and k2 = 0 with M != I."""
    dim, nx, nt, gamma = 2, 3, 6, 1e-3
    pb = D.make_problem(dim, nx, nt, gamma, mass="q1")
    g, f, y0 = W.random_fields(dim, nx, nt, seed=21)
    rng = np.random.default_rng(4)
    fN, g0 = rng.standard_normal(pb.m), rng.standard_normal(pb.m)
    x = spla.spsolve(D.kkt_scaled(pb).tocsc(), D.rhs_scaled(pb, g, f, y0))
    y, p = D.unpack_solution(pb, x)
    yN, p0 = EX.post_solve(pb, y, p, fN, g0, y0)
    M, K, tau = pb.Mm.toarray(), pb.K.toarray(), pb.tau
    r = M @ (yN - y[-1]) / tau + K @ yN - M @ fN              # p^N = 0
    assert np.abs(r).max() < 1e-10 * (1 + np.abs(M @ fN).max())
    r = -M @ (p[0] - p0) / tau + K @ p0 - M @ (g0 - y0)
    assert np.abs(r).max() < 1e-10 * (1 + np.abs(M @ g0).max() / tau)


@pytest.mark.parametrize("dim,nx,nt", [(2, 3, 6), (3, 2, 5)])
def test_fem_ideal_rbd_apply_equals_dense_inverse(dim, nx, nt):
    """P^{-1} v by the two sequential substitutions with T_0 = (1 + alpha) M +
    tau K and the coupling M to the neighbouring level equals the inverse of
    eq. matrix_P assembled densely with M != I."""
    pb = D.make_problem(dim, nx, nt, 1e-3, mass="q1")
    v = np.random.default_rng(9).standard_normal(2 * pb.n * pb.m)
    w = P.IdealRBD(pb).apply(v)
    assert rel(w, np.linalg.solve(P.ideal_rbd_dense(pb), v)) < 1e-12

"""Oracle: discretisation and the all-at-once KKT system (Section 1).

Test infrastructure only.  Plain SciPy sparse matrices in float64, built from
the formulas of Section 1 so that a reader can check them against the paper.

Layout: a spatial grid vector has m = nx**d entries in lexicographic order
with x1 fastest; an all-at-once vector stacks the n = N-1 time blocks
(levels 1..n) with the time index slowest; the scaled unknown x = [sqrt(g) y; p]
stacks the two such block vectors (eq. main_system).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# spatial operator K_m = -L_m (finite differences, M_m = I_m; Section 1)
# ---------------------------------------------------------------------------

def _axis_kron(op1d: sp.spmatrix, dim: int, nx: int, axis: int) -> sp.csr_matrix:
    """Embed a 1-D operator acting along ``axis`` (0 = x1, fastest)."""
    left = sp.identity(nx ** (dim - 1 - axis), format="csr")
    right = sp.identity(nx ** axis, format="csr")
    return sp.kron(left, sp.kron(op1d, right, format="csr"), format="csr")


def laplacian_1d(nx: int) -> sp.csr_matrix:
    """h^-2 tridiag(-1, 2, -1), the 1-D negative Dirichlet Laplacian."""
    h = 1.0 / (nx + 1)
    main = 2.0 * np.ones(nx)
    off = -np.ones(nx - 1)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr") / h ** 2


def stiffness(dim: int, nx: int, coeff: Optional[Callable] = None) -> sp.csr_matrix:
    """K = -L_h with zero Dirichlet data.

    ``coeff is None``: the constant-coefficient (a = 1) 5-point (2-D) or
    7-point (3-D) stencil, K = sum over axes of I (x) T (x) I.

    ``coeff`` callable a(x1, .., xd): the conservative flux form
    (K u)_i = h^-2 sum_d [a_{i+e_d/2}(u_i - u_{i+e_d}) + a_{i-e_d/2}(u_i - u_{i-e_d})]
    with a evaluated at the face midpoints and u = 0 outside the grid.
    This is the finite-difference reading of L = div(a grad) (Section 1)."""
    if coeff is None:
        K = sp.csr_matrix((nx ** dim, nx ** dim))
        T1 = laplacian_1d(nx)
        for axis in range(dim):
            K = K + _axis_kron(T1, dim, nx, axis)
        return K.tocsr()

    h = 1.0 / (nx + 1)
    m = nx ** dim
    idx = np.arange(m)
    # per-axis integer coordinates (0-based) of every point
    sub = [(idx // nx ** axis) % nx for axis in range(dim)]
    xs = [(s + 1) * h for s in sub]
    diag = np.zeros(m)
    rows, cols, vals = [], [], []
    for axis in range(dim):
        plus = list(xs)
        plus[axis] = xs[axis] + 0.5 * h
        minus = list(xs)
        minus[axis] = xs[axis] - 0.5 * h
        a_plus = coeff(*plus)
        a_minus = coeff(*minus)
        diag += (a_plus + a_minus) / h ** 2
        has_next = sub[axis] < nx - 1
        rows.append(idx[has_next])
        cols.append(idx[has_next] + nx ** axis)
        vals.append(-a_plus[has_next] / h ** 2)
        has_prev = sub[axis] > 0
        rows.append(idx[has_prev])
        cols.append(idx[has_prev] - nx ** axis)
        vals.append(-a_minus[has_prev] / h ** 2)
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, m))
    return K.tocsr()


# ---------------------------------------------------------------------------
# bilinear (d = 2) or trilinear (d = 3) finite elements on the uniform grid:
# the mass and stiffness matrices M_m, K_m of Section 1 for a = 1
# ---------------------------------------------------------------------------

def fem_q1_1d(nx: int):
    """1-D piecewise-linear mass and stiffness matrices with zero Dirichlet
    data: M1 = (h/6) tridiag(1, 4, 1), K1 = (1/h) tridiag(-1, 2, -1)."""
    h = 1.0 / (nx + 1)
    M1 = sp.diags([np.ones(nx - 1), 4.0 * np.ones(nx), np.ones(nx - 1)], [-1, 0, 1], format="csr") * (h / 6.0)
    K1 = sp.diags([-np.ones(nx - 1), 2.0 * np.ones(nx), -np.ones(nx - 1)], [-1, 0, 1], format="csr") / h
    return M1, K1


def fem_q1(dim: int, nx: int):
    """Tensor-product (Q1) mass and stiffness matrices on the interior nodes:
    M = M1 (x) .. (x) M1 and K = sum over axes of the product with K1 on that
    axis and M1 on the others (the element integrals of phi_a phi_b and
    grad phi_a . grad phi_b factor by axis for tensor-product shape
    functions)."""
    M1, K1 = fem_q1_1d(nx)

    def prod(factors):
        out = factors[dim - 1]
        for a in range(dim - 2, -1, -1):      # axis 0 = x1 fastest: rightmost factor
            out = sp.kron(out, factors[a], format="csr")
        return out

    M = prod([M1] * dim)
    K = None
    for axis in range(dim):
        fs = [M1] * dim
        fs[axis] = K1
        K = prod(fs) if K is None else K + prod(fs)
    return M.tocsr(), K.tocsr()


def dst_eigenvalues(dim: int, nx: int) -> np.ndarray:
    """Eigenvalues mu of the constant-coefficient K, one per DST-I mode in
    lexicographic order (x1 fastest): mu = (4/h^2) sum_d sin^2(pi j_d h / 2)."""
    h = 1.0 / (nx + 1)
    lam1 = 4.0 / h ** 2 * np.sin(np.pi * np.arange(1, nx + 1) * h / 2.0) ** 2
    mu = np.zeros(nx ** dim)
    idx = np.arange(nx ** dim)
    for axis in range(dim):
        mu += lam1[(idx // nx ** axis) % nx]
    return mu


# ---------------------------------------------------------------------------
# time matrices (eq. Toeplitz_Mat_B and eq. matrix_C_eps_n)
# ---------------------------------------------------------------------------

def toeplitz_B(n: int) -> sp.csr_matrix:
    """B_n: ones on the diagonal, minus ones on the first sub-diagonal."""
    return sp.diags([np.ones(n), -np.ones(n - 1)], [0, -1], format="csr")


def eps_circulant(n: int, eps: float) -> np.ndarray:
    """C_{eps,n}: B_n with -eps in the top-right corner (dense)."""
    C = toeplitz_B(n).toarray()
    C[0, n - 1] -= eps
    return C


# ---------------------------------------------------------------------------
# problem container
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    """Parameters of the discrete optimal-control problem (Section 1).

    N = nt backward-Euler steps of size tau = T/N; n = N-1 unknown time levels;
    alpha = tau/sqrt(gamma) (below eq. matrix_A)."""

    dim: int
    nx: int
    nt: int
    T: float
    gamma: float
    eps: float
    K: sp.csr_matrix
    M: Optional[sp.csr_matrix] = None   # mass matrix; None means M_m = I (finite differences)

    @property
    def Mm(self) -> sp.csr_matrix:
        return sp.identity(self.m, format="csr") if self.M is None else self.M

    @property
    def n(self) -> int:
        return self.nt - 1

    @property
    def m(self) -> int:
        return self.nx ** self.dim

    @property
    def tau(self) -> float:
        return self.T / self.nt

    @property
    def h(self) -> float:
        return 1.0 / (self.nx + 1)

    @property
    def alpha(self) -> float:
        return self.tau / math.sqrt(self.gamma)


def make_problem(dim: int, nx: int, nt: int, gamma: float, T: float = 1.0,
                 eps: Optional[float] = None, coeff: Optional[Callable] = None,
                 mass: str = "identity") -> Problem:
    """mass = "identity": finite differences (M_m = I, K_m = -L_h);
    mass = "q1": bilinear/trilinear finite elements (a = 1 only)."""
    tau = T / nt
    e = math.sqrt(tau) if eps is None else float(eps)
    if mass == "q1":
        if coeff is not None:
            raise ValueError("the finite-element matrices are built for a = 1")
        M, K = fem_q1(dim, nx)
        return Problem(dim, nx, nt, T, gamma, e, K, M)
    if mass != "identity":
        raise ValueError(mass)
    return Problem(dim, nx, nt, T, gamma, e, stiffness(dim, nx, coeff))


# ---------------------------------------------------------------------------
# all-at-once systems
# ---------------------------------------------------------------------------

def kkt_unscaled(pb: Problem) -> sp.csr_matrix:
    """The matrix of eq. matrix_A_before:
        [[tau I (x) M,          B^T (x) M + tau I (x) K],
         [B (x) M + tau I (x) K,       -tau/gamma I (x) M]]
    acting on [y; p] with y = (y^1..y^n), p = (p^1..p^n)."""
    n, tau = pb.n, pb.tau
    Mm = pb.Mm
    In = sp.identity(n, format="csr")
    B = toeplitz_B(n)
    Tm = sp.kron(B, Mm) + tau * sp.kron(In, pb.K)
    Tt = sp.kron(B.T, Mm) + tau * sp.kron(In, pb.K)
    InM = sp.kron(In, Mm, format="csr")
    return sp.bmat([[tau * InM, Tt], [Tm, -(tau / pb.gamma) * InM]], format="csr")


def kkt_scaled(pb: Problem) -> sp.csr_matrix:
    """The scaled matrix A of eq. matrix_A, obtained from eq. matrix_A_before
    by the change of variables x = [sqrt(gamma) y; p] and multiplying the
    second block row by -sqrt(gamma) (eq. main_system)."""
    nm = pb.n * pb.m
    sg = math.sqrt(pb.gamma)
    Inm = sp.identity(nm, format="csr")
    left = sp.block_diag([Inm, -sg * Inm], format="csr")
    right = sp.block_diag([Inm / sg, Inm], format="csr")
    return (left @ kkt_unscaled(pb) @ right).tocsr()


def rhs_unscaled(pb: Problem, g: np.ndarray, f: np.ndarray, y0: np.ndarray,
                 pN: Optional[np.ndarray] = None) -> np.ndarray:
    """Right-hand side [g; f] of eq. main_system_before:
    g-block tau M g^j (+ M p^N at j = n), f-block tau M f^j (+ M y^0 at j = 1)."""
    Mm = pb.Mm
    gb = pb.tau * (Mm @ np.array(g, dtype=np.float64).reshape(pb.n, pb.m).T).T
    fb = pb.tau * (Mm @ np.array(f, dtype=np.float64).reshape(pb.n, pb.m).T).T
    if pN is not None:
        gb[-1] += Mm @ np.asarray(pN, dtype=np.float64)
    fb[0] += Mm @ np.asarray(y0, dtype=np.float64)
    return np.concatenate([gb.ravel(), fb.ravel()])


def rhs_scaled(pb: Problem, g, f, y0) -> np.ndarray:
    """b = [g; -sqrt(gamma) f] of eq. main_system."""
    r = rhs_unscaled(pb, g, f, y0)
    nm = pb.n * pb.m
    return np.concatenate([r[:nm], -math.sqrt(pb.gamma) * r[nm:]])


def unpack_solution(pb: Problem, x: np.ndarray):
    """y = x_1/sqrt(gamma), p = x_2, each [n][m]."""
    nm = pb.n * pb.m
    y = x[:nm].reshape(pb.n, pb.m) / math.sqrt(pb.gamma)
    p = x[nm:].reshape(pb.n, pb.m).copy()
    return y, p


def kkt_apply(pb: Problem, x: np.ndarray, transpose: bool = False) -> np.ndarray:
    """y = A x (or A^T x) with the assembled sparse A."""
    A = kkt_scaled(pb)
    return (A.T @ x) if transpose else (A @ x)


def kkt_apply_blocks(pb: Problem, x: np.ndarray, transpose: bool = False) -> np.ndarray:
    """y = A x (or A^T x) written out block by block from eq. matrix_A without
    assembling A:  with E = M + tau K,
        y_1^j = alpha M x_1^j + E x_2^j - M x_2^{j+1},
        y_2^j = -(E x_1^j - M x_1^{j-1}) + alpha M x_2^j,
    x^0 = x^{n+1} = 0 (B_n has ones on the diagonal and -1 below it); A^T flips
    the sign of both off-diagonal blocks (M and K are symmetric).  Used where
    the assembled matrix is too large to build."""
    n, m = pb.n, pb.m
    X = np.asarray(x, dtype=np.float64).reshape(2, n, m)
    x1, x2 = X[0], X[1]
    Mm = pb.Mm
    Mx1 = (Mm @ x1.T).T
    Mx2 = (Mm @ x2.T).T
    Ex1 = Mx1 + pb.tau * (pb.K @ x1.T).T
    Ex2 = Mx2 + pb.tau * (pb.K @ x2.T).T
    x2next = np.vstack([Mx2[1:], np.zeros((1, m))])
    x1prev = np.vstack([np.zeros((1, m)), Mx1[:-1]])
    sgn = -1.0 if transpose else 1.0
    y1 = pb.alpha * Mx1 + sgn * (Ex2 - x2next)
    y2 = -sgn * (Ex1 - x1prev) + pb.alpha * Mx2
    return np.concatenate([y1.ravel(), y2.ravel()])

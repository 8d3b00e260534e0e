"""Oracle: the RBD preconditioners (Section 1 eq. matrix_P and eq. matrix_P_eps;
Section 2.1 four-step implementation).

Test infrastructure only.  The epsilon-circulant preconditioner is applied
exactly as the four steps of Section 2.1 describe, with an explicit dense
Fourier matrix F_n along time and a sparse LU factorisation per frequency.

Readings of the text (both fixed by checking the factorisation numerically):
  * D_eps = diag(eps^{(i-1)/n}), i = 1..n, as in eq. decomposition_eps (the
    Implementation subsection prints the exponent over N instead).
  * The first diagonal block of U is (F_n^* D_eps)^* (x) I_m = D_eps F_n (x) I_m,
    paired with conj(Lambda); the transpose printed there does not
    reproduce C_eps^T.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretize import Problem, eps_circulant, toeplitz_B


def fourier_matrix(n: int) -> np.ndarray:
    """F_n = n^{-1/2} [theta^{(i-1)(j-1)}], theta = exp(2 pi i / n) (eq. decomposition_eps)."""
    k = np.arange(n)
    return np.exp(2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


def d_eps(n: int, eps: float) -> np.ndarray:
    """Diagonal of D_eps: eps^{(i-1)/n}, i = 1..n."""
    return eps ** (np.arange(n) / n)


def lambda_eps(n: int, eps: float) -> np.ndarray:
    """lambda_k = 1 - eps^{1/n} theta^{-k}, k = 0..n-1."""
    return 1.0 - eps ** (1.0 / n) * np.exp(-2j * np.pi * np.arange(n) / n)


class EpsCirculantRBD:
    """w = P_eps^{-1} v by the four steps of Section 2.1.

    ``spatial="lu"`` solves the shifted systems of Step 2 exactly (sparse
    LU per frequency); ``spatial="mg"`` replaces each solve by one V-cycle of
    the multigrid in :mod:`oracle.multigrid` (Section 3, Example 2), which
    needs the coefficient function ``coeff`` (None means a = 1) and takes
    the V-cycle's ``smoother`` ("rb", "lex" or "sym")."""

    def __init__(self, pb: Problem, spatial: str = "lu", coeff=None, smoother: str = "rb"):
        self.pb = pb
        n, m = pb.n, pb.m
        self.F = fourier_matrix(n)
        self.D = d_eps(n, pb.eps)
        self.lam = lambda_eps(n, pb.eps)
        self.spatial = spatial
        if spatial == "lu":
            Kc = pb.K.tocsc().astype(np.complex128)
            Mc = pb.Mm.tocsc().astype(np.complex128)
            # one factorisation per frequency of (lambda_k + alpha) M + tau K;
            # block 1 needs conj(lambda_k) = lambda_{(n-k) mod n}
            self.lu = [spla.splu(((self.lam[k] + pb.alpha) * Mc + pb.tau * Kc).tocsc()) for k in range(n)]
        elif spatial == "mg":
            from .multigrid import ShiftedVCycle
            self.mg = ShiftedVCycle(pb.dim, pb.nx, pb.tau, coeff, smoother)
        else:
            raise ValueError(spatial)

    def _solve(self, k: int, rhs: np.ndarray) -> np.ndarray:
        if self.spatial == "lu":
            return self.lu[k].solve(rhs)
        return self.mg.apply(rhs, self.lam[k] + self.pb.alpha)

    def apply(self, v: np.ndarray) -> np.ndarray:
        pb = self.pb
        n, m = pb.n, pb.m
        v = np.asarray(v, dtype=np.float64).reshape(2, n, m)
        F, Fh = self.F, self.F.conj().T
        D = self.D[:, None]
        # step 1: v_hat = U^{-1} v with U = blockdiag(D F, D^{-1} F) (x) I
        v1h = Fh @ (v[0] / D)
        v2h = Fh @ (D * v[1])
        # step 2: frequency-wise shifted spatial solves
        t1 = np.empty_like(v1h)
        t2 = np.empty_like(v2h)
        for k in range(n):
            t1[k] = self._solve((n - k) % n, v1h[k])  # conj(lambda_k) + alpha
            t2[k] = self._solve(k, v2h[k])            # lambda_k + alpha
        # step 3: w_tilde = U v_tilde
        w1t = D * (F @ t1)
        w2t = (F @ t2) / D
        # the products are real up to rounding
        w1t = w1t.real
        w2t = w2t.real
        # step 4: w = [[I, -I], [I, I]] w_tilde
        return np.concatenate([(w1t - w2t).ravel(), (w1t + w2t).ravel()])


def eps_circulant_dense(pb: Problem) -> np.ndarray:
    """P_eps of eq. matrix_P_eps assembled densely (tiny grids only)."""
    n, m = pb.n, pb.m
    Md = pb.Mm.toarray()
    C = np.kron(eps_circulant(n, pb.eps), Md) + pb.tau * np.kron(np.eye(n), pb.K.toarray())
    A = pb.alpha * np.kron(np.eye(n), Md)
    H = np.block([[C.T + A, np.zeros_like(C)], [np.zeros_like(C), C + A]])
    I = np.eye(n * m)
    G = np.block([[I, I], [-I, I]])
    return 0.5 * H @ G


def ideal_rbd_dense(pb: Problem) -> np.ndarray:
    """P of eq. matrix_P assembled densely (tiny grids only)."""
    n, m = pb.n, pb.m
    Md = pb.Mm.toarray()
    Tm = np.kron(toeplitz_B(n).toarray(), Md) + pb.tau * np.kron(np.eye(n), pb.K.toarray())
    A = pb.alpha * np.kron(np.eye(n), Md)
    H = np.block([[Tm.T + A, np.zeros_like(Tm)], [np.zeros_like(Tm), Tm + A]])
    I = np.eye(n * m)
    G = np.block([[I, I], [-I, I]])
    return 0.5 * H @ G


class IdealRBD:
    """w = P^{-1} v for the ideal RBD preconditioner of eq. matrix_P.

    P^{-1} = G^{-1} blockdiag(T^T + alpha I, T + alpha I)^{-1}: the two block
    bidiagonal systems are solved by sequential substitution in time
    (T + alpha I forward from level 1, T^T + alpha I backward from level n),
    each step a solve with T_0 = (1 + alpha) M + tau K and the coupling
    -M to the neighbouring level (Section 2, the block lower-triangular
    Toeplitz structure of (T + alpha I (x) M)^{-1}).

    ``spatial="lu"`` solves with T_0 exactly (sparse LU); ``spatial="mg"``
    takes one V-cycle of :mod:`oracle.multigrid` with the real shift
    1 + alpha instead, as for the non-diagonalisable K of Example 2
    (Section 3)."""

    def __init__(self, pb: Problem, spatial: str = "lu", coeff=None, smoother: str = "rb"):
        self.pb = pb
        m = pb.m
        self.spatial = spatial
        if spatial == "lu":
            T0 = (1.0 + pb.alpha) * pb.Mm.tocsc() + pb.tau * pb.K.tocsc()
            self.lu = spla.splu(T0.tocsc())
        elif spatial == "mg":
            from .multigrid import ShiftedVCycle
            self.mg = ShiftedVCycle(pb.dim, pb.nx, pb.tau, coeff, smoother)
        else:
            raise ValueError(spatial)

    def _solve(self, r: np.ndarray) -> np.ndarray:
        if self.spatial == "lu":
            return self.lu.solve(r)
        return self.mg.apply(r, complex(1.0 + self.pb.alpha, 0.0)).real

    def apply(self, v: np.ndarray) -> np.ndarray:
        pb = self.pb
        n, m = pb.n, pb.m
        v = np.asarray(v, dtype=np.float64).reshape(2, n, m)
        z1 = np.zeros((n, m))
        z2 = np.zeros((n, m))
        Mm = pb.Mm
        for j in range(n):                       # (T + alpha I (x) M) z2 = v2
            r = v[1, j] + (Mm @ z2[j - 1] if j > 0 else 0.0)
            z2[j] = self._solve(r)
        for j in range(n - 1, -1, -1):           # (T^T + alpha I (x) M) z1 = v1
            r = v[0, j] + (Mm @ z1[j + 1] if j < n - 1 else 0.0)
            z1[j] = self._solve(r)
        return np.concatenate([(z1 - z2).ravel(), (z1 + z2).ravel()])


def eps_circulant_apply(pb: Problem, w: np.ndarray) -> np.ndarray:
    """v = P_eps w for P_eps of eq. matrix_P_eps without assembling it:
    with [u_1; u_2] = [[I, I], [-I, I]] w,
        v_1 = (C_eps^T + alpha I (x) M) u_1 / 2,  v_2 = (C_eps + alpha I (x) M) u_2 / 2,
    C_eps = C_{eps,n} (x) M + tau I (x) K, and C_{eps,n} = B_n with -eps in the
    top-right corner.  Checks a computed P_eps^{-1} v at any size."""
    n, m = pb.n, pb.m
    W = np.asarray(w, dtype=np.float64).reshape(2, n, m)
    u1 = W[0] + W[1]
    u2 = -W[0] + W[1]
    Mm = pb.Mm

    def c_apply(u, transpose):
        tK = pb.tau * (pb.K @ u.T).T
        Mu = (Mm @ u.T).T
        out = Mu + tK + pb.alpha * Mu
        if not transpose:   # (C u)_j = M u_j - M u_{j-1}, j = 0 wraps with -eps
            out[1:] -= Mu[:-1]
            out[0] -= pb.eps * Mu[-1]
        else:               # (C^T u)_j = M u_j - M u_{j+1}, j = n-1 wraps with -eps
            out[:-1] -= Mu[1:]
            out[-1] -= pb.eps * Mu[0]
        return out

    v1 = 0.5 * c_apply(u1, True)
    v2 = 0.5 * c_apply(u2, False)
    return np.concatenate([v1.ravel(), v2.ravel()])

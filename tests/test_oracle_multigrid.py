"""Pins for oracle.multigrid (the complex-shifted V-cycle).  Section 3 fixes
only 'one V-cycle, Gauss-Seidel pre-smoother, no post-smoother'; the tests
check the textbook properties of the cycle that the oracle implements."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import discretize as D
from oracle.multigrid import ShiftedVCycle, prolongation, red_mask, restriction


def test_transfer_operators():
    for dim in (1, 2, 3):
        P = prolongation(dim, 3)
        R = restriction(dim, 3)
        assert P.shape == (7 ** dim, 3 ** dim)
        assert abs(R - P.T / 2 ** dim).max() < 1e-15
        # linear interpolation reproduces a linear function of x1 that vanishes
        # at both ends only where it is linear: check interior constants
        ones_c = np.ones(3 ** dim)
        fine = P @ ones_c
        # the centre fine point of every coarse cell sees weight 1
        assert fine.max() == pytest.approx(1.0)
        # full weighting has unit row sums
        assert np.allclose(np.asarray(R.sum(axis=1)).ravel(), 1.0)


def test_prolongation_is_exact_for_linear_functions():
    """Multilinear interpolation reproduces functions linear in each x_d that
    vanish on the boundary (the piecewise-linear hat basis)."""
    nxc = 3
    xc = np.arange(1, nxc + 1) / (nxc + 1)
    xf = np.arange(1, 2 * nxc + 2) / (2 * nxc + 2)
    hat = lambda x: np.minimum(x, 1 - x)      # piecewise linear with kink at 1/2
    P = prolongation(1, nxc)
    assert np.allclose(P @ hat(xc), hat(xf))


def test_coarsest_level_is_exact():
    mg = ShiftedVCycle(2, 1, 0.01)
    sigma = 1.3 - 0.4j
    r = np.array([2.0 + 1.0j])
    z = mg.apply(r, sigma)
    A = sigma + 0.01 * D.stiffness(2, 1).toarray()[0, 0]
    assert abs(z[0] - r[0] / A) < 1e-15


def test_red_black_colouring():
    m = red_mask(2, 5)
    K = D.stiffness(2, 5).toarray()
    # red points only couple to black points
    off = K - np.diag(np.diag(K))
    assert np.all(off[np.ix_(m, m)] == 0) and np.all(off[np.ix_(~m, ~m)] == 0)


@pytest.mark.parametrize("dim,nx,coeff,tau,sigma", [
    (2, 31, None, 1 / 32, 1.1 + 0.3j),
    (2, 15, None, 1 / 16, 0.05 - 0.2j),
    (3, 15, W.coeff_sines3d, 1 / 128, 2.47 + 0.05j),
    (3, 7, W.coeff_sines3d, 1 / 8, 0.9 - 0.6j),
])
def test_vcycle_is_a_convergent_iteration(dim, nx, coeff, tau, sigma):
    """Used as a stationary iteration z <- z + V(r - A z), the V-cycle
    converges to the exact solution of (sigma I + tau K_a) z = r with a
    contraction factor well below one."""
    mg = ShiftedVCycle(dim, nx, tau, coeff)
    K = D.stiffness(dim, nx, coeff)
    A = (sigma * sp.identity(nx ** dim) + tau * K).tocsc()
    r = np.random.default_rng(0).standard_normal(nx ** dim) + 0j
    z_ex = spla.spsolve(A, r)
    z = np.zeros_like(r)
    errs = []
    for _ in range(8):
        z = z + mg.apply(r - A @ z, sigma)
        errs.append(np.linalg.norm(z - z_ex) / np.linalg.norm(z_ex))
    rates = np.array(errs[1:]) / np.array(errs[:-1])
    assert rates.max() < 0.6
    assert errs[-1] < 1e-2


def test_vcycle_is_linear():
    mg = ShiftedVCycle(2, 7, 0.05)
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(49) + 1j * rng.standard_normal(49), rng.standard_normal(49)
    s = 0.7 + 0.2j
    assert np.allclose(mg.apply(a + 2 * b, s), mg.apply(a, s) + 2 * mg.apply(b, s), atol=1e-13)


def test_vcycle_rejects_non_dyadic_grid():
    with pytest.raises(ValueError):
        ShiftedVCycle(2, 6, 0.1)


def _gauss_seidel_points(A, r, order):
    """Gauss-Seidel by its definition, one point at a time in the given order
    (dense, tiny grids only)."""
    A = A.toarray()
    z = np.zeros_like(r)
    for i in order:
        z[i] = (r[i] - A[i] @ z + A[i, i] * z[i]) / A[i, i]
    return z


@pytest.mark.parametrize("dim,nx,coeff", [(2, 7, None), (2, 7, W.coeff_example2), (3, 3, W.coeff_sines3d)])
@pytest.mark.parametrize("smoother", ["lex", "sym", "rb"])
def test_smoother_is_gauss_seidel_in_its_order(dim, nx, coeff, smoother):
    """The smoothers are Gauss-Seidel sweeps from z = 0: lexicographic (natural
    index order), symmetric (that order, then the reverse), red-black (even
    index sums first); checked against point-by-point sweeps."""
    tau, sigma = 0.1, 0.7 - 0.3j
    mg = ShiftedVCycle(dim, nx, tau, coeff, smoother=smoother)
    A = (sigma * sp.identity(nx ** dim) + tau * D.stiffness(dim, nx, coeff)).astype(np.complex128).tocsr()
    r = np.random.default_rng(3).standard_normal(nx ** dim) + 1j * np.random.default_rng(4).standard_normal(nx ** dim)
    m = nx ** dim
    if smoother == "rb":
        red = red_mask(dim, nx)
        order = list(np.flatnonzero(red)) + list(np.flatnonzero(~red))
    else:
        order = list(range(m))
        if smoother == "sym":
            order = order + order[::-1]
    z_ref = _gauss_seidel_points(A, r, order)
    assert np.linalg.norm(mg.smooth(0, r, sigma) - z_ref) < 1e-13 * np.linalg.norm(z_ref)


@pytest.mark.parametrize("smoother", ["lex", "sym"])
def test_lexicographic_vcycle_is_a_convergent_iteration(smoother):
    dim, nx, tau, sigma = 2, 31, 1 / 32, 1.1 + 0.3j
    mg = ShiftedVCycle(dim, nx, tau, W.coeff_example2, smoother=smoother)
    A = (sigma * sp.identity(nx ** dim) + tau * D.stiffness(dim, nx, W.coeff_example2)).tocsc()
    r = np.random.default_rng(0).standard_normal(nx ** dim) + 0j
    z_ex = spla.spsolve(A, r)
    z = np.zeros_like(r)
    for _ in range(8):
        z = z + mg.apply(r - A @ z, sigma)
    assert np.linalg.norm(z - z_ex) < 1e-3 * np.linalg.norm(z_ex)

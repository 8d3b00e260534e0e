"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds problem *data* only: the shapes of the five benchmark
workloads, the seeds, and generators for the fields g, f, y0 and the
diffusion coefficient a(x).  It contains none of the solver's arithmetic
(no discretisation, no right-hand-side assembly, no preconditioner), so the
oracle and the HIP path can both draw their inputs from here without sharing
any of the method.

Conventions (Section 1 of the paper, backward Euler with tau = T/N):
  * Omega = (0,1)^d, nx interior points per dimension, h = 1/(nx+1),
    grid points x_i = i*h, i = 1..nx, lexicographic order with x1 fastest.
  * N = nt time steps, the all-at-once system has n = N-1 time blocks
    holding the levels t_j = j*tau, j = 1..n.
  * Field arrays are float64 with shape [n][m] (levels 1..n) for g and f and
    [m] for y0, m = nx**d.

The smooth parts follow Example 1 of Section 3 (sine products, e^{-t}
decay); the noise is i.i.d. normal with variance 1e-2 (sigma = 0.1) on every
interior node, drawn from ``numpy.random.default_rng([config_id, member])``
in the order y0, g (levels 1..n), f (levels 1..n).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

NOISE_SIGMA = 0.1  # N(0, 1e-2): variance 1e-2


@dataclass(frozen=True)
class Workload:
    """Shape and parameters of one synthetic workload."""

    config_id: int
    name: str
    dim: int
    nx: int
    nt: int
    T: float
    gammas: tuple
    eps: Optional[float] = None  # None -> sqrt(tau)
    coeff: str = "one"  # "one" or "sines3d" (variable a(x))
    noise: float = NOISE_SIGMA
    precision: str = "fp64"
    spatial: str = "dst"
    batch: int = 1

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

    def eps_value(self) -> float:
        return math.sqrt(self.tau) if self.eps is None else float(self.eps)


def _batch_gammas(batch: int = 64) -> tuple:
    rng = np.random.default_rng([4, 10 ** 6])
    return tuple(float(v) for v in 10.0 ** rng.uniform(-8.0, -2.0, size=batch))


CONFIGS = {
    1: Workload(1, "2d-nx31-nt32", 2, 31, 32, 1.0, (1e-4,)),
    2: Workload(2, "2d-nx255-nt256", 2, 255, 256, 1.0, (1e-2, 1e-6, 1e-10)),
    3: Workload(3, "2d-nx511-nt512-mixed", 2, 511, 512, 1.0, (1e-6,), precision="mixed"),
    4: Workload(4, "2d-nx127-nt128-batch64", 2, 127, 128, 1.0, _batch_gammas(64), batch=64),
    5: Workload(5, "3d-nx63-nt128-vara-mg", 3, 63, 128, 1.0, (1e-5,), coeff="sines3d",
                precision="mixed", spatial="mg"),
}
# the same workloads by name
WORKLOADS = {w.name: w for w in CONFIGS.values()}


def grid_points(nx: int) -> np.ndarray:
    """Interior grid coordinates i*h, i = 1..nx."""
    return np.arange(1, nx + 1, dtype=np.float64) / (nx + 1)


def mesh(dim: int, nx: int) -> list:
    """Coordinate arrays X_1..X_d of shape [m] in lexicographic order, x1 fastest."""
    x = grid_points(nx)
    grids = np.meshgrid(*([x] * dim), indexing="ij")  # grids[k] varies along axis k
    # axis 0 of the ij-mesh must be the slowest index (x_d), the last axis x1
    out = []
    for d in range(dim):
        # coordinate x_{d+1} varies along array axis (dim-1-d)
        out.append(np.ascontiguousarray(grids[dim - 1 - d]).reshape(-1))
    return out


def sine_product(coords: Sequence[np.ndarray]) -> np.ndarray:
    s = np.ones_like(coords[0])
    for c in coords:
        s = s * np.sin(np.pi * c)
    return s


def smooth_fields(dim: int, nx: int, nt: int, T: float = 1.0):
    """Example-1 fields sampled on the grid (Section 3, Example 1; the 3-D
    case uses the triple product with the coefficient 3*pi^2 - 1).

    Returns g [n][m], f [n][m] at t_j = j*tau (j = 1..n) and y0 [m]."""
    n = nt - 1
    tau = T / nt
    s = sine_product(mesh(dim, nx))
    t = tau * np.arange(1, n + 1, dtype=np.float64)
    decay = np.exp(-t)[:, None]
    g = decay * s[None, :]
    f = (dim * np.pi ** 2 - 1.0) * g
    y0 = s.copy()
    return g, f, y0


def fields(w: Workload, member: int = 0, noise: Optional[float] = None):
    """Smooth-plus-noise g, f, y0 for member ``member`` of workload ``w``."""
    sigma = w.noise if noise is None else noise
    g, f, y0 = smooth_fields(w.dim, w.nx, w.nt, w.T)
    if sigma > 0:
        rng = np.random.default_rng([w.config_id, member])
        y0 += sigma * rng.standard_normal(y0.shape)
        g += sigma * rng.standard_normal(g.shape)
        f += sigma * rng.standard_normal(f.shape)
    return g, f, y0


def random_fields(dim: int, nx: int, nt: int, seed: int, sigma: float = 1.0):
    """Pure-noise g, f, y0 (used by parity tests on small grids)."""
    n, m = nt - 1, nx ** dim
    rng = np.random.default_rng(seed)
    y0 = sigma * rng.standard_normal(m)
    g = sigma * rng.standard_normal((n, m))
    f = sigma * rng.standard_normal((n, m))
    return g, f, y0


def random_vector(dim: int, nx: int, nt: int, seed: int, batch: int = 1) -> np.ndarray:
    """A random all-at-once vector of shape [batch][2][n][m]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch, 2, nt - 1, nx ** dim))


# ---------------------------------------------------------------------------
# diffusion coefficients a(x) (problem data; Section 1, L = div(a grad))
# ---------------------------------------------------------------------------

def coeff_one(*coords):
    return np.ones_like(coords[0])


def coeff_sines3d(*coords):
    """a(x) = 1 + 0.5 * prod_d sin(2 pi x_d)."""
    p = np.ones_like(coords[0])
    for c in coords:
        p = p * np.sin(2.0 * np.pi * c)
    return 1.0 + 0.5 * p


def coeff_example2(x1, x2):
    """a(x1, x2) = 1e-5 sin(pi x1 x2) (Section 3, Example 2)."""
    return 1e-5 * np.sin(np.pi * x1 * x2)


COEFFS: dict = {"one": coeff_one, "sines3d": coeff_sines3d, "example2": coeff_example2}


def coeff_function(name: str) -> Callable:
    return COEFFS[name]


# ---------------------------------------------------------------------------
# analytic test problems of Section 3
# ---------------------------------------------------------------------------

def example1_exact(dim: int, nx: int, t: float):
    """Example 1: y = e^{-t} prod sin(pi x_d), p = 0."""
    s = sine_product(mesh(dim, nx))
    return np.exp(-t) * s, np.zeros_like(s)


def example1_source(dim: int, nx: int, t: float):
    """Example 1 data at time t: f = (d pi^2 - 1) e^{-t} prod sin, g = e^{-t} prod sin."""
    s = sine_product(mesh(dim, nx))
    g = np.exp(-t) * s
    return (dim * np.pi ** 2 - 1.0) * g, g


def example2_exact(nx: int, t: float, gamma: float):
    """Example 2 (2-D): y = e^{-t} x1(1-x1) x2(1-x2), p = gamma sin(pi t) sin(pi x1) sin(pi x2)."""
    x1, x2 = mesh(2, nx)
    y = np.exp(-t) * x1 * (1 - x1) * x2 * (1 - x2)
    p = gamma * np.sin(np.pi * t) * np.sin(np.pi * x1) * np.sin(np.pi * x2)
    return y, p


def example2_source(nx: int, t: float, gamma: float):
    """Example 2 data f, g at time t.  The factor printed as ``x(1-2x_2)`` in
    f is read as x1(1-2x2), the only reading for which the printed y, p, a
    satisfy the state equation."""
    x1, x2 = mesh(2, nx)
    pi = np.pi
    s12 = np.sin(pi * x1 * x2)
    c12 = np.cos(pi * x1 * x2)
    et = np.exp(-t)
    f = (-np.sin(pi * t) * np.sin(pi * x1) * np.sin(pi * x2)
         + et * x1 * (1 - x1) * (2e-5 * s12 - x2 * (1 - x2) - 1e-5 * pi * c12 * x1 * (1 - 2 * x2))
         + et * x2 * (1 - x2) * (2e-5 * s12 - 1e-5 * pi * c12 * x2 * (1 - 2 * x1)))
    g = (-gamma * pi * np.cos(pi * t) * np.sin(pi * x1) * np.sin(pi * x2)
         + et * x1 * (1 - x1) * x2 * (1 - x2)
         - 1e-5 * gamma * pi ** 2 * np.sin(pi * t) * (
             -2 * s12 * np.sin(pi * x1) * np.sin(pi * x2)
             + c12 * (x1 * np.sin(pi * x1) * np.cos(pi * x2) + x2 * np.cos(pi * x1) * np.sin(pi * x2))))
    return f, g


def example_fields(example: int, dim: int, nx: int, nt: int, T: float = 1.0, gamma: float = 1.0):
    """g [n][m], f [n][m] at levels 1..n and y0 [m] for Example 1 or 2."""
    n = nt - 1
    tau = T / nt
    gs, fs = [], []
    for j in range(1, n + 1):
        t = j * tau
        if example == 1:
            f, g = example1_source(dim, nx, t)
        else:
            f, g = example2_source(nx, t, gamma)
        gs.append(g)
        fs.append(f)
    if example == 1:
        y0, _ = example1_exact(dim, nx, 0.0)
    else:
        y0, _ = example2_exact(nx, 0.0, gamma)
    return np.array(gs), np.array(fs), y0

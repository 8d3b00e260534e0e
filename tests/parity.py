"""Comparison helpers of the GPU parity tests.

A whole-vector relative 2-norm can hide a small wrong part (one ragged tile,
one member, the last time level) under a loose floating-point bar, so
``check`` also compares every (member, block, time level) slice element by
element against the largest value of its member."""
from __future__ import annotations

import numpy as np


def rel(a, b) -> float:
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def level_errors(a, b, batch: int, n: int, m: int) -> np.ndarray:
    """max |a - b| over each (member, block, time level) slice of
    [batch][2][n][m] vectors, divided by max |b| over that member."""
    a = np.asarray(a).reshape(batch, 2, n, m)
    b = np.asarray(b).reshape(batch, 2, n, m)
    scale = np.maximum(np.abs(b).reshape(batch, -1).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=3) / scale[:, None, None]


def check(a, b, tol: float, batch: int, n: int, m: int, level_factor: float = 10.0, label: str = "") -> float:
    """Whole-vector relative error <= tol, and on every time level of every
    block and member the largest elementwise error <= level_factor * tol
    times the member's largest value.  Returns the relative error."""
    r = rel(a, b)
    lev = level_errors(a, b, batch, n, m)
    worst = np.unravel_index(int(np.argmax(lev)), lev.shape)
    print(f"  {label} rel {r:.2e}  worst level err {lev.max():.2e} at (member, block, level) {tuple(int(v) for v in worst)}",
          flush=True)
    assert r <= tol, (label, r, tol)
    assert lev.max() <= level_factor * tol, (label, lev.max(), worst, level_factor * tol)
    return r

"""Banded LU without pivoting and line-by-line forward/back substitution
(Appendix: the 1D matrices are banded, M_ij = 0 for |i-j| > p; each
direction is a 1D banded system with many right-hand sides, one per grid
line, factorized once).

All matrices factored here are symmetric positive definite (mass plus a
non-negative multiple of stiffness, after Dirichlet elimination), so
elimination without pivoting is stable.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class BandLU:
    p: int
    L: np.ndarray   # (m, p+1): L[i, k] = multiplier l_{i, i-k}, k = 1..p (col 0 unused)
    U: np.ndarray   # (m, p+1): U[i, k] = u_{i, i+k}, k = 0..p

    @property
    def m(self) -> int:
        return self.L.shape[0]


def band_lu(A: np.ndarray, p: int) -> BandLU:
    """Doolittle elimination restricted to the band |i-j| <= p."""
    m = A.shape[0]
    L = np.zeros((m, m))
    U = np.zeros((m, m))
    for i in range(m):
        L[i, i] = 1.0
        for j in range(i, min(m, i + p + 1)):
            s = sum(L[i, k] * U[k, j] for k in range(max(0, j - p), i))
            U[i, j] = A[i, j] - s
        for r in range(i + 1, min(m, i + p + 1)):
            s = sum(L[r, k] * U[k, i] for k in range(max(0, r - p), i))
            L[r, i] = (A[r, i] - s) / U[i, i]
    Lb = np.zeros((m, p + 1))
    Ub = np.zeros((m, p + 1))
    for i in range(m):
        for k in range(1, p + 1):
            if i - k >= 0:
                Lb[i, k] = L[i, i - k]
        for k in range(0, p + 1):
            if i + k < m:
                Ub[i, k] = U[i, i + k]
    return BandLU(p, Lb, Ub)


def solve_lines(f: BandLU, b: np.ndarray, axis: int) -> np.ndarray:
    """Solve A x = b along ``axis`` of ``b`` for every line at once
    (forward substitution with L, then back substitution with U)."""
    y = np.moveaxis(np.array(b, dtype=np.float64, copy=True), axis, 0)
    m, p = f.m, f.p
    assert y.shape[0] == m
    for i in range(m):
        for k in range(1, min(p, i) + 1):
            y[i] -= f.L[i, k] * y[i - k]
    for i in range(m - 1, -1, -1):
        for k in range(1, min(p, m - 1 - i) + 1):
            y[i] -= f.U[i, k] * y[i + k]
        y[i] /= f.U[i, 0]
    return np.moveaxis(y, 0, axis)

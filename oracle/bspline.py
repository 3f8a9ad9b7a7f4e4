"""B-spline basis on an open uniform knot vector (Section 2: the 1D B-splines
n_a, m_b whose tensor products form the discrete space).

The paper never states the knot vector.  Reading used here: open (clamped)
uniform knots on [0, 1] with E elements and maximal continuity C^{p-1}, so
there are n = E + p basis functions per direction.
"""
from __future__ import annotations

import numpy as np


def open_uniform_knots(E: int, p: int) -> np.ndarray:
    """[0]*(p+1) + [k/E for k=1..E-1] + [1]*(p+1)."""
    inner = np.arange(1, E, dtype=np.float64) / E
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def _degree0(t: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Degree-0 functions: indicator of [t_i, t_{i+1}); the last non-empty
    interval is closed on the right so that x = 1 is covered."""
    m = t.size - 1
    B = np.zeros((x.size, m))
    for i in range(m):
        if t[i + 1] > t[i]:
            B[:, i] = (x >= t[i]) & (x < t[i + 1])
    last = max(i for i in range(m) if t[i + 1] > t[i])
    B[x == t[last + 1], last] = 1.0
    return B


def _ratio(num, den):
    """num / den with the Cox-de Boor convention 0/0 := 0."""
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def basis_upto(t: np.ndarray, p: int, x) -> list:
    """Cox-de Boor recursion; returns [B^0, B^1, ..., B^p] where B^k has shape
    (len(x), len(t)-1-k) and B^k[:, i] = B_{i,k}(x)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    out = [_degree0(t, x)]
    for k in range(1, p + 1):
        prev = out[-1]
        m = t.size - 1 - k
        B = np.zeros((x.size, m))
        for i in range(m):
            left = _ratio(x - t[i], np.full_like(x, t[i + k] - t[i]))
            right = _ratio(t[i + k + 1] - x, np.full_like(x, t[i + k + 1] - t[i + 1]))
            B[:, i] = left * prev[:, i] + right * prev[:, i + 1]
        out.append(B)
    return out


def basis(t: np.ndarray, p: int, x) -> np.ndarray:
    """Values of all n = len(t)-p-1 degree-p B-splines at x, shape (len(x), n)."""
    return basis_upto(t, p, x)[p]


def basis_deriv(t: np.ndarray, p: int, x) -> np.ndarray:
    """First derivatives: B'_{i,p} = p/(t_{i+p}-t_i) B_{i,p-1}
    - p/(t_{i+p+1}-t_{i+1}) B_{i+1,p-1}, with 0/0 := 0."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if p == 0:
        return np.zeros((x.size, t.size - 1))
    Bm = basis_upto(t, p - 1, x)[p - 1]
    n = t.size - p - 1
    D = np.zeros((x.size, n))
    for i in range(n):
        a = t[i + p] - t[i]
        b = t[i + p + 1] - t[i + 1]
        if a > 0:
            D[:, i] += p / a * Bm[:, i]
        if b > 0:
            D[:, i] -= p / b * Bm[:, i + 1]
    return D


def greville(t: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae xi_i = (t_{i+1} + ... + t_{i+p}) / p: the coefficients
    that reproduce the linear function x exactly."""
    n = t.size - p - 1
    return np.array([t[i + 1:i + p + 1].mean() for i in range(n)])

"""Dense 1D matrices (Section 2: M_x = (n_a, n_c), K_x = (n_a', n_c');
Section 5: the mixed matrices (n_a', n_c), (n_a, n_c')).

Every entry is an integral over [0,1] computed with the Gauss rule of
``quadrature`` (exact for these integrands).  Matrices are returned DENSE on
the full index set 0..n-1; ``free_index`` gives the rows/columns that remain
after zero Dirichlet conditions are imposed by eliminating the first and last
basis function (the only ones non-zero on the boundary of an open knot
vector).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import bspline, quadrature


@dataclasses.dataclass
class Basis1D:
    E: int
    p: int
    q: int
    knots: np.ndarray
    x: np.ndarray       # Gauss points, flat (E*q,)
    w: np.ndarray       # Gauss weights (already scaled by element length)
    N: np.ndarray       # (E*q, n) basis values at the points
    D: np.ndarray       # (E*q, n) basis derivatives at the points

    @property
    def n(self) -> int:
        return self.E + self.p


def basis_1d(E: int, p: int, q: int | None = None) -> Basis1D:
    q = p + 1 if q is None else q
    t = bspline.open_uniform_knots(E, p)
    x, w = quadrature.element_points(E, q)
    x = x.reshape(-1)
    w = w.reshape(-1)
    return Basis1D(E, p, q, t, x, w, bspline.basis(t, p, x), bspline.basis_deriv(t, p, x))


def mass(b: Basis1D) -> np.ndarray:
    """M[i,j] = int B_i B_j."""
    return b.N.T @ (b.w[:, None] * b.N)


def stiffness(b: Basis1D) -> np.ndarray:
    """K[i,j] = int B_i' B_j'."""
    return b.D.T @ (b.w[:, None] * b.D)


def mixed(b: Basis1D) -> np.ndarray:
    """G[i,j] = int B_i B_j'  (test function undifferentiated, trial
    differentiated); its transpose is int B_i' B_j."""
    return b.N.T @ (b.w[:, None] * b.D)


def free_index(n: int, bc: str = "dirichlet") -> np.ndarray:
    if bc == "dirichlet":
        return np.arange(1, n - 1)
    if bc == "neumann":
        return np.arange(n)
    raise ValueError(bc)


def restrict(A: np.ndarray, idx: np.ndarray) -> np.ndarray:
    return A[np.ix_(idx, idx)]

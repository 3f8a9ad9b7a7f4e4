"""Gauss-Legendre quadrature per element.

The paper leaves the quadrature unstated; the reading used here is q Gauss
points per element per direction (q = p+1 by default), which integrates the
products B_i B_j, B_i' B_j', B_i B_j' (polynomials of degree <= 2p on each
element) exactly, so the quadrature route and exact integration coincide.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss


def element_points(E: int, q: int):
    """Physical Gauss points and weights on the uniform mesh of [0,1] with E
    elements; both returned with shape (E, q)."""
    xi, om = leggauss(q)
    edges = np.arange(E + 1, dtype=np.float64) / E
    a = edges[:-1, None]
    b = edges[1:, None]
    x = 0.5 * (a + b) + 0.5 * (b - a) * xi[None, :]
    w = 0.5 * (b - a) * om[None, :]
    return x, w


def points_1d(E: int, q: int) -> np.ndarray:
    """All Gauss points of one direction in element-major order (E*q,)."""
    return element_points(E, q)[0].reshape(-1)

"""Kronecker-structured applies and the direction-split solve.

Coefficient arrays are indexed [z, y, x] (x fastest).  Direction d = 0, 1, 2
means x, y, z.  A 1D operator T_d "in direction d" acts on the index of that
direction only; a tensor product T_x (x) T_y (x) T_z applies each factor
along its own direction (eq. pwave2 and the Appendix's three 1D problems).
"""
from __future__ import annotations

import numpy as np

from .banded import BandLU, solve_lines

AXIS = {0: 2, 1: 1, 2: 0}   # direction -> numpy axis of a [z, y, x] array


def apply_dir(T: np.ndarray, U: np.ndarray, d: int) -> np.ndarray:
    """out = T applied along direction d (dense matrix; O(n^4) for n^3 data)."""
    ax = AXIS[d]
    out = np.tensordot(T, U, axes=([1], [ax]))   # new axis 0
    return np.moveaxis(out, 0, ax)


def kron3(Tx: np.ndarray, Ty: np.ndarray, Tz: np.ndarray, U: np.ndarray) -> np.ndarray:
    """(Tx (x) Ty (x) Tz) U with each factor acting along its direction."""
    return apply_dir(Tx, apply_dir(Ty, apply_dir(Tz, U, 2), 1), 0)


def ads_solve(fx: BandLU, fy: BandLU, fz: BandLU, b: np.ndarray) -> np.ndarray:
    """Solve (A_x (x) A_y (x) A_z) x = b as three sets of 1D banded solves:
    every x-line, then every y-line, then every z-line (Appendix)."""
    t = solve_lines(fx, b, AXIS[0])
    t = solve_lines(fy, t, AXIS[1])
    return solve_lines(fz, t, AXIS[2])


def dense_kron(Tx: np.ndarray, Ty: np.ndarray, Tz: np.ndarray) -> np.ndarray:
    """Assembled matrix of Tx (x) Ty (x) Tz acting on a C-order flattened
    [z, y, x] array (z slowest, so Tz is the outer Kronecker factor)."""
    return np.kron(Tz, np.kron(Ty, Tx))

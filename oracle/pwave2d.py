"""The P-wave problem in two dimensions, the dimension of the paper's
exposition (Section 2): tensor-product B-splines on the unit square, the
Galerkin stiffness K = K_x (x) M_y + M_x (x) K_y, and the Newmark step with
the direction-split left-hand side G = (M_x + eta K_x) (x) (M_y + eta K_y) of
eq. pwave2, inverted by x-line then y-line banded solves (Appendix).

Arrays are indexed [y, x] (x fastest).  Test infrastructure only: the HIP
library is never built on this module.  Same readings as the 3D oracle
(standard Newmark beta = 1/4, gamma = 1/2; open uniform knots; q = p + 1
Gauss points; zero Dirichlet by elimination or natural conditions).
"""
from __future__ import annotations

import numpy as np

from . import matrices as mx
from .banded import band_lu, solve_lines


class PWave2D:
    def __init__(self, nelem, p: int, q: int | None = None, tau: float = 1e-2,
                 bc: str = "dirichlet"):
        self.nelem = tuple(int(e) for e in nelem)
        assert len(self.nelem) == 2
        self.p = p
        self.q = p + 1 if q is None else q
        self.tau = float(tau)
        self.eta = self.tau ** 2 / 4.0
        self.b1 = [mx.basis_1d(E, p, self.q) for E in self.nelem]
        self.idx = [mx.free_index(b.n, bc) for b in self.b1]
        self.M = [mx.restrict(mx.mass(b), i) for b, i in zip(self.b1, self.idx)]
        self.K = [mx.restrict(mx.stiffness(b), i) for b, i in zip(self.b1, self.idx)]
        self.A = [M + self.eta * K for M, K in zip(self.M, self.K)]
        self.fA = [band_lu(A, p) for A in self.A]
        self.fM = [band_lu(M, p) for M in self.M]

    # -- layout -----------------------------------------------------------
    @property
    def free_shape(self):
        return (len(self.idx[1]), len(self.idx[0]))

    @property
    def full_shape(self):
        return (self.b1[1].n, self.b1[0].n)

    def to_full(self, U: np.ndarray) -> np.ndarray:
        out = np.zeros(U.shape[:-2] + self.full_shape)
        out[..., self.idx[1][:, None], self.idx[0][None, :]] = U
        return out

    def to_free(self, Ufull: np.ndarray) -> np.ndarray:
        return Ufull[..., self.idx[1][:, None], self.idx[0][None, :]]

    # -- operators ----------------------------------------------------------
    @staticmethod
    def kron2(Tx: np.ndarray, Ty: np.ndarray, U: np.ndarray) -> np.ndarray:
        """(Tx (x) Ty) U: Tx along x (axis 1), Ty along y (axis 0)."""
        return Ty @ U @ Tx.T

    def stiffness(self, w: np.ndarray) -> np.ndarray:
        return self.kron2(self.K[0], self.M[1], w) + self.kron2(self.M[0], self.K[1], w)

    def mass(self, w: np.ndarray) -> np.ndarray:
        return self.kron2(self.M[0], self.M[1], w)

    def G(self, w: np.ndarray) -> np.ndarray:
        return self.kron2(self.A[0], self.A[1], w)

    def _solve(self, f, r: np.ndarray) -> np.ndarray:
        return solve_lines(f[1], solve_lines(f[0], r, 1), 0)

    def solve_G(self, r: np.ndarray) -> np.ndarray:
        return self._solve(self.fA, r)

    def solve_M(self, r: np.ndarray) -> np.ndarray:
        return self._solve(self.fM, r)

    # -- data -------------------------------------------------------------
    def quad_points(self, d: int) -> np.ndarray:
        return self.b1[d].x

    def project(self, vals: np.ndarray) -> np.ndarray:
        """L2 projection of data at the Gauss points [(Ey q), (Ex q)]."""
        Tx = (self.b1[0].N * self.b1[0].w[:, None]).T[self.idx[0]]
        Ty = (self.b1[1].N * self.b1[1].w[:, None]).T[self.idx[1]]
        return self.solve_M(Ty @ vals @ Tx.T)

    # -- time stepping ------------------------------------------------------
    def initial_accel(self, u0: np.ndarray) -> np.ndarray:
        return self.solve_G(-self.stiffness(u0))

    def step(self, u, v, a):
        w = u + self.tau * v + self.eta * a
        a1 = self.solve_G(-self.stiffness(w))
        v1 = v + 0.5 * self.tau * (a + a1)
        u1 = w + self.eta * a1
        return u1, v1, a1

    def run(self, u0, v0=None, nsteps: int = 1, history: bool = False):
        v = np.zeros_like(u0) if v0 is None else v0
        u, a = u0, self.initial_accel(u0)
        hist = [(u, v, a)] if history else None
        for _ in range(nsteps):
            u, v, a = self.step(u, v, a)
            if history:
                hist.append((u, v, a))
        return ((u, v, a), hist) if history else (u, v, a)

    def energy(self, u, v) -> float:
        """1/2 v^T (G - eta K) v + 1/2 u^T K u (conserved without load)."""
        return (0.5 * float(np.sum(v * (self.G(v) - self.eta * self.stiffness(v))))
                + 0.5 * float(np.sum(u * self.stiffness(u))))

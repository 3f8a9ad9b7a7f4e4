"""Isotropic linear elasticity in two dimensions, the dimension in which
Section 5 writes its blocks: plane strain on the unit square, displacement
(u_x, u_y), rho u'' = div sigma + F with sigma = lambda (div u) I +
2 mu eps(u).  Test infrastructure only: the HIP library is never built on
this module.

Readings (as for the 3D oracle, written here for two components):

* Blocks from the bilinear form a(w, u) = 2 mu (eps(w), eps(u)) +
  lambda (div w, div u).  For a test function phi e_i and a trial function
  psi e_k:
      i == k:  (2mu+lambda) (d_i phi, d_i psi) + mu (d_j phi, d_j psi), j != i
      i != k:  mu (d_k phi, d_i psi) + lambda (d_i phi, d_k psi)
  so with tensor-product splines Upsilon_ii = (2mu+lambda) K (x) M + mu M (x) K
  (K in direction i for the first term) and Upsilon_ik = mu [G in direction
  i, G^T in direction k] + lambda [G^T in direction i, G in direction k],
  G = (B_a, B_c') (trial differentiated).
* Alternating-triangular scheme in its three-level form (eq. pre, eq. corr,
  eq. gen): D Z = tau^2 (f^n - Upsilon U^n), U^{n+1} = 2U^n - U^{n-1} + Z,
  D = (rho M + tau^2/2 U1)(rho M)^{-1}(rho M + tau^2/2 U2), the predictor over
  components x then y, the corrector y then x (the paper's order), the
  diagonal blocks split as in eq. spill: rho (M_x + tau^2 c_{i,x}/(4 rho) K_x)
  (x) (M_y + tau^2 c_{i,y}/(4 rho) K_y), c_{i,i} = 2mu+lambda, mu otherwise.
* Start: Z^0 = D^{-1} tau^2 (f^0 - Upsilon U^0), U^{-1} = U^0 - tau V^0 + Z^0/2.

Arrays are [component, y, x] (x fastest).
"""
from __future__ import annotations

import numpy as np

from . import matrices as mx
from .banded import band_lu, solve_lines


class Elastic2D:
    def __init__(self, nelem, p: int, q: int | None = None, tau: float = 5e-3,
                 rho: float = 1.0, lam: float = 1.0, mu: float = 1.0, bc: str = "dirichlet"):
        self.nelem = tuple(int(e) for e in nelem)
        assert len(self.nelem) == 2
        self.p = p
        self.q = p + 1 if q is None else q
        self.tau = float(tau)
        self.rho, self.lam, self.mu = float(rho), float(lam), float(mu)
        self.b1 = [mx.basis_1d(E, p, self.q) for E in self.nelem]
        self.idx = [mx.free_index(b.n, bc) for b in self.b1]
        self.M = [mx.restrict(mx.mass(b), i) for b, i in zip(self.b1, self.idx)]
        self.K = [mx.restrict(mx.stiffness(b), i) for b, i in zip(self.b1, self.idx)]
        self.G = [mx.restrict(mx.mixed(b), i) for b, i in zip(self.b1, self.idx)]
        self.split = {}
        self.fS = {}
        for d in range(2):
            for c in (self.mu, 2 * self.mu + self.lam):
                A = self.M[d] + self.tau ** 2 * c / (4 * self.rho) * self.K[d]
                self.split[(d, c)] = A
                self.fS[(d, c)] = band_lu(A, p)
        self.fM = [band_lu(M, p) for M in self.M]

    # -- layout -------------------------------------------------------------
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

    def c(self, i: int, d: int) -> float:
        return 2 * self.mu + self.lam if i == d else self.mu

    # -- operators ----------------------------------------------------------
    @staticmethod
    def kron2(Tx: np.ndarray, Ty: np.ndarray, U: np.ndarray) -> np.ndarray:
        """(Tx (x) Ty) U: Tx along x (axis 1), Ty along y (axis 0)."""
        return Ty @ U @ Tx.T

    def _dirs(self, ops_by_dir, U):
        return self.kron2(ops_by_dir[0], ops_by_dir[1], U)

    def block(self, i: int, k: int, U: np.ndarray) -> np.ndarray:
        """Upsilon_ik U (test component i, trial component k)."""
        if i == k:
            out = 0.0
            for d in range(2):
                ops = [self.K[e] if e == d else self.M[e] for e in range(2)]
                out = out + self.c(i, d) * self._dirs(ops, U)
            return out
        t_mu = [None, None]
        t_mu[i], t_mu[k] = self.G[i], self.G[k].T
        t_la = [None, None]
        t_la[i], t_la[k] = self.G[i].T, self.G[k]
        return self.mu * self._dirs(t_mu, U) + self.lam * self._dirs(t_la, U)

    def upsilon(self, U: np.ndarray) -> np.ndarray:
        return np.stack([self.block(i, 0, U[0]) + self.block(i, 1, U[1]) for i in range(2)])

    def mass(self, U: np.ndarray) -> np.ndarray:
        return np.stack([self.kron2(self.M[0], self.M[1], U[i]) for i in range(2)])

    # -- split solves ---------------------------------------------------------
    def split_diag(self, i: int, U: np.ndarray) -> np.ndarray:
        return self.rho * self.kron2(self.split[(0, self.c(i, 0))], self.split[(1, self.c(i, 1))], U)

    def solve_diag(self, i: int, r: np.ndarray) -> np.ndarray:
        """rho^-1 (A_x (x) A_y)^-1 r: x-lines, then y-lines."""
        t = solve_lines(self.fS[(0, self.c(i, 0))], r, 1)
        return solve_lines(self.fS[(1, self.c(i, 1))], t, 0) / self.rho

    def at_solve(self, R: np.ndarray) -> np.ndarray:
        """Z = D^{-1} R: predictor x then y (block lower), corrector y then x
        (block upper, right-hand side rho M Y_i)."""
        h = 0.5 * self.tau ** 2
        Y0 = self.solve_diag(0, R[0])
        Y1 = self.solve_diag(1, R[1] - h * self.block(1, 0, Y0))
        Z1 = self.solve_diag(1, self.rho * self.kron2(self.M[0], self.M[1], Y1))
        Z0 = self.solve_diag(0, self.rho * self.kron2(self.M[0], self.M[1], Y0) - h * self.block(0, 1, Z1))
        return np.stack([Z0, Z1])

    def step(self, Un, Unm1, f=None):
        R = -self.upsilon(Un)
        if f is not None:
            R = R + f
        return 2 * Un - Unm1 + self.at_solve(self.tau ** 2 * R)

    def start(self, U0, V0=None, f0=None):
        V0 = np.zeros_like(U0) if V0 is None else V0
        R = -self.upsilon(U0)
        if f0 is not None:
            R = R + f0
        return U0 - self.tau * V0 + 0.5 * self.at_solve(self.tau ** 2 * R)

    def run(self, U0, V0=None, nsteps: int = 1, history=False):
        """(U^n, U^{n-1}) after nsteps steps without load."""
        Unm1 = self.start(U0, V0)
        Un = U0
        hist = [(Un, Unm1)] if history else None
        for _ in range(nsteps):
            Un, Unm1 = self.step(Un, Unm1), Un
            if history:
                hist.append((Un, Unm1))
        return ((Un, Unm1), hist) if history else (Un, Unm1)

    # -- invariants -------------------------------------------------------------
    def D_apply(self, V: np.ndarray) -> np.ndarray:
        """D V = L (rho M)^{-1} L^T V, L = rho M + tau^2/2 U1 (split diagonal)."""
        h = 0.5 * self.tau ** 2
        w0 = self.split_diag(0, V[0]) + h * self.block(0, 1, V[1])
        w1 = self.split_diag(1, V[1])
        s = [solve_lines(self.fM[1], solve_lines(self.fM[0], w, 1), 0) / self.rho for w in (w0, w1)]
        return np.stack([self.split_diag(0, s[0]), self.split_diag(1, s[1]) + h * self.block(1, 0, s[0])])

    def energy(self, Unp1, Un) -> float:
        """1/2 |V|^2_{D - tau^2 Upsilon/4} + 1/2 |W|^2_Upsilon with
        V = (U^{n+1}-U^n)/tau, W = (U^{n+1}+U^n)/2: constant without load."""
        V = (Unp1 - Un) / self.tau
        W = 0.5 * (Unp1 + Un)
        kin = float(np.sum(V * self.D_apply(V))) - 0.25 * self.tau ** 2 * float(np.sum(V * self.upsilon(V)))
        return 0.5 * kin + 0.5 * float(np.sum(W * self.upsilon(W)))

"""Isotropic linear elasticity rho u'' = div sigma + F (Section 5) with the
alternating-triangular (AT) decoupling and a direction split per component.

Readings of the paper:

* Operator.  The 2D blocks printed for Upsilon repeat K_x (x) M_y where the
  second term must be M_x (x) K_y, and the constitutive law carries a stray
  sigma_ij where delta_ij is meant.  The blocks are therefore taken from the
  bilinear form a(w, u) = 2 mu (eps(w), eps(u)) + lambda (div w, div u):

    Upsilon_ii = (2mu+lambda) K in direction i, mu K in the other two,
                 M in the remaining directions of each term;
    Upsilon_ik = mu  [G in direction i, G^T in direction k, M in the third]
               + lam [G^T in direction i, G in direction k, M in the third]
  for i != k, with G = (B_a, B_c') (mixed matrix, trial differentiated).
* AT split (eq. decom): Upsilon^(1) is block lower with half diagonal,
  Upsilon^(2) block upper with half diagonal.
* Scheme (eq. pre, eq. corr).  Subtracting the predictor from the corrector
  shows the pair is equivalent to the three-level "Z-form"
      (rho M + tau^2/2 U1) Zt = tau^2 (f^n - Upsilon U^n)
      (rho M + tau^2/2 U2) Z  = rho M Zt
      U^{n+1} = 2 U^n - U^{n-1} + Z,
  i.e. eq. gen with D = (rho M + tau^2/2 U1)(rho M)^{-1}(rho M + tau^2/2 U2).
  Each block-triangular solve runs component by component: x, y, z in the
  predictor, z, y, x in the corrector (the order the paper gives for 2D).
* Split diagonal blocks (eq. spill): rho M + tau^2/4 Upsilon_ii is replaced by
  rho (x)_d (M_d + tau^2 c_{i,d} / (4 rho) K_d), c_{i,i} = 2mu+lambda,
  c_{i,d} = mu otherwise.  The residual keeps the exact Upsilon.
* Start (unstated): Z^0 = D^{-1} tau^2 (f^0 - Upsilon U^0) and
  U^{-1} = U^0 - tau V^0 + Z^0 / 2.
* Zero Dirichlet conditions on every component (traction-free is the
  paper's; Dirichlet is the workload's).
"""
from __future__ import annotations

import numpy as np

from . import matrices as mx
from .banded import band_lu
from .kron import ads_solve, apply_dir


class Elastic:
    def __init__(self, nelem, p: int, q: int | None = None, tau: float = 5e-3,
                 rho: float = 1.0, lam: float = 1.0, mu: float = 1.0,
                 bc: str = "dirichlet"):
        if np.isscalar(nelem):
            nelem = (nelem,) * 3
        self.nelem = tuple(int(e) for e in nelem)
        self.p = p
        self.q = p + 1 if q is None else q
        self.tau = float(tau)
        self.rho, self.lam, self.mu = float(rho), float(lam), float(mu)
        self.bc = bc
        self.b1 = [mx.basis_1d(E, p, self.q) for E in self.nelem]
        self.idx = [mx.free_index(b.n, bc) for b in self.b1]
        self.M = [mx.restrict(mx.mass(b), i) for b, i in zip(self.b1, self.idx)]
        self.K = [mx.restrict(mx.stiffness(b), i) for b, i in zip(self.b1, self.idx)]
        self.G = [mx.restrict(mx.mixed(b), i) for b, i in zip(self.b1, self.idx)]
        # split diagonal-block factors: per direction, one per distinct c
        self._split = {}
        self.fS = {}
        for d in range(3):
            for c in (self.mu, 2 * self.mu + self.lam):
                A = self.M[d] + self.tau ** 2 * c / (4 * self.rho) * self.K[d]
                self._split[(d, c)] = A
                self.fS[(d, c)] = band_lu(A, p)
        self.fM = [band_lu(M, p) for M in self.M]

    # -- layout -------------------------------------------------------------
    @property
    def free_shape(self):
        return tuple(len(self.idx[d]) for d in (2, 1, 0))

    @property
    def full_shape(self):
        return tuple(self.b1[d].n for d in (2, 1, 0))

    def to_full(self, U):
        out = np.zeros(U.shape[:-3] + self.full_shape)
        out[..., self.idx[2][:, None, None], self.idx[1][None, :, None],
            self.idx[0][None, None, :]] = U
        return out

    def to_free(self, Ufull):
        return Ufull[..., self.idx[2][:, None, None], self.idx[1][None, :, None],
                     self.idx[0][None, None, :]]

    def c(self, i: int, d: int) -> float:
        return 2 * self.mu + self.lam if i == d else self.mu

    # -- operator ---------------------------------------------------------
    def _tensor(self, ops, U):
        """Apply ops[d] along direction d, d = z, y, x."""
        for d in (2, 1, 0):
            U = apply_dir(ops[d], U, d)
        return U

    def block(self, i: int, k: int, U: np.ndarray) -> np.ndarray:
        """Upsilon_ik U (test component i, trial component k)."""
        if i == k:
            out = 0.0
            for d in range(3):
                ops = [self.M[e] if e != d else self.K[e] for e in range(3)]
                out = out + self.c(i, d) * self._tensor(ops, U)
            return out
        j = 3 - i - k
        t_mu = [None] * 3
        t_mu[i], t_mu[k], t_mu[j] = self.G[i], self.G[k].T, self.M[j]
        t_la = [None] * 3
        t_la[i], t_la[k], t_la[j] = self.G[i].T, self.G[k], self.M[j]
        return self.mu * self._tensor(t_mu, U) + self.lam * self._tensor(t_la, U)

    def upsilon(self, U: np.ndarray) -> np.ndarray:
        return np.stack([sum(self.block(i, k, U[k]) for k in range(3)) for i in range(3)])

    def mass(self, U: np.ndarray) -> np.ndarray:
        return np.stack([self._tensor(self.M, U[i]) for i in range(3)])

    # -- split solves --------------------------------------------------------
    def split_diag(self, i: int, U: np.ndarray) -> np.ndarray:
        """rho (x)_d (M_d + tau^2 c_{i,d}/(4 rho) K_d) applied to U."""
        ops = [self._split[(d, self.c(i, d))] for d in range(3)]
        return self.rho * self._tensor(ops, U)

    def solve_diag(self, i: int, r: np.ndarray) -> np.ndarray:
        f = [self.fS[(d, self.c(i, d))] for d in range(3)]
        return ads_solve(*f, r) / self.rho

    def at_solve(self, R: np.ndarray) -> np.ndarray:
        """Z = D^{-1} R: predictor sweep over components x, y, z with the
        block-lower operator, then corrector z, y, x with the block-upper one."""
        h = 0.5 * self.tau ** 2
        Y = [None] * 3
        for i in range(3):
            r = R[i].copy()
            for j in range(i):
                r -= h * self.block(i, j, Y[j])
            Y[i] = self.solve_diag(i, r)
        Z = [None] * 3
        for i in (2, 1, 0):
            r = self.rho * self._tensor(self.M, Y[i])
            for j in range(i + 1, 3):
                r -= h * self.block(i, j, Z[j])
            Z[i] = self.solve_diag(i, r)
        return np.stack(Z)

    def step(self, Un, Unm1, f=None):
        R = -self.upsilon(Un)
        if f is not None:
            R = R + f
        Z = self.at_solve(self.tau ** 2 * R)
        return 2 * Un - Unm1 + Z

    def start(self, U0, V0=None, f0=None):
        V0 = np.zeros_like(U0) if V0 is None else V0
        R = -self.upsilon(U0)
        if f0 is not None:
            R = R + f0
        Z0 = self.at_solve(self.tau ** 2 * R)
        return U0 - self.tau * V0 + 0.5 * Z0

    def run(self, U0, V0=None, nsteps: int = 1, b=None, amps=None, history=False):
        """Returns (U^n, U^{n-1}) after ``nsteps`` steps; the load at step k
        is amps[k] * b (time level n, eq. pre)."""
        F = (lambda k: None) if b is None else (lambda k: amps[k] * b)
        Unm1 = self.start(U0, V0, F(0))
        Un = U0
        hist = [(Un, Unm1)] if history else None
        for k in range(nsteps):
            Un, Unm1 = self.step(Un, Unm1, F(k)), Un
            if history:
                hist.append((Un, Unm1))
        return ((Un, Unm1), hist) if history else (Un, Unm1)

    # -- invariants -------------------------------------------------------------
    def LT(self, V: np.ndarray) -> np.ndarray:
        """L^T V with L = rho M + tau^2/2 Upsilon^(1) (split diagonal)."""
        h = 0.5 * self.tau ** 2
        out = []
        for i in range(3):
            r = self.split_diag(i, V[i])
            for j in range(i + 1, 3):
                r = r + h * self.block(i, j, V[j])
            out.append(r)
        return np.stack(out)

    def D_norm2(self, V: np.ndarray) -> float:
        """V^T D V with D = L (rho M)^{-1} L^T."""
        w = self.LT(V)
        s = np.stack([ads_solve(*self.fM, w[i]) for i in range(3)]) / self.rho
        return float(np.sum(w * s))

    def energy(self, Unp1, Un) -> float:
        """1/2 |V|^2_{D - tau^2 Upsilon/4} + 1/2 |W|^2_Upsilon with
        V = (U^{n+1}-U^n)/tau, W = (U^{n+1}+U^n)/2: constant for f = 0 (inner
        product of eq. gen with U^{n+1} - U^{n-1})."""
        V = (Unp1 - Un) / self.tau
        W = 0.5 * (Unp1 + Un)
        kin = self.D_norm2(V) - 0.25 * self.tau ** 2 * float(np.sum(V * self.upsilon(V)))
        pot = float(np.sum(W * self.upsilon(W)))
        return 0.5 * kin + 0.5 * pot

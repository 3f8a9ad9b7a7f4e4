"""Scalar P-wave equation u'' - Laplace(u) = f on the unit cube (Section 2),
implicit Newmark step with the direction-split left-hand side.

Reading of the paper (its printed scheme is not self-consistent):

* The paper cites Newmark with beta = 1/4 and treats u_n, u'_n, u''_n as three
  independent variables, but the displayed predictor and updates (eq. scheme,
  eq. pwave2) drop every u''_n term.  Taken literally they reduce to
  u_{n+1} = u_n + tau u'_n, which per spectral mode propagates waves at speed
  1/sqrt(2) (see ``literal_step``).  The oracle therefore implements standard
  Newmark, beta = 1/4, gamma = 1/2:

      w       = u_n + tau u'_n + eta u''_n,          eta = tau^2 / 4
      G a     = F_{n+1} - K w                        (split LHS, eq. pwave2)
      u'_{n+1} = u'_n + (tau/2)(u''_n + a)
      u_{n+1}  = w + eta a,                          u''_{n+1} = a

  with G = (M_x + eta K_x) (x) (M_y + eta K_y) (x) (M_z + eta K_z), the 3D
  form of eq. pwave2 (the dropped terms are eta^2 (K(x)K(x)M + ...) +
  eta^3 K(x)K(x)K).
* K is the Galerkin stiffness (grad w, grad u); the right-hand side of the
  weak form (w, Laplace u) becomes -K u after integration by parts.
* Initial acceleration (unstated): u''_0 = G^{-1}(F_0 - K u_0).
* Zero Dirichlet conditions (unstated for the P-wave) by eliminating the
  first/last basis function per direction.
* The load is F(t) = r(t) b with a fixed load vector b.
"""
from __future__ import annotations

import numpy as np

from . import matrices as mx
from .banded import band_lu
from .kron import AXIS, ads_solve, apply_dir, kron3


class PWave:
    def __init__(self, nelem, p: int, q: int | None = None, tau: float = 1e-2,
                 bc: str = "dirichlet", coef: np.ndarray | None = None, c2ref: float = 1.0):
        """coef: squared wave speed c^2 at every Gauss point [(Ez q), (Ey q),
        (Ex q)] (None: c^2 = 1).  With it the stiffness is the element-loop
        quadrature of (c^2 grad B_i, grad w) and the direction-split
        left-hand side uses the constant c2ref (the ADS step then solves with
        an approximation of M + eta K, a preconditioned step)."""
        if np.isscalar(nelem):
            nelem = (nelem,) * 3
        self.nelem = tuple(int(e) for e in nelem)
        self.p = p
        self.q = p + 1 if q is None else q
        self.tau = float(tau)
        self.eta = self.tau ** 2 / 4.0
        self.bc = bc
        self.b1 = [mx.basis_1d(E, p, self.q) for E in self.nelem]
        self.idx = [mx.free_index(b.n, bc) for b in self.b1]
        self.M = [mx.restrict(mx.mass(b), i) for b, i in zip(self.b1, self.idx)]
        self.K = [mx.restrict(mx.stiffness(b), i) for b, i in zip(self.b1, self.idx)]
        self.coef = None if coef is None else np.asarray(coef, dtype=np.float64)
        self.c2ref = float(c2ref)
        self.A = [M + self.eta * self.c2ref * K for M, K in zip(self.M, self.K)]
        self.fA = [band_lu(A, p) for A in self.A]
        self.fM = [band_lu(M, p) for M in self.M]

    # -- layout -----------------------------------------------------------
    @property
    def n(self):
        return tuple(b.n for b in self.b1)

    @property
    def free_shape(self):
        """(nz, ny, nx) of the free-coefficient arrays."""
        return tuple(len(self.idx[d]) for d in (2, 1, 0))

    @property
    def full_shape(self):
        return tuple(self.b1[d].n for d in (2, 1, 0))

    def to_full(self, U: np.ndarray) -> np.ndarray:
        out = np.zeros(U.shape[:-3] + self.full_shape)
        out[..., self.idx[2][:, None, None], self.idx[1][None, :, None],
            self.idx[0][None, None, :]] = U
        return out

    def to_free(self, Ufull: np.ndarray) -> np.ndarray:
        return Ufull[..., self.idx[2][:, None, None], self.idx[1][None, :, None],
                     self.idx[0][None, None, :]]

    # -- operators (Section 2, the 1D matrices in Kronecker form) ----------
    def stiffness(self, w: np.ndarray) -> np.ndarray:
        """K w with K = K_x(x)M_y(x)M_z + M_x(x)K_y(x)M_z + M_x(x)M_y(x)K_z
        (constant coefficient), else the element-loop quadrature with c^2."""
        if self.coef is not None:
            from .quadref import stiffness_action
            return self.to_free(stiffness_action(self.b1, self.to_full(w), self.coef))
        Mx, My, Mz = self.M
        Kx, Ky, Kz = self.K
        return kron3(Kx, My, Mz, w) + kron3(Mx, Ky, Mz, w) + kron3(Mx, My, Kz, w)

    def mass(self, w: np.ndarray) -> np.ndarray:
        return kron3(*self.M, w)

    def G(self, w: np.ndarray) -> np.ndarray:
        """The split operator G = (M_x+eta K_x)(x)(M_y+eta K_y)(x)(M_z+eta K_z)."""
        return kron3(*self.A, w)

    def solve_G(self, r: np.ndarray) -> np.ndarray:
        return ads_solve(*self.fA, r)

    def solve_M(self, r: np.ndarray) -> np.ndarray:
        return ads_solve(*self.fM, r)

    # -- data -------------------------------------------------------------
    def quad_points(self, d: int) -> np.ndarray:
        return self.b1[d].x

    def project(self, vals: np.ndarray) -> np.ndarray:
        """Isogeometric L2 projection (Appendix, last paragraph): solve
        M u = b with b_i = int B_i g, g given at the Gauss points as an array
        [(Ez q), (Ey q), (Ex q)]."""
        b = vals
        for d in (0, 1, 2):
            T = (self.b1[d].N * self.b1[d].w[:, None]).T[self.idx[d]]
            b = apply_dir(T, b, d)
        return self.solve_M(b)

    def point_load(self, xs) -> np.ndarray:
        """b_{ijk} = B_i(x_s) B_j(y_s) B_k(z_s): a point source tested against
        the basis."""
        from .bspline import basis
        v = [basis(self.b1[d].knots, self.p, [xs[d]])[0][self.idx[d]] for d in range(3)]
        return v[2][:, None, None] * v[1][None, :, None] * v[0][None, None, :]

    # -- time stepping ------------------------------------------------------
    def initial_accel(self, u0: np.ndarray, F0=None) -> np.ndarray:
        r = -self.stiffness(u0)
        if F0 is not None:
            r = r + F0
        return self.solve_G(r)

    def step(self, u, v, a, F1=None):
        w = u + self.tau * v + self.eta * a
        r = -self.stiffness(w)
        if F1 is not None:
            r = r + F1
        a1 = self.solve_G(r)
        v1 = v + 0.5 * self.tau * (a + a1)
        u1 = w + self.eta * a1
        return u1, v1, a1

    def literal_step(self, u, v, a, F1=None):
        """The coefficient set exactly as printed in eq. pwave2 (diagnostic
        only): G a = F - K(u + tau v), v += tau/2 a, u += tau v_new - tau^2/2 a."""
        r = -self.stiffness(u + self.tau * v)
        if F1 is not None:
            r = r + F1
        a1 = self.solve_G(r)
        v1 = v + 0.5 * self.tau * a1
        u1 = u + self.tau * v1 - 0.5 * self.tau ** 2 * a1
        return u1, v1, a1

    def run(self, u0, v0=None, nsteps: int = 1, b=None, amps=None,
            literal: bool = False, history: bool = False):
        """Start (u''_0 from the equation) and take ``nsteps`` steps; the load
        at step k -> k+1 is amps[k+1] * b.  Returns (u, v, a) and, with
        ``history``, the list of states after every step."""
        v0 = np.zeros_like(u0) if v0 is None else v0
        F = (lambda k: None) if b is None else (lambda k: amps[k] * b)
        u, v = u0, v0
        a = self.initial_accel(u0, F(0))
        hist = [(u, v, a)] if history else None
        stepper = self.literal_step if literal else self.step
        for k in range(nsteps):
            u, v, a = stepper(u, v, a, F(k + 1))
            if history:
                hist.append((u, v, a))
        return ((u, v, a), hist) if history else (u, v, a)

    # -- invariants ---------------------------------------------------------
    def energy(self, u, v) -> float:
        """E = 1/2 v^T (G - eta K) v + 1/2 u^T K u: conserved exactly (F = 0)
        by the scheme from step 1 on, because the split step is Newmark with
        the modified mass G - eta K >= M (with a coefficient field: when
        c2ref >= max c^2)."""
        mt = self.G(v) - self.eta * self.stiffness(v)
        return 0.5 * float(np.sum(v * mt)) + 0.5 * float(np.sum(u * self.stiffness(u)))

    def plain_energy(self, u, v) -> float:
        return 0.5 * float(np.sum(v * self.mass(v))) + 0.5 * float(np.sum(u * self.stiffness(u)))

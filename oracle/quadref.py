"""Element-by-element Gauss quadrature of the weak forms (Section 2, the
tested equation (w, u'') + (grad w, grad u) = (w, f); Section 5, the weak form
rho (w_i, u_i'') + (w_(i,j), sigma_ij) = (F_i, w)).

Used only to pin the Kronecker routes of ``pwave``/``elastic``: every element
is visited, the discrete field and its gradient are evaluated at every Gauss
point from the element's (p+1)^3 coefficients, and the integrand is tested
against every basis function supported on the element.  No sum factorization,
no Kronecker structure.  Arrays are on the FULL index set (no boundary
elimination).  Intended for small meshes only.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import matrices as mx


def _element_tables(b: mx.Basis1D, e: int):
    q, p = b.q, b.p
    rows = slice(e * q, (e + 1) * q)
    cols = slice(e, e + p + 1)         # basis functions active on element e
    return b.N[rows, cols], b.D[rows, cols], b.w[rows]


def stiffness_action(b1, u: np.ndarray, coef: np.ndarray | None = None) -> np.ndarray:
    """out_i = int c(x) grad B_i . grad u_h over the cube, u: full [z, y, x];
    coef: c at every Gauss point, [(Ez q), (Ey q), (Ex q)] (None: c = 1)."""
    bx, by, bz = b1
    p = bx.p
    q = bx.q
    out = np.zeros_like(u)
    for ez, ey, ex in itertools.product(range(bz.E), range(by.E), range(bx.E)):
        Nx, Dx, wx = _element_tables(bx, ex)
        Ny, Dy, wy = _element_tables(by, ey)
        Nz, Dz, wz = _element_tables(bz, ez)
        c = u[ez:ez + p + 1, ey:ey + p + 1, ex:ex + p + 1]          # [a_z, a_y, a_x]
        # fields at Gauss points [gz, gy, gx]
        ux = np.einsum("ka,jb,ic,abc->kji", Nz, Ny, Dx, c)
        uy = np.einsum("ka,jb,ic,abc->kji", Nz, Dy, Nx, c)
        uz = np.einsum("ka,jb,ic,abc->kji", Dz, Ny, Nx, c)
        W = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
        if coef is not None:
            W = W * coef[ez * q:(ez + 1) * q, ey * q:(ey + 1) * q, ex * q:(ex + 1) * q]
        out[ez:ez + p + 1, ey:ey + p + 1, ex:ex + p + 1] += (
            np.einsum("ka,jb,ic,kji->abc", Nz, Ny, Dx, W * ux)
            + np.einsum("ka,jb,ic,kji->abc", Nz, Dy, Nx, W * uy)
            + np.einsum("ka,jb,ic,kji->abc", Dz, Ny, Nx, W * uz))
    return out


def mass_action(b1, u: np.ndarray) -> np.ndarray:
    """out_i = int B_i u_h."""
    bx, by, bz = b1
    p = bx.p
    out = np.zeros_like(u)
    for ez, ey, ex in itertools.product(range(bz.E), range(by.E), range(bx.E)):
        Nx, _, wx = _element_tables(bx, ex)
        Ny, _, wy = _element_tables(by, ey)
        Nz, _, wz = _element_tables(bz, ez)
        c = u[ez:ez + p + 1, ey:ey + p + 1, ex:ex + p + 1]
        v = np.einsum("ka,jb,ic,abc->kji", Nz, Ny, Nx, c)
        W = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
        out[ez:ez + p + 1, ey:ey + p + 1, ex:ex + p + 1] += np.einsum(
            "ka,jb,ic,kji->abc", Nz, Ny, Nx, W * v)
    return out


def elastic_action(b1, U: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """out_{i, node} = int 2 mu eps(B_node e_i) : eps(u_h)
    + lam div(B_node e_i) div(u_h);  U: full [3, z, y, x]."""
    bx, by, bz = b1
    p = bx.p
    out = np.zeros_like(U)
    for ez, ey, ex in itertools.product(range(bz.E), range(by.E), range(bx.E)):
        Nx, Dx, wx = _element_tables(bx, ex)
        Ny, Dy, wy = _element_tables(by, ey)
        Nz, Dz, wz = _element_tables(bz, ez)
        W = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
        # derivative tables per direction j: (z-table, y-table, x-table)
        tabs = [(Nz, Ny, Dx), (Nz, Dy, Nx), (Dz, Ny, Nx)]
        grad = np.zeros((3, 3) + W.shape)     # grad[k, j] = d_j u_k
        for k in range(3):
            c = U[k, ez:ez + p + 1, ey:ey + p + 1, ex:ex + p + 1]
            for j in range(3):
                tz, ty, tx = tabs[j]
                grad[k, j] = np.einsum("ka,jb,ic,abc->kji", tz, ty, tx, c)
        eps = 0.5 * (grad + grad.transpose(1, 0, 2, 3, 4))
        div = grad[0, 0] + grad[1, 1] + grad[2, 2]
        sig = 2 * mu * eps
        for i in range(3):
            sig[i, i] += lam * div
        # test function B e_i: d_j (B e_i) has only row i -> integrand sig[i, j] d_j B
        for i in range(3):
            acc = 0.0
            for j in range(3):
                tz, ty, tx = tabs[j]
                acc = acc + np.einsum("ka,jb,ic,kji->abc", tz, ty, tx, W * sig[i, j])
            out[i, ez:ez + p + 1, ey:ey + p + 1, ex:ex + p + 1] += acc
    return out

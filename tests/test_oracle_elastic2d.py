"""Pins of the two-dimensional (plane strain) elasticity oracle: strain
energies of linear displacement fields on the unit square in closed form
(each block and each of mu, lambda separately), the rigid-body null space,
agreement with the 3D oracle on fields constant in z, the alternating-
triangular solve against a dense D, the literal predictor/corrector against
the Z-form, the energy identity, and a rigid motion kept at rest."""
import numpy as np
import pytest

from oracle import bspline, elastic, elastic2d

PARS = dict(rho=1.3, lam=0.8, mu=0.6)


def _linear_fields(el):
    """Spline coefficients of x and y (Greville abscissae) on the free
    index set, broadcast to [y, x]."""
    ny, nx = el.free_shape
    gx = bspline.greville(el.b1[0].knots, el.p)[el.idx[0]]
    gy = bspline.greville(el.b1[1].knots, el.p)[el.idx[1]]
    X = np.broadcast_to(gx[None, :], (ny, nx)).copy()
    Y = np.broadcast_to(gy[:, None], (ny, nx)).copy()
    return X, Y, np.zeros((ny, nx)), np.ones((ny, nx))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_strain_energies_of_linear_fields(p):
    """Natural conditions, unit square: w^T Upsilon u equals the integral of
    2 mu eps(w):eps(u) + lam div w div u, in closed form for linear fields."""
    el = elastic2d.Elastic2D((3, 4), p, tau=0.1, bc="neumann", **PARS)
    X, Y, O, _ = _linear_fields(el)
    mu, lam = PARS["mu"], PARS["lam"]
    F = {"x0": np.stack([X, O]), "y0": np.stack([Y, O]), "0x": np.stack([O, X]), "0y": np.stack([O, Y]),
         "yx": np.stack([Y, X]), "xy": np.stack([X, Y]), "rot": np.stack([-Y, X])}

    def a(w, u):
        return float(np.sum(F[w] * el.upsilon(F[u])))

    cases = [("x0", "x0", 2 * mu + lam), ("0y", "0y", 2 * mu + lam), ("y0", "y0", mu), ("0x", "0x", mu),
             ("yx", "yx", 4 * mu), ("xy", "xy", 4 * mu + 4 * lam), ("rot", "rot", 0.0),
             ("x0", "0y", lam),     # lambda part of the off-diagonal block alone
             ("y0", "0x", mu),      # mu part of the off-diagonal block alone
             ("0y", "x0", lam), ("0x", "y0", mu)]
    for w, u, ref in cases:
        assert abs(a(w, u) - ref) < 1e-12 * (1 + abs(ref)), (w, u, a(w, u), ref)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rigid_modes_natural(p):
    """Two translations and the rotation are in the null space with natural
    (traction-free) conditions."""
    el = elastic2d.Elastic2D((4, 3), p, tau=0.1, bc="neumann", **PARS)
    X, Y, O, I = _linear_fields(el)
    for U in (np.stack([I, O]), np.stack([O, I]), np.stack([-Y, X])):
        r = el.upsilon(U)
        assert np.abs(r).max() < 1e-12 * (1 + np.abs(U).max()), np.abs(r).max()


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("p", [2, 3])
def test_matches_3d_oracle_on_z_constant_fields(bc, p):
    """On a 3D field constant in z with no z-displacement, the 3D operator's x-
    and y-rows are the 2D operator times the z mass row sums (K_z and G_z
    annihilate constants).  The 3D oracle, pinned against element-loop
    quadrature of the bilinear form, takes natural conditions (so that the
    constant in z is in its space); with zero Dirichlet in x and y the 2D
    field sits on the interior x, y indices and the rows are compared there."""
    el2 = elastic2d.Elastic2D((3, 4), p, tau=0.1, bc=bc, **PARS)
    el3 = elastic.Elastic((3, 4, 2), p, tau=0.1, bc="neumann", **PARS)
    U2 = np.random.default_rng(p).normal(size=(2,) + el2.free_shape)
    ix, iy = el2.idx[0], el2.idx[1]
    U3 = np.zeros((3,) + el3.free_shape)
    for c in range(2):
        U3[c][:, iy[:, None], ix[None, :]] = U2[c][None]
    r3 = el3.upsilon(U3)
    r2 = el2.upsilon(U2)
    mz = el3.M[2].sum(axis=1)
    for c in range(2):
        np.testing.assert_allclose(r3[c][:, iy[:, None], ix[None, :]], mz[:, None, None] * r2[c][None],
                                   atol=1e-12 * np.abs(r2).max())


def _dense(el):
    nf = int(np.prod(el.free_shape))
    Ups = np.zeros((2 * nf, 2 * nf))
    e = np.zeros((2,) + el.free_shape)
    for c in range(2 * nf):
        e.flat[c] = 1.0
        Ups[:, c] = el.upsilon(e).ravel()
        e.flat[c] = 0.0
    Mf = np.kron(el.M[1], el.M[0])
    M2 = np.block([[Mf, np.zeros_like(Mf)], [np.zeros_like(Mf), Mf]])
    return Ups, M2, nf


@pytest.mark.parametrize("tau", [0.05, 2.0])
def test_at_solve_against_dense(tau):
    """The component-wise solve (x then y, y then x) equals a dense solve with
    D = L (rho M)^{-1} L^T, L block lower with the split diagonal blocks."""
    el = elastic2d.Elastic2D((3, 4), 2, tau=tau, **PARS)
    Ups, M2, nf = _dense(el)
    np.testing.assert_allclose(Ups, Ups.T, atol=1e-13 * np.abs(Ups).max())
    L = np.zeros_like(Ups)
    for i in range(2):
        c = [2 * el.mu + el.lam if d == i else el.mu for d in range(2)]
        A = [el.M[d] + tau ** 2 * c[d] / (4 * el.rho) * el.K[d] for d in range(2)]
        L[i * nf:(i + 1) * nf, i * nf:(i + 1) * nf] = el.rho * np.kron(A[1], A[0])
    L[nf:, :nf] = 0.5 * tau ** 2 * Ups[nf:, :nf]
    D = L @ np.linalg.solve(el.rho * M2, L.T)
    R = np.random.default_rng(4).normal(size=(2,) + el.free_shape)
    ref = np.linalg.solve(D, R.ravel()).reshape(R.shape)
    np.testing.assert_allclose(el.at_solve(R), ref, atol=1e-11 * np.abs(ref).max())
    V = np.random.default_rng(5).normal(size=(2,) + el.free_shape)
    np.testing.assert_allclose(el.D_apply(V).ravel(), D @ V.ravel(), atol=1e-11 * np.abs(D @ V.ravel()).max())


def test_predictor_corrector_equals_zform():
    """The predictor and corrector (eq. pre, eq. corr) solved literally with
    unsplit blocks give the Z-form's U^{n+1}."""
    el = elastic2d.Elastic2D((3, 3), 2, tau=0.07, **PARS)
    Ups, M2, nf = _dense(el)
    U1 = np.zeros_like(Ups)
    U2 = np.zeros_like(Ups)
    U1[nf:, :nf] = Ups[nf:, :nf]
    U2[:nf, nf:] = Ups[:nf, nf:]
    for i in range(2):
        s = slice(i * nf, (i + 1) * nf)
        U1[s, s] = 0.5 * Ups[s, s]
        U2[s, s] = 0.5 * Ups[s, s]
    rho, tau = el.rho, el.tau
    Un, Unm1, f = np.random.default_rng(9).normal(size=(3, 2 * nf))
    A = rho * M2 / tau ** 2
    Ut = np.linalg.solve(A + 0.5 * U1, f + A @ (2 * Un - Unm1) - 0.5 * U1 @ Unm1 - U2 @ Un)
    Unp1 = np.linalg.solve(A + 0.5 * U2, f + A @ (2 * Un - Unm1) - 0.5 * U1 @ (Ut + Unm1) - 0.5 * U2 @ Unm1)
    Zt = np.linalg.solve(rho * M2 + 0.5 * tau ** 2 * U1, tau ** 2 * (f - Ups @ Un))
    Z = np.linalg.solve(rho * M2 + 0.5 * tau ** 2 * U2, rho * M2 @ Zt)
    np.testing.assert_allclose(2 * Un - Unm1 + Z, Unp1, atol=1e-12 * np.abs(Unp1).max())


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("tau", [5e-3, 0.5])
def test_energy_conserved(tau, bc):
    el = elastic2d.Elastic2D((5, 4), 2, tau=tau, bc=bc, **PARS)
    U0 = np.random.default_rng(2).normal(size=(2,) + el.free_shape)
    (_, hist) = el.run(U0, nsteps=30, history=True)
    E = np.array([el.energy(hist[k + 1][0], hist[k][0]) for k in range(len(hist) - 1)])
    assert E[0] > 0
    np.testing.assert_allclose(E / E[0], 1.0, atol=1e-11)


def test_rigid_motion_at_rest():
    el = elastic2d.Elastic2D((4, 3), 3, tau=0.05, bc="neumann", **PARS)
    X, Y, O, I = _linear_fields(el)
    U0 = np.stack([0.3 * I - 0.7 * Y, -0.1 * I + 0.7 * X])
    (_, hist) = el.run(U0, nsteps=6, history=True)
    for Un, Unm1 in hist:
        np.testing.assert_allclose(Un, U0, atol=1e-12)
        np.testing.assert_allclose(Unm1, U0, atol=1e-12)


def test_temporal_order_semidiscrete_exact():
    """Against rho M U'' + Upsilon U = 0 solved exactly by a dense generalized
    eigendecomposition, the error ratio on halving tau tends to 4 (second
    order, which needs the start's + Z^0 / 2 term)."""
    import scipy.linalg
    T = 0.6
    el0 = elastic2d.Elastic2D((4, 3), 2, tau=0.1, **PARS)
    Ups, M2, nf = _dense(el0)
    w2, Phi = scipy.linalg.eigh(Ups, el0.rho * M2)
    coef = np.zeros(w2.size)
    coef[:6] = np.random.default_rng(3).normal(size=6)
    U0 = (Phi @ coef).reshape((2,) + el0.free_shape)
    exact = (Phi @ (coef * np.cos(np.sqrt(w2) * T))).reshape(U0.shape)
    errs = []
    for N in (30, 60, 120, 240):
        el = elastic2d.Elastic2D((4, 3), 2, tau=T / N, **PARS)
        Un, _ = el.run(U0, nsteps=N)
        errs.append(np.linalg.norm(Un - exact) / np.linalg.norm(exact))
    r = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(r - 4.0) < 0.35), (errs, r)

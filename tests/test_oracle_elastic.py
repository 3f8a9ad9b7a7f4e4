"""Pins of the oracle's elasticity operator and alternating-triangular step
(P12-P14) against element-by-element quadrature of the bilinear form, the
rigid-body null space, the literal predictor/corrector equations, an
independently assembled dense operator, the energy identity of eq. gen and the
exact semi-discrete solution."""
import numpy as np
import pytest
import scipy.linalg

from oracle import bspline, elastic, kron, quadref

PARS = dict(rho=1.3, lam=0.8, mu=0.6)


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_operator_matches_bilinear_form(bc, p):
    """P12: Upsilon from the (corrected) Kronecker blocks equals quadrature of
    2 mu eps(w):eps(u) + lam div w div u."""
    el = elastic.Elastic((2, 3, 2), p, tau=0.1, bc=bc, **PARS)
    U = np.random.default_rng(p).normal(size=(3,) + el.free_shape)
    ref = el.to_free(quadref.elastic_action(el.b1, el.to_full(U), PARS["lam"], PARS["mu"]))
    np.testing.assert_allclose(el.upsilon(U), ref, atol=1e-13 * np.abs(ref).max())


def _dense_ops(el):
    """Dense Upsilon (from quadrature on unit vectors, independent of the
    oracle's block formula) and dense block-diagonal M."""
    nf = int(np.prod(el.free_shape))
    Ups = np.zeros((3 * nf, 3 * nf))
    e = np.zeros((3,) + el.free_shape)
    for c in range(3 * nf):
        e.flat[c] = 1.0
        Ups[:, c] = el.to_free(quadref.elastic_action(el.b1, el.to_full(e), el.lam, el.mu)).ravel()
        e.flat[c] = 0.0
    Mf = kron.dense_kron(*el.M)
    M3 = scipy.linalg.block_diag(Mf, Mf, Mf)
    return Ups, M3, nf


def test_operator_spd_dirichlet():
    el = elastic.Elastic((2, 3, 3), 2, tau=0.1, **PARS)
    Ups, _, _ = _dense_ops(el)
    np.testing.assert_allclose(Ups, Ups.T, atol=1e-14)
    assert np.linalg.eigvalsh(Ups).min() > 1e-6


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_rigid_modes_neumann(p):
    """P12: with traction-free (Neumann) assembly the 3 translations and 3
    rotations (linear fields via Greville coefficients) are in the null space."""
    el = elastic.Elastic((3, 2, 4), p, tau=0.1, bc="neumann", **PARS)
    nz, ny, nx = el.free_shape
    xi = [bspline.greville(el.b1[d].knots, p) for d in range(3)]
    X = np.broadcast_to(xi[0][None, None, :], (nz, ny, nx))
    Y = np.broadcast_to(xi[1][None, :, None], (nz, ny, nx))
    Z = np.broadcast_to(xi[2][:, None, None], (nz, ny, nx))
    zero, one = np.zeros((nz, ny, nx)), np.ones((nz, ny, nx))
    modes = [np.stack([one, zero, zero]), np.stack([zero, one, zero]), np.stack([zero, zero, one]),
             np.stack([-Y, X, zero]), np.stack([zero, -Z, Y]), np.stack([Z, zero, -X])]
    rnd = np.random.default_rng(0).normal(size=(3, nz, ny, nx))
    scale = np.linalg.norm(el.upsilon(rnd)) / np.linalg.norm(rnd)
    for r in modes:
        assert np.linalg.norm(el.upsilon(r)) < 1e-12 * scale * np.linalg.norm(r)


def _lower_upper(el, Ups, nf):
    U1 = np.zeros_like(Ups)
    U2 = np.zeros_like(Ups)
    for i in range(3):
        for j in range(3):
            blk = Ups[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf]
            if i == j:
                U1[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = 0.5 * blk
                U2[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = 0.5 * blk
            elif j < i:
                U1[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = blk
            else:
                U2[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = blk
    return U1, U2


def test_predictor_corrector_equals_zform():
    """P13 (i): the predictor (eq. pre) and corrector (eq. corr), solved
    literally for U~ and U^{n+1} with unsplit operators, give the same U^{n+1}
    as the Z-form (rho M + tau^2/2 U1)(rho M)^{-1}(rho M + tau^2/2 U2) Z =
    tau^2 (f - Upsilon U^n)."""
    el = elastic.Elastic((2, 3, 2), 2, tau=0.07, **PARS)
    Ups, M3, nf = _dense_ops(el)
    U1, U2 = _lower_upper(el, Ups, nf)
    rho, tau = el.rho, el.tau
    rng = np.random.default_rng(9)
    Un, Unm1, f = rng.normal(size=(3, 3 * nf))
    A = rho * M3 / tau ** 2
    rhs_pre = f + A @ (2 * Un - Unm1) - 0.5 * U1 @ Unm1 - U2 @ Un
    Ut = np.linalg.solve(A + 0.5 * U1, rhs_pre)
    rhs_cor = f + A @ (2 * Un - Unm1) - 0.5 * U1 @ (Ut + Unm1) - 0.5 * U2 @ Unm1
    Unp1 = np.linalg.solve(A + 0.5 * U2, rhs_cor)
    Zt = np.linalg.solve(rho * M3 + 0.5 * tau ** 2 * U1, tau ** 2 * (f - Ups @ Un))
    Z = np.linalg.solve(rho * M3 + 0.5 * tau ** 2 * U2, rho * M3 @ Zt)
    np.testing.assert_allclose(2 * Un - Unm1 + Z, Unp1, atol=1e-12 * np.abs(Unp1).max())


@pytest.mark.parametrize("tau", [0.05, 2.0])
def test_split_at_solve_against_dense(tau):
    """P13 (ii): the oracle's component-wise AT solve equals a dense solve with
    D = L (rho M)^{-1} L^T, L = block lower with split diagonal blocks
    rho (x)(M_d + tau^2 c_{i,d}/(4 rho) K_d); D is symmetric positive definite."""
    el = elastic.Elastic((2, 3, 2), 2, tau=tau, **PARS)
    Ups, M3, nf = _dense_ops(el)
    L = np.zeros_like(Ups)
    for i in range(3):
        c = [2 * el.mu + el.lam if d == i else el.mu for d in range(3)]
        A = [el.M[d] + tau ** 2 * c[d] / (4 * el.rho) * el.K[d] for d in range(3)]
        L[i * nf:(i + 1) * nf, i * nf:(i + 1) * nf] = el.rho * kron.dense_kron(*A)
        for j in range(i):
            L[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = 0.5 * tau ** 2 * Ups[i * nf:(i + 1) * nf,
                                                                            j * nf:(j + 1) * nf]
    D = L @ np.linalg.solve(el.rho * M3, L.T)
    np.testing.assert_allclose(D, D.T, atol=1e-12 * np.abs(D).max())
    assert np.linalg.eigvalsh(0.5 * (D + D.T)).min() > 0
    R = np.random.default_rng(4).normal(size=(3,) + el.free_shape)
    Z = el.at_solve(R)
    ref = np.linalg.solve(D, R.ravel()).reshape(R.shape)
    np.testing.assert_allclose(Z, ref, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("tau", [5e-3, 5e-2, 0.5])
def test_energy_conserved(tau, bc):
    """P13 (iii): with f = 0 the three-level energy is constant."""
    el = elastic.Elastic((4, 3, 3), 2, tau=tau, bc=bc, **PARS)
    U0 = np.random.default_rng(2).normal(size=(3,) + el.free_shape)
    (_, hist) = el.run(U0, nsteps=30, history=True)
    E = np.array([el.energy(hist[k + 1][0], hist[k][0]) for k in range(len(hist) - 1)])
    np.testing.assert_allclose(E / E[0], 1.0, atol=1e-11)
    assert E[0] > 0


def test_temporal_order_semidiscrete_exact():
    """P14: against rho M U'' + Upsilon U = 0 solved exactly by a dense
    generalized eigendecomposition, the error ratio tends to 4."""
    T = 0.6
    el0 = elastic.Elastic(3, 2, tau=0.1, **PARS)
    Ups, M3, nf = _dense_ops(el0)
    w2, Phi = scipy.linalg.eigh(Ups, el0.rho * M3)
    coef = np.zeros(w2.size)
    coef[:8] = np.random.default_rng(3).normal(size=8)
    U0 = (Phi @ coef).reshape((3,) + el0.free_shape)
    exact = (Phi @ (coef * np.cos(np.sqrt(w2) * T))).reshape(U0.shape)
    errs = []
    for N in (30, 60, 120, 240):
        el = elastic.Elastic(3, 2, tau=T / N, **PARS)
        Un, _ = el.run(U0, nsteps=N)
        errs.append(np.linalg.norm(Un - exact) / np.linalg.norm(exact))
    r = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(r - 4.0) < 0.35), (errs, r)


@pytest.mark.parametrize("p", [2, 3])
def test_traction_free_rigid_motion_at_rest(p):
    """Traction-free conditions (Section 5): a rigid displacement (translation
    plus rotation, linear fields through Greville coefficients) has zero
    strain, so the three-level scheme keeps it exactly at rest."""
    el = elastic.Elastic((3, 4, 2), p, tau=0.05, bc="neumann", **PARS)
    nz, ny, nx = el.free_shape
    xi = [bspline.greville(el.b1[d].knots, p) for d in range(3)]
    X = np.broadcast_to(xi[0][None, None, :], (nz, ny, nx))
    Y = np.broadcast_to(xi[1][None, :, None], (nz, ny, nx))
    Z = np.broadcast_to(xi[2][:, None, None], (nz, ny, nx))
    U0 = np.stack([0.3 - 0.7 * Y + 0.2 * Z, -0.1 + 0.7 * X - 0.4 * Z, 0.5 - 0.2 * X + 0.4 * Y])
    (_, hist) = el.run(U0, nsteps=6, history=True)
    for Un, Unm1 in hist:
        np.testing.assert_allclose(Un, U0, atol=1e-12)
        np.testing.assert_allclose(Unm1, U0, atol=1e-12)

"""Pins of the 2D P-wave oracle (Section 2's exposition dimension) against
the scalar recursion of a separable eigenmode, energy conservation, and a
dense brute-force run of the assembled 2D matrices."""
import numpy as np
import pytest
import scipy.linalg

from oracle import pwave2d


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("tau", [1e-2, 0.5])
@pytest.mark.parametrize("p", [2, 3])
def test_eigenmode_recursion_2d(p, tau, bc):
    """On phi_y (x) phi_x (generalized eigenvectors of K_d, M_d) the 2D scheme
    reduces to the scalar Newmark recursion with s = lam_x + lam_y and
    g = (1 + eta lam_x)(1 + eta lam_y)."""
    pw = pwave2d.PWave2D((6, 5), p, tau=tau, bc=bc)
    lam, vec = [], []
    for d, k in enumerate((2, 1)):
        w, V = scipy.linalg.eigh(pw.K[d], pw.M[d])
        lam.append(w[k])
        vec.append(V[:, k])
    phi = vec[1][:, None] * vec[0][None, :]
    s, eta = lam[0] + lam[1], pw.eta
    g = (1 + eta * lam[0]) * (1 + eta * lam[1])
    _, hist = pw.run(0.6 * phi, nsteps=10, history=True)
    c, v = 0.6, 0.0
    a = -(s / g) * c
    for k, (uu, vv, aa) in enumerate(hist):
        if k > 0:
            w = c + tau * v + eta * a
            a1 = -(s / g) * w
            v = v + 0.5 * tau * (a + a1)
            c = w + eta * a1
            a = a1
        np.testing.assert_allclose(uu, c * phi, atol=1e-12)
        np.testing.assert_allclose(vv, v * phi, atol=1e-11 * max(1, abs(v)))
        np.testing.assert_allclose(aa, a * phi, atol=1e-10 * max(1, abs(a)))


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_energy_conserved_2d(bc):
    pw = pwave2d.PWave2D((7, 6), 2, tau=0.3, bc=bc)
    u0 = np.random.default_rng(9).normal(size=pw.free_shape)
    _, hist = pw.run(u0, nsteps=30, history=True)
    E = np.array([pw.energy(u, v) for (u, v, a) in hist[1:]])
    np.testing.assert_allclose(E / E[0], 1.0, atol=1e-12)


@pytest.mark.parametrize("p", [2, 3])
def test_brute_force_dense_2d(p):
    """The same Newmark step with the assembled 2D matrices and dense solves
    (x fastest in the flattened index, so T_x (x) T_y = kron(T_y, T_x))."""
    pw = pwave2d.PWave2D((4, 5), p, tau=0.05)
    Md = np.kron(pw.M[1], pw.M[0])
    Kd = np.kron(pw.M[1], pw.K[0]) + np.kron(pw.K[1], pw.M[0])
    Gd = np.kron(pw.A[1], pw.A[0])
    u0 = np.random.default_rng(2).normal(size=pw.free_shape)
    (u, v, a) = pw.run(u0, nsteps=6)
    uf = u0.ravel()
    vf = np.zeros_like(uf)
    af = np.linalg.solve(Gd, -Kd @ uf)
    eta, tau = pw.eta, pw.tau
    for _ in range(6):
        w = uf + tau * vf + eta * af
        a1 = np.linalg.solve(Gd, -Kd @ w)
        vf = vf + 0.5 * tau * (af + a1)
        uf = w + eta * a1
        af = a1
    np.testing.assert_allclose(u.ravel(), uf, atol=1e-12 * np.abs(uf).max())
    np.testing.assert_allclose(a.ravel(), af, atol=1e-11 * np.abs(af).max())
    # in 2D the split operator is M + eta K + eta^2 K_x (x) K_y exactly
    np.testing.assert_allclose(Gd - (Md + eta * Kd), eta ** 2 * np.kron(pw.K[1], pw.K[0]),
                               atol=1e-14 * np.abs(Gd).max())

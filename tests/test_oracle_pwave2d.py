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


def _scipy_design(knots, p, x):
    """Values of all degree-p B-splines at x from scipy's own B-spline
    evaluator (independent of the oracle's Cox-de Boor recursion)."""
    from scipy.interpolate import BSpline
    return BSpline.design_matrix(np.asarray(x, dtype=np.float64), knots, p).toarray()


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("p", [2, 3])
def test_projection_2d_reproduces_spline(p, bc):
    """The 2D L2 projection (Appendix, last paragraph, in the dimension of
    Section 2) returns a function of the spline space exactly, on a
    non-square grid: random coefficients c are evaluated at the Gauss points
    with scipy's B-spline evaluator, projected, and the projection must give
    c back.  A transposed operand, a swapped weight or a wrong basis fails."""
    pw = pwave2d.PWave2D((5, 3), p, bc=bc)
    c = np.random.default_rng(17).normal(size=pw.free_shape)
    By = _scipy_design(pw.b1[1].knots, p, pw.quad_points(1))[:, pw.idx[1]]
    Bx = _scipy_design(pw.b1[0].knots, p, pw.quad_points(0))[:, pw.idx[0]]
    vals = By @ c @ Bx.T
    np.testing.assert_allclose(pw.project(vals), c, atol=1e-12 * np.abs(c).max())


def test_projection_2d_convergence():
    """The 2D projection of a smooth function converges at h^{p+1} in L2
    (errors measured at 5 Gauss points per element with scipy's evaluator
    and numpy's Gauss rule)."""
    from numpy.polynomial.legendre import leggauss
    errs = []
    for E in (4, 8, 16):
        pw = pwave2d.PWave2D((E, E + 2), 2, bc="dirichlet")
        gy, gx = pw.quad_points(1), pw.quad_points(0)
        u = pw.project(np.sin(np.pi * gy)[:, None] * (gx * np.exp(gx) * (1 - gx))[None, :])
        xi, om = leggauss(5)
        pts, wts = [], []
        for n in (pw.nelem[1], pw.nelem[0]):
            e = np.arange(n)[:, None]
            pts.append(((e + 0.5 + 0.5 * xi[None, :]) / n).ravel())
            wts.append(np.broadcast_to(0.5 * om[None, :] / n, (n, 5)).ravel())
        By = _scipy_design(pw.b1[1].knots, 2, pts[0])[:, pw.idx[1]]
        Bx = _scipy_design(pw.b1[0].knots, 2, pts[1])[:, pw.idx[0]]
        uh = By @ u @ Bx.T
        g = np.sin(np.pi * pts[0])[:, None] * (pts[1] * np.exp(pts[1]) * (1 - pts[1]))[None, :]
        errs.append(np.sqrt(np.sum(wts[0][:, None] * wts[1][None, :] * (uh - g) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.8), (errs, rates)

"""Pins of the oracle's P-wave step (P7-P11, P15, P16 and the literal-scheme
diagnostic) against element-by-element quadrature, the paper's own spectral
decomposition, exact semi-discrete solutions, invariants and brute force."""
import numpy as np
import pytest
import scipy.linalg

from oracle import kron, matrices as mx, pwave, quadref


@pytest.mark.parametrize("E,p", [((3, 4, 2), 2), ((3, 2, 3), 3), ((4, 3, 2), 1), ((2, 3, 2), 4), ((2, 2, 3), 5)])
def test_stiffness_quadrature_route(E, p):
    """P7: element-loop quadrature of (grad B_i, grad u_h) equals the
    Kronecker route sum_d K_d (x) M (x) M, also on the full index set."""
    pw = pwave.PWave(E, p, tau=0.1)
    u = np.random.default_rng(5).normal(size=pw.free_shape)
    ref = pw.to_free(quadref.stiffness_action(pw.b1, pw.to_full(u)))
    np.testing.assert_allclose(pw.stiffness(u), ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
    refm = pw.to_free(quadref.mass_action(pw.b1, pw.to_full(u)))
    np.testing.assert_allclose(pw.mass(u), refm, atol=1e-15 * 1e3 * np.abs(refm).max())


def _mode(pw, k):
    """Separable generalized eigenmode phi_x (x) phi_y (x) phi_z (eq. sd0/eigKM0)."""
    lam, vec = [], []
    for d in range(3):
        w, V = scipy.linalg.eigh(pw.K[d], pw.M[d])
        lam.append(w[k[d]])
        vec.append(V[:, k[d]])
    phi = vec[2][:, None, None] * vec[1][None, :, None] * vec[0][None, None, :]
    return np.array(lam), phi


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("tau", [1e-2, 0.3, 10.0])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_eigenmode_recursion(tau, p, bc):
    """P8: on a separable eigenmode the 3D scheme reduces to the scalar
    recursion with s = sum lam_d and g = prod(1 + eta lam_d) (with natural
    conditions the z-factor of mode (1, 2, 0) is the constant, lam_z = 0)."""
    pw = pwave.PWave((5, 4, 6), p, tau=tau, bc=bc)
    lam, phi = _mode(pw, (1, 2, 0))
    s, eta = lam.sum(), pw.eta
    g = np.prod(1 + eta * lam)
    (_, hist) = pw.run(0.7 * phi, nsteps=12, history=True)
    c = 0.7
    a = -(s / g) * c
    v = 0.0
    for k, (u, vv, aa) in enumerate(hist):
        if k > 0:
            w = c + tau * v + eta * a
            a1 = -(s / g) * w
            v = v + 0.5 * tau * (a + a1)
            c = w + eta * a1
            a = a1
        np.testing.assert_allclose(u, c * phi, atol=1e-12 * max(1, abs(c)))
        np.testing.assert_allclose(vv, v * phi, atol=1e-11 * max(1, abs(v)))
        np.testing.assert_allclose(aa, a * phi, atol=1e-11 * max(1, abs(a)))


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("tau", [1e-2, 1.0, 100.0])
def test_energy_conserved(tau, bc):
    """P9: with F = 0 the energy 1/2 v^T (G - eta K) v + 1/2 u^T K u is constant
    for n >= 1 (unconditional stability), and the plain energy stays below it."""
    pw = pwave.PWave((6, 5, 4), 2, tau=tau, bc=bc)
    u0 = np.random.default_rng(11).normal(size=pw.free_shape)
    (_, hist) = pw.run(u0, nsteps=40, history=True)
    E = np.array([pw.energy(u, v) for (u, v, a) in hist[1:]])
    np.testing.assert_allclose(E / E[0], 1.0, atol=1e-12)
    Ep = np.array([pw.plain_energy(u, v) for (u, v, a) in hist[1:]])
    assert np.all(Ep <= E * (1 + 1e-12))


def _dense(pw):
    Mf = kron.dense_kron(*pw.M)
    Kf = (kron.dense_kron(pw.K[0], pw.M[1], pw.M[2]) + kron.dense_kron(pw.M[0], pw.K[1], pw.M[2])
          + kron.dense_kron(pw.M[0], pw.M[1], pw.K[2]))
    return Mf, Kf


def test_temporal_order_semidiscrete_exact():
    """P10: against the exact semi-discrete solution of M u'' + K u = 0
    (dense generalized eigendecomposition), the error ratio tends to 4."""
    T = 1.0
    pw0 = pwave.PWave(4, 2, tau=0.1)
    Mf, Kf = _dense(pw0)
    w2, Phi = scipy.linalg.eigh(Kf, Mf)
    coef = np.zeros(w2.size)
    coef[:6] = np.random.default_rng(7).normal(size=6)
    u0 = (Phi @ coef).reshape(pw0.free_shape)
    exact = (Phi @ (coef * np.cos(np.sqrt(w2) * T))).reshape(pw0.free_shape)
    errs = []
    for N in (20, 40, 80, 160):
        pw = pwave.PWave(4, 2, tau=T / N)
        u, _, _ = pw.run(u0, nsteps=N)
        errs.append(np.linalg.norm(u - exact) / np.linalg.norm(exact))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.25), (errs, ratios)


def test_temporal_order_forced_selfconvergence():
    """P10 (forced): load b = (B_i, sin pi x sin pi y sin pi z) cos t, the
    manufactured problem of u = sin sin sin cos t; self-convergence ratio 4."""
    T = 0.5
    res = []
    for N in (40, 80, 160, 320):
        pw = pwave.PWave(4, 2, tau=T / N)
        g = [np.sin(np.pi * pw.quad_points(d)) for d in range(3)]
        vals = g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
        u0 = pw.project(vals)
        b = pw.mass(pw.project((3 * np.pi ** 2 - 1) * vals))   # b_i = int B_i f
        amps = np.cos(pw.tau * np.arange(N + 1))
        u, _, _ = pw.run(u0, nsteps=N, b=b, amps=amps)
        res.append(u)
    d = [np.linalg.norm(res[i] - res[i + 1]) for i in range(3)]
    r = np.array(d[:-1]) / np.array(d[1:])
    # e(tau) = C2 tau^2 + C4 tau^4: the ratio decreases monotonically to 4
    assert r[0] > r[1] > 4.0 and r[1] < 4.5, (d, r)


def test_spatial_order_projection():
    """P11: the L2 projection of a smooth function converges at h^{p+1}."""
    errs = []
    for E in (4, 8):
        pw = pwave.PWave(E, 2, tau=0.1)
        g = [np.sin(np.pi * pw.quad_points(d)) for d in range(3)]
        vals = g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
        u = pw.project(vals)
        # evaluate the projection at the Gauss points and compare
        uh = pw.to_full(u)
        for d in (0, 1, 2):
            uh = kron.apply_dir(pw.b1[d].N, uh, d)
        W = [pw.b1[d].w for d in range(3)]
        Wt = W[2][:, None, None] * W[1][None, :, None] * W[0][None, None, :]
        errs.append(np.sqrt(np.sum(Wt * (uh - vals) ** 2)))
    assert np.log2(errs[0] / errs[1]) > 2.7


def test_projection_reproduces_spline():
    """The projection of a function inside the Dirichlet spline space returns
    it exactly: x(1-x) y(1-y) z(1-z) is a p=2 spline vanishing on the
    boundary, so its projection evaluates back to the same values."""
    pw = pwave.PWave((3, 4, 5), 2, tau=0.1)
    g = [pw.quad_points(d) * (1 - pw.quad_points(d)) for d in range(3)]
    vals = g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
    uh = pw.to_full(pw.project(vals))
    for d in (0, 1, 2):
        uh = kron.apply_dir(pw.b1[d].N, uh, d)
    np.testing.assert_allclose(uh, vals, atol=1e-14)


def test_point_load_partition_of_unity():
    pw = pwave.PWave(5, 3, tau=0.1, bc="neumann")
    b = pw.point_load([0.31, 0.52, 0.77])
    assert abs(b.sum() - 1.0) < 1e-14 and b.min() >= 0


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_brute_force_dense_run(p):
    """P16: everything assembled densely (np.kron) and solved with dense
    solves matches the oracle's line-solve path."""
    tau = 0.05
    pw = pwave.PWave((3, 4, 3), p, tau=tau)
    Mf, Kf = _dense(pw)
    Gf = kron.dense_kron(*[pw.M[d] + pw.eta * pw.K[d] for d in range(3)])
    rng = np.random.default_rng(p)
    u0 = rng.normal(size=pw.free_shape)
    b = rng.normal(size=pw.free_shape)
    amps = np.sin(np.arange(9))
    u, v, a = pw.run(u0, nsteps=8, b=b, amps=amps)
    U = u0.ravel()
    V = np.zeros_like(U)
    A = np.linalg.solve(Gf, amps[0] * b.ravel() - Kf @ U)
    for k in range(8):
        W = U + tau * V + pw.eta * A
        A1 = np.linalg.solve(Gf, amps[k + 1] * b.ravel() - Kf @ W)
        V = V + 0.5 * tau * (A + A1)
        U = W + pw.eta * A1
        A = A1
    # two FP64 routes differ by rounding amplified by the condition number of
    # G (7e6 for p = 5 on this mesh: boundary splines of high degree)
    tol = max(1e-12, 1e-15 * np.linalg.cond(Gf))
    np.testing.assert_allclose(u.ravel(), U, rtol=tol, atol=tol * np.abs(U).max())
    np.testing.assert_allclose(a.ravel(), A, rtol=tol, atol=tol * np.abs(A).max())


def test_splitting_error_order():
    """P15: one split step differs from one unsplit step (M + eta K) by
    O(tau^4) in the acceleration on a smooth field."""
    diffs = []
    for tau in (0.04, 0.02, 0.01):
        pw = pwave.PWave(4, 2, tau=tau)
        Mf, Kf = _dense(pw)
        g = [np.sin(np.pi * pw.quad_points(d)) for d in range(3)]
        u0 = pw.project(g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :])
        r = -pw.stiffness(u0)
        a_split = pw.solve_G(r)
        a_full = np.linalg.solve(Mf + pw.eta * Kf, r.ravel()).reshape(r.shape)
        diffs.append(np.linalg.norm(a_split - a_full))
    r = np.array(diffs[:-1]) / np.array(diffs[1:])
    assert np.all(r > 14.0), (diffs, r)


def test_literal_scheme_wave_speed():
    """The coefficient set exactly as printed (u''_n terms dropped) propagates
    a mode at omega/sqrt(2); the standard-Newmark reading at omega."""
    tau = 1e-3
    pw = pwave.PWave(4, 2, tau=tau)
    lam, phi = _mode(pw, (0, 0, 0))
    s, g = lam.sum(), np.prod(1 + pw.eta * lam)
    nrm = np.sum(phi * phi)
    # literal scheme: (u, v) -> (u, v) is linear and does not use u''_n
    cols = []
    for (cu, cv) in ((1.0, 0.0), (0.0, 1.0)):
        u1, v1, _ = pw.literal_step(cu * phi, cv * phi, 0 * phi)
        cols.append([np.sum(u1 * phi) / nrm, np.sum(v1 * phi) / nrm])
    th_lit = np.arccos(0.5 * np.trace(np.array(cols).T))
    assert abs(th_lit / (tau * np.sqrt(s)) - 1 / np.sqrt(2)) < 1e-3
    # standard reading: for n >= 1 the amplitude obeys the three-level
    # recursion with cos(theta) = 1 - tau^2 s / (2 g), theta / tau -> sqrt(s)
    (_, hist) = pw.run(phi, nsteps=400, history=True)
    c = np.array([np.sum(h[0] * phi) / nrm for h in hist])[1:]
    th = np.arccos(1 - tau ** 2 * s / (2 * g))
    assert abs(th / (tau * np.sqrt(s)) - 1) < 1e-3
    n = np.arange(1, 401)
    X = np.stack([np.cos(th * n), np.sin(th * n)], 1)
    coef = np.linalg.lstsq(X, c, rcond=None)[0]
    np.testing.assert_allclose(X @ coef, c, atol=1e-10)


@pytest.mark.parametrize("p", [2, 3])
def test_natural_bc_constant_field_at_rest(p):
    """With natural (zero normal derivative) conditions the constant function
    (all coefficients 1, partition of unity) is in the null space of K: the
    scheme keeps it at rest exactly, u = 1, u' = u'' = 0 for every step."""
    pw = pwave.PWave((4, 3, 5), p, tau=0.05, bc="neumann")
    assert pw.free_shape == tuple(n + p for n in (5, 3, 4))
    (_, hist) = pw.run(np.ones(pw.free_shape), nsteps=8, history=True)
    # rounding of K 1 = 0 is amplified by |M^-1 K| ~ 1/h^2 in u''; a wrong row
    # sum would give O(1) values
    for u, v, a in hist:
        np.testing.assert_allclose(u, 1.0, atol=1e-12)
        assert np.abs(v).max() < 1e-11 and np.abs(a).max() < 1e-10


def _coef_grid(pw, fx, fy, fz):
    """c^2 at every Gauss point [(Ez q), (Ey q), (Ex q)] of a separable field."""
    x, y, z = (pw.quad_points(d) for d in range(3))
    return fz(z)[:, None, None] * fy(y)[None, :, None] * fx(x)[None, None, :]


@pytest.mark.parametrize("p", [2, 3])
def test_unit_coefficient_is_the_kronecker_route(p):
    """A coefficient field equal to 1 reproduces K = sum_d K_d (x) M (x) M."""
    E = (3, 4, 2)
    ref = pwave.PWave(E, p, tau=0.1)
    pw = pwave.PWave(E, p, tau=0.1, coef=np.ones([e * (p + 1) for e in E[::-1]]))
    u = np.random.default_rng(3).normal(size=pw.free_shape)
    a, b = pw.stiffness(u), ref.stiffness(u)
    np.testing.assert_allclose(a, b, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("p", [2, 3])
def test_separable_coefficient_kronecker(p):
    """c^2 = f(x) g(y) h(z): the element-loop quadrature equals the Kronecker
    sum of 1D mass and stiffness matrices weighted by f, g, h, each built
    here from the Gauss tables (N^T diag(w f) N, D^T diag(w f) D)."""
    E = (4, 3, 5)
    fx, fy, fz = (lambda x: 1.0 + 0.5 * np.sin(3 * x), lambda y: 2.0 - y, lambda z: 0.5 + z * z)
    pw = pwave.PWave(E, p, tau=0.1)
    pw = pwave.PWave(E, p, tau=0.1, coef=_coef_grid(pw, fx, fy, fz))
    Mw, Kw = [], []
    for d, f in enumerate((fx, fy, fz)):
        b = pw.b1[d]
        wf = b.w * f(b.x)
        i = pw.idx[d]
        Mw.append(((b.N * wf[:, None]).T @ b.N)[np.ix_(i, i)])
        Kw.append(((b.D * wf[:, None]).T @ b.D)[np.ix_(i, i)])
    u = np.random.default_rng(4).normal(size=pw.free_shape)
    ref = (kron.kron3(Kw[0], Mw[1], Mw[2], u) + kron.kron3(Mw[0], Kw[1], Mw[2], u)
           + kron.kron3(Mw[0], Mw[1], Kw[2], u))
    np.testing.assert_allclose(pw.stiffness(u), ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_variable_coefficient_energy_conserved(bc):
    """With c^2 in [0.5, 1.5] and the split left-hand side at c2ref = 1.5 >= max
    c^2, the preconditioned ADS step still conserves E = 1/2 v(G - eta K)v +
    1/2 uKu exactly (G - eta K stays SPD)."""
    E = (5, 4, 6)
    base = pwave.PWave(E, 2, tau=0.2, bc=bc)
    x, y, z = (base.quad_points(d) for d in range(3))
    c2 = 1.0 + 0.5 * np.sin(5 * z)[:, None, None] * np.cos(4 * y)[None, :, None] * np.sin(7 * x + 1)[None, None, :]
    pw = pwave.PWave(E, 2, tau=0.2, bc=bc, coef=c2, c2ref=1.5)
    u0 = np.random.default_rng(6).normal(size=pw.free_shape)
    (_, hist) = pw.run(u0, nsteps=15, history=True)
    En = np.array([pw.energy(u, v) for (u, v, a) in hist[1:]])
    np.testing.assert_allclose(En / En[0], 1.0, atol=1e-12)


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
@pytest.mark.parametrize("p", [2, 3])
def test_point_load_evaluates_the_spline(p, bc):
    """The point load b_ijk = B_i(x_s) B_j(y_s) B_k(z_s) is the functional
    c -> u_h(x_s): for random coefficients c, b . c equals the spline
    u_h = sum c_ijk B_i(x) B_j(y) B_k(z) evaluated at x_s by scipy's B-spline
    evaluator.  Three different element counts and three distinct
    coordinates, so an exchange of axes or a wrong basis fails."""
    from scipy.interpolate import BSpline
    pw = pwave.PWave((3, 4, 5), p, tau=0.1, bc=bc)
    xs = [0.31, 0.52, 0.77]
    c = np.random.default_rng(23).normal(size=pw.free_shape)
    ref = c
    for d in (2, 1, 0):          # contract z, then y, then x
        B = BSpline.design_matrix(np.array([xs[d]]), pw.b1[d].knots, p).toarray()[0, pw.idx[d]]
        ref = np.tensordot(B, ref, axes=([0], [0]))
    b = pw.point_load(xs)
    assert b.shape == pw.free_shape
    np.testing.assert_allclose(np.sum(b * c), float(ref), rtol=1e-13, atol=1e-14)

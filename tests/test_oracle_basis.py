"""Pins of the oracle's basis, quadrature and 1D matrices (P1-P5) against
closed forms and properties fixed by the mathematics, not by the oracle."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import bspline, matrices as mx

GOLD = os.path.join(os.path.dirname(__file__), "golden", "stencils.json")


@pytest.mark.parametrize("E,p", [(1, 1), (3, 2), (7, 2), (5, 3), (9, 3), (6, 4), (7, 5)])
def test_partition_of_unity_and_support(E, p):
    """P1: sum_i B_i = 1, sum_i B_i' = 0, B_i >= 0, supp B_i = [t_i, t_{i+p+1}]."""
    t = bspline.open_uniform_knots(E, p)
    x = np.concatenate([np.random.default_rng(1).uniform(0, 1, 200), [0.0, 1.0], t])
    B = bspline.basis(t, p, x)
    D = bspline.basis_deriv(t, p, x)
    assert B.shape[1] == E + p
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-11)
    assert B.min() >= -1e-15
    for i in range(E + p):
        outside = (x < t[i]) | (x > t[i + p + 1])
        assert np.all(B[outside, i] == 0.0)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_derivative_matches_finite_difference(p):
    t = bspline.open_uniform_knots(6, p)
    x = np.random.default_rng(2).uniform(0.01, 0.99, 50)
    x = x[np.abs(np.subtract.outer(x, t)).min(axis=1) > 1e-4]   # avoid knots
    h = 1e-6
    fd = (bspline.basis(t, p, x + h) - bspline.basis(t, p, x - h)) / (2 * h)
    np.testing.assert_allclose(bspline.basis_deriv(t, p, x), fd, atol=1e-7)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_greville_reproduces_linear(p):
    t = bspline.open_uniform_knots(5, p)
    x = np.linspace(0, 1, 37)
    np.testing.assert_allclose(bspline.basis(t, p, x) @ bspline.greville(t, p), x, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_interior_stencils_closed_form(p):
    """P2: interior rows equal the cardinal-spline autocorrelation values
    (tests/golden/stencils.json, exact rationals)."""
    gold = json.load(open(GOLD))[f"p{p}"]
    m_ref = np.array([float(Fraction(a, b)) for a, b in gold["mass_over_h"]])
    k_ref = np.array([float(Fraction(a, b)) for a, b in gold["stiffness_times_h"]])
    E = 4 * p + 6
    h = 1.0 / E
    b = mx.basis_1d(E, p)
    M, K = mx.mass(b), mx.stiffness(b)
    i = (E + p) // 2
    np.testing.assert_allclose(M[i, i - p:i + p + 1] / h, m_ref, rtol=1e-13)
    np.testing.assert_allclose(K[i, i - p:i + p + 1] * h, k_ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("E,p", [(4, 2), (7, 2), (5, 3), (8, 3)])
def test_matrix_properties(E, p):
    """P3: sum M = |domain| = 1, K 1 = 0 (before BC), row sums of M equal
    int B_i = (t_{i+p+1} - t_i)/(p+1), symmetry, bandwidth |i-j| <= p."""
    b = mx.basis_1d(E, p)
    M, K, G = mx.mass(b), mx.stiffness(b), mx.mixed(b)
    t = b.knots
    assert abs(M.sum() - 1.0) < 1e-14
    np.testing.assert_allclose(K @ np.ones(b.n), 0.0, atol=1e-12)
    np.testing.assert_allclose(M.sum(axis=1), [(t[i + p + 1] - t[i]) / (p + 1) for i in range(b.n)],
                               rtol=1e-13)
    np.testing.assert_allclose(M, M.T, atol=1e-16)
    np.testing.assert_allclose(K, K.T, atol=1e-13)
    # G + G^T = boundary term: int (B_i B_j)' = B_i B_j |_0^1
    bd = np.zeros((b.n, b.n))
    bd[0, 0] = -1.0
    bd[-1, -1] = 1.0
    np.testing.assert_allclose(G + G.T, bd, atol=1e-12)
    ii, jj = np.indices(M.shape)
    far = np.abs(ii - jj) > p
    assert np.all(M[far] == 0) and np.all(K[far] == 0) and np.all(G[far] == 0)


@pytest.mark.parametrize("p", [2, 3])
def test_quadrature_exactness(p):
    """P4: q = p+1 and q = p+3 Gauss points give the same matrices."""
    b1 = mx.basis_1d(5, p, p + 1)
    b2 = mx.basis_1d(5, p, p + 3)
    for f in (mx.mass, mx.stiffness, mx.mixed):
        np.testing.assert_allclose(f(b1), f(b2), atol=2e-15)


@pytest.mark.parametrize("p", [2, 3])
def test_dirichlet_eigenvalues_converge(p):
    """P5: lowest Dirichlet generalized eigenvalues of (K, M) approach
    (k pi)^2 at rate h^{2p}."""
    errs = []
    for E in (8, 16):
        b = mx.basis_1d(E, p)
        idx = mx.free_index(b.n)
        lam = scipy.linalg.eigh(mx.restrict(mx.stiffness(b), idx),
                                mx.restrict(mx.mass(b), idx), eigvals_only=True)
        errs.append(abs(lam[1] - (2 * np.pi) ** 2) / (2 * np.pi) ** 2)
    rate = np.log2(errs[0] / errs[1])
    assert rate > 2 * p - 0.3, (errs, rate)

"""Pins of the oracle's banded LU, line solves and direction-split solve (P6)
against LAPACK's pivoting banded solver and against dense Kronecker solves."""
import numpy as np
import pytest
import scipy.linalg

from oracle import banded, kron, matrices as mx


def _spd_band(m, p, seed):
    b = mx.basis_1d(m + 2 - p, p)  # n = m + 2 basis functions, m free ones
    idx = mx.free_index(b.n)
    A = mx.restrict(mx.mass(b) + 0.37 * mx.stiffness(b), idx)
    return A


@pytest.mark.parametrize("m,p", [(1, 2), (2, 2), (5, 2), (16, 2), (4, 3), (13, 3), (40, 3), (9, 1), (30, 4), (25, 5)])
def test_band_lu_against_lapack(m, p):
    A = _spd_band(m, p, 0)
    assert A.shape == (m, m)
    f = banded.band_lu(A, p)
    rhs = np.random.default_rng(m).normal(size=(m, 7))
    x = banded.solve_lines(f, rhs, 0)
    ab = np.zeros((2 * p + 1, m))
    for i in range(m):
        for j in range(max(0, i - p), min(m, i + p + 1)):
            ab[p + i - j, j] = A[i, j]
    ref = scipy.linalg.solve_banded((p, p), ab, rhs)
    np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-13)


def test_band_lu_reconstructs_matrix():
    A = _spd_band(11, 3, 1)
    f = banded.band_lu(A, 3)
    m = 11
    L = np.eye(m)
    U = np.zeros((m, m))
    for i in range(m):
        for k in range(1, 4):
            if i - k >= 0:
                L[i, i - k] = f.L[i, k]
        for k in range(4):
            if i + k < m:
                U[i, i + k] = f.U[i, k]
    np.testing.assert_allclose(L @ U, A, atol=1e-15)


@pytest.mark.parametrize("shape,p", [((3, 4, 5), 2), ((4, 4, 4), 3), ((2, 6, 3), 3), ((5, 3, 4), 2), ((4, 3, 5), 1), ((2, 3, 2), 4), ((2, 2, 3), 5)])
def test_kronecker_identity_dense(shape, p):
    """P6: three line-solve passes equal a dense solve of the assembled
    Kronecker product, (A_x(x)A_y(x)A_z)^{-1} = A_x^{-1}(x)A_y^{-1}(x)A_z^{-1}."""
    Ex, Ey, Ez = shape
    A = []
    for d, E in enumerate((Ex, Ey, Ez)):
        b = mx.basis_1d(E, p)
        idx = mx.free_index(b.n)
        A.append(mx.restrict(mx.mass(b) + (0.1 + d) * mx.stiffness(b), idx))
    f = [banded.band_lu(a, p) for a in A]
    nz, ny, nx = A[2].shape[0], A[1].shape[0], A[0].shape[0]
    b = np.random.default_rng(3).normal(size=(nz, ny, nx))
    x = kron.ads_solve(*f, b)
    ref = np.linalg.solve(kron.dense_kron(*A), b.ravel()).reshape(b.shape)
    np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
    # and the forward operator round-trips
    np.testing.assert_allclose(kron.kron3(*A, x), b, atol=1e-12)

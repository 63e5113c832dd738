"""Pins of the oracle's reference-element operators (closed forms, SBP)."""
import math

import numpy as np
import pytest

from oracle.basis import lgl, derivative_matrix, legendre_vandermonde, Basis, gauss_legendre, interpolation_matrix


def test_lgl_closed_forms():
    x, w = lgl(3)
    s = 1.0 / math.sqrt(5.0)
    assert np.allclose(x, [-1, -s, s, 1], atol=1e-15, rtol=0)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15, rtol=0)
    x, w = lgl(4)
    s = math.sqrt(3.0 / 7.0)
    assert np.allclose(x, [-1, -s, 0, s, 1], atol=1e-15, rtol=0)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15, rtol=0)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 7])
def test_sbp_and_exactness(N):
    x, w = lgl(N)
    D = derivative_matrix(x)
    M = np.diag(w)
    B = np.zeros((N + 1, N + 1))
    B[0, 0] = -1.0
    B[N, N] = 1.0
    assert np.abs(M @ D + (M @ D).T - B).max() < 1e-14
    assert abs(D[0, 0] + N * (N + 1) / 4.0) < 1e-13
    assert np.abs(np.diag(D)[1:-1]).max() < 1e-13
    for k in range(N + 1):
        assert np.abs(D @ x ** k - (k * x ** (k - 1) if k else 0 * x)).max() < 1e-12
    # quadrature exact to degree 2N-1
    for k in range(2 * N):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14


def test_legendre_modes_orthonormal():
    xg, wg = gauss_legendre(8)
    V = legendre_vandermonde(xg)[:, :6]
    assert np.abs(V.T @ np.diag(wg) @ V - np.eye(6)).max() < 1e-13


def test_interpolation_matrix_reproduces_polynomials():
    x, _ = lgl(4)
    y = np.linspace(-1, 1, 7)
    I = interpolation_matrix(x, y)
    for k in range(5):
        assert np.abs(I @ x ** k - y ** k).max() < 1e-13

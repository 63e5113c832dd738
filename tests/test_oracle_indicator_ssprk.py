"""Pins of the oracle's shock indicator and SSPRK3 integrator.

Indicator: an indicator field made of exactly two orthonormal Legendre
modes, built with NumPy's Legendre routines on LGL nodes from NumPy's root
finder (not the oracle's basis), has the energy ratio the definition gives in
closed form: a constant plus the top mode P_N gives c_N^2 / (c_0^2 + c_N^2),
a constant plus P_{N-1} gives c_{N-1}^2 / (c_0^2 + c_{N-1}^2), and a
constant plus modes of degree <= N-2 gives 0.  The logistic map gives
a = 1e-4 at E = 0 (so alpha = 0 below the alpha_min cut), 1/2 at the
threshold, and alpha_max far above it.

SSPRK3: one step of u' = lambda u multiplies u by the stability polynomial
1 + z + z^2/2 + z^3/6 (z = lambda dt); third-order convergence on the
nonlinear u' = -u^2 (exact 1/(1 + t)); and on u' = cos t (exact sin t) the
step is a quadrature whose weights 1/6, 1/6, 2/3 at the stage times t,
t + dt, t + dt/2 form Simpson's rule, fourth order: a wrong stage time
drops it.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import ssprk
from oracle.basis import Basis
from oracle.indicator import blending_factor, modal_energy_ratio


def lgl_numpy(N):
    inner = npleg.Legendre.basis(N).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def onp(k, x):
    """Orthonormal Legendre polynomial of degree k on [-1, 1]."""
    c = np.zeros(k + 1)
    c[k] = 1.0
    return math.sqrt((2 * k + 1) / 2.0) * npleg.legval(x, c)


def two_mode_field(N, dim, k, a, b):
    """a P0(xi)P0(eta).. + b Pk(xi)P0(eta).. at the LGL nodes, node order
    i + (N+1)(j + (N+1) k) with i along the first direction."""
    x = lgl_numpy(N)
    p0, pk = onp(0, x), onp(k, x)
    f = a * p0 + b * pk                 # along direction 0
    for _ in range(dim - 1):
        f = np.multiply.outer(p0, f)    # other directions: P0 (constant)
    return f.reshape(1, -1)


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("dim", [2, 3])
def test_energy_ratio_of_two_modes(N, dim):
    basis = Basis(N)
    assert np.allclose(basis.xi, lgl_numpy(N), atol=1e-14)
    a, b = 1.3, 0.4
    E = modal_energy_ratio(two_mode_field(N, dim, N, a, b), basis, dim)[0]
    assert abs(E - b * b / (a * a + b * b)) < 1e-13
    E = modal_energy_ratio(two_mode_field(N, dim, N - 1, a, b), basis, dim)[0]
    assert abs(E - b * b / (a * a + b * b)) < 1e-13
    for k in range(N - 1):
        E = modal_energy_ratio(two_mode_field(N, dim, k, a, b), basis, dim)[0]
        assert abs(E) < 1e-13


@pytest.mark.parametrize("N", [3, 4])
def test_blending_map(N):
    thr = 0.5 * 10.0 ** (-1.8 * (N + 1) ** 0.25)
    alpha, raw = blending_factor(np.array([0.0, thr, 50 * thr]), N, alpha_max=0.5, alpha_min=1e-3)
    assert abs(raw[0] - 1e-4) < 1e-15 and alpha[0] == 0.0
    assert abs(raw[1] - 0.5) < 1e-15 and alpha[1] == 0.5
    assert alpha[2] == 0.5 and raw[2] > 1 - 1e-12


def test_stability_polynomial():
    for z in (-2.5, -1.0, -0.1, 0.3, 1.0):
        dt, lam = 0.1, z / 0.1
        u1 = ssprk.step(lambda v, t: lam * v, np.array([1.0]), 0.0, dt)[0]
        assert abs(u1 - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-14


def order(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_third_order_nonlinear_and_time_dependent():
    errs_nl, errs_t = [], []
    for m in (10, 20, 40, 80):
        dt = 1.0 / m
        u, _ = ssprk.run(lambda v, t: -v * v, np.array([1.0]), 0.0, dt, m)
        errs_nl.append(abs(u[0] - 0.5))
        u, _ = ssprk.run(lambda v, t: np.cos(t) + 0 * v, np.array([0.0]), 0.0, dt, m)
        errs_t.append(abs(u[0] - math.sin(1.0)))
    for p in order(errs_nl):
        assert 2.9 < p < 3.2
    for p in order(errs_t):
        assert 3.9 < p < 4.1


def test_smoothing_on_a_ring():
    """Four elements in a periodic ring, alpha = (0, 0.8, 0, 0.1): by hand,
    each element takes the larger of its own alpha and half its neighbours'."""
    from oracle.indicator import smooth
    faces = np.array([[0, 1, 1, 0], [1, 1, 2, 0], [2, 1, 3, 0], [3, 1, 0, 0]])
    out = smooth(np.array([0.0, 0.8, 0.0, 0.1]), faces)
    assert np.allclose(out, [0.4, 0.8, 0.4, 0.1], rtol=0, atol=1e-15)

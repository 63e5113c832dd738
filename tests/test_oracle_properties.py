"""Property tests of the oracle over generated inputs (hypothesis, derandomized
so that every run draws the same examples).

* The Ranocha two-point flux satisfies Tadmor's condition
  (w_R - w_L) . f = psi_R - psi_L for any pair of admissible states, from
  nearly equal ones (the logarithmic mean's series branch) to ratios of
  1e6 in density and pressure, and is symmetric in its arguments.
* The logarithmic mean lies between the geometric and the arithmetic mean.
* The mixture temperature solve inverts rho e(T) for any composition and
  any T from 50 to 30000 K.
* The species sources conserve mass and N and O atoms for any composition
  and temperature.
"""
import math

import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import gas
from oracle.kinetics import Kinetics
from oracle.thermo import Mixture
from paper_2511_17551_amd import workloads as W

SET = settings(max_examples=150, deadline=None, derandomize=True)
pos = st.floats(min_value=1e-3, max_value=1e3, allow_nan=False, allow_infinity=False)
vel = st.floats(min_value=-50.0, max_value=50.0, allow_nan=False, allow_infinity=False)
unit = st.floats(min_value=-1.0, max_value=1.0, allow_nan=False, allow_infinity=False)


def pg(rho, v, p, gamma=1.4):
    v = np.asarray(v, float)
    u = np.concatenate([[rho], rho * v, [p / (gamma - 1.0) + 0.5 * rho * (v * v).sum()]])[:, None]
    return gas.pg_state(u, 3, gamma)


@SET
@given(pos, st.tuples(vel, vel, vel), pos, pos, st.tuples(vel, vel, vel), pos, st.tuples(unit, unit, unit),
       st.floats(min_value=0.0, max_value=1.0))
def test_tadmor_condition_and_symmetry(rL, vL, pL, rR, vR, pR, n, near):
    # with `near` close to 1 the right state approaches the left one
    rR = near * rL + (1.0 - near) * rR
    pR = near * pL + (1.0 - near) * pR
    vR = tuple(near * a + (1.0 - near) * b for a, b in zip(vL, vR))
    n = np.asarray(n, float)[:, None] + np.array([[1e-3], [0.0], [0.0]])
    sL, sR = pg(rL, vL, pL), pg(rR, vR, pR)
    f = gas.ranocha(sL, sR, n)
    wL, wR = gas.entropy_variables(sL), gas.entropy_variables(sR)
    lhs = ((wR - wL) * f).sum(0)
    rhs = gas.entropy_potential(sR, n) - gas.entropy_potential(sL, n)
    scale = np.abs((wR - wL) * f).sum(0) + np.abs(rhs) + 1e-300
    assert np.all(np.abs(lhs - rhs) <= 1e-10 * scale + 1e-13)
    g = gas.ranocha(sR, sL, n)
    assert np.all(np.abs(f - g) <= 1e-12 * (np.abs(f) + np.abs(g)) + 1e-300)


@SET
@given(st.floats(min_value=1e-6, max_value=1e6), st.floats(min_value=-0.999, max_value=1e3))
def test_ln_mean_between_geometric_and_arithmetic(x, rel):
    y = x * (1.0 + rel)
    L = gas.ln_mean(np.array([x]), np.array([y]))[0]
    geo, ari = np.sqrt(x * y), 0.5 * (x + y)
    assert geo * (1 - 1e-13) <= L <= ari * (1 + 1e-13)
    # symmetric up to rounding: log(y/x) and log(x/y) round differently.  The
    # rounding of the quotient y/x (relative eps) is an absolute error of eps
    # in its logarithm, so the far branch carries a relative error of about
    # eps / |ln(y/x)| (up to ~50 eps where the series takes over, z = 1e-4,
    # |ln(y/x)| ~ 0.02); the series branch is symmetric to a few eps
    bound = (8.0 + 4.0 / max(abs(math.log(y / x)), 1e-300)) * np.finfo(float).eps * L
    assert abs(L - gas.ln_mean(np.array([y]), np.array([x]))[0]) <= bound


mixture = Mixture(W.Species())
kinetics = Kinetics(W.Species(), W.park17_reactions(4))
frac = st.floats(min_value=0.0, max_value=1.0)


@SET
@given(st.tuples(frac, frac, frac, frac, frac), st.floats(min_value=1e-4, max_value=10.0),
       st.floats(min_value=50.0, max_value=30000.0))
def test_temperature_round_trip(y, rho, T):
    Y = np.asarray(y) + np.array([1e-3, 0, 0, 0, 0])
    rs = (Y / Y.sum() * rho)[:, None]
    rhoe = mixture.rho_e(rs, np.array([T]))
    T2, _ = mixture.solve_T(rs, rhoe, np.array([300.0]), tol=1e-14, maxit=100)
    assert abs(T2[0] - T) <= 1e-11 * T


@SET
@given(st.tuples(frac, frac, frac, frac, frac), st.floats(min_value=1e-4, max_value=10.0),
       st.floats(min_value=200.0, max_value=20000.0))
def test_sources_conserve_mass_and_atoms(y, rho, T):
    Y = np.asarray(y) + 1e-3
    rs = (Y / Y.sum() * rho)[:, None]
    w = kinetics.omega_dot(rs, np.array([T]))[:, 0]
    W_ = W.Species().W
    scale = np.abs(w).sum() + 1e-300
    assert abs(w.sum()) <= 1e-12 * scale
    for atoms in (np.array([2, 0, 1, 1, 0]), np.array([0, 2, 1, 0, 1])):
        c = atoms * w / W_
        assert abs(c.sum()) <= 1e-12 * (np.abs(c).sum() + 1e-300)

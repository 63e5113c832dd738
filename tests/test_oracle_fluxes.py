"""Pins of the oracle's two-point and Riemann fluxes (Tadmor, consistency, symmetry)."""
import numpy as np

from oracle import gas


def random_states(rng, n, dim=3):
    rho = rng.uniform(0.2, 3.0, n)
    v = rng.uniform(-2, 2, (dim, n))
    p = rng.uniform(0.2, 5.0, n)
    u = np.concatenate([rho[None], rho * v, (p / 0.4 + 0.5 * rho * (v * v).sum(0))[None]])
    return u


def test_ranocha_tadmor_condition():
    rng = np.random.default_rng(0)
    uL = random_states(rng, 2000)
    uR = random_states(rng, 2000)
    n = rng.normal(size=(3, 2000))
    sL, sR = gas.pg_state(uL, 3, 1.4), gas.pg_state(uR, 3, 1.4)
    f = gas.ranocha(sL, sR, n)
    wL, wR = gas.entropy_variables(sL), gas.entropy_variables(sR)
    lhs = ((wR - wL) * f).sum(0)
    rhs = gas.entropy_potential(sR, n) - gas.entropy_potential(sL, n)
    scale = np.abs((wR - wL) * f).sum(0) + 1.0
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-12


def test_two_point_consistency_and_symmetry():
    rng = np.random.default_rng(1)
    u = random_states(rng, 500)
    u2 = random_states(rng, 500)
    n = rng.normal(size=(3, 500))
    s, s2 = gas.pg_state(u, 3, 1.4), gas.pg_state(u2, 3, 1.4)
    fphys = gas.physical_flux(s, n)
    for flux in (gas.ranocha, gas.ducros):
        assert np.abs(flux(s, s, n) - fphys).max() < 1e-12 * np.abs(fphys).max()
        assert np.abs(flux(s, s2, n) - flux(s2, s, n)).max() < 1e-13 * np.abs(fphys).max()


def test_rusanov_consistency_and_direction():
    rng = np.random.default_rng(2)
    u = random_states(rng, 300, 2)
    u2 = random_states(rng, 300, 2)
    n = rng.normal(size=(2, 300))
    s, s2 = gas.pg_state(u, 2, 1.4), gas.pg_state(u2, 2, 1.4)
    assert np.abs(gas.rusanov(s, s, n) - gas.physical_flux(s, n)).max() < 1e-12
    assert np.abs(gas.rusanov(s, s2, n) + gas.rusanov(s2, s, -n)).max() < 1e-12


def test_ln_mean_branches_agree():
    x = np.linspace(0.5, 2.0, 1001)
    y = x * (1 + np.linspace(-0.05, 0.05, 1001))
    exact = np.where(np.abs(x - y) > 0, (y - x) / (np.log(y) - np.log(x) + 1e-300), x)
    m = gas.ln_mean(x, y)
    ok = np.abs(x - y) > 1e-3 * x
    assert np.max(np.abs(m[ok] - exact[ok]) / exact[ok]) < 1e-12
    assert np.allclose(gas.ln_mean(x, x), x, rtol=1e-15)

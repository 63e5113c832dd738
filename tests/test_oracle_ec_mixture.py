"""Pins of the oracle's entropy-conservative flux for the RRHO mixture
(oracle/gas.py ec_mixture).

* Tadmor's condition, sum (w_R - w_L) . F = psi_R - psi_L, with the entropy
  variables computed from the species entropies in closed form (an
  independent route to the thermodynamics: the flux uses divided
  differences, log means and sinh(z)/z), over random pairs of mixture states
  (compositions, 300-8000 K, pressures over two decades) to 1e-13 of the
  jump terms, and over nearly equal pairs (relative jumps 1e-3 to 1e-7),
  where the divided differences meet their limits, to 1e-14 of the rounding
  scale sum |w| |F| of the jumps themselves (measured 3e-16).
* Consistency (equal states give f(u).n) and symmetry.
* A planted mistake, the vibrational divided difference replaced by e_v at
  the mean temperature, breaks Tadmor's condition (the check can fail).
* At the operator level, with the flux in the volume and at the faces, the
  semi-discrete entropy rate sum J w . du vanishes to rounding on the
  curved periodic 5-species field with nodal noise (traces jump across
  every face); with Rusanov faces the same state loses entropy.
"""
import numpy as np
import pytest

from oracle import gas
from oracle.dgsem import Operator
from oracle.thermo import Mixture
from paper_2511_17551_amd import workloads as W
from tests.test_oracle_split_forms import mixture_states


@pytest.fixture(scope="module")
def mix():
    return Mixture(W.Species())


def tadmor(a, b, n, mix, flux=gas.ec_mixture):
    F = flux(a, b, n, mix)
    dw = gas.mixture_entropy_variables(b, mix) - gas.mixture_entropy_variables(a, mix)
    lhs = (dw * F).sum(0)
    rhs = gas.mixture_entropy_potential(b, mix, n) - gas.mixture_entropy_potential(a, mix, n)
    scale = np.abs(dw * F).sum(0) + np.abs(rhs)
    return np.abs(lhs - rhs) / scale


def perturbed(s, mix, rng, rel):
    """A state whose species densities, velocity and temperature differ from
    s by relative amounts of order rel."""
    m = s["rho"].shape[0]
    rs = s["rs"] * (1.0 + rel * rng.uniform(-1, 1, s["rs"].shape))
    T = s["T"] * (1.0 + rel * rng.uniform(-1, 1, m))
    v = s["v"] * (1.0 + rel * rng.uniform(-1, 1, s["v"].shape))
    rho = rs.sum(0)
    u = np.concatenate([rs, rho * v, (mix.rho_e(rs, T) + 0.5 * rho * (v * v).sum(0))[None]])
    return mix.state(u, 3, T)


def test_tadmor_condition(mix):
    rng = np.random.default_rng(21)
    a, b = mixture_states(rng, 3000, mix), mixture_states(rng, 3000, mix)
    n = rng.normal(size=(3, 3000))
    assert tadmor(a, b, n, mix).max() < 1e-13
    # nearly equal states: the jumps of w are differences of nearly equal
    # numbers, so the residual is measured against the rounding scale of
    # those differences, sum |w| |F| (relative to the jump terms themselves
    # it grows like eps / rel)
    for rel in (1e-3, 1e-5, 1e-7):
        c = perturbed(a, mix, rng, rel)
        F = gas.ec_mixture(a, c, n, mix)
        wa = gas.mixture_entropy_variables(a, mix)
        dw = gas.mixture_entropy_variables(c, mix) - wa
        res = (dw * F).sum(0) - (gas.mixture_entropy_potential(c, mix, n) - gas.mixture_entropy_potential(a, mix, n))
        r = np.abs(res) / np.abs(wa * F).sum(0)
        assert r.max() < 1e-14, (rel, r.max())


def test_consistency_and_symmetry(mix):
    rng = np.random.default_rng(22)
    a, b = mixture_states(rng, 500, mix), mixture_states(rng, 500, mix)
    n = rng.normal(size=(3, 500))
    f = gas.physical_flux(a, n)
    sc = np.abs(f).max(1, keepdims=True)
    assert np.all(np.abs(gas.ec_mixture(a, a, n, mix) - f) <= 1e-13 * sc)
    F = gas.ec_mixture(a, b, n, mix)
    assert np.all(np.abs(F - gas.ec_mixture(b, a, n, mix)) <= 1e-13 * np.abs(F).max(1, keepdims=True))


def test_tadmor_check_catches_a_wrong_energy_mean(mix):
    def wrong(sL, sR, n, mix_):
        F = gas.ec_mixture(sL, sR, n, mix_)
        # the vibrational divided difference replaced by e_v at the mean T
        Tm = 2.0 / (1.0 / sL["T"] + 1.0 / sR["T"])
        vn = gas.dot(0.5 * (sL["v"] + sR["v"]), n)
        for k in range(mix_.ns):
            if mix_.mol[k]:
                th, bL, bR = mix_.th[k], 1.0 / sL["T"], 1.0 / sR["T"]
                exact = mix_.Rs[k] * th * np.exp(-th * 0.5 * (bL + bR)) * gas.sinhc(0.5 * th * (bR - bL)) \
                    / gas.ln_mean(-np.expm1(-th * bL), -np.expm1(-th * bR))
                ev = mix_.Rs[k] * th / np.expm1(th / Tm)
                F[-1] += (ev - exact) * gas.ln_mean(sL["rs"][k], sR["rs"][k]) * vn
        return F
    rng = np.random.default_rng(23)
    a, b = mixture_states(rng, 500, mix), mixture_states(rng, 500, mix)
    n = rng.normal(size=(3, 500))
    assert tadmor(a, b, n, mix, wrong).max() > 1e-6


def noisy(c, mix, seed=24):
    """The case's state with independent nodal noise of 1% in the species
    densities and 2% in T, so that the traces jump across every face."""
    rng = np.random.default_rng(seed)
    u = c.u0.copy()
    rs = u[:5] * (1.0 + 0.01 * rng.uniform(-1, 1, u[:5].shape))
    rho = rs.sum(0)
    v = u[5:8] / u[:5].sum(0)
    T = c.extra["T"] * (1.0 + 0.02 * rng.uniform(-1, 1, rho.shape))
    return np.concatenate([rs, rho * v, (mix.rho_e(rs, T) + 0.5 * rho * (v * v).sum(0))[None]])


def test_operator_conserves_entropy(mix):
    c = W.curved_periodic_mixture_case(lambda rs, T: mix.rho_e(rs, T), n=2, N=3,
                                       volume_flux=W.VF_RANOCHA, surface_flux=W.SF_RANOCHA)
    c.u0 = noisy(c, mix)
    op = Operator(c.cfg, c.mesh, species=c.species)
    du = op.rhs(c.u0)
    s = op.states(c.u0)
    w = gas.mixture_entropy_variables(s, mix)
    wq = np.einsum("i,j,k->kji", op.b.w, op.b.w, op.b.w).reshape(-1)
    dens = (w * du).sum(0) * op.J * wq
    assert abs(dens.sum()) < 1e-12 * np.abs(dens).sum(), (dens.sum(), np.abs(dens).sum())
    # with Rusanov faces entropy is dissipated
    c2 = W.curved_periodic_mixture_case(lambda rs, T: mix.rho_e(rs, T), n=2, N=3,
                                        volume_flux=W.VF_RANOCHA, surface_flux=W.SF_RUSANOV)
    op2 = Operator(c2.cfg, c2.mesh, species=c2.species)
    du2 = op2.rhs(c.u0)
    assert ((w * du2).sum(0) * op2.J * wq).sum() < -1e-6 * np.abs(dens).sum()

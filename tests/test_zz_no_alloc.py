"""dgx_thermo_noalloc (the entry point that allocates nothing) against
dgx_thermo: the same temperatures, pressures, statistics and return codes,
bitwise, on two calls in a row, the second with fewer states, and the size
limit rejected before any launch.

Call 1: 200,003 packed 3D mixture states (seeded far-from-equilibrium
compositions, 250-12000 K, random velocities) with the surrogate guess from
a network that predicts 1e20 K, under a 6-iteration Newton budget: about
half of the solves from that guess fail (96,780 in the oracle) and are redone
from the freestream guess, from which every node converges within the
budget.  Call 2: the 27,000 nodes of a curved-shock mesh from the
freestream guess.  T is also checked against the oracle on the nodes that
converge."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle.thermo import Mixture
from tests.helpers import to_dev, to_host

pytestmark = pytest.mark.gpu

KEYS = ("nodes", "iters_total", "iters_max", "iters_wave_max_mean", "nonconverged", "first_bad", "fallbacks", "rc")


@pytest.fixture(scope="module")
def dgx():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_17551_amd import dgx as mod
    return mod


def packed_states(mix, n, seed):
    rs, T = W.far_chem_states(n, seed=seed)
    rng = np.random.default_rng(seed + 1)
    rho = rs.sum(0)
    v = rng.uniform(-2000.0, 2000.0, (3, n))
    E = mix.rho_e(rs, T) + 0.5 * rho * (v * v).sum(0)
    return np.ascontiguousarray(np.concatenate([rs, rho * v, E[None]], 0)), T


def both(dgx, ctx, u, n, guess, nstates):
    import torch
    out = []
    for fn in (dgx.dgx_thermo, dgx.dgx_thermo_noalloc):
        T = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        p = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        st = fn(ctx, u, T, p, guess=guess, nstates=nstates, check=False)
        out.append((to_host(T), to_host(p), st))
        dgx.dgx_check_code(ctx)  # clear the sticky flags between the two
    return out


def test_noalloc_matches_dgx_thermo(dgx):
    mix = Mixture(W.Species())
    fns = (lambda rs, T: mix.rho_e(rs, T)), (lambda rs, T: mix.rho_cv(rs, T))
    c = W.case_c3(*fns, n=6)
    c.cfg["newton_maxit"] = 6
    s = dgx.Solver(c)
    prm = np.zeros(dgx.SUR_PARAMS + dgx.SUR_NORM, np.float32)
    prm[dgx.SUR_PARAMS + 6:dgx.SUR_PARAMS + 12] = 1.0
    prm[dgx.SUR_PARAMS + 12] = 1e20
    prm[dgx.SUR_PARAMS + 13] = 1.0
    dgx.dgx_surrogate_set(s.ctx, prm)

    # call 1: many packed states, surrogate guess
    n1 = 200003
    u1, T1 = packed_states(mix, n1, seed=21)
    (Ta, pa, sa), (Tb, pb, sb) = both(dgx, s.ctx, to_dev(u1), n1, dgx.GUESS_SURROGATE, n1)
    print("call 1:", {k: sb[k] for k in KEYS})
    assert np.array_equal(Ta, Tb, equal_nan=True) and np.array_equal(pa, pb, equal_nan=True)
    for k in KEYS:
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    assert sb["fallbacks"] > 1000
    assert sb["rc"] == (-5 if sb["nonconverged"] else 0)
    rs = u1[:5]
    rhoe = u1[8] - 0.5 * (u1[5:8] ** 2).sum(0) / rs.sum(0)
    Tref, _ = mix.solve_T(rs, rhoe, T1, maxit=50)
    ok = np.isfinite(Tb) & (Tb > 0)
    assert ok.sum() >= n1 - sb["nonconverged"]
    assert np.max(np.abs(Tb[ok] - Tref[ok]) / Tref[ok]) < 1e-10

    # call 2: fewer states (the mesh's 27,000 nodes), freestream guess
    u2 = to_dev(c.u0)
    n2 = c.u0.shape[1] * c.u0.shape[2]
    (Ta, pa, sa), (Tb, pb, sb) = both(dgx, s.ctx, u2, n2, dgx.GUESS_FREESTREAM, 0)
    print("call 2:", {k: sb[k] for k in KEYS})
    assert np.array_equal(Ta, Tb) and np.array_equal(pa, pb)
    for k in KEYS:
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    assert sb["nodes"] == n2 and sb["nonconverged"] == 0 and sb["fallbacks"] == 0 and sb["rc"] == 0
    uu = c.u0.reshape(9, -1)
    Tref, _ = mix.solve_T(uu[:5], uu[8] - 0.5 * (uu[5:8] ** 2).sum(0) / uu[:5].sum(0), 300.0)
    assert np.max(np.abs(Tb - Tref) / Tref) < 1e-10
    s.close()


def test_noalloc_rejects_oversized_input(dgx):
    import torch
    mix = Mixture(W.Species())
    fns = (lambda rs, T: mix.rho_e(rs, T)), (lambda rs, T: mix.rho_cv(rs, T))
    c = W.case_c3(*fns, n=3)
    s = dgx.Solver(c)
    u = torch.zeros(9, 4, dtype=torch.float64, device="cuda")
    T = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(dgx.DgxError) as ei:
        dgx.dgx_thermo_noalloc(s.ctx, u, T, nstates=dgx.NOALLOC_MAX_STATES + 1)
    assert ei.value.code == -1 and "DGX_NOALLOC_MAX_STATES" in str(ei.value)
    s.close()

"""The boundary's helper entry points, called directly.

* dgx_species_energy: the context's species energies and heat capacities
  against the oracle's rigid-rotor / harmonic-oscillator tables from 50 K to
  20000 K (host arithmetic on both sides, different code).
* dgx_mixture_energy: rho e and rho cv of seeded mixture states against the
  oracle's sums over species (Eq. Internal_energy), one temperature per
  state, and its argument checks.
* dgx_kernel_times: the kernels of one right-hand side, named in launch
  order (gradient pass before the fused right-hand side for Navier-Stokes;
  the indicator, with the temperature solve fused into it, before the
  right-hand side for the shocked mixture), each with a positive average
  duration, and the state left untouched.
* dgx_last_error: after a rejected call the message names what was wrong;
  the binding's exception carries the same text.
* dgx_get_launch returns the launch shape dgx_set_launch set, unchanged by
  a rejected dgx_set_launch."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle.thermo import Mixture
from tests.helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dgx():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_17551_amd import dgx as mod
    return mod


@pytest.fixture(scope="module")
def thermo_fns():
    mix = Mixture(W.Species())
    return (lambda rs, T: mix.rho_e(rs, T)), (lambda rs, T: mix.rho_cv(rs, T))


def test_species_energy_matches_oracle(dgx, thermo_fns):
    c = W.case_c4(*thermo_fns, nr=4, nth=8, hot=True)
    mix = Mixture(c.species)
    s = dgx.Solver(c)
    worst_e = worst_cv = 0.0
    for T in (50.0, 300.0, 1000.0, 3371.0, 8000.0, 20000.0):
        e, cv = dgx.dgx_species_energy(s.ctx, T)
        er, cvr = mix.e_species(np.array(T)), mix.cv_species(np.array(T))
        worst_e = max(worst_e, float(np.max(np.abs(e - er) / np.abs(er))))
        worst_cv = max(worst_cv, float(np.max(np.abs(cv - cvr) / cvr)))
    s.close()
    print("species tables: max rel err e %.2e, cv %.2e" % (worst_e, worst_cv))
    assert worst_e < 1e-13 and worst_cv < 1e-13


def test_mixture_energy_matches_oracle(dgx, thermo_fns):
    c = W.case_c4(*thermo_fns, nr=4, nth=8, hot=True)
    mix = Mixture(c.species)
    rs, T = W.far_chem_states(997, seed=13)
    s = dgx.Solver(c)
    rhoe, rhocv = dgx.dgx_mixture_energy(s.ctx, rs, T)
    ref_e, ref_cv = mix.rho_e(rs, T), mix.rho_cv(rs, T)
    scale = np.abs(rs * mix.e_species(T)).sum(0)
    err_e = float(np.max(np.abs(rhoe - ref_e) / scale))
    err_cv = float(np.max(np.abs(rhocv - ref_cv) / ref_cv))
    print("mixture sums: max rel err rho e %.2e (of sum |rho_s e_s|), rho cv %.2e" % (err_e, err_cv))
    assert err_e < 1e-13 and err_cv < 1e-13
    # the binding's energy functions broadcast through the same entry point
    energy, cv = dgx.mixture_energy_fns(s.ctx)
    Tb = np.full((3, 4), 2500.0)
    rsb = np.broadcast_to(rs[:, :1, None], (5, 3, 4))
    assert np.allclose(energy(rsb, Tb), mix.rho_e(np.ascontiguousarray(rsb), Tb), rtol=1e-13)
    assert np.allclose(cv(rs, 2500.0), mix.rho_cv(rs, np.full(rs.shape[1], 2500.0)), rtol=1e-13)
    # a non-positive temperature is rejected, nothing written
    bad = T.copy()
    bad[5] = 0.0
    with pytest.raises(dgx.DgxError):
        dgx.dgx_mixture_energy(s.ctx, rs, bad)
    s.close()


def timed(dgx, c, expect):
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    times = dgx.dgx_kernel_times(s.ctx, u, reps=3)
    s.check()
    s.close()
    print(c.cfg.get("eq"), times)
    names = list(times)
    assert [n for n in names if n in expect] == expect
    assert names[-1] == "k_rhs"
    assert all(ms > 0.0 for ms in times.values())
    assert np.array_equal(to_host(u), c.u0)


def test_kernel_times_name_the_launches(dgx, thermo_fns):
    timed(dgx, W.case_c2(n=4), ["k_grad", "k_rhs"])
    timed(dgx, W.case_c3(*thermo_fns, n=2), ["k_indicator_T", "k_rhs"])


def test_last_error_names_the_cause(dgx):
    c = W.case_c2(n=2)
    s = dgx.Solver(c)
    dgx.dgx_set_launch(s.ctx, 2, 0)
    assert dgx.dgx_get_launch(s.ctx) == (2, 0)
    with pytest.raises(dgx.DgxError) as ei:
        dgx.dgx_set_launch(s.ctx, 3, 1)          # not one of 1, 2, 4, 8
    assert dgx.dgx_get_launch(s.ctx) == (2, 0)   # unchanged by the rejected call
    msg = dgx.dgx_last_error(s.ctx)
    assert dgx.ERRORS[ei.value.code] == "DGX_E_INVAL"
    assert "elements per workgroup" in msg and msg in str(ei.value)
    print("last error:", msg)
    # the context still works after the rejected call
    s.rhs(to_dev(c.u0))
    s.check()
    s.close()

"""The boundary's helper entry points, called directly.

* dgx_species_energy: the context's species energies and heat capacities
  against the oracle's rigid-rotor / harmonic-oscillator tables from 50 K to
  20000 K (host arithmetic on both sides, different code).
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

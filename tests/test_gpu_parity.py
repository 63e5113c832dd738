"""GPU right-hand side and SSPRK3 against the oracle (perfect gas)."""
import math

import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle.dgsem import Operator
from oracle import ssprk
from tests.helpers import rel_err, parity_err, flux_scale, to_dev, to_host, eps_units, ld_reference, oracle_dt

pytestmark = pytest.mark.gpu

# RHS: max_v ||du_gpu - du_ora||_inf / max(||du_ora||_inf, S_v) with the
# flux-divergence scale S_v (see helpers.flux_scale); states after SSPRK3
# steps: plain per-variable relative max norm.
RHS_TOL = 1e-11
STEP_TOL = 1e-9
# distance from the extended-precision value of the operator, in eps_64 S_v
# units (tests/test_oracle_rounding.py: the float64 oracle itself sits ~100-200
# units away on affine meshes and ~1e3 on curved ones)
AFFINE_EPS = 400.0
CURVED_EPS = 2500.0
EPS64 = float(np.finfo(np.float64).eps)


def check_rhs(label, op, u, got, ref):
    e = parity_err(got, ref, flux_scale(op, u))
    print("%s: parity %.3e (plain per-variable relative %.3e)" % (label, e, rel_err(got, ref)))
    assert e < RHS_TOL


def check_rhs_exact(label, case, op, got, ref, bound):
    """Both float64 evaluations against the operator's extended-precision
    value: the GPU within `bound` eps_64 S_v of it per variable; then the
    plain per-variable relative bound that implies, asserted against the
    float64 oracle: |du_gpu - du_ora|_v <= 2 bound eps_64 S_v, i.e. relative to
    ||du_ora_v|| the conditioning factor S_v / ||du_ora_v|| times 2 bound eps_64."""
    u = case.u0
    S = flux_scale(op, u)
    dld = ld_reference(case, u)
    g = eps_units(got, dld, S)
    o = eps_units(ref, dld, S)
    refmax = np.abs(ref).reshape(ref.shape[0], -1).max(1)
    plain = np.abs(got - ref).reshape(ref.shape[0], -1).max(1) / refmax
    plain_bound = 2.0 * bound * EPS64 * S / refmax
    print("%s: eps*S_v units from the extended value: gpu %s, float64 oracle %s; plain per-variable "
          "%s (bound %s)" % (label, np.round(g, 1), np.round(o, 1), np.array2string(plain, precision=2),
                             np.array2string(plain_bound, precision=2)))
    assert np.all(g < bound), g
    assert np.all(plain <= plain_bound), (plain, plain_bound)


@pytest.fixture(scope="module")
def dgx():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_17551_amd import dgx as mod
    return mod


def gpu_rhs(dgx, case, u=None):
    s = dgx.Solver(case)
    uu = to_dev(case.u0 if u is None else u)
    du = s.rhs(uu)
    s.check()
    out = to_host(du)
    s.close()
    return out


@pytest.mark.parametrize("sf", [W.SF_RUSANOV, W.SF_RANOCHA])
def test_vortex_rhs(dgx, sf):
    c = W.case_c1(surface_flux=sf)
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    got = gpu_rhs(dgx, c)
    check_rhs("vortex", op, c.u0, got, ref)
    assert rel_err(got, ref) < RHS_TOL
    check_rhs_exact("vortex", c, op, got, ref, AFFINE_EPS)


def test_vortex_ssprk3_100_steps(dgx):
    c = W.case_c1()
    op = Operator(c.cfg, c.mesh)
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    dt = oracle_dt(op, c.u0, 0.5)
    # the library's own CFL estimate is the same rule
    assert abs(dgx.dgx_max_dt(s.ctx, u, 0.5) - dt) <= 1e-12 * dt
    s.ssprk3(u, dt, 100)
    s.check()
    got = to_host(u)
    s.close()
    ref, _ = ssprk.run(lambda v, t: op.rhs(v, t), c.u0, 0.0, dt, 100)
    print("vortex 100 steps rel err", rel_err(got, ref), "dt", dt)
    assert rel_err(got, ref) < STEP_TOL


@pytest.mark.parametrize("eq", [W.EQ_EULER, W.EQ_NS])
def test_tgv_small_rhs(dgx, eq):
    c = W.case_c2(n=4, eq=eq)
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    got = gpu_rhs(dgx, c)
    check_rhs("tgv n=4 eq=%d" % eq, op, c.u0, got, ref)
    check_rhs_exact("tgv n=4 eq=%d" % eq, c, op, got, ref, AFFINE_EPS)


def test_tgv_8cube_rhs_extended(dgx):
    c = W.case_c2(n=8)
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    got = gpu_rhs(dgx, c)
    check_rhs("tgv n=8", op, c.u0, got, ref)
    check_rhs_exact("tgv n=8", c, op, got, ref, AFFINE_EPS)


def test_tgv_small_ssprk3(dgx):
    c = W.case_c2(n=4)
    op = Operator(c.cfg, c.mesh)
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    dt = 0.01
    s.ssprk3(u, dt, 20)
    s.check()
    got = to_host(u)
    s.close()
    ref, _ = ssprk.run(lambda v, t: op.rhs(v, t), c.u0, 0.0, dt, 20)
    assert rel_err(got, ref) < STEP_TOL


def test_tgv_8cube_ns_200_steps(dgx):
    """The Navier-Stokes TGV (8^3 elements, N = 3, BR1) over 200 SSPRK3 steps
    at the oracle's CFL-0.5 time step (to t ~ 0.65)."""
    c = W.case_c2(n=8)
    op = Operator(c.cfg, c.mesh)
    dt = oracle_dt(op, c.u0, 0.5)
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    s.ssprk3(u, dt, 200)
    s.check()
    got = to_host(u)
    s.close()
    ref, _ = ssprk.run(lambda v, t: op.rhs(v, t), c.u0, 0.0, dt, 200)
    print("tgv 8^3 NS 200 steps (dt %.4e) rel err %.3e" % (dt, rel_err(got, ref)))
    assert rel_err(got, ref) < STEP_TOL


@pytest.mark.parametrize("N", [3, 4])
def test_curved_channel_outflow(dgx, N):
    """Supersonic perfect-gas channel on the curved mesh: Dirichlet inflow at
    x = 0, outflow (external state = interior) at x = 1; right-hand side and
    20 SSPRK3 steps."""
    c = W.curved_channel_case(n=3, N=N)
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    got = gpu_rhs(dgx, c)
    check_rhs("channel outflow N=%d" % N, op, c.u0, got, ref)
    dt = oracle_dt(op, c.u0, 0.5)
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    s.ssprk3(u, dt, 20)
    s.check()
    gotu = to_host(u)
    s.close()
    refu, _ = ssprk.run(lambda v, t: op.rhs(v, t), c.u0, 0.0, dt, 20)
    print("channel outflow N=%d 20 steps rel err %.3e" % (N, rel_err(gotu, refu)))
    assert rel_err(gotu, refu) < STEP_TOL


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("vf", [W.VF_RANOCHA, W.VF_DUCROS])
def test_curved_rhs_forced_alpha(dgx, N, alpha, vf):
    c = W.curved_periodic_case(n=3, N=N, shock=True, force_alpha=alpha, volume_flux=vf)
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    got = gpu_rhs(dgx, c)
    check_rhs("curved N=%d alpha=%g vf=%d" % (N, alpha, vf), op, c.u0, got, ref)
    check_rhs_exact("curved N=%d alpha=%g vf=%d" % (N, alpha, vf), c, op, got, ref, CURVED_EPS)


@pytest.mark.parametrize("N", [3, 4])
def test_curved_freestream(dgx, N):
    c = W.curved_periodic_case(n=3, N=N, shock=True, force_alpha=0.5)
    u = np.empty_like(c.u0)
    rho, v, p = 1.3, np.array([0.4, -0.7, 0.2]), 2.1
    u[0] = rho
    u[1:4] = (rho * v)[:, None, None]
    u[4] = p / 0.4 + 0.5 * rho * (v @ v)
    got = gpu_rhs(dgx, c, u)
    op = Operator(c.cfg, c.mesh)
    S = (np.abs(op.Ja).max() / op.J.min()) * (u[4].max() + p)
    assert np.abs(got).max() < 1e-12 * S * 3


def test_tgv_full_size_rhs(dgx):
    """32^3 N=3 Navier-Stokes TGV (the benchmark workload), whole field."""
    c = W.case_c2()
    got = gpu_rhs(dgx, c)
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    check_rhs("tgv 32^3", op, c.u0, got, ref)
    # the plain per-variable norm (the float64 oracle is itself ~6.5e-9 from
    # the exact value in it: du_rho is 1.6e5 times below S_rho here)
    check_rhs_exact("tgv 32^3", c, op, got, ref, AFFINE_EPS)

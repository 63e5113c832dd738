"""BR1 Navier-Stokes on the GPU beyond the periodic affine mesh, against the
oracle: curved elements (N = 3 and 4), no-slip isothermal and adiabatic
walls, Dirichlet, outflow and slip boundaries, Sutherland viscosity at the
walls, and 2:1 non-conforming meshes with viscous mortars.

Each right-hand side is checked twice: whole, in the parity norm of the
other tests (per variable, the max-norm difference over max(||ref_v||,
S_v), S_v the advective flux scale), and for its viscous part alone,
GPU(Navier-Stokes) - GPU(Euler) on the same mesh against the oracle's
viscous terms, relative to their own per-variable max norm, so that a
mistake in the viscous terms cannot hide under the larger advective ones.
Time integration: 50 SSPRK3 steps (20 on the octree mesh) at the smaller of the oracle's advective
(CFL 0.5) and diffusive step bounds."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle.dgsem import Operator
from oracle.br1 import viscous_rhs
from oracle import ssprk
from tests.helpers import rel_err, parity_err, flux_scale, to_dev, to_host, oracle_dt_ns

pytestmark = pytest.mark.gpu
RHS_TOL = 1e-11
VISC_TOL = 1e-10
STEP_TOL = 1e-9


@pytest.fixture(scope="module")
def dgx():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_17551_amd import dgx as mod
    return mod


def gpu_rhs(dgx, case, cfg=None):
    import copy
    c = copy.copy(case)
    if cfg is not None:
        c.cfg = cfg
    s = dgx.Solver(c)
    du = s.rhs(to_dev(c.u0))
    s.check()
    out = to_host(du)
    s.close()
    return out


def curved_ns(N):
    c = W.curved_periodic_case(n=2, N=N, eq=W.EQ_NS, mu=0.02)
    return c


def wall_channel(T_hi=1.6, **kw):
    return W.wall_channel_case(T_hi=T_hi, mu=0.02, **kw)


def wall_channel_other_bcs():
    """The wall channel with a slip wall at y = 0 and outflow at y = 1."""
    c = W.wall_channel_case(T_hi=1.6, mu=0.02)
    c.mesh.bc_kind[:] = (W.BC_SLIPWALL, W.BC_OUTFLOW)
    return c


def curved_channel_ns(N):
    """Supersonic channel on the curved map: Dirichlet inflow, outflow."""
    c = W.curved_channel_case(n=2, N=N)
    c.cfg = dict(c.cfg, eq=W.EQ_NS, mu=0.02)
    return c


def amr_ns():
    """The small 2:1 octree mesh (periodic) with the density wave plus a
    smooth velocity perturbation (the wave alone has uniform velocity)."""
    c = W.case_amr(base=4, radii=(0.4, 0.25), centre=(0.45, 0.5, 0.55))
    c.cfg = dict(c.cfg, eq=W.EQ_NS, mu=0.02)
    x = c.mesh.x
    rho = c.u0[0]
    v = c.u0[1:4] / rho
    p = 0.4 * (c.u0[4] - 0.5 * rho * (v * v).sum(0))
    v = v + 0.1 * np.stack([np.sin(2 * np.pi * x[1]), np.cos(2 * np.pi * x[2]), np.sin(2 * np.pi * (x[0] + x[1]))])
    c.u0 = W._pg_conserved(rho, v, p, 1.4)
    return c


CASES = [
    ("curved_periodic_N3", lambda: curved_ns(3)),
    ("curved_periodic_N4", lambda: curved_ns(4)),
    ("wall_channel_isothermal", lambda: wall_channel()),
    ("wall_channel_adiabatic_top", lambda: wall_channel(T_hi=None)),
    ("wall_channel_sutherland", lambda: wall_channel(sutherland_S=0.4, sutherland_T0=1.0)),
    ("wall_channel_slip_outflow", wall_channel_other_bcs),
    ("curved_channel_N3", lambda: curved_channel_ns(3)),
    ("curved_channel_N4", lambda: curved_channel_ns(4)),
    ("amr_periodic", amr_ns),
]


@pytest.mark.parametrize("which", range(len(CASES)))
def test_ns_rhs(dgx, which):
    name, make = CASES[which]
    c = make()
    print("case", name, flush=True)
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    got = gpu_rhs(dgx, c)
    e = parity_err(got, ref, flux_scale(op, c.u0))
    # the viscous part alone
    s = op.states(c.u0)
    vref = viscous_rhs(op, c.u0, s)
    gotE = gpu_rhs(dgx, c, dict(c.cfg, eq=W.EQ_EULER))
    vgot = got - gotE
    vs = np.abs(vref).reshape(5, -1).max(1)
    assert np.all(vs[1:] > 1e-3 * vs[1:].max())   # every viscous row is exercised
    ve = (np.abs(vgot - vref).reshape(5, -1).max(1)[1:] / vs[1:]).max()
    print("%s: parity %.3e, viscous part %.3e (scale %s)" % (name, e, ve, vs[1:]))
    assert e < RHS_TOL, (name, e)
    assert ve < VISC_TOL, (name, ve)


@pytest.mark.parametrize("which,steps", [(1, 50), (2, 50), (3, 50), (8, 20)])
def test_ns_ssprk3_steps(dgx, which, steps):
    name, make = CASES[which]
    c = make()
    print("case", name, flush=True)
    op = Operator(c.cfg, c.mesh)
    dt = oracle_dt_ns(op, c.u0)
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    s.ssprk3(u, dt, steps)
    s.check()
    got = to_host(u)
    s.close()
    ref, _ = ssprk.run(lambda v, t: op.rhs(v, t), c.u0, 0.0, dt, steps)
    e = rel_err(got, ref)
    print("%s: %d steps rel err %.3e" % (name, steps, e))
    assert e < STEP_TOL, (name, e)

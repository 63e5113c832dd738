"""Edge cases of the boundary on the GPU, against the oracle.

* Ragged workgroups: 27 elements (3^3) with 1, 2, 4 and 8 elements per
  workgroup and both workgroup numberings, so the last workgroup is partly
  empty; the perfect-gas Navier-Stokes TGV (N = 3) and the curved 5-species
  shock case (N = 4), right-hand side against the oracle.
* The one-element periodic mesh: every face of the element is its own
  neighbour's; right-hand side and one SSPRK3 step against the oracle.
* Calls that do nothing: zero SSPRK3 steps and a chemistry step over dt = 0
  leave the state bitwise unchanged; an empty mesh and an empty state set
  are rejected with DGX_E_INVAL.
* The largest reaction table (32 reactions: the 17 of the workload and 15
  of them again with halved rates): the reacting right-hand side against the
  oracle."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle.dgsem import Operator
from oracle import ssprk
from oracle.thermo import Mixture
from tests.helpers import flux_scale, parity_err, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
RHS_TOL = 1e-11
STEP_TOL = 1e-9


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


def ragged_cases(thermo_fns):
    return [("tgv_ns_3cube_N3", W.case_c2(n=3)), ("curved_air5_shock_3cube_N4", W.case_c3(*thermo_fns, n=3))]


@pytest.mark.parametrize("which", [0, 1])
def test_ragged_workgroups(dgx, thermo_fns, which):
    name, c = ragged_cases(thermo_fns)[which]
    print("case", name, flush=True)
    op = Operator(c.cfg, c.mesh, species=c.species, reactions=c.reactions)
    ref = op.rhs(c.u0)
    scale = flux_scale(op, c.u0)
    tried = 0
    for epb in (1, 2, 4, 8):
        for order in (0, 1):
            s = dgx.Solver(c)
            try:
                dgx.dgx_set_launch(s.ctx, epb, order)
            except dgx.DgxError:
                s.close()
                continue          # does not fit (threads or LDS)
            tried += 1
            got = to_host(s.rhs(to_dev(c.u0)))
            s.check()
            s.close()
            e = parity_err(got, ref, scale)
            print("%s epb %d order %d: parity %.3e" % (name, epb, order, e), flush=True)
            assert e < RHS_TOL, (name, epb, order, e)
    assert tried >= 4
    assert c.mesh.nelem % 2 == 1


def test_single_element_periodic(dgx):
    c = W.case_c2(n=1)
    assert c.mesh.nelem == 1
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    got = to_host(s.rhs(u))
    e = parity_err(got, ref, flux_scale(op, c.u0))
    dt = 1e-3
    s.ssprk3(u, dt, 1)
    s.check()
    step = to_host(u)
    s.close()
    ref1 = ssprk.step(lambda v, t: op.rhs(v, t), c.u0, 0.0, dt)
    print("one element: rhs parity %.3e, step %.3e" % (e, rel_err(step, ref1)))
    assert e < RHS_TOL
    assert rel_err(step, ref1) < STEP_TOL


def test_calls_that_do_nothing(dgx, thermo_fns):
    import torch
    # zero SSPRK3 steps
    c = W.case_c2(n=2)
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    s.ssprk3(u, 0.01, 0)
    s.check()
    assert np.array_equal(to_host(u), c.u0)
    # an empty mesh is rejected
    empty = W.Mesh(c.mesh.dim, c.mesh.N, c.mesh.x[:, :0], c.mesh.faces[:0], c.mesh.bfaces[:0],
                   c.mesh.mortars[:0], c.mesh.bc_kind, c.mesh.bc_state)
    with pytest.raises(dgx.DgxError) as ei:
        dgx.dgx_set_mesh(s.ctx, empty)
    assert dgx.ERRORS[ei.value.code] == "DGX_E_INVAL"
    s.close()
    # chemistry over dt = 0, and an empty state set for the surrogate
    h = W.case_c4(*thermo_fns, nr=4, nth=8, hot=True)
    h.cfg = dict(h.cfg, eq=W.EQ_EULER_MIX)
    s = dgx.Solver(h)
    u = to_dev(h.u0)
    st = dgx.dgx_chem_step(s.ctx, u, 0.0)
    s.check()
    assert st["nonconverged"] == 0 and st["substeps_max"] == 1
    assert np.array_equal(to_host(u), h.u0)
    with pytest.raises(dgx.DgxError) as ei:
        dgx.dgx_surrogate_predict(s.ctx, u.reshape(u.shape[0], -1)[:, :0].contiguous(),
                                  torch.empty(0, dtype=torch.float64, device="cuda"))
    assert dgx.ERRORS[ei.value.code] == "DGX_E_INVAL"
    s.close()


def test_largest_reaction_table(dgx, thermo_fns):
    c = W.case_c4(*thermo_fns, nr=8, nth=16, hot=True)
    rx = c.reactions
    rows = np.concatenate([np.arange(17), np.arange(15)])
    A = rx.A[rows].copy()
    A[17:] *= 0.5
    c.reactions = W.Reactions(A=A, b=rx.b[rows], theta_a=rx.theta_a[rows], nu=rx.nu[rows], nup=rx.nup[rows])
    assert c.reactions.nreactions == 32
    op = Operator(c.cfg, c.mesh, species=c.species, reactions=c.reactions)
    ref = op.rhs(c.u0)
    s = dgx.Solver(c)
    got = to_host(s.rhs(to_dev(c.u0)))
    s.check()
    s.close()
    e = parity_err(got, ref, flux_scale(op, c.u0))
    print("32 reactions: parity %.3e" % e)
    assert e < RHS_TOL

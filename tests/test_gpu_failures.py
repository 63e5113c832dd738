"""Failure paths, forced from the host with inputs that every kernel handles
and exits from normally (NaN arithmetic, bounded iterations; no index is
derived from the data).

* A NaN or a negative density in the state: the right-hand side raises the
  non-physical flag, and dgx_check reports DGX_E_NONPHYSICAL (perfect gas
  and mixture, where a negative species density counts too).
* An iteration budget of one for the temperature Newton solve, started from
  the freestream guess on hot states: dgx_thermo reports DGX_E_NOCONV with
  the count of nodes that needed more, and the first of them.
* NaN surrogate weights: every guess is NaN, the solve falls back to the
  freestream guess and converges to the plain solve's temperatures,
  bitwise.
* Malformed mesh tables (a face row that is not a (+d, -d) pair, a
  boundary face with an unknown boundary condition, an element index out of
  range) are rejected with DGX_E_INVAL before any launch, and the context
  keeps its previous mesh."""
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


def code(dgx, ex):
    return dgx.ERRORS[ex.value.code]


def expect_nonphysical(dgx, c, u):
    s = dgx.Solver(c)
    s.rhs(to_dev(u))
    with pytest.raises(dgx.DgxError) as ei:
        s.check()
    assert code(dgx, ei) == "DGX_E_NONPHYSICAL"
    # the flag is cleared by the check: a clean state passes again
    s.rhs(to_dev(c.u0))
    s.check()
    s.close()


def test_nonphysical_states_are_reported(dgx, thermo_fns):
    c = W.case_c2(n=2)
    u = c.u0.copy()
    u[0, 3, 5] = np.nan
    expect_nonphysical(dgx, c, u)
    u = c.u0.copy()
    u[0, 6, 1] = -0.5
    expect_nonphysical(dgx, c, u)
    h = W.case_c4(*thermo_fns, nr=4, nth=8, hot=True)
    h.cfg = dict(h.cfg, eq=W.EQ_EULER_MIX)
    u = h.u0.copy()
    u[3, 5, 2] = -1e-3 * u[:5, 5, 2].sum()
    expect_nonphysical(dgx, h, u)


def test_newton_budget_exhaustion_is_counted(dgx, thermo_fns):
    import torch
    h = W.case_c4(*thermo_fns, nr=4, nth=8, hot=True)
    h.cfg = dict(h.cfg, eq=W.EQ_EULER_MIX)
    s = dgx.Solver(h)
    u = to_dev(h.u0)
    n = h.u0.shape[1] * h.u0.shape[2]
    T = torch.empty(n, dtype=torch.float64, device="cuda")
    full = dgx.dgx_thermo(s.ctx, u, T)           # the context's budget (50)
    assert full["nonconverged"] == 0 and full["iters_max"] > 1
    s.close()
    h.cfg = dict(h.cfg, newton_maxit=1)
    s = dgx.Solver(h)
    st = dgx.dgx_thermo(s.ctx, to_dev(h.u0), T, check=False)
    s.close()
    print("budget 1: %d of %d nodes not converged, first %d (full budget: max %d iterations)"
          % (st["nonconverged"], n, st["first_bad"], full["iters_max"]))
    assert dgx.ERRORS[st["rc"]] == "DGX_E_NOCONV"
    assert 0 < st["nonconverged"] <= n
    assert 0 <= st["first_bad"] < n


def test_nan_surrogate_weights_fall_back(dgx, thermo_fns):
    import torch
    h = W.case_c4(*thermo_fns, nr=4, nth=8, hot=True)
    h.cfg = dict(h.cfg, eq=W.EQ_EULER_MIX)
    s = dgx.Solver(h)
    u = to_dev(h.u0)
    n = h.u0.shape[1] * h.u0.shape[2]
    Tp = torch.empty(n, dtype=torch.float64, device="cuda")
    Ts = torch.empty_like(Tp)
    plain = dgx.dgx_thermo(s.ctx, u, Tp)
    dgx.dgx_surrogate_set(s.ctx, np.full(8847, np.nan, np.float32))
    sur = dgx.dgx_thermo(s.ctx, u, Ts, guess=dgx.GUESS_SURROGATE)
    s.check()
    s.close()
    assert sur["nonconverged"] == 0
    assert sur["iters_total"] == plain["iters_total"]
    assert np.array_equal(to_host(Ts), to_host(Tp))


def test_malformed_mesh_tables_are_rejected(dgx):
    c = W.case_c2(n=2)
    m = c.mesh
    s = dgx.Solver(c)
    bad_pair = m.faces.copy()
    bad_pair[0, 1] -= 1                  # an even face id on the "+" side
    out_of_range = m.faces.copy()
    out_of_range[1, 2] = m.nelem         # no such element
    for faces in (bad_pair, out_of_range):
        bad = W.Mesh(m.dim, m.N, m.x, faces, m.bfaces, m.mortars, m.bc_kind, m.bc_state)
        with pytest.raises(dgx.DgxError) as ei:
            dgx.dgx_set_mesh(s.ctx, bad)
        assert code(dgx, ei) == "DGX_E_INVAL"
    # a boundary face naming a boundary condition that does not exist
    e0 = W.case_c1(n=4)
    m1 = e0.mesh
    s1 = dgx.Solver(e0)
    if m1.bfaces.shape[0] == 0:
        faces = m1.faces[1:]
        bf = np.array([[int(m1.faces[0, 0]), int(m1.faces[0, 1]), 5]], np.int32)
    else:
        faces = m1.faces
        bf = m1.bfaces.copy()
        bf[0, 2] = m1.bc_kind.shape[0]
    bad = W.Mesh(m1.dim, m1.N, m1.x, faces, bf, m1.mortars, m1.bc_kind, m1.bc_state)
    with pytest.raises(dgx.DgxError) as ei:
        dgx.dgx_set_mesh(s1.ctx, bad)
    assert code(dgx, ei) == "DGX_E_INVAL"
    # the contexts keep their valid meshes
    s.rhs(to_dev(c.u0))
    s.check()
    s.close()
    s1.close()

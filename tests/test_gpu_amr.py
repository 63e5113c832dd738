"""GPU mortars, the 2-level AMR mesh and batched independent cases against
the oracle; batched execution against separate per-case runs."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle.dgsem import Operator
from oracle import ssprk
from tests.helpers import rel_err, parity_err, flux_scale, to_dev, to_host, oracle_dt

pytestmark = pytest.mark.gpu
RHS_TOL = 1e-11


@pytest.fixture(scope="module")
def dgx():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_17551_amd import dgx as mod
    return mod


def gpu_rhs(dgx, case, u=None):
    s = dgx.Solver(case)
    du = s.rhs(to_dev(case.u0 if u is None else u))
    s.check()
    out = to_host(du)
    s.close()
    return out


@pytest.mark.parametrize("sf", [W.SF_RUSANOV, W.SF_RANOCHA])
def test_small_amr_rhs(dgx, sf):
    c = W.case_amr(base=4, radii=(0.4, 0.25), centre=(0.45, 0.5, 0.55))
    c.cfg["surface_flux"] = sf
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    got = gpu_rhs(dgx, c)
    e = parity_err(got, ref, flux_scale(op, c.u0))
    print("small amr sf=%d parity %.3e plain %.3e" % (sf, e, rel_err(got, ref)))
    assert e < RHS_TOL


@pytest.mark.parametrize("vf", [W.VF_KENNEDY_GRUBER, W.VF_PIROZZOLI, W.VF_CENTRAL, W.VF_MORINISHI])
def test_small_amr_rhs_other_volume_forms(dgx, vf):
    """The Kennedy-Gruber, Pirozzoli, Morinishi and standard-DG volume forms on the
    2:1 non-conforming mesh (Rusanov faces and mortars)."""
    c = W.case_amr(base=4, radii=(0.4, 0.25), centre=(0.45, 0.5, 0.55))
    c.cfg["volume_flux"] = vf
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    got = gpu_rhs(dgx, c)
    e = parity_err(got, ref, flux_scale(op, c.u0))
    print("small amr vf=%d parity %.3e" % (vf, e))
    assert e < RHS_TOL


def test_small_amr_ssprk3(dgx):
    """100 SSPRK3 steps on the small 2:1 mesh (498 elements, mortars), dt
    from the oracle's CFL rule (0.5)."""
    c = W.case_amr(base=4, radii=(0.4, 0.25), centre=(0.45, 0.5, 0.55))
    op = Operator(c.cfg, c.mesh)
    dt = oracle_dt(op, c.u0, 0.5)
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    s.ssprk3(u, dt, 100)
    s.check()
    got = to_host(u)
    s.close()
    ref, _ = ssprk.run(lambda v, t: op.rhs(v, t), c.u0, 0.0, dt, 100)
    print("small amr 100 steps rel err %.3e" % rel_err(got, ref))
    assert rel_err(got, ref) < 1e-9


def test_full_amr_rhs_and_conservation(dgx):
    """The ~60k-element 2-level mesh (base 16^3, seeded sphere)."""
    c = W.case_amr()
    got = gpu_rhs(dgx, c)
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    e = parity_err(got, ref, flux_scale(op, c.u0))
    print("amr %d elements, %d mortars: parity %.3e" % (c.mesh.nelem, len(c.mesh.mortars), e))
    assert e < RHS_TOL
    w = op.b.w
    wq = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
    tot = (got * op.J[None] * wq).sum(axis=(1, 2))
    scale = np.abs(got * op.J[None] * wq).sum(axis=(1, 2))
    assert np.all(np.abs(tot) < 1e-12 * scale)


def test_batched_equals_separate(dgx):
    """One launch over the AMR domain + 4 vortex-tube cases gives the same
    right-hand side as each case run on its own (to roundoff: the batched mesh
    has mortars and runs the mortar-enabled kernel variant, a lone tube the
    conforming one, whose instruction schedules differ)."""
    sizes = [5, 7, 4, 6]
    c = W.case_c5(base=4, radii=(0.4, 0.25), sizes=sizes)
    got = gpu_rhs(dgx, c)
    offs = c.mesh.case_offsets
    amr = W.case_amr(base=4, radii=(0.4, 0.25))
    parts = [gpu_rhs(dgx, amr)]
    for n in sizes:
        x, faces, u0 = W.vortex_tube_case(n)
        m = W.Mesh(3, 3, x, faces, np.zeros((0, 3), np.int32), np.zeros((0, 7), np.int32),
                   np.zeros(0, np.int32), np.zeros((0, 5)))
        parts.append(gpu_rhs(dgx, W.Case("tube", W.base_cfg(3, 3, W.EQ_EULER), m, u0)))
    for i, ref in enumerate(parts):
        sl = got[:, offs[i]:offs[i + 1]]
        assert rel_err(sl, ref) < 1e-13, (i, rel_err(sl, ref))


def test_c5_full_rhs(dgx):
    """AMR domain + 16 seeded vortex-tube cases (8^3..24^3) in one mesh."""
    c = W.case_c5()
    got = gpu_rhs(dgx, c)
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    e = parity_err(got, ref, flux_scale(op, c.u0))
    print("c5 %d elements parity %.3e" % (c.mesh.nelem, e))
    assert e < RHS_TOL

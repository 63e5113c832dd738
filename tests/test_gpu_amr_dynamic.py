"""Dynamic AMR on the GPU against the oracle (oracle/amr.py): octree mesh
construction, the Loehner and Hennemann-Gassner indicators, one adaptation
pass (leaves and solution transfer) and cycles of indicator, adaptation and
time steps on a Gaussian density pulse carried across the periodic unit
cube (4^3 level-0 cells, levels 0-2, thresholds 0.05 and 0.1 on Loehner's
estimate of the density), for the Euler and (one pass plus steps) the
Navier-Stokes equations.

Leaves are integers: the GPU's leaf list (element order) must equal the
oracle's Morton-ordered list exactly.  To keep the decision in one
precision, the single-pass test feeds the oracle's indicator values to both
sides; the cycle test lets each side use its own indicator and first checks
that no oracle value lies within 1e-8 of a threshold (so that rounding
cannot flip a decision)."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle import amr, ssprk
from oracle.dgsem import Operator
from tests.helpers import rel_err, parity_err, flux_scale, to_dev, to_host, oracle_dt

pytestmark = pytest.mark.gpu
BASE, N = 4, 3
CTRL = dict(base_level=0, med_level=1, max_level=2, med_threshold=0.05, max_threshold=0.1)


@pytest.fixture(scope="module")
def dgx():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_17551_amd import dgx as mod
    return mod


def uniform_leaves():
    return [(0, i, j, k) for k in range(BASE) for j in range(BASE) for i in range(BASE)]


def oracle_case(order):
    x, faces, mortars, level = amr.mesh(BASE, N, order)
    cfg = W.base_cfg(3, N, W.EQ_EULER)
    mesh = W.Mesh(3, N, x, faces, np.zeros((0, 3), np.int32), mortars, np.zeros(0, np.int32),
                  np.zeros((0, 5)), level=level)
    return W.Case("amr_blob", cfg, mesh, W.blob_state(x))


def solver(dgx, leaves):
    c = W.case_amr(base=4, radii=(0.4,), centre=(0.5, 0.5, 0.5))
    s = dgx.Solver(c)
    order = s.set_octree(BASE, np.asarray(leaves, np.int32))
    return s, order


def test_octree_mesh_and_rhs(dgx):
    leaves = amr.morton_order(BASE, uniform_leaves())
    # one refined round first, from the oracle, so that the mesh has mortars
    c0 = oracle_case(leaves)
    ind = amr.indicator(c0.u0, N, amr.IND_LOEHNER, amr.VAR_DENSITY)
    tgt = amr.controller(ind, **{k: CTRL[k] for k in ("base_level", "med_level", "max_level",
                                                     "med_threshold", "max_threshold")})
    new, _ = amr.adapt(BASE, leaves, {c: int(t) for c, t in zip(leaves, tgt)})
    order = amr.morton_order(BASE, new)
    s, got_order = solver(dgx, list(new)[::-1])     # any input order
    assert [tuple(r) for r in got_order] == order
    c = oracle_case(order)
    assert len(c.mesh.mortars) > 0
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    got = to_host(s.rhs(to_dev(c.u0)))
    s.check()
    s.close()
    e = parity_err(got, ref, flux_scale(op, c.u0))
    print("octree mesh (%d elements, %d mortars): rhs parity %.3e" % (len(order), len(c.mesh.mortars), e))
    assert e < 1e-11


@pytest.mark.parametrize("kind", [amr.IND_LOEHNER, amr.IND_HENNEMANN_GASSNER])
@pytest.mark.parametrize("var", [amr.VAR_DENSITY, amr.VAR_PRESSURE, amr.VAR_DENSITY_PRESSURE, amr.VAR_VELOCITY])
def test_indicator(dgx, kind, var):
    order = amr.morton_order(BASE, uniform_leaves())
    c = oracle_case(order)
    u = c.u0.copy()
    # a pressure and velocity perturbation as well, so that every variable varies
    x = c.mesh.x
    u[4] += 0.2 * np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1])
    u[1] += 0.3 * u[0] * np.cos(2 * np.pi * x[2])
    s, got_order = solver(dgx, order)
    ind = to_host(s.amr_indicator(to_dev(u), kind, var))
    s.check()
    s.close()
    ref = amr.indicator(u, N, kind, var)
    e = np.abs(ind - ref).max()
    print("indicator kind %d var %d: max |diff| %.3e (range %.3g .. %.3g)" % (kind, var, e, ref.min(), ref.max()))
    assert ref.max() > (1e-3 if kind == amr.IND_LOEHNER else 1.2e-4)   # above the cut-off of 1e-4
    assert e < (1e-12 if kind == amr.IND_LOEHNER else 1e-9)


def test_one_adaptation_pass(dgx):
    """From a mesh with two levels: refinement, 2:1 balancing and merging in
    one pass, the oracle's indicator values fed to both sides."""
    leaves = amr.morton_order(BASE, uniform_leaves())
    c0 = oracle_case(leaves)
    ind0 = amr.indicator(c0.u0, N, amr.IND_LOEHNER, amr.VAR_DENSITY)
    tg0 = amr.controller(ind0, 0, 1, 2, 0.05, 0.1)
    l1, _ = amr.adapt(BASE, leaves, {c: int(t) for c, t in zip(leaves, tg0)})
    order = amr.morton_order(BASE, l1)
    # move the pulse so that some refined regions merge and others split
    x, _, _, _ = amr.mesh(BASE, N, order)
    u = W.blob_state(x, centre=(0.6, 0.45, 0.5))
    ind = amr.indicator(u, N, amr.IND_LOEHNER, amr.VAR_DENSITY)
    tgt = amr.controller(ind, 0, 1, 2, 0.05, 0.1)
    new, plan = amr.adapt(BASE, order, {c: int(t) for c, t in zip(order, tgt)})
    kinds = [p[0] for p in plan.values()]
    assert "refine" in kinds and "coarsen" in kinds
    new_order = amr.morton_order(BASE, new)
    ref = amr.transfer(u, order, new_order, plan, N)
    s, got_order = solver(dgx, order)
    assert [tuple(r) for r in got_order] == order
    got = to_host(s.amr_adapt(to_dev(u), ind, CTRL))
    s.check()
    assert [tuple(r) for r in s.octree()] == new_order
    e = rel_err(got, ref)
    print("adaptation: %d -> %d elements (%d split, %d merged), transfer rel err %.3e"
          % (len(order), len(new_order), kinds.count("refine"), kinds.count("coarsen"), e))
    assert e < 1e-13
    # and the right-hand side on the adapted mesh
    c = oracle_case(new_order)
    op = Operator(c.cfg, c.mesh)
    du = to_host(s.rhs(to_dev(ref)))
    s.check()
    s.close()
    assert parity_err(du, op.rhs(ref), flux_scale(op, ref)) < 1e-11


def test_amr_cycles(dgx):
    """Three cycles of: indicator, adaptation, 10 SSPRK3 steps."""
    order = amr.morton_order(BASE, uniform_leaves())
    c = oracle_case(order)
    u_ref = c.u0
    s, _ = solver(dgx, order)
    u = to_dev(c.u0)
    for cyc in range(3):
        ind_ref = amr.indicator(u_ref, N, amr.IND_LOEHNER, amr.VAR_DENSITY)
        margin = min(np.abs(ind_ref - CTRL["med_threshold"]).min(), np.abs(ind_ref - CTRL["max_threshold"]).min())
        assert margin > 1e-8, margin
        tgt = amr.controller(ind_ref, 0, 1, 2, 0.05, 0.1)
        new, plan = amr.adapt(BASE, order, {cc: int(t) for cc, t in zip(order, tgt)})
        new_order = amr.morton_order(BASE, new)
        u_ref = amr.transfer(u_ref, order, new_order, plan, N)
        order = new_order
        ind = to_host(s.amr_indicator(u, amr.IND_LOEHNER, amr.VAR_DENSITY))
        u = s.amr_adapt(u, ind, CTRL)
        s.check()
        assert [tuple(r) for r in s.octree()] == order
        cc = oracle_case(order)
        op = Operator(cc.cfg, cc.mesh)
        dt = oracle_dt(op, u_ref, 0.5)
        u_ref, _ = ssprk.run(lambda v, t: op.rhs(v, t), u_ref, 0.0, dt, 10)
        s.ssprk3(u, dt, 10)
        s.check()
        e = rel_err(to_host(u), u_ref)
        print("cycle %d: %d elements, levels %s, rel err %.3e"
              % (cyc, len(order), np.bincount([o[0] for o in order]), e))
        assert e < 1e-11
    s.close()


def test_navier_stokes_adaptation(dgx):
    """Navier-Stokes on the octree: one adaptation pass (the oracle's
    indicator values fed to both sides) and 10 SSPRK3 steps with the BR1
    terms across the new mortars (mu = 0.01)."""
    from tests.helpers import oracle_dt_ns
    leaves = amr.morton_order(BASE, uniform_leaves())
    c0 = oracle_case(leaves)
    ind = amr.indicator(c0.u0, N, amr.IND_LOEHNER, amr.VAR_DENSITY)
    new, plan = amr.adapt(BASE, leaves, {c: int(t) for c, t in zip(leaves, amr.controller(ind, 0, 1, 2, 0.05, 0.1))})
    order = amr.morton_order(BASE, new)
    ref = amr.transfer(c0.u0, leaves, order, plan, N)
    base_case = W.case_amr(base=4, radii=(0.4,), centre=(0.5, 0.5, 0.5))
    base_case.cfg = dict(base_case.cfg, eq=W.EQ_NS, mu=0.01)
    s = dgx.Solver(base_case)
    s.set_octree(BASE, np.asarray(leaves, np.int32))
    u = s.amr_adapt(to_dev(c0.u0), ind, CTRL)
    s.check()
    assert [tuple(r) for r in s.octree()] == order
    c = oracle_case(order)
    c.cfg = dict(c.cfg, eq=W.EQ_NS, mu=0.01)
    op = Operator(c.cfg, c.mesh)
    du = to_host(s.rhs(u))
    e_rhs = parity_err(du, op.rhs(ref), flux_scale(op, ref))
    dt = oracle_dt_ns(op, ref)
    s.ssprk3(u, dt, 10)
    s.check()
    got = to_host(u)
    s.close()
    r10, _ = ssprk.run(lambda v, t: op.rhs(v, t), ref, 0.0, dt, 10)
    e = rel_err(got, r10)
    print("NS on the adapted octree (%d elements, %d mortars): rhs parity %.3e, 10 steps %.3e"
          % (len(order), len(c.mesh.mortars), e_rhs, e))
    assert e_rhs < 1e-11 and e < 1e-11


def test_octree_and_adaptation_errors(dgx):
    """Rejected inputs leave the context usable: leaves that overlap, leave a
    hole, break the 2:1 balance or lie out of range; a bad controller or a
    non-finite indicator; apply without a plan."""
    import pytest as _pt
    leaves = uniform_leaves()
    s, _ = solver(dgx, leaves)
    split = [c for c in leaves if c != (0, 1, 1, 1)] + amr.children((0, 1, 1, 1))
    bad = {
        "overlap": leaves + [(1, 2, 2, 2)],
        "hole": leaves[1:],
        "duplicate": leaves + [leaves[0]],
        "out of range": leaves[:-1] + [(0, 4, 0, 0)],
        # a leaf split twice next to unsplit neighbours: 2:1 broken
        "unbalanced": [c for c in split if c != (1, 2, 2, 2)] + amr.children((1, 2, 2, 2)),
    }
    for name, lv in bad.items():
        with _pt.raises(dgx.DgxError) as ei:
            s.set_octree(BASE, np.asarray(lv, np.int32))
        assert ei.value.code == -1, name          # DGX_E_INVAL
    # the context still holds the last good octree
    assert len(s.octree()) == 64
    s.set_octree(BASE, np.asarray(split, np.int32))
    assert len(s.octree()) == 71
    ind = np.zeros(71)
    with _pt.raises(dgx.DgxError):
        dgx.dgx_amr_plan(s.ctx, ind, dict(CTRL, max_level=1, med_level=2))
    ind[3] = np.nan
    with _pt.raises(dgx.DgxError):
        dgx.dgx_amr_plan(s.ctx, ind, CTRL)
    import torch
    u = torch.zeros((5, 71, (N + 1) ** 3), dtype=torch.float64, device="cuda")
    with _pt.raises(dgx.DgxError) as ei:
        dgx.dgx_amr_apply(s.ctx, u, torch.empty_like(u))
    assert ei.value.code == -6                    # DGX_E_STATE
    s.close()


def test_finest_level(dgx):
    """An octree refined toward one corner down to the finest level (12,
    base 1, 540 leaves after 2:1 balancing): accepted, its right-hand side
    matches the oracle, and a plan that would split a level-12 leaf is
    rejected."""
    leaves = [(0, 0, 0, 0)]
    for _ in range(12):
        tgt = {c: (c[0] + 1 if c[1:] == (0, 0, 0) else c[0]) for c in leaves}
        new, _ = amr.adapt(1, leaves, tgt)
        leaves = sorted(new)
    c = W.case_amr(base=4, radii=(0.4,), centre=(0.5, 0.5, 0.5))
    s = dgx.Solver(c)
    order = [tuple(r) for r in s.set_octree(1, np.asarray(leaves, np.int32))]
    assert order == amr.morton_order(1, leaves) and max(o[0] for o in order) == 12
    x, faces, mortars, level = amr.mesh(1, N, order)
    cfg = W.base_cfg(3, N, W.EQ_EULER)
    mesh = W.Mesh(3, N, x, faces, np.zeros((0, 3), np.int32), mortars, np.zeros(0, np.int32),
                  np.zeros((0, 5)), level=level)
    u0 = W.blob_state(x, centre=(0.02, 0.03, 0.01), width=0.05)
    op = Operator(cfg, mesh)
    got = to_host(s.rhs(to_dev(u0)))
    s.check()
    e = parity_err(got, op.rhs(u0), flux_scale(op, u0))
    print("finest-level octree (%d elements, %d mortars): rhs parity %.3e" % (len(order), len(mortars), e))
    assert e < 1e-11
    # a controller beyond the finest level is rejected; at the finest level a
    # plan that keeps the level-12 leaves is accepted
    ind = np.where(np.array([o[0] for o in order]) == 12, 1.0, 0.0)
    with pytest.raises(dgx.DgxError) as ei:
        dgx.dgx_amr_plan(s.ctx, ind, dict(base_level=0, med_level=13, max_level=13, med_threshold=0.5,
                                          max_threshold=0.5))
    assert ei.value.code == -1                    # DGX_E_INVAL
    n = dgx.dgx_amr_plan(s.ctx, ind, dict(base_level=0, med_level=12, max_level=12, med_threshold=0.5,
                                          max_threshold=0.5))
    assert n > 0
    s.close()

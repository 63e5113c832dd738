"""The captured SSPRK3 step (dgx_ssprk3_step replays a HIP graph) against
the same step taken eagerly: three right-hand sides (dgx_rhs) combined on
the host side of the boundary with torch arithmetic, and the positivity
limiter (dgx_limit_positivity) after each stage when the case uses it.

One context replays its graph once per step, five times, with the eager
work and a device synchronisation between the replays; a second context
replays its graph five times back to back in one call.  The two must agree
bitwise (a replay computes what the first one did).  The graph and the
eager path differ in rounding only (the graph's stage update is fused into
the RHS kernel), and the flow amplifies rounding: the low-Mach TGV carries
its pressure as a small difference of large energies.  The scale of that
amplification is measured by a second eager path started from the state
perturbed in its last bits (seeded); the graph must stay within ten times
it at every step.  Each path has its own context with the same history
(the mixture temperature solves start from a node's previous T)."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle.thermo import Mixture
from tests.helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
STEPS = 5


@pytest.fixture(scope="module")
def dgx():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_17551_amd import dgx as mod
    return mod


def cases():
    mix = Mixture(W.Species())
    c3 = W.case_c3(lambda rs, T: mix.rho_e(rs, T), lambda rs, T: mix.rho_cv(rs, T), n=6)
    c3.cfg = dict(c3.cfg, positivity=True)
    return [("tgv_ns_8cube_N3", W.case_c2(n=8), 0.2), ("curved_air5_shock_6cube_N4_limiter", c3, 0.01)]


@pytest.mark.parametrize("which", [0, 1])
def test_graph_replays_match_eager_steps(dgx, which):
    import torch
    name, c, cfl = cases()[which]
    print("case", name, flush=True)
    lim = bool(c.cfg.get("positivity", False))
    sg, sb, se, sp = (dgx.Solver(c) for _ in range(4))
    ug, ub, ue = to_dev(c.u0), to_dev(c.u0), to_dev(c.u0)
    rng = np.random.default_rng(9)
    up = to_dev(c.u0 * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], c.u0.shape)))
    # the same call on every context: it also refreshes the per-node
    # temperatures that the mixture solves start from
    dt = dgx.dgx_max_dt(sg.ctx, ug, cfl)
    for s, v in ((sb, ub), (se, ue), (sp, up)):
        dgx.dgx_max_dt(s.ctx, v, cfl)
    du = torch.empty_like(ue)

    def eager_step(s, v):
        def stage(w):
            dgx.dgx_rhs(s.ctx, w, 0.0, du)
            return w + dt * du
        v1 = stage(v)
        if lim:
            dgx.dgx_limit_positivity(s.ctx, v1)
        v2 = 0.75 * v + 0.25 * stage(v1)
        if lim:
            dgx.dgx_limit_positivity(s.ctx, v2)
        v3 = v / 3.0 + (2.0 / 3.0) * stage(v2)
        if lim:
            dgx.dgx_limit_positivity(s.ctx, v3)
        return v3

    errs, scales = [], []
    for step in range(STEPS):
        sg.ssprk3(ug, dt, 1)
        ue = eager_step(se, ue)
        up = eager_step(sp, up)
        torch.cuda.synchronize()
        g, e, p = to_host(ug), to_host(ue), to_host(up)
        errs.append(rel_err(g, e))
        scales.append(rel_err(p, e))
        print("%s step %d: graph vs eager %.3e, eager vs perturbed eager %.3e" % (name, step, errs[-1], scales[-1]),
              flush=True)
    sb.ssprk3(ub, dt, STEPS)
    torch.cuda.synchronize()
    for s in (sg, sb, se, sp):
        s.check()
    back_to_back = to_host(ub)
    moved = rel_err(g, c.u0)
    for s in (sg, sb, se, sp):
        s.close()
    print("%s: %d replays, graph vs eager worst %.3e, perturbation scale worst %.3e, state moved %.3e"
          % (name, STEPS, max(errs), max(scales), moved))
    assert np.array_equal(back_to_back, g)
    assert moved > 1e-8
    for err, scale in zip(errs, scales):
        assert err <= 10.0 * scale + 1e-15

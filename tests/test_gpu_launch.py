"""The launch shape does not change the results: every elements-per-workgroup
choice that fits and both workgroup numberings (round-robin over the XCDs,
XCD-contiguous) give bitwise identical right-hand sides and SSPRK3 steps, on
the Navier-Stokes TGV (flat elements, BR1) and on the curved N=4 mixture
shock case (chunked work items, subcell FV, per-node temperature), and the
autotuner leaves a context that still reproduces them."""
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


def cases():
    mix = Mixture(W.Species())
    energy = lambda rs, T: mix.rho_e(rs, T)
    cv = lambda rs, T: mix.rho_cv(rs, T)
    c3 = W.case_c3(energy, cv, n=6)
    # species that start at zero density dip below it in a step without the
    # limiter (in the oracle too); stepped here with the positivity limiter
    c3.cfg = dict(c3.cfg, positivity=True)
    return [("tgv_ns_8cube_N3", W.case_c2(n=8)), ("curved_air5_shock_6cube_N4", c3)]


@pytest.mark.parametrize("which", [0, 1])
def test_launch_shape_is_bitwise_neutral(dgx, which):
    """Each launch configuration on a fresh context: mixture right-hand sides
    start their T(e) solves from the node's previous temperature, so only the
    same history gives the same last bits."""
    name, c = cases()[which]
    print("case", name, flush=True)
    ref = ref_step = None
    s = dgx.Solver(c)
    # the shock case is a right-hand-side workload: its steps here are
    # short, to exercise the graph path only
    dt = dgx.dgx_max_dt(s.ctx, to_dev(c.u0), 0.2 if which == 0 else 0.01)
    s.close()
    tried = 0
    for epb in (1, 2, 4, 8):
        for order in (0, 1):
            s = dgx.Solver(c)
            u = to_dev(c.u0)
            try:
                dgx.dgx_set_launch(s.ctx, epb, order)
            except dgx.DgxError:
                s.close()
                continue          # does not fit (threads or LDS)
            tried += 1
            du = to_host(s.rhs(u))
            s.ssprk3(u, dt, 2)
            step = to_host(u)
            s.check()
            s.close()
            if ref is None:
                ref, ref_step = du, step
            else:
                assert np.array_equal(du, ref), (name, epb, order)
                assert np.array_equal(step, ref_step), (name, epb, order)
    assert tried >= 4


def test_autotuned_context_reproduces(dgx):
    name, c = cases()[0]
    s = dgx.Solver(c)
    u = to_dev(c.u0)
    ref = to_host(s.rhs(u))
    dgx.dgx_autotune(s.ctx, u, reps=2)
    assert np.array_equal(to_host(s.rhs(u)), ref)
    s.check()
    s.close()

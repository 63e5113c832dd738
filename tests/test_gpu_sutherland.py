"""Sutherland viscosity (Eq. sutherland) on the GPU: the Navier-Stokes
Taylor-Green right-hand side, whose temperature varies from node to node,
with mu(T) = mu (T/T0)^(3/2) (T0 + S)/(T + S), against the oracle."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle import gas
from oracle.dgsem import Operator
from tests.helpers import flux_scale, parity_err, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dgx():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_17551_amd import dgx as mod
    return mod


def test_sutherland_rhs(dgx):
    c = W.case_c2(n=3)
    s = gas.pg_state(c.u0, 3, c.cfg["gamma"])
    T = s["p"] / (s["rho"] * c.cfg["R"])
    assert T.max() > 1.01 * T.min()
    c.cfg = dict(c.cfg, sutherland_S=0.4042 * T.mean(), sutherland_T0=T.mean())
    op = Operator(c.cfg, c.mesh)
    ref = op.rhs(c.u0)
    plain = Operator(dict(c.cfg, sutherland_S=0.0), c.mesh).rhs(c.u0)
    sol = dgx.Solver(c)
    got = to_host(sol.rhs(to_dev(c.u0)))
    sol.check()
    sol.close()
    scale = flux_scale(op, c.u0)
    e = parity_err(got, ref, scale)
    print("Sutherland TGV: parity %.3e (law changes the rhs by %.2e)" % (e, parity_err(plain, ref, scale)))
    assert e < 1e-11
    assert parity_err(plain, ref, scale) > 1e3 * e


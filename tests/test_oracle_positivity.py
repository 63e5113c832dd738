"""Pins of the oracle's Zhang-Shu limiter: element means unchanged,
admissible elements untouched, every node admissible afterwards, and each
element changed by one common scaling toward its mean."""
import numpy as np

from paper_2511_17551_amd import workloads as W
from oracle.dgsem import Operator
from oracle.positivity import limit, psi
from oracle.thermo import Mixture


def _mix_case():
    mix = Mixture(W.Species())
    return W.case_c4(lambda rs, T: mix.rho_e(rs, T), lambda rs, T: mix.rho_cv(rs, T), nr=4, nth=8, hot=True)


def test_limiter_properties_mixture():
    c = _mix_case()
    op = Operator(c.cfg, c.mesh, species=c.species, reactions=c.reactions)
    rng = np.random.default_rng(3)
    u = c.u0.copy()
    # push some nodes out of the admissible set: negative species and low energy
    for e in (1, 5, 9):
        u[3, e, rng.integers(0, 16, 3)] *= -0.2
        u[7, e, rng.integers(0, 16, 2)] *= 0.3
    wq = np.outer(op.b.w, op.b.w).reshape(-1)
    e0 = c.species.e0
    out, th = limit(u, op.J, wq, 2, e0)
    wJ = op.J * wq
    mean_in = (u * wJ).sum(2)
    mean_out = (out * wJ).sum(2)
    assert np.allclose(mean_out, mean_in, rtol=1e-13, atol=1e-13 * np.abs(mean_in).max())
    assert (out[:5] >= 0).all()
    rho_bar = mean_in[:5].sum(0) / wJ.sum(1)
    assert (psi(out, 2, e0) >= np.minimum(1e-13 * rho_bar * 1e5, psi((mean_in / wJ.sum(1))[:, :, None], 2, e0)[:, 0])[:, None] * (1 - 1e-12)).all()
    untouched = [k for k in range(u.shape[1]) if k not in (1, 5, 9)]
    assert np.array_equal(out[:, untouched], u[:, untouched])


def test_limiter_is_a_scaling_toward_the_mean():
    c = W.case_c1(n=4)
    op = Operator(c.cfg, c.mesh)
    u = c.u0.copy()
    u[0, 2, 5] = -0.2                     # negative density at one node
    wq = np.outer(op.b.w, op.b.w).reshape(-1)
    out, th = limit(u, op.J, wq, 2)
    wJ = op.J * wq
    ubar = (u * wJ).sum(2) / wJ.sum(1)
    d_in = u[1:, 2] - ubar[1:, 2][:, None]
    d_out = out[1:, 2] - ubar[1:, 2][:, None]
    ratio = d_out[np.abs(d_in) > 1e-12] / d_in[np.abs(d_in) > 1e-12]
    assert np.allclose(ratio, ratio[0], rtol=1e-12)
    assert out[0, 2].min() >= 0.0

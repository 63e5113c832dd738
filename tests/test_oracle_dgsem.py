"""Pins of the oracle's semi-discrete operator: free-stream, conservation,
entropy conservation, metric identities, convergence, viscous dissipation."""
import math

import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle import gas, ssprk
from oracle.dgsem import Operator
from oracle.geometry import tensor, flat, ref_deriv


def quad_weights(op):
    w = op.b.w
    if op.dim == 2:
        return np.outer(w, w).reshape(-1)
    return np.einsum("i,j,k->kji", w, w, w).reshape(-1)


def test_metric_identities_curved():
    c = W.curved_periodic_case(n=2, N=4)
    op = Operator(c.cfg, c.mesh)
    n1 = op.b.n1
    for comp in range(3):
        s = sum(ref_deriv(tensor(op.Ja[d, comp], 3, n1), op.b.D, d, 3) for d in range(3))
        assert np.abs(s).max() < 1e-13 * np.abs(op.Ja).max()


def _mapped_volume(lo, hi, amp, q=12):
    """Volume of the box [lo, hi] under the curved map x = X + amp s(X)(1,1,1),
    s = sin(pi X) sin(pi Y) sin(pi Z): Gauss-Legendre quadrature of the map's
    analytic Jacobian determinant 1 + amp (s_X + s_Y + s_Z)."""
    g, w = np.polynomial.legendre.leggauss(q)
    pts = [0.5 * (lo[d] + hi[d]) + 0.5 * (hi[d] - lo[d]) * g for d in range(3)]
    X, Y, Z = np.meshgrid(*pts, indexing="ij")
    p = math.pi
    det = 1.0 + amp * p * (np.cos(p * X) * np.sin(p * Y) * np.sin(p * Z)
                           + np.sin(p * X) * np.cos(p * Y) * np.sin(p * Z)
                           + np.sin(p * X) * np.sin(p * Y) * np.cos(p * Z))
    w3 = np.einsum("i,j,k->ijk", w, w, w) * np.prod([(hi[d] - lo[d]) / 2 for d in range(3)])
    return float((det * w3).sum())


@pytest.mark.parametrize("N", [3, 4])
def test_curved_jacobian_volumes(N):
    """Eq. jacobian on the curved map: the quadrature of J over each element is
    that element's volume under the analytic map (to the interpolation error of
    the map, converging at order >= N + 1), and the elements tile the unit cube
    (the map takes [0,1]^3 onto itself): sum_k sum_n w_n J_n = 1 to roundoff.
    The elements' volumes differ from the uniform 1/n^3 by up to 24%, so a
    wrong or dropped term in the determinant fails here."""
    errs = []
    for n in (2, 3):
        c = W.curved_periodic_case(n=n, N=N)
        op = Operator(c.cfg, c.mesh)
        vol = (op.J * quad_weights(op)).sum(1)
        assert abs(vol.sum() - 1.0) < 1e-14
        exact = []
        for e in range(n ** 3):
            i, j, k = e % n, (e // n) % n, e // (n * n)
            exact.append(_mapped_volume((i / n, j / n, k / n), ((i + 1) / n, (j + 1) / n, (k + 1) / n), 0.1))
        exact = np.array(exact)
        assert np.abs(exact * n ** 3 - 1.0).max() > 0.2
        errs.append(np.abs(vol - exact).max() * n ** 3)
    assert errs[0] < (2e-5 if N == 3 else 5e-8), errs
    assert errs[0] / errs[1] > 1.5 ** (N + 1), errs


@pytest.mark.parametrize("N", [3, 4])
def test_curved_metric_terms_against_the_map(N):
    """Eqs. mapped_equation, jacobian: the curl-form metric terms Ja^i (rows
    of the adjugate of dx/dxi) against the cofactors of the analytic map's
    Jacobian, (h/2)^2 (a_j x a_k) with a_d = dx/dX_d, at every node.  The
    curl form differentiates a degree-N interpolant, so its nodal error
    falls like h^N (asserted: EOC >= N - 0.2 on 4^3 -> 8^3); a wrong index,
    sign or cyclic order in the curl gives an O(1) error."""
    errs = []
    for n in (4, 8):
        c = W.curved_periodic_case(n=n, N=N)
        op = Operator(c.cfg, c.mesh)
        X = W.structured_mesh(3, N, (n,) * 3, (0.0,) * 3, (1.0,) * 3, (True,) * 3)[0]
        p, a, h = math.pi, 0.1, 1.0 / n
        g = a * p * np.array([np.cos(p * X[0]) * np.sin(p * X[1]) * np.sin(p * X[2]),
                              np.sin(p * X[0]) * np.cos(p * X[1]) * np.sin(p * X[2]),
                              np.sin(p * X[0]) * np.sin(p * X[1]) * np.cos(p * X[2])])
        A = np.array([[(1.0 if cc == d else 0.0) + g[d] for d in range(3)] for cc in range(3)]) * (h / 2)
        Ja = np.array([np.cross(A[:, (i + 1) % 3], A[:, (i + 2) % 3], axis=0) for i in range(3)])
        errs.append(np.abs(op.Ja - Ja).max() / np.abs(Ja).max())
    eoc = math.log2(errs[0] / errs[1])
    assert errs[1] < (1e-3 if N == 3 else 5e-5), errs
    assert eoc >= N - 0.2, (errs, eoc)


@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("N", [3, 4])
def test_freestream_curved(alpha, N):
    c = W.curved_periodic_case(n=2, N=N, shock=True, force_alpha=alpha)
    op = Operator(c.cfg, c.mesh)
    u = np.empty_like(c.u0)
    rho, v, p = 1.3, np.array([0.4, -0.7, 0.2]), 2.1
    u[0] = rho
    u[1:4] = (rho * v)[:, None, None]
    u[4] = p / 0.4 + 0.5 * rho * (v @ v)
    du = op.rhs(u)
    # per-variable scale S_v = max_n sum_d |f_v(u0)| |Ja^d_n| / J_n
    f = np.array([rho, rho * v[0] + p, rho * v[1] + p, rho * v[2] + p,
                  (u[4, 0, 0] + p)]) * np.abs(v).max()
    f[1:4] += p
    S = f * (sum(np.sqrt((op.Ja[d] ** 2).sum(0)) for d in range(3)) / op.J).max()
    assert np.all(np.abs(du).max(axis=(1, 2)) < 1e-12 * S)


@pytest.mark.parametrize("alpha", [0.0, 0.3, 1.0])
def test_conservation_curved(alpha):
    c = W.curved_periodic_case(n=2, N=3, shock=True, force_alpha=alpha)
    op = Operator(c.cfg, c.mesh)
    du = op.rhs(c.u0)
    wq = quad_weights(op)
    tot = (du * op.J[None] * wq).sum(axis=(1, 2))
    scale = np.abs(du * op.J[None] * wq).sum(axis=(1, 2))
    assert np.all(np.abs(tot) < 1e-13 * scale)


def test_entropy_conservation_ec_surface():
    for c in (W.case_c1(n=6, surface_flux=W.SF_RANOCHA),
              W.curved_periodic_case(n=2, N=3, surface_flux=W.SF_RANOCHA)):
        op = Operator(c.cfg, c.mesh)
        du = op.rhs(c.u0)
        s = gas.pg_state(c.u0, op.dim, 1.4)
        w = gas.entropy_variables(s)
        prod = w * du * op.J[None] * quad_weights(op)
        assert abs(prod.sum()) < 1e-13 * np.abs(prod).sum()


def test_entropy_dissipation_rusanov_and_fv():
    """Rusanov faces and the FV subcells only remove entropy (jumps make it strict)."""
    for alpha in (0.0, 1.0):
        c = W.curved_periodic_case(n=2, N=3, shock=True, force_alpha=alpha)
        op = Operator(c.cfg, c.mesh)
        rng = np.random.default_rng(5)
        u = c.u0 * (1.0 + 0.02 * rng.uniform(-1, 1, (1, c.u0.shape[1], 1)))
        du = op.rhs(u)
        w = gas.entropy_variables(gas.pg_state(u, 3, 1.4))
        prod = (w * du * op.J[None] * quad_weights(op)).sum()
        assert prod < -1e-6


def test_telescoped_equals_diagonal_free_split_form():
    """(Fbar_{n+1} - Fbar_n)/w_n == sum_{j != n} 2 D_nj F#(u_n, u_j)."""
    c = W.curved_periodic_case(n=2, N=4)
    op = Operator(c.cfg, c.mesh)
    s = gas.pg_state(c.u0, 3, 1.4)
    G = op.volume_terms(s, np.zeros(op.mesh.nelem))
    from oracle.geometry import line_view, line_unview
    n1 = op.b.n1
    ref = np.zeros_like(G)
    for d in range(3):
        sl = {k: (line_view(v, d, 3, n1) if isinstance(v, np.ndarray) else v) for k, v in s.items()}
        Jl = line_view(op.Ja[d], d, 3, n1)
        acc = np.zeros((5,) + Jl.shape[1:])
        for nn in range(n1):
            for j in range(n1):
                if j != nn:
                    f = gas.ranocha(gas.take(sl, nn), gas.take(sl, j), 0.5 * (Jl[..., nn] + Jl[..., j]))
                    acc[..., nn] += 2 * op.b.D[nn, j] * f
        ref += line_unview(acc, d, 3, n1)
    assert np.abs(G - ref).max() < 1e-12 * np.abs(ref).max()


def test_vortex_convergence():
    """Advected isentropic vortex: max error of rho falls faster than h^3 (N = 3)."""
    errs = []
    T = 0.2
    for n in (24, 48):
        c = W.case_c1(n=n, N=3, length=14.0)
        op = Operator(c.cfg, c.mesh)
        h = 14.0 / n
        steps = int(math.ceil(T / (0.01 * h)))
        dt = T / steps
        u, _ = ssprk.run(lambda v, t: op.rhs(v, t), c.u0, 0.0, dt, steps)
        rho, vel, p = W.isentropic_vortex(c.mesh.x[0] - T, c.mesh.x[1] - T, xc=7.0, yc=7.0)
        errs.append(np.abs(u[0] - rho).max())
    eoc = math.log(errs[0] / errs[1], 2)
    assert eoc > 3.0, (errs, eoc)


def test_tgv_initial_dissipation():
    """-dKE/dt(0) = mu <|omega|^2> = 3 mu / 4 for the TGV (closed form)."""
    c = W.case_c2(n=8)
    op = Operator(c.cfg, c.mesh)
    du = op.rhs(c.u0)
    u = c.u0
    v = u[1:4] / u[0]
    dke = (v * du[1:4]).sum(0) - 0.5 * (v * v).sum(0) * du[0]
    wq = quad_weights(op)
    rate = (dke * op.J * wq).sum() / (op.J * wq).sum()
    mu = c.cfg["mu"]
    assert abs(rate + 0.75 * mu) < 1e-5 * 0.75 * mu


def test_br1_uniform_flow_and_linear_gradient():
    c = W.case_c2(n=3)
    op = Operator(c.cfg, c.mesh)
    u = np.empty_like(c.u0)
    u[0] = 1.0
    u[1:4] = np.array([0.3, -0.2, 0.1])[:, None, None]
    u[4] = 50.0 + 0.5 * 0.14
    from oracle.br1 import viscous_rhs, gradients, primitives
    s = gas.pg_state(u, 3, 1.4)
    assert np.abs(viscous_rhs(op, u, s)).max() < 1e-12
    # gradient of a field that is periodic and degree <= N per element is exact:
    # a single Fourier mode is not, but its error must be small and shrink.
    x = c.mesh.x
    W_ = np.stack([np.sin(x[0]), np.cos(x[1]), np.sin(x[2]), np.cos(x[0] + x[1])])
    q = gradients(op, W_)
    exact = np.zeros_like(q)
    exact[0, 0] = np.cos(x[0])
    exact[1, 1] = -np.sin(x[1])
    exact[2, 2] = np.cos(x[2])
    exact[0, 3] = -np.sin(x[0] + x[1])
    exact[1, 3] = -np.sin(x[0] + x[1])
    assert np.abs(q - exact).max() < 0.1

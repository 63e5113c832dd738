"""BR1 viscous terms for the perfect-gas Navier-Stokes equations (oracle).

Test infrastructure: only the tests, the smoke check and the CPU baseline
of the benchmark use this package.

Paper: Sec. Methodology, Viscous Fluxes, Eqs. visfluxcalc, auxil,
auxstrongf (gradients of primitive variables as auxiliary unknowns, interface
value = arithmetic mean, averaged viscous interface flux); Governing
Equations, Eq. visc_fluxes; Appendix, Transport, Eq. stress (bulk
viscosity neglected); Sec. New Developments, parabolic solver on P4est
meshes (gradient and viscous-flux patching across interfaces and 1:2 / 1:4
mortars, interpolation to the small sides and L2 projection back);
Sec. Results, boundary conditions (weak boundaries; for the viscous terms
the external state is averaged with the interior one; no-slip adiabatic and
isothermal walls).

Readings:
* Eq. auxstrongf has the wrong sign on the boundary term; the strong form
  used is  Q = (1/J) sum_d Ja^d [ D_d W + M^{-1} B (W* - W) ]  with the
  nodal metric terms (curved elements included).
* Eq. visc_fluxes is inconsistent in sign between momentum and energy and
  uses q_1 in the third direction; the viscous flux used is
  F_v^c = (0, tau_{.c}, (tau v)_c - q_c), q = -kappa grad T, and the
  equation is du/dt = ... + div F_v.
* Primitive set W = (v, T) with T = p / (rho R); constant mu, or
  Sutherland's law mu(T) = mu (T/T0)^(3/2) (T0 + S)/(T + S) (Eq. sutherland)
  when sutherland_S > 0; Stokes hypothesis, kappa = mu gamma R / ((gamma -
  1) Pr).
* The divergence is taken in strong form with the averaged interface flux,
  one scaled normal per face (from the element on the face's minus side).
* Boundary faces: the interface value W* is the mean of W and the external
  state's primitives (Dirichlet: the boundary state; outflow: the interior
  state, so W* = W; slip wall: the mirrored velocity); at a no-slip wall
  W* = (0, T_wall) (isothermal, T_wall = bc_state[bc][0]) or (0, T)
  (adiabatic).  The viscous boundary flux is F_v(W*, Q).n with the
  interior gradient Q (viscosity at the temperature of W*); at an
  adiabatic wall its energy row is zero (no heat flux, no work).  At a
  slip wall this rule keeps the interior shear stress; no closed form pins
  it (parity unpinned there).
* Mortars: the large side's conserved trace is interpolated to each
  sub-face (the operators of oracle.mortar); there W* = (W_small +
  W(I_s u_large))/2, and the large side takes W*_L = sum_s (P_a x P_b) W*_s.
  The viscous sub-face flux is the mean of the small side's F_v.n_s and the
  interpolated Cartesian viscous flux of the large side contracted with the
  small side's normal n_s; the large side takes 2^(dim-1) sum_s (P_a x P_b)
  F*_s, as the advective mortar flux does.
"""
import numpy as np

from .geometry import tensor, flat, ref_deriv
from . import gas

BC_DIRICHLET, BC_OUTFLOW, BC_SLIPWALL, BC_WALL_ISOTHERMAL, BC_WALL_ADIABATIC = 0, 1, 2, 3, 4


def primitives(s, R):
    """W = (v_1..v_dim, T), shape (dim+1, ...)."""
    T = s["p"] / (s["rho"] * R)
    return np.concatenate([s["v"], T[None]], 0)


def _lift(arr, e, nodes, side, val, b):
    """Strong-form surface term at the nodes of one local face: + val / w_N on
    the xi_d = +1 face, - val / w_0 on the xi_d = -1 face."""
    sc = 1.0 / b.w[b.N] if side == 1 else -1.0 / b.w[0]
    np.add.at(arr, (slice(None), e, nodes), sc * val)


def _boundary_groups(op):
    """Boundary faces grouped by local face index and boundary index:
    yields (d, side, elements (m, 1), face nodes (1, nf), bc)."""
    bf = op.mesh.bfaces
    for f in range(2 * op.dim):
        rows = bf[bf[:, 1] == f]
        if len(rows) == 0:
            continue
        d, side = divmod(f, 2)
        nodes = op.fn[f]
        for bc in np.unique(rows[:, 2]):
            e = rows[rows[:, 2] == bc, 0]
            yield d, side, e[:, None], nodes[None, :], int(bc)


def boundary_value(op, u, s, W, d, e, nodes, bc):
    """W* at the nodes of boundary faces of one group, shape (nw, m, nf)."""
    mesh = op.mesh
    kind = int(mesh.bc_kind[bc])
    idx = (e, nodes)
    Wo = W[(slice(None),) + idx]
    if kind == BC_OUTFLOW:
        return Wo
    if kind in (BC_WALL_ISOTHERMAL, BC_WALL_ADIABATIC):
        Wb = np.zeros_like(Wo)
        Wb[op.dim] = mesh.bc_state[bc][0] if kind == BC_WALL_ISOTHERMAL else Wo[op.dim]
        return Wb
    ui = u[(slice(None),) + idx]
    si = gas.take(s, idx)
    n = op.Ja[d][(slice(None),) + idx]
    se = op.external_state(si, ui, kind, mesh.bc_state[bc], n, si.get("T"),
                           x_face=mesh.x[(slice(None),) + idx])
    return 0.5 * (Wo + primitives(se, op.cfg["R"]))


def _mortar_rows(op):
    from .mortar import operators, face_op
    nsub = 2 ** (op.dim - 1)
    Iops, Pops = operators(op.b)
    for row in op.mesh.mortars:
        eL, fL = int(row[0]), int(row[1])
        smalls = [int(v) for v in row[2:2 + nsub]]
        fS = int(row[2 + nsub])
        I = [face_op(Iops, s, op.dim) for s in range(nsub)]
        Pm = [face_op(Pops, s, op.dim) for s in range(nsub)]
        yield eL, fL, smalls, fS, I, Pm


def gradients(op, W, u=None, s=None):
    """q[c] = dW/dx_c at every node, shape (dim, nw, E, nn)."""
    b = op.b
    dim, N, n1 = op.dim, op.N, op.b.n1
    mesh = op.mesh
    nw = W.shape[0]
    # reference derivatives with the strong-form lifting of (W* - W)
    dref = []
    for d in range(dim):
        Wt = tensor(W, dim, n1)
        dW = flat(ref_deriv(Wt, b.D, d, dim), dim)
        dref.append(dW)
    for d in range(dim):
        sel = mesh.faces[mesh.faces[:, 1] == 2 * d + 1]
        eL, eR = sel[:, 0], sel[:, 2]
        nl, nr = op.fn[2 * d + 1], op.fn[2 * d]
        WL = W[:, eL[:, None], nl[None, :]]
        WR = W[:, eR[:, None], nr[None, :]]
        Ws = 0.5 * (WL + WR)
        _lift(dref[d], eL[:, None], nl[None, :], 1, Ws - WL, b)
        _lift(dref[d], eR[:, None], nr[None, :], 0, Ws - WR, b)
    for d, side, e, nodes, bc in _boundary_groups(op):
        Wb = boundary_value(op, u, s, W, d, e, nodes, bc)
        _lift(dref[d], e, nodes, side, Wb - W[:, e, nodes], b)
    if len(mesh.mortars):
        R, gam = op.cfg["R"], op.cfg["gamma"]
        for eL, fL, smalls, fS, I, Pm in _mortar_rows(op):
            d, sideL = divmod(fL, 2)
            nlf, nsf = op.fn[fL], op.fn[fS]
            uL = u[:, eL, nlf]
            WstarL = 0.0
            for k, es in enumerate(smalls):
                Wi = primitives(gas.pg_state(uL @ I[k].T, dim, gam), R)
                Wsm = W[:, es, nsf]
                Wst = 0.5 * (Wsm + Wi)
                _lift(dref[d], es, nsf, fS & 1, Wst - Wsm, b)
                WstarL = WstarL + Wst @ Pm[k].T
            _lift(dref[d], eL, nlf, sideL, WstarL - W[:, eL, nlf], b)
    q = np.zeros((dim, nw) + W.shape[1:], W.dtype)
    for c in range(dim):
        for d in range(dim):
            q[c] += op.Ja[d, c][None] * dref[d]
        q[c] /= op.J[None]
    return q


def viscous_flux_w(v, q, mu, kappa, dim, heat=True):
    """F_v^c for c = 1..dim, each (dim + 1, ...) (momentum and energy rows),
    with the velocity v of the work term and the gradients q."""
    gv = q[:, :dim]          # gv[c][k] = d v_k / d x_c
    gT = q[:, dim]
    div = sum(gv[k, k] for k in range(dim))
    out = []
    for c in range(dim):
        rows = []
        tau_c = []
        for k in range(dim):
            t = mu * (gv[c, k] + gv[k, c])
            if k == c:
                t = t - 2.0 / 3.0 * mu * div
            tau_c.append(t)
            rows.append(t)
        energy = sum(tau_c[k] * v[k] for k in range(dim))
        if heat:
            energy = energy + kappa * gT[c]
        rows.append(energy)
        out.append(np.stack(rows, 0))
    return out


def viscous_flux(s, q, mu, kappa, dim):
    """F_v^c for c = 1..dim, each (nvar, ...) (zero mass row)."""
    return [np.concatenate([np.zeros_like(f[:1]), f], 0) for f in viscous_flux_w(s["v"], q, mu, kappa, dim)]


def transport(cfg, T):
    """mu and kappa at temperature T (constant mu, or Sutherland's law)."""
    mu = cfg["mu"]
    if cfg.get("sutherland_S", 0.0) > 0.0:
        S, T0 = cfg["sutherland_S"], cfg["sutherland_T0"]
        mu = mu * (T / T0) ** 1.5 * (T0 + S) / (T + S)
    kappa = mu * cfg["gamma"] * cfg["R"] / ((cfg["gamma"] - 1.0) * cfg["Pr"])
    return mu, kappa


def viscous_rhs(op, u, s):
    cfg = op.cfg
    dim, N, n1 = op.dim, op.N, op.b.n1
    b = op.b
    mesh = op.mesh
    W = primitives(s, cfg["R"])
    mu, kappa = transport(cfg, W[dim])
    q = gradients(op, W, u, s)
    Fv = viscous_flux(s, q, mu, kappa, dim)            # list over c
    out = np.zeros_like(u)
    Ft = [sum(op.Ja[d, c][None] * Fv[c] for c in range(dim)) for d in range(dim)]   # contravariant
    div = [flat(ref_deriv(tensor(Ft[d], dim, n1), b.D, d, dim), dim) for d in range(dim)]
    for d in range(dim):
        sel = mesh.faces[mesh.faces[:, 1] == 2 * d + 1]
        eL, eR = sel[:, 0], sel[:, 2]
        nl, nr = op.fn[2 * d + 1], op.fn[2 * d]
        n = op.Ja[d][:, eL[:, None], nl[None, :]]
        FL = sum(Fv[c][:, eL[:, None], nl[None, :]] * n[c][None] for c in range(dim))
        FR = sum(Fv[c][:, eR[:, None], nr[None, :]] * n[c][None] for c in range(dim))
        Fstar = 0.5 * (FL + FR)
        _lift(div[d], eL[:, None], nl[None, :], 1, Fstar - Ft[d][:, eL[:, None], nl[None, :]], b)
        _lift(div[d], eR[:, None], nr[None, :], 0, Fstar - Ft[d][:, eR[:, None], nr[None, :]], b)
    for d, side, e, nodes, bc in _boundary_groups(op):
        idx = (e, nodes)
        Wb = boundary_value(op, u, s, W, d, e, nodes, bc)
        mub, kb = transport(cfg, Wb[dim])
        heat = int(mesh.bc_kind[bc]) != BC_WALL_ADIABATIC
        Fb = viscous_flux_w(Wb[:dim], q[(slice(None), slice(None)) + idx], mub, kb, dim, heat)
        n = op.Ja[d][(slice(None),) + idx]
        Fstar = sum(Fb[c] * n[c][None] for c in range(dim))
        Fstar = np.concatenate([np.zeros_like(Fstar[:1]), Fstar], 0)
        _lift(div[d], e, nodes, side, Fstar - Ft[d][(slice(None),) + idx], b)
    if len(mesh.mortars):
        nsub = 2 ** (dim - 1)
        for eL, fL, smalls, fS, I, Pm in _mortar_rows(op):
            d, sideL = divmod(fL, 2)
            nlf, nsf = op.fn[fL], op.fn[fS]
            FstarL = 0.0
            for k, es in enumerate(smalls):
                n = op.Ja[d][:, es, nsf]                      # small element's normal
                Fs = sum(Fv[c][:, es, nsf] * n[c][None] for c in range(dim))
                Fi = sum((Fv[c][:, eL, nlf] @ I[k].T) * n[c][None] for c in range(dim))
                Fst = 0.5 * (Fs + Fi)
                _lift(div[d], es, nsf, fS & 1, Fst - Ft[d][:, es, nsf], b)
                FstarL = FstarL + nsub * (Fst @ Pm[k].T)
            _lift(div[d], eL, nlf, sideL, FstarL - Ft[d][:, eL, nlf], b)
    for d in range(dim):
        out += div[d]
    return out / op.J[None]

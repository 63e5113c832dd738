"""BR1 viscous terms for the perfect-gas Navier-Stokes equations (oracle).

Paper: Sec. Methodology, Viscous Fluxes, Eqs. visfluxcalc, auxil,
auxstrongf (gradients of primitive variables as auxiliary unknowns, interface
value = arithmetic mean, averaged viscous interface flux); Governing
Equations, Eq. visc_fluxes; Appendix, Transport, Eq. stress (bulk
viscosity neglected).

Readings:
* Eq. auxstrongf has the wrong sign on the boundary term; the strong form
  used is  Q = (1/J) sum_d Ja^d [ D_d W + M^{-1} B (W* - W) ]  (affine
  elements: Ja^d constant per element).
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
"""
import numpy as np

from .geometry import tensor, flat, ref_deriv


def primitives(s, R):
    """W = (v_1..v_dim, T), shape (dim+1, E, nn)."""
    T = s["p"] / (s["rho"] * R)
    return np.concatenate([s["v"], T[None]], 0)


def gradients(op, W):
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
        np.add.at(dref[d], (slice(None), eL[:, None], nl[None, :]), (Ws - WL) / b.w[N])
        np.add.at(dref[d], (slice(None), eR[:, None], nr[None, :]), -(Ws - WR) / b.w[0])
    if len(mesh.bfaces):
        raise NotImplementedError("BR1 boundary conditions are not part of this operator")
    q = np.zeros((dim, nw) + W.shape[1:], W.dtype)
    for c in range(dim):
        for d in range(dim):
            q[c] += op.Ja[d, c][None] * dref[d]
        q[c] /= op.J[None]
    return q


def viscous_flux(s, q, mu, kappa, dim):
    """F_v^c for c = 1..dim, each (nvar, ...)."""
    gv = q[:, :dim]          # gv[c][k] = d v_k / d x_c
    gT = q[:, dim]
    div = sum(gv[k, k] for k in range(dim))
    out = []
    for c in range(dim):
        rows = [np.zeros_like(div)]
        tau_c = []
        for k in range(dim):
            t = mu * (gv[c, k] + gv[k, c])
            if k == c:
                t = t - 2.0 / 3.0 * mu * div
            tau_c.append(t)
            rows.append(t)
        energy = sum(tau_c[k] * s["v"][k] for k in range(dim)) + kappa * gT[c]
        rows.append(energy)
        out.append(np.stack(rows, 0))
    return out


def viscous_rhs(op, u, s):
    cfg = op.cfg
    dim, N, n1 = op.dim, op.N, op.b.n1
    b = op.b
    mesh = op.mesh
    R = cfg["R"]
    W = primitives(s, R)
    mu = cfg["mu"]
    if cfg.get("sutherland_S", 0.0) > 0.0:
        # Sutherland's law (Eq. sutherland), node by node
        S, T0 = cfg["sutherland_S"], cfg["sutherland_T0"]
        T = W[dim]
        mu = mu * (T / T0) ** 1.5 * (T0 + S) / (T + S)
    kappa = mu * cfg["gamma"] * R / ((cfg["gamma"] - 1.0) * cfg["Pr"])
    q = gradients(op, W)
    Fv = viscous_flux(s, q, mu, kappa, dim)            # list over c
    out = np.zeros_like(u)
    for d in range(dim):
        Ft = sum(op.Ja[d, c][None] * Fv[c] for c in range(dim))   # contravariant
        div = flat(ref_deriv(tensor(Ft, dim, n1), b.D, d, dim), dim)
        sel = mesh.faces[mesh.faces[:, 1] == 2 * d + 1]
        eL, eR = sel[:, 0], sel[:, 2]
        nl, nr = op.fn[2 * d + 1], op.fn[2 * d]
        n = op.Ja[d][:, eL[:, None], nl[None, :]]
        FL = sum(Fv[c][:, eL[:, None], nl[None, :]] * n[c][None] for c in range(dim))
        FR = sum(Fv[c][:, eR[:, None], nr[None, :]] * n[c][None] for c in range(dim))
        Fstar = 0.5 * (FL + FR)
        FLown = Ft[:, eL[:, None], nl[None, :]]
        FRown = Ft[:, eR[:, None], nr[None, :]]
        np.add.at(div, (slice(None), eL[:, None], nl[None, :]), (Fstar - FLown) / b.w[N])
        np.add.at(div, (slice(None), eR[:, None], nr[None, :]), -(Fstar - FRown) / b.w[0])
        out += div
    return out / op.J[None]

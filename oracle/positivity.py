"""Zhang-Shu positivity-preserving scaling limiter (oracle).

Paper: Sec. Results (blast wave, supersonic TGV, P8 inlet): the scheme of
Zhang and Shu weakly enforces positive species densities and pressure.

Per element, with the quadrature mean  u_bar = sum_n J_n w_n u_n / sum_n J_n w_n
(w_n the tensor LGL weights):

1. densities: for every species (the total density for a perfect gas) with
   nodal minimum m below eps_rho, scale that variable toward its mean,
   rho_n <- rho_bar + theta (rho_n - rho_bar), theta = (rho_bar - eps_rho) / (rho_bar - m);
2. pressure: psi(u) = rho E - |m|^2 / (2 rho) - sum_s rho_s e0_s (the internal
   energy above the T -> 0 limit; psi > 0 <=> p > 0, concave in u).  For each
   node with psi(u_n) < eps_p, t_n is the largest t in [0, 1] with
   psi(u_bar + t (u_n - u_bar)) >= eps_p, found by 64 bisection steps; then
   u_n <- u_bar + theta_p (u_n - u_bar) with theta_p = min_n t_n.

Readings (the paper gives no parameters): eps_rho = 1e-14 rho_s_bar for the
species of a mixture (absent species are admissible; the small margin keeps
the scaled minimum non-negative after rounding), min(1e-13, rho_bar) for a
perfect gas; eps_p = min(1e-13 * rho_bar * c_scale, psi(u_bar)) with c_scale = 1 for
the perfect gas and 1e5 (J/kg) for the mixture; an element whose mean is
itself inadmissible is left unchanged.
"""
import numpy as np


def psi(u, dim, e0=None):
    if e0 is None:
        rho = u[0]
        m = u[1:1 + dim]
        E = u[1 + dim]
        return E - 0.5 * np.sum(m * m, axis=0) / rho
    rs = u[:5]
    rho = rs.sum(0)
    m = u[5:5 + dim]
    E = u[5 + dim]
    return E - 0.5 * np.sum(m * m, axis=0) / rho - np.tensordot(e0, rs, axes=(0, 0))


def limit(u, J, wq, dim, e0=None):
    """Return the limited copy of u (nvar, E, nn) and the per-element thetas."""
    u = u.copy()
    mix = e0 is not None
    wJ = J * wq[None, :]
    vol = wJ.sum(1)
    ubar = (u * wJ[None]).sum(2) / vol[None]            # (nvar, E)
    dens = range(5) if mix else [0]
    for s in dens:
        eps = 1e-14 * np.maximum(ubar[s], 0.0) if mix else np.minimum(1e-13, ubar[s])
        mn = u[s].min(1)
        bad = (mn < eps) & (ubar[s] > eps)
        theta = np.where(bad, (ubar[s] - eps) / np.where(bad, ubar[s] - mn, 1.0), 1.0)
        k = np.flatnonzero(bad)
        u[s, k] = ubar[s, k][:, None] + theta[k][:, None] * (u[s, k] - ubar[s, k][:, None])
    rho_bar = ubar[:5].sum(0) if mix else ubar[0]
    pb = psi(ubar[:, :, None], dim, e0)[:, 0]
    eps_p = np.minimum(1e-13 * rho_bar * (1e5 if mix else 1.0), pb)
    pn = psi(u, dim, e0)
    E = u.shape[1]
    theta_p = np.ones(E)
    for k in range(E):
        if pb[k] <= 0 or not np.any(pn[k] < eps_p[k]):
            continue
        tmin = 1.0
        for n in np.flatnonzero(pn[k] < eps_p[k]):
            d = u[:, k, n] - ubar[:, k]
            lo, hi = 0.0, 1.0
            for _ in range(64):
                mid = 0.5 * (lo + hi)
                if psi((ubar[:, k] + mid * d)[:, None], dim, e0)[0] >= eps_p[k]:
                    lo = mid
                else:
                    hi = mid
            tmin = min(tmin, lo)
        theta_p[k] = tmin
        u[:, k] = ubar[:, k][:, None] + tmin * (u[:, k] - ubar[:, k][:, None])
    return u, theta_p

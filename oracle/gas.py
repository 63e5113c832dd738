"""Advective fluxes, two-point volume fluxes and Riemann fluxes (oracle).

Paper: Sec. Governing Equations, Eq. adevctive_flux (physical flux),
Sec. Methodology, Eqs. riemann_problem1-3 (interface Riemann flux, Lax-
Friedrichs named), Eqs. fluxdiff/fluxdiffcons/conssymm (symmetric,
consistent two-point fluxes: entropy-conservative or the Ducros split form).

A state is a dict with 'rho' (total density), 'rs' (species densities, mixture
only), 'v' (dim, ...), 'p', 'rhoE', 'c' (sound speed) and, for the perfect
gas, 'gamma'.  Conserved layout: (rho | rho_1..rho_5, rho v_1..rho v_dim,
rho E).  Normal vectors are scaled (not unit) and have shape (dim, ...).

Readings where the paper is silent:
* the entropy-conservative flux for the perfect gas is Ranocha's
  (ln-mean of rho and rho/p, with the small-difference series of the
  logarithmic mean);
* the Lax-Friedrichs (Rusanov) dissipation uses the Davis estimate
  max(|v_L.n| + c_L|n|, |v_R.n| + c_R|n|).
"""
import numpy as np


def pg_state(u, dim, gamma):
    """Perfect-gas primitives from conserved u (nvar, ...)."""
    rho = u[0]
    v = u[1:1 + dim] / rho
    rhoE = u[1 + dim]
    p = (gamma - 1.0) * (rhoE - 0.5 * rho * np.sum(v * v, axis=0))
    c = np.sqrt(gamma * p / rho)
    return dict(rho=rho, v=v, p=p, rhoE=rhoE, c=c, gamma=gamma, mix=False)


def dot(a, b):
    return np.sum(a * b, axis=0)


def physical_flux(s, n):
    """f(u).n for the Euler equations (perfect gas or mixture)."""
    vn = dot(s["v"], n)
    rows = []
    if s["mix"]:
        rows += [rs * vn for rs in s["rs"]]
    else:
        rows.append(s["rho"] * vn)
    for c in range(s["v"].shape[0]):
        rows.append(s["rho"] * s["v"][c] * vn + s["p"] * n[c])
    rows.append((s["rhoE"] + s["p"]) * vn)
    return np.stack(rows, 0)


def conserved(s):
    rows = list(s["rs"]) if s["mix"] else [s["rho"]]
    rows += [s["rho"] * s["v"][c] for c in range(s["v"].shape[0])]
    rows.append(s["rhoE"])
    return np.stack(rows, 0)


def rusanov(sL, sR, n):
    """Local Lax-Friedrichs flux  1/2 (f_L + f_R).n - 1/2 lambda (u_R - u_L)."""
    nn = np.sqrt(dot(n, n))
    lam = np.maximum(np.abs(dot(sL["v"], n)) + sL["c"] * nn,
                     np.abs(dot(sR["v"], n)) + sR["c"] * nn)
    return 0.5 * (physical_flux(sL, n) + physical_flux(sR, n)) \
        - 0.5 * lam * (conserved(sR) - conserved(sL))


def ln_mean(x, y):
    """Logarithmic mean (y - x)/ln(y/x) with the series for nearby arguments."""
    z = (x * (x - 2.0 * y) + y * y) / (x * (x + 2.0 * y) + y * y)
    small = z < 1e-4
    with np.errstate(divide="ignore", invalid="ignore"):
        big = (y - x) / np.log(y / x)
    ser = (x + y) / (2.0 + z * (2.0 / 3.0 + z * (2.0 / 5.0 + 2.0 / 7.0 * z)))
    return np.where(small, ser, big)


def ranocha(sL, sR, n):
    """Entropy-conservative, kinetic-energy-preserving two-point flux (perfect gas)."""
    g = sL["gamma"]
    rho_hat = ln_mean(sL["rho"], sR["rho"])
    beta_hat = ln_mean(sL["rho"] / sL["p"], sR["rho"] / sR["p"])
    vbar = 0.5 * (sL["v"] + sR["v"])
    pbar = 0.5 * (sL["p"] + sR["p"])
    q = 0.5 * dot(sL["v"], sR["v"])
    f_rho = rho_hat * dot(vbar, n)
    rows = [f_rho]
    for c in range(vbar.shape[0]):
        rows.append(f_rho * vbar[c] + pbar * n[c])
    rows.append(f_rho * (q + 1.0 / ((g - 1.0) * beta_hat))
                + 0.5 * (sL["p"] * dot(sR["v"], n) + sR["p"] * dot(sL["v"], n)))
    return np.stack(rows, 0)


def ducros(sL, sR, n):
    """Ducros et al. split-form two-point flux (perfect gas or mixture)."""
    vn = dot(0.5 * (sL["v"] + sR["v"]), n)
    pbar = 0.5 * (sL["p"] + sR["p"])
    rows = []
    if sL["mix"]:
        rows += [0.5 * (a + b) * vn for a, b in zip(sL["rs"], sR["rs"])]
    else:
        rows.append(0.5 * (sL["rho"] + sR["rho"]) * vn)
    for c in range(sL["v"].shape[0]):
        mbar = 0.5 * (sL["rho"] * sL["v"][c] + sR["rho"] * sR["v"][c])
        rows.append(mbar * vn + pbar * n[c])
    rows.append((0.5 * (sL["rhoE"] + sR["rhoE"]) + pbar) * vn)
    return np.stack(rows, 0)


def entropy_variables(s):
    """w = dU/du for U = -rho s/(gamma-1), s = ln p - gamma ln rho."""
    g = s["gamma"]
    beta = s["rho"] / s["p"]
    ent = np.log(s["p"]) - g * np.log(s["rho"])
    v2 = dot(s["v"], s["v"])
    rows = [(g - ent) / (g - 1.0) - 0.5 * beta * v2]
    rows += [beta * s["v"][c] for c in range(s["v"].shape[0])]
    rows.append(-beta)
    return np.stack(rows, 0)


def entropy_potential(s, n):
    """psi = rho v.n, the flux potential of the Tadmor condition."""
    return s["rho"] * dot(s["v"], n)


def take(s, idx):
    """Sub-state s[..., idx] (fancy index along the trailing axes)."""
    out = {}
    for k, val in s.items():
        if isinstance(val, np.ndarray):
            out[k] = val[(Ellipsis,) + idx] if isinstance(idx, tuple) else val[..., idx]
        else:
            out[k] = val
    return out

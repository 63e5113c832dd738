"""Per-node stiff chemistry: one backward-Euler step of the species sources
at fixed internal energy (oracle).

Test infrastructure only: the library does not import this module.

Paper: Governing Equations, Eq. source_term (the species sources, with the
transport terms split off); Appendix, Chemical Kinetics (the rates).  The
paper integrates the sources inside its explicit schemes and warns that the
iterative thermochemistry is the overhead risk of a reacting step
(Introduction); it gives no implicit treatment.  Reading: the stiff sources
are integrated per node by operator splitting, one backward-Euler step over
dt on the species densities while rho, momentum and total energy stay
fixed (so rho e = rho E - |m|^2 / (2 rho) is fixed as well):

    G(rho_s) = rho_s - rho_s^n - dt * omega_s(rho_s, T(rho_s, rho e)) = 0.

The reactions conserve mass, so sum_s omega_s = 0 and the step keeps
rho = sum_s rho_s.  The root is found by Newton's method with a
central-difference Jacobian (columns scaled to the node's density), a step
restricted so that no density becomes negative and the thermal energy
rho e - sum_s rho_s e0_s stays positive (else no temperature exists), and
the stop max_s |delta_s| <= tol * rho on the full Newton step.  The Jacobian only steers the iteration; the
root is what both implementations must agree on.
"""
import numpy as np


def residual(mix, kin, rs, rs0, rhoe, dt, Tg):
    """G(rs) and the temperature it used, per node (rs: (ns, n))."""
    T, _ = mix.solve_T(rs, rhoe, Tg, tol=1e-14, maxit=100)
    return rs - rs0 - dt * kin.omega_dot(rs, T), T


def backward_euler(mix, kin, rs0, rhoe, dt, T0, tol=1e-13, maxit=100):
    """One implicit step for every node.  rs0: (ns, n); rhoe, T0: (n,).

    Returns (rs, T, iterations).  Raises if a node does not converge.
    """
    ns, n = rs0.shape
    rs = rs0.copy()
    rho = rs0.sum(0)
    T = np.array(np.broadcast_to(T0, (n,)), float)
    it = np.zeros(n, np.int64)
    active = np.ones(n, bool)
    for _ in range(maxit):
        if not active.any():
            break
        idx = np.flatnonzero(active)
        ra, r0, ea, Ta, rhoa = rs[:, idx], rs0[:, idx], rhoe[idx], T[idx], rho[idx]
        G, Ta = residual(mix, kin, ra, r0, ea, dt, Ta)
        # central-difference Jacobian, column k: dG/drho_k
        h = 1e-7 * rhoa
        Jm = np.empty((len(idx), ns, ns))
        for k in range(ns):
            up = ra.copy()
            dn = ra.copy()
            up[k] += h
            dn[k] -= h
            Gp, _ = residual(mix, kin, up, r0, ea, dt, Ta)
            Gm, _ = residual(mix, kin, dn, r0, ea, dt, Ta)
            Jm[:, :, k] = ((Gp - Gm) / (2.0 * h)).T
        delta = -np.linalg.solve(Jm, G.T[:, :, None])[:, :, 0].T
        # keep every density non-negative, and keep a positive thermal
        # energy rho e - sum_s rho_s e0_s (at or below zero no T exists)
        theta = np.ones(len(idx))
        neg = ra + delta < 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            lim = np.where(neg, -0.9 * ra / delta, np.inf)
            e0 = mix.e0[:, None]
            thermal = ea - (ra * e0).sum(0)
            de0 = (delta * e0).sum(0)
            lim_e = np.where(de0 > 0.0, 0.9 * thermal / de0, np.inf)
        theta = np.minimum(np.minimum(theta, lim.min(0)), lim_e)
        rs[:, idx] = ra + theta * delta
        T[idx] = Ta
        it[idx] += 1
        # converged when the full (undamped) Newton step is below tolerance
        done = np.max(np.abs(delta), axis=0) <= tol * rhoa
        active[idx[done]] = False
    if active.any():
        raise RuntimeError("backward-Euler chemistry did not converge")
    T, _ = mix.solve_T(rs, rhoe, T, tol=1e-14, maxit=100)
    return rs, T, it

"""Per-node stiff chemistry: backward-Euler steps of the species sources at
fixed internal energy (oracle).

Test infrastructure only: the library does not import this module.

Paper: Governing Equations, Eq. source_term (the species sources, with the
transport terms split off); Appendix, Chemical Kinetics (the rates).  The
paper integrates the sources inside its explicit schemes and warns that the
iterative thermochemistry is the overhead risk of a reacting step
(Introduction); it gives no implicit treatment.  Reading: the stiff sources
are integrated per node by operator splitting, backward Euler on the species
densities while rho, momentum and total energy stay fixed (so
rho e = rho E - |m|^2 / (2 rho) is fixed as well).  One backward-Euler step
over h from rho_s^a solves

    G(rho_s) = rho_s - rho_s^a - h * omega_s(rho_s, T(rho_s, rho e)) = 0.

The reactions conserve mass, so sum_s omega_s = 0 and the step keeps
rho = sum_s rho_s.  The root is found by Newton's method with a
central-difference Jacobian (steps of 1e-7 rho, cut where the thermal energy
could not pay for the perturbed formation energy), a step
restricted so that no density becomes negative and the thermal energy
rho e - sum_s rho_s e0_s stays positive (else no temperature exists), and
the stop max_s |delta_s| <= tol * rho on the full Newton step.  An iterate
whose temperature solve fails ends the iteration as failed.  The Jacobian
only steers the iteration; the root is what both implementations must agree
on.

Substeps.  A mode that grows (atom-impact dissociation makes [X] grow at a
rate k [X2]) turns the step's Jacobian singular as h times the growth rate
reaches 1; beyond that the root near rho^a is gone and the Newton step
points out of the admissible set, so the positivity limit shrinks it to
nothing.  Such a Newton iteration is declared failed when the limit cuts the
step to below STALL of its length on two consecutive iterations, or after
maxit iterations, and the node then covers the step with backward-Euler
substeps of dt / 2^k: a failed substep is retried at half the size, and
after a successful one the node returns to the next larger size when its
position in the step is a multiple of it.  Positions are kept as integers in
units of dt / 2^KMAX; a node that fails at the smallest size does not
converge.  Where the single step converges (the usual case) the result is
that step's root.

Rounding.  Far from equilibrium a Newton iteration can wander for tens of
iterations before it converges; its path then depends on rounding (of the
Jacobian above all), and so may whether it lands within maxit.  Two
implementations of this procedure can therefore take different substep
sequences at such a node: both results are backward-Euler integrations over
dt, they differ by the substeps' truncation error, and both keep every
invariant.
"""
import numpy as np

KMAX = 20      # smallest substep dt / 2^20
STALL = 1e-3   # a step cut below this fraction twice in a row has failed


def residual(mix, kin, rs, rs0, rhoe, dt, Tg, strict=True):
    """G(rs) and the temperature it used, per node (rs: (ns, n); dt scalar or
    per node).  A node whose T(e) solve fails raises, or with strict=False
    gets NaN."""
    T, _ = mix.solve_T(rs, rhoe, Tg, tol=1e-14, maxit=100, strict=strict)
    with np.errstate(invalid="ignore"):
        return rs - rs0 - dt * kin.omega_dot(rs, T), T


def newton(mix, kin, rs0, rhoe, dt, T0, tol=1e-13, maxit=50):
    """Damped Newton for one backward-Euler step per node (dt: (n,)).

    Returns (rs, T, iterations, converged); nodes that stall or run out of
    iterations are reported as not converged (their rs is meaningless).
    """
    ns, n = rs0.shape
    rs = rs0.copy()
    rho = rs0.sum(0)
    T = np.array(np.broadcast_to(T0, (n,)), float)
    it = np.zeros(n, np.int64)
    low = np.zeros(n, np.int64)
    ok = np.zeros(n, bool)
    active = np.ones(n, bool)
    for _ in range(maxit):
        if not active.any():
            break
        idx = np.flatnonzero(active)
        ra, r0, ea, Ta, rhoa, dta = rs[:, idx], rs0[:, idx], rhoe[idx], T[idx], rho[idx], dt[idx]
        G, Ta = residual(mix, kin, ra, r0, ea, dta, Ta, strict=False)
        # central-difference Jacobian, column k: dG/drho_k; the perturbation
        # is 1e-7 rho, cut to a quarter of the thermal energy over e0_k so
        # that the perturbed state still has a temperature
        thermal0 = ea - (ra * mix.e0[:, None]).sum(0)
        Jm = np.empty((len(idx), ns, ns))
        for k in range(ns):
            h = 1e-7 * rhoa
            if mix.e0[k] > 0.0:
                h = np.minimum(h, 0.25 * thermal0 / mix.e0[k])
            up = ra.copy()
            dn = ra.copy()
            up[k] += h
            dn[k] -= h
            Gp, _ = residual(mix, kin, up, r0, ea, dta, Ta, strict=False)
            Gm, _ = residual(mix, kin, dn, r0, ea, dta, Ta, strict=False)
            Jm[:, :, k] = ((Gp - Gm) / (2.0 * h)).T
        # an iterate without a temperature (its T(e) solve failed) ends that
        # node's iteration as failed
        nan = ~(np.isfinite(Jm).all((1, 2)) & np.isfinite(G).all(0))
        Jm[nan] = np.eye(ns)
        G = np.where(nan[None], 0.0, G)
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
        done = (np.max(np.abs(delta), axis=0) <= tol * rhoa) & ~nan
        low[idx] = np.where(theta < STALL, low[idx] + 1, 0)
        stalled = nan | (~done & (low[idx] >= 2))
        ok[idx[done]] = True
        active[idx[done | stalled]] = False
    T[ok], _ = mix.solve_T(rs[:, ok], rhoe[ok], T[ok], tol=1e-14, maxit=100)
    return rs, T, it, ok


def backward_euler(mix, kin, rs0, rhoe, dt, T0, tol=1e-13, maxit=50):
    """Chemistry over dt for every node.  rs0: (ns, n); rhoe, T0: (n,).

    Returns (rs, T, iterations, substeps): the Newton iterations summed over
    a node's substeps and its number of substeps (1 where the single step
    converged).  Raises if a node fails at the smallest substep.
    """
    ns, n = rs0.shape
    unit = 1 << KMAX
    pos = np.zeros(n, np.int64)
    lev = np.zeros(n, np.int64)
    rs = rs0.copy()
    T = np.array(np.broadcast_to(T0, (n,)), float)
    its = np.zeros(n, np.int64)
    nsub = np.zeros(n, np.int64)
    while True:
        act = np.flatnonzero(pos < unit)
        if len(act) == 0:
            break
        if np.any(lev[act] > KMAX):
            raise RuntimeError("backward-Euler chemistry did not converge")
        h = dt * np.ldexp(1.0, -lev[act].astype(np.int32))
        r1, T1, it, ok = newton(mix, kin, rs[:, act], rhoe[act], h, T[act], tol, maxit)
        its[act] += it
        good = act[ok]
        rs[:, good] = r1[:, ok]
        T[good] = T1[ok]
        pos[good] += unit >> lev[good]
        nsub[good] += 1
        # back to the next larger substep once the position is a multiple of it
        up = (lev[good] > 0) & (pos[good] % (unit >> np.maximum(lev[good] - 1, 0)) == 0)
        lev[good[up]] -= 1
        lev[act[~ok]] += 1
    return rs, T, its, nsub

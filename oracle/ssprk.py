"""Three-stage, third-order strong-stability-preserving Runge-Kutta (oracle).

The paper integrates with SSPRK43 and other explicit schemes (Sec. Results);
the workloads fix the Shu-Osher SSPRK3 at a constant time step:

  u1 = u + dt L(u, t)
  u2 = 3/4 u + 1/4 (u1 + dt L(u1, t + dt))
  u  = 1/3 u + 2/3 (u2 + dt L(u2, t + dt/2))
"""


def step(L, u, t, dt, limiter=None):
    """One step; ``limiter`` (optional) is applied to every stage value."""
    lim = limiter if limiter is not None else (lambda v: v)
    u1 = lim(u + dt * L(u, t))
    u2 = lim(0.75 * u + 0.25 * (u1 + dt * L(u1, t + dt)))
    return lim(u / 3.0 + 2.0 / 3.0 * (u2 + dt * L(u2, t + 0.5 * dt)))


def run(L, u, t, dt, nsteps, limiter=None):
    for _ in range(nsteps):
        u = step(L, u, t, dt, limiter)
        t += dt
    return u, t

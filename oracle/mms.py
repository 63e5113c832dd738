"""Manufactured solution for the operator's order of accuracy (oracle).

Paper: Sec. Governing Equations, Eq. system_equation: dU/dt + div F(U) = S
on the domain, U = Phi on its boundary.  Choosing a smooth steady U(x) and
setting S = div F(U) makes U an exact solution of the forced system with
Dirichlet data Phi = U on the boundary; the discrete solution of the DGSEM
of degree N then converges to it at order N + 1.

The source is derived symbolically (SymPy) from the primitive fields below
and turned into NumPy functions; no part of the discretisation is involved,
so this module checks the operator from outside.  The solution is steady so
that the time integrator's accuracy and the order reduction of Runge-Kutta
stages under time-dependent boundary data play no part: only the spatial
discretisation is measured.

Primitive fields on the unit cube, a quarter wave in each direction, every
component non-constant and every direction varying (a wrong metric term,
Jacobian, index or sign in any direction shows up as an error that does not
converge):
  rho = 2 + (sin(k (x + 0.3)) + cos(k (y + 0.2)) + sin(k (z + 0.1))) / 10
  v1  = 0.6 + cos(k (y + 0.2)) / 10
  v2  = 0.4 + sin(k (z + 0.1)) / 10
  v3  = 0.3 + cos(k (x + 0.3)) / 10
  p   = 1.5 + (sin(k (x + 0.3)) + cos(k (z + 0.1))) / 10,   k = pi / 2,
with the perfect-gas energy rho E = p / (gamma - 1) + rho |v|^2 / 2.
"""
import functools

import numpy as np


@functools.lru_cache(maxsize=4)
def euler3d_steady(gamma=1.4):
    """(u_exact(x, y, z), source(x, y, z)) for the 3D Euler equations, each
    returning an array (5, ...) in the conserved layout
    (rho, rho v1, rho v2, rho v3, rho E)."""
    import sympy as sp

    x, y, z = sp.symbols("x y z", real=True)
    k = sp.pi / 2
    a = sp.Rational(1, 10)
    X, Y, Z = x + sp.Rational(3, 10), y + sp.Rational(1, 5), z + sp.Rational(1, 10)
    rho = 2 + a * (sp.sin(k * X) + sp.cos(k * Y) + sp.sin(k * Z))
    v = [sp.Rational(3, 5) + a * sp.cos(k * Y),
         sp.Rational(2, 5) + a * sp.sin(k * Z),
         sp.Rational(3, 10) + a * sp.cos(k * X)]
    p = sp.Rational(3, 2) + a * (sp.sin(k * X) + sp.cos(k * Z))
    g = sp.nsimplify(gamma)
    rhoE = p / (g - 1) + rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) / 2
    U = [rho, rho * v[0], rho * v[1], rho * v[2], rhoE]
    xs = (x, y, z)
    # physical flux F_j (j = Cartesian direction) of each equation
    F = [[rho * v[j] for j in range(3)]]
    for c in range(3):
        F.append([rho * v[c] * v[j] + (p if c == j else 0) for j in range(3)])
    F.append([(rhoE + p) * v[j] for j in range(3)])
    S = [sum(sp.diff(F[q][j], xs[j]) for j in range(3)) for q in range(5)]
    fu = sp.lambdify((x, y, z), U, "numpy")
    fs = sp.lambdify((x, y, z), S, "numpy")

    def as_array(f):
        def call(xx, yy, zz):
            vals = f(xx, yy, zz)
            shape = np.broadcast(xx, yy, zz).shape
            return np.stack([np.broadcast_to(np.asarray(q, float), shape) for q in vals], 0)
        return call

    return as_array(fu), as_array(fs)

"""Pin of the oracle's Sutherland viscosity (Eq. sutherland, as used for the
hypersonic inlet: mu = mu0 (T/T0)^(3/2) (T0 + S)/(T + S)).

The paper prints the same law a second time for its viscous TGV, in the form
mu = 1.4042 (T/T0)^1.5 / (T/T0 + 0.4042) mu0, i.e. S = 0.4042 T0.  On a
state of uniform temperature T (uniform density and pressure, varying
velocity) the viscous terms are those of a constant viscosity, so the
Navier-Stokes right-hand side with Sutherland's law (S = 0.4042 T0) must
equal the constant-viscosity one with mu set from that second form at T,
for T = T0 (where mu = mu0), T0/2 and 3 T0."""
import numpy as np

from oracle.dgsem import Operator
from paper_2511_17551_amd import workloads as W


def uniform_T_case(T):
    c = W.case_c2(n=2)
    g, R = c.cfg["gamma"], c.cfg["R"]
    rho = c.u0[0]
    v = c.u0[1:4] / rho
    p = rho * R * T
    u = c.u0.copy()
    u[4] = p / (g - 1.0) + 0.5 * rho * (v * v).sum(0)
    c.u0 = u
    return c


def test_sutherland_matches_the_tgv_form_at_uniform_temperature():
    T0 = 2.0
    for T in (T0, 0.5 * T0, 3.0 * T0):
        c = uniform_T_case(T)
        mu0 = c.cfg["mu"]
        suth = Operator(dict(c.cfg, sutherland_S=0.4042 * T0, sutherland_T0=T0), c.mesh).rhs(c.u0)
        th = T / T0
        mu_tgv = 1.4042 * th ** 1.5 / (th + 0.4042) * mu0
        const = Operator(dict(c.cfg, mu=mu_tgv), c.mesh).rhs(c.u0)
        scale = np.abs(const).max()
        assert np.abs(suth - const).max() < 1e-12 * scale, (T, np.abs(suth - const).max(), scale)
        if T != T0:   # and differs from the unscaled viscosity there
            plain = Operator(c.cfg, c.mesh).rhs(c.u0)
            assert np.abs(plain - const).max() > 1e-6 * scale

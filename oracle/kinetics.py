"""Finite-rate chemistry: Arrhenius rates and species sources (oracle).

Paper: Appendix, Chemical Kinetics, Eqs. chemreact, nrp, forward_rate,
backward, kedef, gibbs, trans_gibbs, rot, vib, elec, calc_prod; Governing
Equations, Eq. source_term.

Readings of garbled or silent passages:
* Eq. backward: k_b = k_f / K_eq (concentration-based K_c).
* Eq. nrp: the products use nu'_{sr} and concentrations [X_s] = rho_s/W_s;
  with the collision partner written explicitly in each reaction, no
  third-body efficiencies are needed.
* Eq. gibbs omits the formation energy; it is added (g_s includes e_s^0).
* Eqs. rot, vib and elec carry sign errors; the modal Gibbs energies are
  -R_s T ln q_mode:  g_r = -R_s T [L/2 ln(T/theta_r) - ln sigma],
  g_v = +R_s T ln(1 - exp(-theta_v/T)),  g_e = -R_s T ln Q_e.
  Eq. trans_gibbs is taken as printed.  These signs are the ones for which
  d(g_s/T)/dT = -h_s/T^2 with h_s = e_s + R_s T (Gibbs-Helmholtz).
* Eq. calc_prod runs over species s = 1..N_s.
"""
import numpy as np


class Kinetics:
    def __init__(self, sp, rx):
        self.sp = sp
        self.rx = rx
        self.Rs = sp.Ru / sp.W
        self.dnu = (rx.nup - rx.nu).astype(float)   # (nr, ns)

    def gibbs_species(self, T):
        """Specific Gibbs energies g_s(T, p_ref), shape (ns,) + T.shape."""
        sp = self.sp
        T = np.asarray(T, float)
        out = []
        for s in range(len(sp.W)):
            R = self.Rs[s]
            arg = (sp.Ru * T / (sp.NA * sp.p_ref)) * \
                (2.0 * np.pi * sp.W[s] * sp.Ru * T / (sp.NA ** 2 * sp.hP ** 2)) ** 1.5
            g = -R * T * np.log(arg)
            if sp.molecule[s]:
                g = g - R * T * (1.0 * np.log(T / sp.theta_r[s]) - np.log(sp.sigma[s]))
                g = g + R * T * np.log(-np.expm1(-sp.theta_v[s] / T))
            g = g - R * T * np.log(sp.Qe[s])
            g = g + sp.e0[s]
            out.append(g)
        return np.stack(out, 0)

    def enthalpy_species(self, T, mixture):
        return mixture.e_species(T) + self.Rs.reshape((-1,) + (1,) * np.ndim(T)) * T

    def ln_Kc(self, T):
        """ln K_c per reaction: -sum dnu G_s/(R_u T) + sum dnu ln(p_ref/(R_u T))."""
        sp = self.sp
        G = self.gibbs_species(T) * sp.W.reshape((-1,) + (1,) * np.ndim(T))  # J/mol
        dG = np.tensordot(self.dnu, G, axes=(1, 0))
        dn = self.dnu.sum(1).reshape((-1,) + (1,) * np.ndim(T))
        return -dG / (sp.Ru * T) + dn * np.log(sp.p_ref / (sp.Ru * T))

    def ln_kf(self, T):
        """ln k_f = ln A + b ln T - theta_a / T (Eq. forward_rate)."""
        rx = self.rx
        sh = (-1,) + (1,) * np.ndim(T)
        return np.log(rx.A).reshape(sh) + rx.b.reshape(sh) * np.log(T) - rx.theta_a.reshape(sh) / T

    def kf(self, T):
        return np.exp(self.ln_kf(T))

    def kb(self, T):
        """k_b = k_f / K_c (Eq. backward), formed as exp(ln k_f - ln K_c): at low
        T both factors underflow while their ratio stays finite."""
        return np.exp(self.ln_kf(T) - self.ln_Kc(T))

    def rates(self, rs, T):
        """Molar rates of progress R_r (mol m^-3 s^-1), shape (nr,) + T.shape."""
        rx = self.rx
        conc = rs / self.sp.W.reshape((-1,) + (1,) * np.ndim(T))
        kf = self.kf(T)
        kb = self.kb(T)
        out = []
        for r in range(rx.nreactions):
            fwd = np.ones_like(T)
            bwd = np.ones_like(T)
            for s in range(len(self.sp.W)):
                if rx.nu[r, s]:
                    fwd = fwd * conc[s] ** rx.nu[r, s]
                if rx.nup[r, s]:
                    bwd = bwd * conc[s] ** rx.nup[r, s]
            out.append(kf[r] * fwd - kb[r] * bwd)
        return np.stack(out, 0)

    def omega_dot(self, rs, T):
        """omega_s = W_s sum_r (nu'_sr - nu_sr) R_r  (kg m^-3 s^-1)."""
        R = self.rates(rs, T)
        return self.sp.W.reshape((-1,) + (1,) * np.ndim(T)) * np.tensordot(self.dnu.T, R, axes=(1, 0))

"""RRHO mixture thermodynamics and the T(e) Newton solve (oracle).

Paper: Appendix, Thermodynamics, Eqs. Internal_energy, trans_energ,
rot_energ, vib_energ, elec_energ; Governing Equations, Eqs.
internal_energies and eos (Dalton's law p = sum rho_s R_s T).

e_s(T) = 3/2 R_s T  (+ L_s/2 R_s T + R_s theta_v/(exp(theta_v/T) - 1) for
molecules) + e_s^0, with L_s = 2 for the linear diatomics.

Readings:
* the electronic mode has no level data in the paper; it is dropped
  (e_e = 0, ground-state degeneracy only);
* the paper asks for iterative T(e) at least cost but does not give the
  iteration: Newton on f(T) = sum rho_s e_s(T) - rho e with
  f' = sum rho_s cv_s(T) > 0, stopped when |dT| <= tol * T.
* the frozen sound speed a_f = sqrt(gamma_f p / rho),
  gamma_f = 1 + sum rho_s R_s / sum rho_s cv_s, is used in the Lax-Friedrichs
  dissipation.
"""
import numpy as np


class Mixture:
    def __init__(self, sp):
        self.sp = sp
        self.Rs = sp.Ru / sp.W
        self.mol = sp.molecule.astype(bool)
        self.th = sp.theta_v
        self.e0 = sp.e0
        self.ns = len(sp.W)

    def _col(self, a, nd):
        return a.reshape((-1,) + (1,) * nd)

    def e_species(self, T):
        """Specific energies e_s(T), shape (ns,) + T.shape."""
        nd = np.ndim(T)
        R = self._col(self.Rs, nd)
        e = 1.5 * R * T + self._col(self.e0, nd)
        out = np.array(np.broadcast_to(e, (self.ns,) + np.shape(T)))
        for s in range(self.ns):
            if self.mol[s]:
                # R theta/(e^x - 1), x = theta/T, in the overflow-free form
                # R theta e^-x / (1 - e^-x)
                x = self.th[s] / T
                out[s] = out[s] + self.Rs[s] * T + self.Rs[s] * self.th[s] * np.exp(-x) / (-np.expm1(-x))
        return out

    def cv_species(self, T):
        nd = np.ndim(T)
        out = np.array(np.broadcast_to(1.5 * self._col(self.Rs, nd), (self.ns,) + np.shape(T)))
        for s in range(self.ns):
            if self.mol[s]:
                # d/dT of R theta/(e^x - 1), x = theta/T, in the overflow-free
                # form R x^2 e^-x / (1 - e^-x)^2
                x = self.th[s] / T
                em = np.exp(-x)
                out[s] = out[s] + self.Rs[s] + self.Rs[s] * x * x * em / (-np.expm1(-x)) ** 2
        return out

    def rho_e(self, rs, T):
        """sum_s rho_s e_s(T)."""
        return np.sum(rs * self.e_species(T), axis=0)

    def rho_cv(self, rs, T):
        return np.sum(rs * self.cv_species(T), axis=0)

    def solve_T(self, rs, rhoe, T0, tol=1e-10, maxit=50, strict=True):
        """Per-node Newton iteration; every node stops on its own test:
        |dT| <= tol * |T|, or a residual at the rounding level of the
        energies it is made of, |rho e(T) - target| <= 8 eps (|target| +
        sum_s |rho_s e0_s|) (a thermal energy of that size, T ~ 1e-10 K, is
        determined no better than that).

        Returns T and the iteration count per node.  A node that fails to
        converge within maxit raises, or with strict=False gets T = NaN.
        """
        shape = np.shape(rhoe)
        rs = rs.reshape(self.ns, -1)
        target = np.reshape(rhoe, -1)
        T = np.array(np.broadcast_to(T0, shape), float).reshape(-1)
        it = np.zeros(T.shape, np.int64)
        active = np.ones(T.shape, bool)
        floor = 8.0 * np.finfo(float).eps * (np.abs(target) + (np.abs(rs) * np.abs(self.e0)[:, None]).sum(0))
        for _ in range(maxit):
            if not active.any():
                break
            idx = np.flatnonzero(active)
            Ta = T[idx]
            rsa = rs[:, idx]
            f = self.rho_e(rsa, Ta) - target[idx]
            fp = self.rho_cv(rsa, Ta)
            dT = f / fp
            Tn = Ta - dT
            T[idx] = Tn
            it[idx] += 1
            done = (np.abs(dT) <= tol * np.abs(Tn)) | (np.abs(f) <= floor[idx])
            active[idx[done]] = False
        if active.any():
            if strict:
                raise RuntimeError("Newton for T(e) did not converge")
            T[active] = np.nan
        return T.reshape(shape), it.reshape(shape)

    def pressure(self, rs, T):
        return np.sum(rs * self.Rs.reshape((-1,) + (1,) * np.ndim(T)), axis=0) * T

    def sound_speed(self, rs, T):
        nd = np.ndim(T)
        rho = rs.sum(0)
        rR = np.sum(rs * self._col(self.Rs, nd), axis=0)
        gam = 1.0 + rR / self.rho_cv(rs, T)
        return np.sqrt(gam * rR * T / rho)

    def state(self, u, dim, T):
        """Mixture flux state from conserved u and a converged T."""
        rs = u[:self.ns]
        rho = rs.sum(0)
        v = u[self.ns:self.ns + dim] / rho
        rhoE = u[self.ns + dim]
        p = self.pressure(rs, T)
        c = self.sound_speed(rs, T)
        return dict(rho=rho, rs=rs, v=v, p=p, rhoE=rhoE, c=c, T=T, mix=True)

    def temperature(self, u, dim, T0, tol=1e-10, maxit=50):
        rs = u[:self.ns]
        rho = rs.sum(0)
        m = u[self.ns:self.ns + dim]
        rhoe = u[self.ns + dim] - 0.5 * np.sum(m * m, axis=0) / rho
        return self.solve_T(rs, rhoe, T0, tol, maxit)

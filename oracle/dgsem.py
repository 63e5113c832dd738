"""Semi-discrete DGSEM operator du/dt = L(u) (oracle).

Paper: Sec. Methodology.  Per element k and node n, with n_d the node's
index along reference direction d,

  du_n/dt = -(1/J_n) sum_d { (1/w_{n_d}) [ (1-alpha_k)(Fbar_{n_d+1} - Fbar_{n_d})
                                           + alpha_k (Ffv_{n_d+1} - Ffv_{n_d}) ]
                             + delta_{n_d N} F*_N / w_N - delta_{n_d 0} F*_0 / w_0 }
            + S_n  (+ viscous terms, see br1)

* Fbar: the telescoped high-order subcell flux of Eq. DGvec,
  Fbar_j = sum_{p>=j} sum_{q<j} 2 w_q D_qp F#(u_q, u_p), j = 1..N, with the
  two-point flux F# of Eq. fluxdiffcons evaluated with the averaged metric
  n = (Ja^d_q + Ja^d_p)/2.
* Ffv: the first-order subcell flux of Eq. finitevolumeflux, the Riemann
  flux between neighbouring nodes through the telescoped subcell normal.
* F*: interface Riemann flux of Eqs. riemann_problem1-3 (Rusanov), with one
  scaled normal per face taken from the element on the face's minus side
  (its xi_d = +1 face), so both elements see the same flux.
* S: species sources of Eq. source_term.

Reading of the endpoint conflict (Eq. DGvec sets Fbar_0 = F(U_0),
Eq. finitevolumeflux sets the FV endpoints to 0): both subcell fluxes have
zero end values and the surface terms are not blended.  At alpha = 0 this
is the strong form of Eq. fluxes_discrete_fluxdifferencing (it uses
2 D_00 + 1/w_0 = 0); for any alpha it is conservative.
Garbles taken as: the time derivative missing on the left of Eqs.
divergenc_quadrature/strong_form, the surface terms act only at the end
nodes, and the right-face labels of Eqs. riemann_problem2-3 name the
xi_2 = P and xi_3 = P faces.
"""
import numpy as np

from . import gas
from .basis import Basis
from .geometry import metrics, face_nodes, line_view, line_unview, subcell_normals
from .indicator import modal_energy_ratio, blending_factor, smooth
from .thermo import Mixture
from .kinetics import Kinetics

EQ_EULER, EQ_NS, EQ_EULER_MIX, EQ_REACT_MIX = 0, 1, 2, 3
BC_DIRICHLET, BC_OUTFLOW, BC_SLIPWALL, BC_WALL_ISOTHERMAL, BC_WALL_ADIABATIC = 0, 1, 2, 3, 4


class Operator:
    def __init__(self, cfg, mesh, species=None, reactions=None, dtype=np.float64):
        """``dtype`` float64 (the oracle) or np.longdouble (x87 80-bit, for
        measuring the rounding of float64 evaluations: operators, metrics and
        every step run in that precision on the same inputs)."""
        self.cfg = cfg
        self.mesh = mesh
        self.dim = mesh.dim
        self.N = mesh.N
        self.dtype = dtype
        self.b = Basis(self.N, dtype)
        self.Ja, self.J = metrics(np.asarray(mesh.x, dtype), self.b, self.dim)
        self.fn = [face_nodes(self.dim, self.N, f) for f in range(2 * self.dim)]
        self.eq = cfg["eq"]
        self.mix = Mixture(species) if self.eq in (EQ_EULER_MIX, EQ_REACT_MIX) else None
        self.kin = Kinetics(species, reactions) if self.eq == EQ_REACT_MIX else None
        self.nsub = subcell_normals(self.Ja, self.b, self.dim) if cfg.get("shock") else None
        self.boundary_exact = None   # optional Phi(x) of Dirichlet boundaries (manufactured solutions)
        self.last = {}

    # ------------------------------------------------------------------
    def states(self, u, T=None):
        if self.mix is None:
            return gas.pg_state(u, self.dim, self.cfg["gamma"])
        if T is None:
            T, _ = self.mix.temperature(u, self.dim, self.cfg["T_guess"],
                                        self.cfg["newton_tol"], self.cfg["newton_maxit"])
        return self.mix.state(u, self.dim, T)

    # volume and surface flux choices (the library's DGX_VF_* / DGX_SF_*
    # numbering; for mixtures the entropy-conservative choice 0 / 1 is
    # gas.ec_mixture); "kg" / "pirozzoli" / "morinishi" as a surface flux serve the oracle's
    # own kinetic-energy checks
    VOLUME = {0: gas.ranocha, 1: gas.ducros, 2: gas.kennedy_gruber, 3: gas.pirozzoli, 4: gas.central,
              5: gas.morinishi}
    SURFACE = {0: gas.rusanov, 1: gas.ranocha, 2: gas.hll, 3: gas.hllc, "kg": gas.kennedy_gruber,
               "pirozzoli": gas.pirozzoli, "morinishi": gas.morinishi}

    def volume_flux(self, sL, sR, n):
        if self.mix is not None and self.cfg["volume_flux"] == 0:
            return gas.ec_mixture(sL, sR, n, self.mix)
        return self.VOLUME[self.cfg["volume_flux"]](sL, sR, n)

    def surface_flux(self, sL, sR, n):
        if self.mix is not None and self.cfg["surface_flux"] == 1:
            return gas.ec_mixture(sL, sR, n, self.mix)
        return self.SURFACE[self.cfg["surface_flux"]](sL, sR, n)

    # ------------------------------------------------------------------
    def blending(self, s):
        cfg = self.cfg
        E = self.mesh.nelem
        if cfg.get("force_alpha", -1.0) >= 0.0:
            return np.full(E, cfg["force_alpha"], self.dtype), None
        if not cfg.get("shock"):
            return np.zeros(E, self.dtype), None
        eps = s["p"] if cfg.get("ind_var", 0) == 1 else s["rho"] * s["p"]
        Erat = modal_energy_ratio(eps, self.b, self.dim)
        alpha, raw = blending_factor(Erat, self.N, cfg["alpha_max"], cfg["alpha_min"])
        if cfg.get("alpha_smooth"):
            alpha = smooth(alpha, self.mesh.faces, self.mesh.mortars)
        return alpha, raw

    # ------------------------------------------------------------------
    def volume_terms(self, s, alpha):
        """sum_d (1/w) Delta((1-alpha) Fbar + alpha Ffv), shape (nvar, E, nn)."""
        b = self.b
        n1 = b.n1
        N = self.N
        dim = self.dim
        nvar = self.cfg["nvar"]
        E = self.mesh.nelem
        G = np.zeros((nvar, E, n1 ** dim), self.dtype)
        use_fv = np.any(alpha > 0.0)
        for d in range(dim):
            sl = {k: (line_view(v, d, dim, n1) if isinstance(v, np.ndarray) else v)
                  for k, v in s.items()}
            Jl = line_view(self.Ja[d], d, dim, n1)     # (dim, E, lines, n1)
            nodes = [gas.take(sl, q) for q in range(n1)]
            # symmetric two-point fluxes F#(u_q, u_p), q < p
            Fs = {}
            for q in range(n1):
                for p in range(q + 1, n1):
                    nbar = 0.5 * (Jl[..., q] + Jl[..., p])
                    Fs[(q, p)] = self.volume_flux(nodes[q], nodes[p], nbar)
            shape = (nvar,) + Jl.shape[1:-1]
            Fbar = [np.zeros(shape, self.dtype) for _ in range(n1 + 1)]
            for j in range(1, n1):
                acc = np.zeros(shape, self.dtype)
                for p in range(j, n1):
                    for q in range(0, j):
                        acc += 2.0 * b.w[q] * b.D[q, p] * Fs[(q, p)]
                Fbar[j] = acc
            Gl = np.zeros(shape + (n1,), self.dtype)
            a = alpha.reshape((1, E, 1))
            if use_fv:
                ns = self.nsub[d]
                Ffv = [np.zeros(shape, self.dtype) for _ in range(n1 + 1)]
                for m in range(1, n1):
                    Ffv[m] = self.surface_fv(nodes[m - 1], nodes[m], ns[..., m])
            for n in range(n1):
                hi = (1.0 - a) * (Fbar[n + 1] - Fbar[n])
                if use_fv:
                    hi = hi + a * (Ffv[n + 1] - Ffv[n])
                Gl[..., n] = hi / b.w[n]
            G += line_unview(Gl, d, dim, n1)
        return G

    def surface_fv(self, sL, sR, n):
        """Subcell interface flux of the first-order scheme (Rusanov)."""
        return gas.rusanov(sL, sR, n)

    # ------------------------------------------------------------------
    def external_state(self, s_int, u_int, kind, state, n, T_int, x_face=None):
        """External state of a boundary face (Eq. system_equation, U = Phi on
        the boundary, imposed weakly through the surface flux).  Dirichlet
        takes the boundary's constant state, or, when ``boundary_exact`` is
        set (a manufactured solution's Phi(x)), that function at the face
        nodes ``x_face``."""
        if kind == BC_DIRICHLET:
            if self.boundary_exact is not None:
                return self.states(np.asarray(self.boundary_exact(x_face), self.dtype))
            ue = np.broadcast_to(state.reshape((-1,) + (1,) * (u_int.ndim - 1)), u_int.shape).copy()
            return self.states(ue)
        if kind == BC_OUTFLOW:
            return s_int
        ue = u_int.copy()
        off = 5 if self.mix is not None else 1
        m = u_int[off:off + self.dim]
        if kind in (BC_WALL_ISOTHERMAL, BC_WALL_ADIABATIC):
            # no-slip wall: the advective flux sees the state with the whole
            # velocity reversed (same density and energy), which carries no
            # mass or energy through the face
            ue[off:off + self.dim] = -m
            return self.states(ue, T_int)
        # slip wall: mirror the momentum about the face
        nh = n / np.sqrt(gas.dot(n, n))
        mn = gas.dot(m, nh)
        ue[off:off + self.dim] = m - 2.0 * mn * nh
        return self.states(ue, T_int)

    def surface_terms(self, u, s, G):
        b = self.b
        N = self.N
        mesh = self.mesh
        for d in range(self.dim):
            sel = mesh.faces[mesh.faces[:, 1] == 2 * d + 1]
            if len(sel) == 0:
                continue
            eL, eR = sel[:, 0], sel[:, 2]
            nl = self.fn[2 * d + 1]
            nr = self.fn[2 * d]
            sL = gas.take(s, (eL[:, None], nl[None, :]))
            sR = gas.take(s, (eR[:, None], nr[None, :]))
            n = self.Ja[d][:, eL[:, None], nl[None, :]]
            F = self.surface_flux(sL, sR, n)
            np.add.at(G, (slice(None), eL[:, None], nl[None, :]), F / b.w[N])
            np.add.at(G, (slice(None), eR[:, None], nr[None, :]), -F / b.w[0])
        # boundary faces, all faces of one local face index and boundary
        # together (each boundary face node receives its one flux)
        bf = mesh.bfaces
        for f in range(2 * self.dim):
            rows = bf[bf[:, 1] == f]
            if len(rows) == 0:
                continue
            d, side = divmod(f, 2)
            nodes = self.fn[f]
            for bc in np.unique(rows[:, 2]):
                e = rows[rows[:, 2] == bc, 0]
                idx = (e[:, None], nodes[None, :])
                ui = u[(slice(None),) + idx]
                si = gas.take(s, idx)
                n = self.Ja[d][(slice(None),) + idx]
                se = self.external_state(si, ui, int(mesh.bc_kind[bc]), mesh.bc_state[bc], n, si.get("T"),
                                         x_face=mesh.x[(slice(None),) + idx])
                if side == 1:
                    np.add.at(G, (slice(None),) + idx, self.surface_flux(si, se, n) / b.w[N])
                else:
                    np.add.at(G, (slice(None),) + idx, -self.surface_flux(se, si, n) / b.w[0])
        if len(mesh.mortars):
            from .mortar import mortar_surface_terms
            mortar_surface_terms(self, s, G)

    # ------------------------------------------------------------------
    def rhs(self, u, t=0.0, alpha=None):
        u = np.asarray(u, self.dtype)
        s = self.states(u)
        if alpha is None:
            alpha, raw = self.blending(s)
        else:
            raw = None
        G = self.volume_terms(s, alpha)
        self.surface_terms(u, s, G)
        du = -G / self.J[None]
        if self.eq == EQ_NS:
            from .br1 import viscous_rhs
            du += viscous_rhs(self, u, s)
        if self.kin is not None:
            du[:5] += self.kin.omega_dot(s["rs"], s["T"])
        self.last = dict(alpha=alpha, alpha_raw=raw, T=s.get("T"))
        return du

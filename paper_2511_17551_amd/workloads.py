"""Seeded synthetic workloads: meshes, initial states and physical data tables.

This module only builds *inputs*.  It holds no part of the discretisation
(no derivative operators, metrics, fluxes, thermodynamic closures or
kinetics): the HIP library and the CPU oracle each compute those on their
own from the inputs produced here.  Both sides receive

* a mesh: nodal coordinates of every element at the Legendre-Gauss-Lobatto
  (LGL) points (the paper's element mapping, Sec. Methodology, Eq. mapp,
  evaluated at the nodes), plus conforming face, boundary-face and mortar
  tables;
* an initial conserved state ``u[nvar][nelem][(N+1)^dim]`` (Eq. Uconserv);
* physical data: gas constants, species data for 5-species air
  (N2, O2, NO, N, O; Appendix, Thermodynamics) and a seeded
  17-reaction table with the structure of the Park mechanism (Appendix,
  Chemical Kinetics, Eq. reactions).

Node numbering inside an element is ``n = i + (N+1)*(j + (N+1)*k)`` with
``i`` along the first reference direction.  Local face ``f = 2*d + s`` is the
face xi_d = -1 (s = 0) or xi_d = +1 (s = 1).  A conforming face row
``(eL, fL, eR, fR)`` always joins the +d face of eL to the -d face of eR
with the tangential node order aligned.  A mortar row
``(eL, fL, eS_0..eS_{m-1}, fS)`` joins one large face to 2 (2D) or 4 (3D)
small faces; sub-face ``s = a + 2*b`` covers the lower (0) or upper (1)
half of each tangential direction of the large face, in increasing order.

Mixture states need e_s(T); the caller passes an ``energy`` callable so that
this module stays free of thermodynamics.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# Boundary-condition kinds (shared numbering of the mesh input format)
BC_DIRICHLET = 0   # external state is a fixed conserved state
BC_OUTFLOW = 1     # external state equals the interior state
BC_SLIPWALL = 2    # mirror the normal velocity
BC_WALL_ISOTHERMAL = 3  # no-slip wall at the temperature bc_state[bc][0]
BC_WALL_ADIABATIC = 4   # no-slip wall without heat flux

EQ_EULER = 0       # perfect-gas Euler
EQ_NS = 1          # perfect-gas Navier-Stokes (BR1 viscous terms)
EQ_EULER_MIX = 2   # 5-species frozen-chemistry Euler, RRHO thermodynamics
EQ_REACT_MIX = 3   # as above plus Arrhenius species sources

VF_RANOCHA = 0     # entropy-conservative two-point flux
VF_DUCROS = 1      # Ducros split-form two-point flux
VF_KENNEDY_GRUBER = 2  # Kennedy-Gruber split form
VF_PIROZZOLI = 3   # Pirozzoli split form
VF_CENTRAL = 4     # standard-DG form: mean of the physical fluxes
VF_MORINISHI = 5   # Morinishi's skew-symmetric splitting (perfect gas)
SF_RUSANOV = 0     # local Lax-Friedrichs surface flux
SF_RANOCHA = 1     # EC flux at faces (entropy-conservation checks only)
SF_HLL = 2         # HLL with Davis wave-speed bounds
SF_HLLC = 3        # HLLC, Davis bounds and Toro's contact speed

IND_RHO_P = 0      # shock indicator variable rho*p
IND_P = 1          # shock indicator variable p


def _mesh_nodes(N: int) -> np.ndarray:
    """Positions in [-1, 1] at which the mesh places element nodes.

    The LGL points: the end points plus the roots of P_N'.  Only used to
    place coordinates; each consumer builds its own operators.
    """
    c = np.zeros(N + 1)
    c[N] = 1.0
    inner = np.polynomial.legendre.Legendre(c).deriv().roots()
    return np.concatenate(([-1.0], np.sort(inner.real), [1.0]))


@dataclass
class Mesh:
    dim: int
    N: int
    x: np.ndarray                     # (dim, nelem, nnodes) float64
    faces: np.ndarray                 # (nface, 4) int32
    bfaces: np.ndarray                # (nbface, 3) int32 : e, f, bc index
    mortars: np.ndarray               # (nmortar, 2 + 2^(dim-1) + 1) int32
    bc_kind: np.ndarray               # (nbc,) int32
    bc_state: np.ndarray              # (nbc, nvar) float64 (Dirichlet states)
    level: np.ndarray | None = None   # refinement level per element (AMR)
    case_offsets: np.ndarray | None = None  # batched cases: first element of each case

    @property
    def nelem(self) -> int:
        return self.x.shape[1]

    @property
    def nnodes(self) -> int:
        return (self.N + 1) ** self.dim


def structured_mesh(dim, N, shape, lo, hi, periodic, mapping=None,
                    bc_lo=None, bc_hi=None):
    """Block-structured mesh of ``prod(shape)`` elements on a box.

    ``mapping(X) -> x`` (arrays of shape (dim, ...)) deforms the box; element
    e = i + n0*(j + n1*k).  Non-periodic directions get boundary faces with
    bc index ``bc_lo[d]`` / ``bc_hi[d]``.
    """
    nx = tuple(int(s) for s in shape)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    h = (hi - lo) / np.asarray(nx, float)
    xi = _mesh_nodes(N)
    n1 = N + 1
    nelem = int(np.prod(nx))
    nn = n1 ** dim
    # element multi-indices
    eidx = np.stack(np.unravel_index(np.arange(nelem), nx[::-1])[::-1], 0)  # (dim, nelem)
    # node multi-indices (a along dim 0)
    nidx = np.stack(np.unravel_index(np.arange(nn), (n1,) * dim)[::-1], 0)  # (dim, nn)
    X = np.empty((dim, nelem, nn))
    for d in range(dim):
        X[d] = lo[d] + h[d] * (eidx[d][:, None] + 0.5 * (xi[nidx[d]][None, :] + 1.0))
    x = mapping(X) if mapping is not None else X
    faces = []
    bfaces = []
    strides = [1, nx[0], nx[0] * (nx[1] if dim > 1 else 1)]
    for d in range(dim):
        for e in range(nelem):
            c = eidx[d, e]
            if c + 1 < nx[d]:
                faces.append((e, 2 * d + 1, e + strides[d], 2 * d))
            elif periodic[d]:
                faces.append((e, 2 * d + 1, e - (nx[d] - 1) * strides[d], 2 * d))
            else:
                bfaces.append((e, 2 * d + 1, bc_hi[d]))
            if c == 0 and not periodic[d]:
                bfaces.append((e, 2 * d, bc_lo[d]))
    faces = np.asarray(faces, np.int32).reshape(-1, 4)
    bfaces = np.asarray(bfaces, np.int32).reshape(-1, 3)
    return x, faces, bfaces


def ogrid_mesh(N, nr, nth, r0, r1):
    """Annular O-grid: xi along the radius (r0 -> r1), eta along the angle.

    Inner ring (r = r0) is boundary 0, outer ring (r = r1) boundary 1, the
    angle is periodic.
    """
    def polar(X):
        r = X[0]
        th = X[1]
        return np.stack((r * np.cos(th), r * np.sin(th)), 0)
    return structured_mesh(2, N, (nr, nth), (r0, 0.0), (r1, 2.0 * math.pi),
                           (False, True), polar, bc_lo=(0, None), bc_hi=(1, None))


# ----------------------------------------------------------------------------
# Physical data
@dataclass
class Species:
    """5-species air data (N2, O2, NO, N, O).

    Molar masses: IUPAC atomic masses.  theta_v: the values quoted with the
    curvilinear 5-species workload.  theta_r, sigma: textbook spectroscopic
    constants.  Formation energies: NIST-JANAF heats of formation at 298 K.
    Electronic mode: ground-state degeneracy only (the paper prints no level
    data), so e_e = 0 and Q_e is a constant.
    """
    names: tuple = ("N2", "O2", "NO", "N", "O")
    W: np.ndarray = field(default_factory=lambda: np.array(
        [0.0280134, 0.0319988, 0.0300061, 0.0140067, 0.0159994]))
    molecule: np.ndarray = field(default_factory=lambda: np.array([1, 1, 1, 0, 0], np.int32))
    theta_v: np.ndarray = field(default_factory=lambda: np.array([3393.0, 2273.0, 2739.0, 0.0, 0.0]))
    theta_r: np.ndarray = field(default_factory=lambda: np.array([2.88, 2.08, 2.45, 0.0, 0.0]))
    sigma: np.ndarray = field(default_factory=lambda: np.array([2.0, 2.0, 1.0, 1.0, 1.0]))
    Qe: np.ndarray = field(default_factory=lambda: np.array([1.0, 3.0, 4.0, 4.0, 9.0]))
    hf_molar: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, 90.29e3, 472.68e3, 249.18e3]))
    Ru: float = 8.314462618
    NA: float = 6.02214076e23
    hP: float = 6.62607015e-34
    p_ref: float = 1.0  # reference pressure of the equilibrium constants [Pa]

    @property
    def e0(self):
        return self.hf_molar / self.W

    @property
    def nspecies(self):
        return 5


@dataclass
class Reactions:
    """Stoichiometry and Arrhenius data; nu = reactants, nup = products."""
    A: np.ndarray        # m^3 mol^-1 s^-1 (all reactions are bimolecular forward)
    b: np.ndarray
    theta_a: np.ndarray  # K
    nu: np.ndarray       # (nr, ns) int
    nup: np.ndarray      # (nr, ns) int

    @property
    def nreactions(self):
        return self.A.shape[0]


def park17_reactions(seed: int = 4) -> Reactions:
    """17 reactions with the Park 5-species structure, partner made explicit.

    X2 + M <=> X + Y + M for X2 in {N2, O2, NO} and each M in the 5
    species, then N2 + O <=> NO + N and NO + O <=> O2 + N, each written in
    its endothermic direction.  Coefficients are seeded so that they span
    the Park data: b ~ U[-1.6, 0]; A such that log10(A * 5000^b) ~ U[12, 17]
    (cm^3/mol/s, the range of A T^b of those reactions at 5000 K, all below
    the gas-kinetic collision rate); and the activation temperature is the
    reaction heat over R_u plus U[0, 4000] K, as theta_a of a dissociation is
    its dissociation energy over k_B and the exchange reactions sit a few
    hundred kelvin above their heat.  The last keeps k_b = k_f / K_c bounded
    as T falls (an activation temperature away from the heat makes k_b grow
    or vanish like exp(|dtheta|/T)).
    """
    N2, O2, NO, N, O = range(5)
    nu, nup = [], []
    for mol, prod in ((N2, (N, N)), (O2, (O, O)), (NO, (N, O))):
        for M in range(5):
            r = np.zeros(5, int)
            p = np.zeros(5, int)
            r[mol] += 1
            r[M] += 1
            p[prod[0]] += 1
            p[prod[1]] += 1
            p[M] += 1
            nu.append(r)
            nup.append(p)
    for (ra, rb), (pa, pb) in (((N2, O), (NO, N)), ((NO, O), (O2, N))):
        r = np.zeros(5, int)
        p = np.zeros(5, int)
        r[ra] += 1
        r[rb] += 1
        p[pa] += 1
        p[pb] += 1
        nu.append(r)
        nup.append(p)
    rng = np.random.default_rng(seed)
    nr = len(nu)
    b = rng.uniform(-1.6, 0.0, nr)
    logA = rng.uniform(12.0, 17.0, nr) - b * math.log10(5000.0)
    heat = (np.asarray(nup) - np.asarray(nu)) @ Species().hf_molar / Species().Ru
    th = heat + rng.uniform(0.0, 4.0e3, nr)
    return Reactions(A=10.0 ** logA * 1e-6, b=b, theta_a=th,
                     nu=np.asarray(nu, np.int32), nup=np.asarray(nup, np.int32))


# ----------------------------------------------------------------------------
# Workload descriptions
@dataclass
class Case:
    name: str
    cfg: dict
    mesh: Mesh
    u0: np.ndarray
    t0: float = 0.0
    dt: float | None = None
    species: Species | None = None
    reactions: Reactions | None = None
    extra: dict = field(default_factory=dict)


def base_cfg(dim, N, eq, **kw):
    nvar = {EQ_EULER: dim + 2, EQ_NS: dim + 2, EQ_EULER_MIX: 5 + dim + 1, EQ_REACT_MIX: 5 + dim + 1}[eq]
    cfg = dict(dim=dim, N=N, eq=eq, nvar=nvar, gamma=1.4, R=1.0, mu=0.0, Pr=0.72,
               volume_flux=VF_RANOCHA, surface_flux=SF_RUSANOV,
               shock=False, alpha_max=0.5, alpha_min=1e-3, ind_var=IND_RHO_P,
               alpha_smooth=False, force_alpha=-1.0,
               newton_tol=1e-10, newton_maxit=50, T_guess=300.0, positivity=False,
               sutherland_S=0.0, sutherland_T0=1.0)
    cfg.update(kw)
    return cfg


def _pg_conserved(rho, vel, p, gamma):
    """(rho, rho v, rho E) of a calorically perfect gas from primitives."""
    m = [rho * v for v in vel]
    E = p / (gamma - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    return np.stack([rho] + m + [E], 0)


def isentropic_vortex(x, y, gamma=1.4, eps=5.0, xc=5.0, yc=5.0, uinf=(1.0, 1.0)):
    """Shu's isentropic vortex on rho = 1, u = (1, 1), p = 1 (strength 5, radius 1)."""
    xb = x - xc
    yb = y - yc
    r2 = xb * xb + yb * yb
    f = np.exp(0.5 * (1.0 - r2))
    du = eps / (2.0 * math.pi) * f
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi ** 2) * f * f
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return rho, (uinf[0] - du * yb, uinf[1] + du * xb), p


def case_c1(n=16, N=3, surface_flux=SF_RUSANOV, length=10.0):
    """2D Euler isentropic vortex, 16x16 periodic quads on [0,10]^2."""
    x, faces, bfaces = structured_mesh(2, N, (n, n), (0.0, 0.0), (length, length), (True, True))
    cfg = base_cfg(2, N, EQ_EULER, surface_flux=surface_flux)
    rho, v, p = isentropic_vortex(x[0], x[1], cfg["gamma"], xc=0.5 * length, yc=0.5 * length)
    u0 = _pg_conserved(rho, v, p, cfg["gamma"])
    mesh = Mesh(2, N, x, faces, bfaces, np.zeros((0, 5), np.int32),
                np.zeros(0, np.int32), np.zeros((0, 4)))
    return Case("vortex2d", cfg, mesh, u0)


def tgv_state(x, y, z, gamma=1.4, mach=0.1):
    """Taylor-Green vortex initial state (rho0 = U0 = L = 1)."""
    rho = np.ones_like(x)
    v1 = np.sin(x) * np.cos(y) * np.cos(z)
    v2 = -np.cos(x) * np.sin(y) * np.cos(z)
    v3 = np.zeros_like(x)
    p0 = 1.0 / (gamma * mach * mach)
    p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    return rho, (v1, v2, v3), p


def case_c2(n=32, N=3, mu=1.0 / 1600.0, eq=EQ_NS):
    """3D Navier-Stokes Taylor-Green vortex on the periodic cube [0, 2pi]^3."""
    L = 2.0 * math.pi
    x, faces, bfaces = structured_mesh(3, N, (n, n, n), (0.0,) * 3, (L,) * 3, (True,) * 3)
    cfg = base_cfg(3, N, eq, mu=mu if eq == EQ_NS else 0.0, Pr=0.72)
    rho, v, p = tgv_state(x[0], x[1], x[2], cfg["gamma"])
    u0 = _pg_conserved(rho, v, p, cfg["gamma"])
    mesh = Mesh(3, N, x, faces, bfaces, np.zeros((0, 7), np.int32),
                np.zeros(0, np.int32), np.zeros((0, 5)))
    return Case("tgv3d", cfg, mesh, u0)


def curved_periodic_case(n=3, N=3, eq=EQ_EULER, amp=0.1, seed=7, **kw):
    """Perfect-gas state on the curved unit cube, periodic in all directions."""
    x, faces, bfaces = structured_mesh(3, N, (n, n, n), (0.0,) * 3, (1.0,) * 3, (True,) * 3,
                                       lambda X: curved_map(X, amp))
    cfg = base_cfg(3, N, eq, **kw)
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 3, size=(3, 3))
    ph = rng.uniform(0, 2 * math.pi, 3)
    arg = [2 * math.pi * (k[i, 0] * x[0] + k[i, 1] * x[1] + k[i, 2] * x[2]) + ph[i] for i in range(3)]
    rho = 1.0 + 0.3 * np.sin(arg[0])
    v = (0.5 + 0.2 * np.cos(arg[1]), -0.3 + 0.2 * np.sin(arg[2]), 0.1 * np.cos(arg[0]))
    p = 1.0 + 0.25 * np.cos(arg[2])
    u0 = _pg_conserved(rho, v, p, cfg["gamma"])
    mesh = Mesh(3, N, x, faces, bfaces, np.zeros((0, 7), np.int32),
                np.zeros(0, np.int32), np.zeros((0, 5)))
    return Case("curved_periodic", cfg, mesh, u0)


def curved_periodic_mixture_case(energy, n=2, N=4, seed=5, T0=2000.0, p0=1.0e4, uniform_p=False,
                                 **kw):
    """Frozen 5-species air on the curved unit cube, periodic in all
    directions: mass fractions near (0.7, 0.2, 0.04, 0.03, 0.03) with smooth
    seeded variations of a few percent, density and velocity (a third of the
    sound speed) varying smoothly, T around ``T0``.  With ``uniform_p`` the
    temperature follows the density so that p = ``p0`` at every node.
    ``energy(rho_s, T)`` supplies the thermal energy density."""
    sp = Species()
    x, faces, bfaces = structured_mesh(3, N, (n, n, n), (0.0,) * 3, (1.0,) * 3, (True,) * 3,
                                       lambda X: curved_map(X, 0.1))
    Y0 = np.array([0.7, 0.2, 0.04, 0.03, 0.03])
    Y = Y0[:, None, None] * (1.0 + smooth_perturbation(x, seed, amp=0.3))
    Y = Y / Y.sum(0)[None]
    rng = np.random.default_rng(seed + 1)
    k = rng.integers(1, 3, size=(3, 3))
    ph = rng.uniform(0, 2 * math.pi, 3)
    arg = [2 * math.pi * (k[i, 0] * x[0] + k[i, 1] * x[1] + k[i, 2] * x[2]) + ph[i] for i in range(3)]
    Rmix = (Y * (sp.Ru / sp.W)[:, None, None]).sum(0)
    if uniform_p:
        rho = p0 / (Rmix * T0) * (1.0 + 0.3 * np.sin(arg[0]))
        T = p0 / (rho * Rmix)
    else:
        T = T0 * (1.0 + 0.2 * np.cos(arg[1]))
        rho = p0 / (Rmix * T0) * (1.0 + 0.3 * np.sin(arg[0]))
    a = math.sqrt(1.3 * float(Rmix.mean()) * T0)
    vel = (a * (0.3 + 0.1 * np.cos(arg[1])), a * (-0.2 + 0.1 * np.sin(arg[2])), a * 0.1 * np.cos(arg[0]))
    u0 = mixture_state(Y, rho, vel, T, energy)
    mesh = Mesh(3, N, x, faces, bfaces, np.zeros((0, 7), np.int32),
                np.zeros(0, np.int32), np.zeros((0, 10)))
    cfg = base_cfg(3, N, EQ_EULER_MIX, T_guess=T0, **kw)
    return Case("curved_periodic_air5", cfg, mesh, u0, species=sp, extra=dict(T=T))


def curved_channel_case(n=3, N=3, mach=2.0, amp=0.1, seed=7, **kw):
    """Perfect-gas supersonic channel on the curved unit cube: x = 0 is a
    Dirichlet inflow (rho 1, p 1, u = mach * c along x), x = 1 an outflow
    (external state = interior state), y and z periodic.  The initial state
    is the inflow state plus the smooth seeded perturbation of
    ``curved_periodic_case`` at a tenth of its amplitude."""
    x, faces, bfaces = structured_mesh(3, N, (n, n, n), (0.0,) * 3, (1.0,) * 3, (False, True, True),
                                       lambda X: curved_map(X, amp), bc_lo=(0, None, None),
                                       bc_hi=(1, None, None))
    cfg = base_cfg(3, N, EQ_EULER, **kw)
    g = cfg["gamma"]
    uin = mach * math.sqrt(g)
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 3, size=(3, 3))
    ph = rng.uniform(0, 2 * math.pi, 3)
    arg = [2 * math.pi * (k[i, 0] * x[0] + k[i, 1] * x[1] + k[i, 2] * x[2]) + ph[i] for i in range(3)]
    rho = 1.0 + 0.03 * np.sin(arg[0])
    v = (uin + 0.02 * np.cos(arg[1]), 0.02 * np.sin(arg[2]), 0.01 * np.cos(arg[0]))
    p = 1.0 + 0.025 * np.cos(arg[2])
    u0 = _pg_conserved(rho, v, p, g)
    inflow = _pg_conserved(np.array(1.0), (np.array(uin), np.array(0.0), np.array(0.0)), np.array(1.0), g)
    bc_state = np.stack([inflow, inflow])
    mesh = Mesh(3, N, x, faces, bfaces, np.zeros((0, 7), np.int32),
                np.array([BC_DIRICHLET, BC_OUTFLOW], np.int32), bc_state)
    return Case("curved_channel", cfg, mesh, u0)


def curved_map(X, amp=0.1):
    """x = X + amp*sin(pi X)sin(pi Y)sin(pi Z) added to every coordinate."""
    s = amp * np.sin(math.pi * X[0]) * np.sin(math.pi * X[1]) * np.sin(math.pi * X[2])
    return X + s[None]


def smooth_perturbation(x, seed, nmodes=3, amp=1e-3):
    """A few low Fourier modes with seeded coefficients, shape (5, ...)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((5,) + x[0].shape)
    for s in range(5):
        for _ in range(nmodes):
            kvec = rng.integers(1, 3, size=x.shape[0])
            ph = rng.uniform(0, 2 * math.pi)
            a = rng.uniform(-1.0, 1.0)
            out[s] += a * np.sin(2 * math.pi * sum(kvec[d] * x[d] for d in range(x.shape[0])) + ph)
    return amp * out / nmodes


def mixture_state(Y, rho, vel, T, energy):
    """Conserved mixture state from mass fractions, density, velocity and T.

    ``energy(rho_s, T) -> rho*e`` supplies the thermal energy density.
    """
    rho_s = Y * rho[None]
    rhoe = energy(rho_s, T)
    m = [rho * v for v in vel]
    E = rhoe + 0.5 * rho * sum(v * v for v in vel)
    return np.concatenate([rho_s] + [mm[None] for mm in m] + [E[None]], 0)


def far_chem_states(n, seed=11):
    """Seeded compositions far from chemical equilibrium, the hard cases of a
    per-node chemistry step: T 250-12000 K, rho 1e-3-1 kg/m^3 (log-uniform),
    air plus NO, N and O at mass fractions 1e-20-0.1 (log-uniform; all three
    zero in the first node of every 20).  Cold gas carrying atoms and hot
    gas with trace atoms both occur.  Returns (rho_s (5, n), T (n,))."""
    rng = np.random.default_rng(seed)
    rho = 10.0 ** rng.uniform(-3.0, 0.0, n)
    T = 10.0 ** rng.uniform(math.log10(250.0), math.log10(12000.0), n)
    Y = np.stack([np.full(n, 0.767), np.full(n, 0.233)] + [10.0 ** rng.uniform(-20.0, -1.0, n) for _ in range(3)])
    Y[3:, : n // 20] = 0.0
    Y = Y / Y.sum(0)
    return Y * rho, T


def case_c3(energy, cv, n=24, N=4, seed=3, T1=300.0, p1=1.0e4, mach=3.0, xs=0.3,
            shock=True, force_alpha=-1.0, outflow=False):
    """3D frozen 5-species Euler on the curved hex mesh with a planar shock.

    ``energy(rho_s, T)`` and ``cv(rho_s, T)`` (thermal energy and heat
    capacity densities) are supplied by the caller.  Pre-shock state at
    (T1, p1), velocity mach * frozen sound speed along x; post-shock state
    from the gamma = 1.4 Rankine-Hugoniot ratios, expressed through the
    mixture energy at the post-shock temperature.  x = 0 carries the
    pre-shock and x = 1 the post-shock state (Dirichlet; with ``outflow``
    x = 1 is an outflow boundary instead, external state = interior state);
    y and z are periodic.
    """
    sp = Species()
    x, faces, bfaces = structured_mesh(3, N, (n, n, n), (0.0,) * 3, (1.0,) * 3,
                                       (False, True, True), curved_map,
                                       bc_lo=(0, None, None), bc_hi=(1, None, None))
    Y0 = np.array([0.767, 0.233, 0.0, 0.0, 0.0])
    pert = smooth_perturbation(x, seed)
    Y = np.maximum(Y0[:, None, None] + pert, 1e-12)
    Y = Y / Y.sum(0)[None]
    Rs = sp.Ru / sp.W
    Rmix = (Y * Rs[:, None, None]).sum(0)
    rho1 = p1 / (Rmix * T1)
    # frozen sound speed of the reference composition at T1
    Yr = Y0.copy()
    Yr_rs = Yr * (p1 / ((Yr * Rs).sum() * T1))
    Tarr = np.array([T1])
    cvr = cv(Yr_rs[:, None], Tarr)[0]
    rr = Yr_rs.sum()
    gam_f = 1.0 + (Yr_rs * Rs).sum() / cvr
    a1 = math.sqrt(gam_f * p1 / rr)
    u1 = mach * a1
    g = 1.4
    M2 = mach * mach
    r_ratio = (g + 1) * M2 / ((g - 1) * M2 + 2)
    p_ratio = 1 + 2 * g / (g + 1) * (M2 - 1)
    T2 = T1 * p_ratio / r_ratio
    post = x[0] > xs
    rho = np.where(post, rho1 * r_ratio, rho1)
    T = np.where(post, T2, T1)
    ux = np.where(post, u1 / r_ratio, u1)
    zero = np.zeros_like(ux)
    u0 = mixture_state(Y, rho, (ux, zero, zero), T, energy)
    # Dirichlet boundary states (reference composition)
    def st(rho_, T_, ux_):
        rs = Y0 * rho_
        E = energy(rs[:, None], np.array([T_]))[0] + 0.5 * rho_ * ux_ * ux_
        return np.concatenate([rs, [rho_ * ux_, 0.0, 0.0, E]])
    bc_state = np.stack([st(p1 / ((Y0 * Rs).sum() * T1), T1, u1),
                         st(p1 / ((Y0 * Rs).sum() * T1) * r_ratio, T2, u1 / r_ratio)])
    mesh = Mesh(3, N, x, faces, bfaces, np.zeros((0, 7), np.int32),
                np.array([BC_DIRICHLET, BC_OUTFLOW if outflow else BC_DIRICHLET], np.int32), bc_state)
    cfg = base_cfg(3, N, EQ_EULER_MIX, volume_flux=VF_DUCROS, shock=shock,
                   force_alpha=force_alpha, T_guess=T1)
    return Case("curved_shock_air5", cfg, mesh, u0, species=sp,
                extra=dict(T1=T1, T2=T2, u1=u1, rho1=rho1, p1=p1))


def case_c4(energy, cv, nr=64, nth=128, N=3, seed=4, T=300.0, p=1.0e3, mach=8.0,
            r0=1.0, r1=8.0, shock=True, hot=False):
    """2D reacting 5-species Euler around a cylinder on an annular O-grid.

    Freestream (T, p, mach along +x) everywhere at t = 0; slip wall at
    r = r0, freestream Dirichlet state at r = r1.  ``hot=True`` replaces the
    impulsive start by a state with a hot, partly dissociated, decelerated
    layer in front of the cylinder (a seeded stand-in for the post-shock
    region) so that every term of the right-hand side is active.
    """
    sp = Species()
    rx = park17_reactions(seed)
    x, faces, bfaces = ogrid_mesh(N, nr, nth, r0, r1)
    Y0 = np.array([0.767, 0.233, 0.0, 0.0, 0.0])
    Rs = sp.Ru / sp.W
    rho = p / ((Y0 * Rs).sum() * T)
    rs = Y0 * rho
    cvv = cv(rs[:, None], np.array([T]))[0]
    gam_f = 1.0 + (rs * Rs).sum() / cvv
    a = math.sqrt(gam_f * p / rho)
    uinf = mach * a
    E = energy(rs[:, None], np.array([T]))[0] + 0.5 * rho * uinf * uinf
    state = np.concatenate([rs, [rho * uinf, 0.0, E]])
    u0 = np.broadcast_to(state[:, None, None], (8,) + x.shape[1:]).copy()
    if hot:
        rng = np.random.default_rng(seed + 100)
        g = np.exp(-((x[0] + 1.6) ** 2 + 0.5 * x[1] ** 2) / 0.6)
        Tn = 3000.0 + 5000.0 * g         # hot everywhere: finite, well-scaled sources
        f = 0.05 + 0.5 * g               # dissociated fraction
        jit = 1.0 + 0.02 * rng.uniform(-1, 1, (5, 1, 1))
        Y = np.stack([0.767 * (1 - f), 0.233 * (1 - 0.8 * f), 0.05 * f * jit[2],
                      0.767 * f * 0.9 * jit[3], 0.233 * 0.8 * f * jit[4]], 0)
        Y = Y / Y.sum(0)[None]
        rho_n = rho * (1.0 + 4.0 * g)
        ux = uinf * (1.0 - 0.85 * g)
        uy = 0.1 * uinf * g * np.sign(x[1])
        u0 = mixture_state(Y, rho_n, (ux, uy), Tn, energy)
    mesh = Mesh(2, N, x, faces, bfaces, np.zeros((0, 5), np.int32),
                np.array([BC_SLIPWALL, BC_DIRICHLET], np.int32),
                np.stack([state, state]))
    cfg = base_cfg(2, N, EQ_REACT_MIX, volume_flux=VF_DUCROS, shock=shock, T_guess=T, positivity=True)
    return Case("cylinder_air5_react", cfg, mesh, u0, species=sp, reactions=rx,
                extra=dict(T=T, p=p, uinf=uinf, rho=rho))


# ----------------------------------------------------------------------------
# Non-conforming 2:1 octree meshes (mortars) and batched cases
def _periodic_dist(a, b):
    d = np.abs(a - b)
    return np.minimum(d, 1.0 - d)


def _morton3(i, j, k, bits):
    """Interleave the bits of i, j, k (i lowest): the Z-order index."""
    code = 0
    for b in range(bits):
        code |= ((i >> b) & 1) << (3 * b) | ((j >> b) & 1) << (3 * b + 1) | ((k >> b) & 1) << (3 * b + 2)
    return code


def octree_mesh(N, base=16, radii=(0.51, 0.35), centre=(0.5, 0.5, 0.5), element_order="morton"):
    """Periodic unit cube, base^3 level-0 hexes, refined 2:1 inside spheres.

    A leaf of level L is split into 8 children while L < len(radii) and its
    centre lies within radii[L] (periodic distance) of ``centre``; then 2:1
    face balance is enforced.  Returns nodal coordinates, conforming faces
    (+d of eL to -d of eR), mortars (large face, 4 small elements ordered
    s = a + 2b over the two tangential directions in increasing order, small
    face) and the level of every element.  ``element_order`` "morton" numbers
    the leaves along the Z-order curve of their corners at the finest level
    (elements that are close in space, across levels too, are close in
    memory); "level" numbers them level by level, lexicographically.
    """
    centre = np.asarray(centre, float)
    leaves = set()
    for k in range(base):
        for j in range(base):
            for i in range(base):
                leaves.add((0, i, j, k))

    def centre_of(c):
        L, i, j, k = c
        h = 1.0 / (base * 2 ** L)
        return np.array([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h])

    def split(c):
        L, i, j, k = c
        leaves.discard(c)
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    leaves.add((L + 1, 2 * i + dx, 2 * j + dy, 2 * k + dz))

    for L, r in enumerate(radii):
        for c in [c for c in leaves if c[0] == L]:
            if np.sqrt((_periodic_dist(centre_of(c), centre) ** 2).sum()) < r:
                split(c)

    def find_leaf(L, i, j, k):
        """Leaf containing the level-L cell (i, j, k), or None if it is refined."""
        n = base * 2 ** L
        i, j, k = i % n, j % n, k % n
        for LL in range(L, -1, -1):
            s = L - LL
            c = (LL, i >> s, j >> s, k >> s)
            if c in leaves:
                return c
        return None

    # 2:1 balance
    changed = True
    while changed:
        changed = False
        for c in list(leaves):
            if c not in leaves:
                continue
            L, i, j, k = c
            for d in range(3):
                for sgn in (-1, 1):
                    ii = [i, j, k]
                    ii[d] += sgn
                    nb = find_leaf(L, *ii)
                    if nb is None:
                        # neighbour region is refined: its cells adjacent to c
                        # must be at most level L + 1
                        n2 = base * 2 ** (L + 1)
                        q = [2 * i, 2 * j, 2 * k]
                        q[d] = (2 * ii[d] + (1 if sgn < 0 else 0)) % n2
                        for a in (0, 1):
                            for b in (0, 1):
                                t = [x for x in range(3) if x != d]
                                qq = list(q)
                                qq[t[0]] += a
                                qq[t[1]] += b
                                if find_leaf(L + 1, *qq) is None:
                                    split(c)
                                    changed = True
                                    break
                            if c not in leaves:
                                break
                    if c not in leaves:
                        break
                if c not in leaves:
                    break
    if element_order == "morton":
        Lmax = max(c[0] for c in leaves)
        bits = int(base * 2 ** Lmax - 1).bit_length()
        order = sorted(leaves, key=lambda c: _morton3(c[1] << (Lmax - c[0]), c[2] << (Lmax - c[0]),
                                                      c[3] << (Lmax - c[0]), bits))
    else:
        order = sorted(leaves)
    eid = {c: e for e, c in enumerate(order)}
    xi = _mesh_nodes(N)
    n1 = N + 1
    nn = n1 ** 3
    nidx = np.stack(np.unravel_index(np.arange(nn), (n1,) * 3)[::-1], 0)
    E = len(order)
    x = np.empty((3, E, nn))
    level = np.empty(E, np.int32)
    for e, (L, i, j, k) in enumerate(order):
        h = 1.0 / (base * 2 ** L)
        level[e] = L
        for d, cc in enumerate((i, j, k)):
            x[d, e] = h * (cc + 0.5 * (xi[nidx[d]] + 1.0))
    faces, mortars = [], []
    for e, c in enumerate(order):
        L, i, j, k = c
        for d in range(3):
            t = [x_ for x_ in range(3) if x_ != d]
            for sgn in (1, -1):
                ii = [i, j, k]
                ii[d] += sgn
                nb = find_leaf(L, *ii)
                if nb is not None and nb[0] == L:
                    if sgn == 1:
                        faces.append((e, 2 * d + 1, eid[nb], 2 * d))
                    continue
                if nb is not None:
                    continue  # coarser neighbour: recorded by the large element
                # finer neighbour: this element is the large side
                n2 = base * 2 ** (L + 1)
                q = [2 * i, 2 * j, 2 * k]
                q[d] = (2 * ii[d] + (1 if sgn < 0 else 0)) % n2
                small = []
                for b in (0, 1):
                    for a in (0, 1):
                        qq = list(q)
                        qq[t[0]] += a
                        qq[t[1]] += b
                        sc = find_leaf(L + 1, *qq)
                        assert sc is not None and sc[0] == L + 1, "2:1 balance violated"
                        small.append(eid[sc])
                fl = 2 * d + (1 if sgn == 1 else 0)
                fs = 2 * d + (0 if sgn == 1 else 1)
                mortars.append(tuple([e, fl] + small + [fs]))
    return x, np.asarray(faces, np.int32).reshape(-1, 4), np.asarray(mortars, np.int32).reshape(-1, 7), level


def blob_state(x, centre=(0.4, 0.55, 0.45), width=0.1, amp=0.8, vel=(1.0, 0.5, 0.25), gamma=1.4):
    """A Gaussian density pulse on the periodic unit cube carried by a uniform
    flow at uniform pressure: rho = 1 + amp exp(-|x - centre|^2 / width^2)
    (periodic distance), p = 1."""
    d = (np.moveaxis(x, 0, -1) - np.asarray(centre) + 0.5) % 1.0 - 0.5
    rho = 1.0 + amp * np.exp(-(d * d).sum(-1) / width ** 2)
    v = tuple(np.full_like(rho, c) for c in vel)
    return _pg_conserved(rho, v, np.ones_like(rho), gamma)


def density_wave(x):
    """rho = 1 + 0.5 sin(2 pi (x + y + z)), v = (1, 0.5, 0.25), p = 1."""
    rho = 1.0 + 0.5 * np.sin(2.0 * math.pi * (x[0] + x[1] + x[2]))
    return rho, (np.ones_like(rho), 0.5 * np.ones_like(rho), 0.25 * np.ones_like(rho)), np.ones_like(rho)


def cut_periodic(N, x, faces, direction, bc_lo, bc_hi):
    """Turn the faces that close a periodic direction into boundary faces:
    the element face at the low end (-direction) gets boundary ``bc_lo``,
    the one at the high end boundary ``bc_hi``.  Returns (faces, bfaces)."""
    dim = x.shape[0]
    n1 = N + 1
    nidx = np.stack(np.unravel_index(np.arange(n1 ** dim), (n1,) * dim)[::-1], 0)
    d = direction
    lo_node = int(np.flatnonzero(nidx[d] == 0)[0])
    hi_node = int(np.flatnonzero(nidx[d] == N)[0])
    keep, bf = [], []
    for row in faces:
        eL, fL, eR, fR = (int(v) for v in row)
        if fL == 2 * d + 1 and abs(x[d][eL, hi_node] - x[d][eR, lo_node]) > 1e-9:
            bf.append((eL, fL, bc_hi))
            bf.append((eR, fR, bc_lo))
        else:
            keep.append(row)
    return np.asarray(keep, np.int32).reshape(-1, 4), np.asarray(bf, np.int32).reshape(-1, 3)


def wall_channel_case(N=3, base=4, radii=(0.3,), centre=(0.5, 0.5, 0.5), T_lo=1.2, T_hi=None, seed=9,
                      mu=2e-3, element_order="morton", **kw):
    """Navier-Stokes flow between no-slip walls on the 2:1 octree mesh of the
    unit cube: y = 0 is an isothermal wall at ``T_lo``, y = 1 an isothermal
    wall at ``T_hi`` (or an adiabatic wall when ``T_hi`` is None); x and z
    are periodic.  The state is a perturbed shear flow, u = 0.3 sin(pi y)
    plus small smooth modes in all three components, and T between the wall
    temperatures with a bump and a mode, density 1 (Mach about 0.3, R = 1,
    gamma = 1.4); the modes do not vanish at the walls, so the walls act on
    the velocity and temperature traces."""
    x, faces, mortars, level = octree_mesh(N, base, radii, centre, element_order)
    faces, bfaces = cut_periodic(N, x, faces, 1, 0, 1)
    cfg = base_cfg(3, N, EQ_NS, mu=mu, **kw)
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 3, size=(3, 2))
    ph = rng.uniform(0, 2 * math.pi, 3)
    sy = np.sin(math.pi * x[1])
    mode = [np.cos(2 * math.pi * (k[i, 0] * x[0] + k[i, 1] * x[2]) + ph[i]) for i in range(3)]
    vel = (0.3 * sy + 0.05 * mode[0], 0.05 * mode[1], 0.05 * mode[2])
    T_top = T_hi if T_hi is not None else T_lo
    T = T_lo + (T_top - T_lo) * x[1] + 0.1 * sy + 0.05 * mode[1] * mode[2]
    rho = np.ones_like(T)
    u0 = _pg_conserved(rho, vel, rho * cfg["R"] * T, cfg["gamma"])
    kinds = np.array([BC_WALL_ISOTHERMAL, BC_WALL_ISOTHERMAL if T_hi is not None else BC_WALL_ADIABATIC],
                     np.int32)
    bc_state = np.zeros((2, 5))
    bc_state[0, 0] = T_lo
    bc_state[1, 0] = T_hi if T_hi is not None else 0.0
    mesh = Mesh(3, N, x, faces, bfaces, mortars, kinds, bc_state, level=level)
    return Case("wall_channel_ns", cfg, mesh, u0)


def case_amr(N=3, base=16, radii=(0.51, 0.35), seed=5, centre=None, element_order="morton"):
    """3D Euler density wave on the 2-level non-conforming octree mesh."""
    if centre is None:
        rng = np.random.default_rng(seed)
        centre = rng.uniform(0.35, 0.65, 3)
    x, faces, mortars, level = octree_mesh(N, base, radii, centre, element_order)
    cfg = base_cfg(3, N, EQ_EULER)
    rho, v, p = density_wave(x)
    u0 = _pg_conserved(rho, v, p, cfg["gamma"])
    mesh = Mesh(3, N, x, faces, np.zeros((0, 3), np.int32), mortars, np.zeros(0, np.int32),
                np.zeros((0, 5)), level=level)
    return Case("amr_density_wave", cfg, mesh, u0, extra=dict(centre=np.asarray(centre)))


def vortex_tube_case(n, N=3, length=10.0):
    """The isentropic vortex extruded along z (w = 0), periodic n^3 hexes."""
    x, faces, bfaces = structured_mesh(3, N, (n, n, n), (0.0,) * 3, (length,) * 3, (True,) * 3)
    rho, (vx, vy), p = isentropic_vortex(x[0], x[1], 1.4, xc=0.5 * length, yc=0.5 * length)
    u0 = _pg_conserved(rho, (vx, vy, np.zeros_like(vx)), p, 1.4)
    return x, faces, u0


def concat_cases(parts):
    """Concatenate independent meshes (x, faces, mortars, u0) into one."""
    xs, fs, ms, us, offs = [], [], [], [], [0]
    off = 0
    for x, faces, mortars, u0 in parts:
        xs.append(x)
        us.append(u0)
        f = faces.copy()
        f[:, 0] += off
        f[:, 2] += off
        fs.append(f)
        if mortars is not None and len(mortars):
            m = mortars.copy()
            m[:, 0] += off
            m[:, 2:6] += off
            ms.append(m)
        off += x.shape[1]
        offs.append(off)
    mort = np.concatenate(ms, 0) if ms else np.zeros((0, 7), np.int32)
    return (np.concatenate(xs, 1), np.concatenate(fs, 0).astype(np.int32), mort.astype(np.int32),
            np.concatenate(us, 1), np.asarray(offs, np.int64))


def batch_sizes(seed=55, ncases=16, lo=8, hi=24):
    return [int(v) for v in np.random.default_rng(seed).integers(lo, hi + 1, ncases)]


def case_c5(N=3, base=16, radii=(0.51, 0.35), seed=5, batch_seed=55, ncases=16, sizes=None,
            element_order="morton"):
    """The AMR density wave plus a batch of independent vortex-tube cases in
    one mesh (element ranges in ``mesh.case_offsets``: case 0 is the AMR
    domain)."""
    amr = case_amr(N, base, radii, seed, element_order=element_order)
    parts = [(amr.mesh.x, amr.mesh.faces, amr.mesh.mortars, amr.u0)]
    sizes = batch_sizes(batch_seed, ncases) if sizes is None else sizes
    for n in sizes:
        x, faces, u0 = vortex_tube_case(n, N)
        parts.append((x, faces, None, u0))
    x, faces, mortars, u0, offs = concat_cases(parts)
    cfg = base_cfg(3, N, EQ_EULER)
    mesh = Mesh(3, N, x, faces, np.zeros((0, 3), np.int32), mortars, np.zeros(0, np.int32),
                np.zeros((0, 5)), case_offsets=offs)
    return Case("amr_plus_batch", cfg, mesh, u0, extra=dict(sizes=sizes, amr_elements=amr.mesh.nelem))

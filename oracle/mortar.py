"""Non-conforming 2:1 mortars (oracle).

Paper: Sec. New Developments, P4est based Adaptive Parabolic Solver: 1:2 (2D)
and 1:4 (3D) mortars, interpolation from the large to the small sides and
L2 projection back; Sec. Results (AMR Taylor-Green case): the projection is
computed through Gauss-Legendre points.

Reading (the paper names the operators, not their formulas):
* interpolation to the lower/upper half of a face, I_lo[i][j] = l_j((xi_i - 1)/2),
  I_hi[i][j] = l_j((xi_i + 1)/2);
* exact L2 projection back, P_s = 1/2 M^-1 I_s^T M, with the exact mass
  matrix M_ij = int l_i l_j computed by (N+1)-point Gauss-Legendre
  quadrature; in 3D the face operators are tensor products over the two
  tangential directions, sub-face s = a + 2b;
* the Riemann flux of sub-face s uses the small element's trace, the
  interpolated large trace and the small element's scaled normal; the small
  element takes it directly, the large element takes
  2^(dim-1) sum_s (P_a x P_b) F*_s (the factor is the ratio of the reference
  areas), which keeps the scheme exactly conservative.
"""
import numpy as np

from . import gas
from .basis import gauss_legendre, interpolation_matrix


def operators(basis):
    x = basis.xi
    N = basis.N
    I_lo = interpolation_matrix(x, 0.5 * (x - 1.0))
    I_hi = interpolation_matrix(x, 0.5 * (x + 1.0))
    xg, wg = gauss_legendre(N + 1)
    L = interpolation_matrix(x, xg)          # l_j(xg_q)
    M = (L * wg[:, None]).T @ L
    Minv = np.linalg.inv(M)
    P_lo = 0.5 * Minv @ I_lo.T @ M
    P_hi = 0.5 * Minv @ I_hi.T @ M
    return (I_lo, I_hi), (P_lo, P_hi)


def face_op(ops1d, s, dim):
    """Face operator of sub-face s (tensor product in 3D)."""
    if dim == 2:
        return ops1d[s]
    a, b = s & 1, s >> 1
    # face node q = qa + n1 * qb  ->  kron(B_b, A_a)
    return np.kron(ops1d[b], ops1d[a])


def mortar_surface_terms(op, s_all, G):
    b = op.b
    dim, N = op.dim, op.N
    mesh = op.mesh
    if op.mix is not None:
        raise NotImplementedError("mortars are built for the perfect gas")
    Iops, Pops = operators(b)
    nsub = 2 ** (dim - 1)
    u_all = gas.conserved(s_all)
    for row in mesh.mortars:
        eL, fL = int(row[0]), int(row[1])
        smalls = [int(v) for v in row[2:2 + nsub]]
        fS = int(row[2 + nsub])
        d, sideL = divmod(fL, 2)
        nlf = op.fn[fL]
        nsf = op.fn[fS]
        uL = u_all[:, eL, nlf]                               # (nvar, nf)
        Fl = np.zeros_like(uL)
        for s, es in enumerate(smalls):
            ui = uL @ face_op(Iops, s, dim).T                # interpolated large trace
            us = u_all[:, es, nsf]
            n = op.Ja[d][:, es, nsf]                         # small element's normal
            si = gas.pg_state(ui, dim, op.cfg["gamma"])
            ss = gas.pg_state(us, dim, op.cfg["gamma"])
            if sideL == 1:                                   # large element is on the minus side
                F = op.surface_flux(si, ss, n)
                G[:, es, nsf] -= F / b.w[0]
            else:
                F = op.surface_flux(ss, si, n)
                G[:, es, nsf] += F / b.w[N]
            Fl += nsub * (F @ face_op(Pops, s, dim).T)
        if sideL == 1:
            G[:, eL, nlf] += Fl / b.w[N]
        else:
            G[:, eL, nlf] -= Fl / b.w[0]

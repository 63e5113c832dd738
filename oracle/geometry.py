"""Element geometry from nodal coordinates (oracle).

Paper: Sec. Methodology, Eqs. mapp, mapped_equation and jacobian.  The
contravariant flux is F~ = |J| dX_i/dx_j F_j; |J| dX_i/dx_j are the metric
terms Ja^i (rows of the adjugate of dx/dX).

Reading (the paper is silent on how metric terms are discretised): 2D uses
Ja^1 = (y_eta, -x_eta), Ja^2 = (-y_xi, x_xi); 3D uses the conservative curl
form Ja^i_n = -e_i . curl_X( I^N( x_l grad_X x_m ) ), (n, m, l) cyclic, with
every derivative taken by the nodal derivative matrix.  |J| is the
determinant of the nodal Jacobian matrix.  Both are evaluated on coordinates
relative to the element's first node: the discrete curl form is invariant
under a translation (D_p and D_q act on different tensor indices and
commute), and the smaller magnitudes reduce roundoff.  Face normals are +-Ja^d at the
face nodes; subcell normals of the finite-volume blend are the telescoped
sums n_m = Ja^d_0 + sum_{l<m} w_l (D Ja^d)_l along each line.
"""
import numpy as np


def tensor(a, dim, n1):
    """(..., E, nn) -> (..., E, n1, .., n1) with the last axis = direction 0."""
    return a.reshape(a.shape[:-1] + (n1,) * dim)


def flat(a, dim):
    return a.reshape(a.shape[:-dim] + (-1,))


def ref_deriv(a, D, d, dim):
    """Apply D along reference direction d of a tensor-shaped array."""
    ax = a.ndim - 1 - d
    b = np.moveaxis(a, ax, -1)
    b = b @ D.T          # sum_j D_nj a_j
    return np.moveaxis(b, -1, ax)


def metrics(x, basis, dim):
    """Ja[i][c] (i = reference direction, c = Cartesian component) and J.

    x: (dim, E, nn).  Returns Ja with shape (dim, dim, E, nn) and J (E, nn).
    """
    n1 = basis.n1
    D = basis.D
    X = tensor(x - x[:, :, :1], dim, n1)
    # dx_c / dX_d
    dx = np.stack([np.stack([ref_deriv(X[c], D, d, dim) for d in range(dim)], 0)
                   for c in range(dim)], 0)  # dx[c][d]
    if dim == 2:
        Ja = np.empty((2, 2) + X.shape[1:], X.dtype)
        Ja[0, 0] = dx[1, 1]
        Ja[0, 1] = -dx[0, 1]
        Ja[1, 0] = -dx[1, 0]
        Ja[1, 1] = dx[0, 0]
        J = dx[0, 0] * dx[1, 1] - dx[0, 1] * dx[1, 0]
    else:
        Ja = np.empty((3, 3) + X.shape[1:], X.dtype)
        for n in range(3):
            m = (n + 1) % 3
            l = (n + 2) % 3
            # V_d = x_l * d x_m / d X_d  (nodal product = interpolant)
            V = [X[l] * dx[m, d] for d in range(3)]
            # curl components: (d1 V2 - d2 V1, d2 V0 - d0 V2, d0 V1 - d1 V0)
            c0 = ref_deriv(V[2], D, 1, 3) - ref_deriv(V[1], D, 2, 3)
            c1 = ref_deriv(V[0], D, 2, 3) - ref_deriv(V[2], D, 0, 3)
            c2 = ref_deriv(V[1], D, 0, 3) - ref_deriv(V[0], D, 1, 3)
            Ja[0, n] = -c0
            Ja[1, n] = -c1
            Ja[2, n] = -c2
        J = (dx[0, 0] * (dx[1, 1] * dx[2, 2] - dx[1, 2] * dx[2, 1])
             - dx[0, 1] * (dx[1, 0] * dx[2, 2] - dx[1, 2] * dx[2, 0])
             + dx[0, 2] * (dx[1, 0] * dx[2, 1] - dx[1, 1] * dx[2, 0]))
    return flat(Ja, dim), flat(J, dim)


def face_nodes(dim, N, f):
    """Volume node indices of local face f = 2d + s, in tangential order."""
    n1 = N + 1
    d, s = divmod(f, 2)
    idx = np.arange(n1 ** dim).reshape((n1,) * dim)   # idx[k][j][i] (3D)
    ax = dim - 1 - d
    sl = [slice(None)] * dim
    sl[ax] = 0 if s == 0 else N
    return idx[tuple(sl)].reshape(-1)


def line_view(a, d, dim, n1):
    """(..., E, nn) -> (..., E, lines, n1) with the last axis along direction d."""
    t = tensor(a, dim, n1)
    ax = t.ndim - 1 - d
    t = np.moveaxis(t, ax, -1)
    return t.reshape(t.shape[:-dim] + (-1, n1))


def line_unview(b, d, dim, n1):
    """Inverse of line_view."""
    shp = b.shape[:-2] + (n1,) * dim
    t = b.reshape(shp)
    ax = t.ndim - 1 - d
    t = np.moveaxis(t, -1, ax)
    return flat(t, dim)


def subcell_normals(Ja, basis, dim):
    """Telescoped subcell normals for each direction d.

    Returns a list over d of arrays (dim, E, lines, N+2) where entry m is the
    normal of subcell interface m (m = 0 and N+1 are the element faces).
    """
    n1 = basis.n1
    out = []
    for d in range(dim):
        Jd = np.stack([tensor(Ja[d, c], dim, n1) for c in range(dim)], 0)
        dJ = np.stack([ref_deriv(Jd[c], basis.D, d, dim) for c in range(dim)], 0)
        Jl = np.stack([line_view(flat(Jd[c], dim), d, dim, n1) for c in range(dim)], 0)
        dl = np.stack([line_view(flat(dJ[c], dim), d, dim, n1) for c in range(dim)], 0)
        ns = np.zeros(Jl.shape[:-1] + (n1 + 1,), Jl.dtype)
        ns[..., 0] = Jl[..., 0]
        for m in range(1, n1 + 1):
            ns[..., m] = ns[..., m - 1] + basis.w[m - 1] * dl[..., m - 1]
        out.append(ns)
    return out

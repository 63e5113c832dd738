"""Dynamic adaptive mesh refinement on a periodic octree (oracle).

Test infrastructure: only the tests, the smoke check and the CPU baseline
of the benchmark use this package.

Paper: Sec. New Developments (AMR with the parabolic solver; elements split
into 4 or 8; mortars with interpolation from large to small sides and exact
L2 projection back) and Sec. Results (AMR Taylor-Green case: an indicator
on a derived variable, Loehner's weighted second-derivative estimate or the
Hennemann-Gassner modal-energy coefficient in [0, 1]; a base, a medium and
a maximum level with two thresholds).

Readings (the paper names the pieces, not their formulas):
* indicator variables: density, pressure, density times pressure, or the
  velocity magnitude (perfect gas);
* Loehner's estimate, per element: the element's polynomial is sampled at
  N+1 equidistant points per direction (the estimate is a difference
  formula for uniform spacing; on the LGL nodes a linear field would not
  give 0), then along every line of samples in every reference direction,
  at every interior sample i,
    |phi_{i+1} - 2 phi_i + phi_{i-1}| /
    (|phi_{i+1} - phi_i| + |phi_i - phi_{i-1}| + f (|phi_{i+1}| + 2|phi_i| + |phi_{i-1}|)),
  f = 0.2 (0 where the denominator is 0); the element takes the maximum;
* Hennemann-Gassner: the blending coefficient of oracle.indicator with
  alpha_max = 1 and alpha_min = 1e-4;
* controller: target level = max_level where the indicator is >=
  max_threshold, else med_level where it is >= med_threshold, else
  base_level;
* one adaptation pass: every leaf whose target exceeds its level is split
  once; then leaves are split until every pair of face neighbours differs
  by at most one level (2:1 balance, periodic neighbours included); then
  every family of 8 sibling leaves that were not split, whose targets are
  all below their level, is merged into its parent, unless the parent would
  face a leaf two levels finer;
* element order: Z-order (Morton) of the leaves' lower corners on the
  finest grid;
* solution transfer: a child c = (c_x, c_y, c_z) of a split element takes
  (I_{c_z} x I_{c_y} x I_{c_x}) u_parent, I_0 / I_1 the interpolation to the
  lower / upper half of the reference interval; a merged parent takes
  sum_c (P_{c_z} x P_{c_y} x P_{c_x}) u_c with the L2 projections P of
  oracle.mortar.
"""
import math

import numpy as np

from .basis import Basis
from .indicator import modal_energy_ratio, blending_factor
from .mortar import operators

VAR_DENSITY, VAR_PRESSURE, VAR_DENSITY_PRESSURE, VAR_VELOCITY = 0, 1, 2, 3
IND_LOEHNER, IND_HENNEMANN_GASSNER = 0, 1


def variable(u, kind, gamma):
    """Indicator variable at every node, shape (E, nn) (3D perfect gas)."""
    rho = u[0]
    v = u[1:4] / rho
    p = (gamma - 1.0) * (u[4] - 0.5 * rho * (v * v).sum(0))
    if kind == VAR_DENSITY:
        return rho
    if kind == VAR_PRESSURE:
        return p
    if kind == VAR_DENSITY_PRESSURE:
        return rho * p
    return np.sqrt((v * v).sum(0))


def loehner(phi, N, f=0.2):
    """Loehner's estimate per element from nodal phi (E, (N+1)^3)."""
    from .basis import interpolation_matrix, lgl
    n1 = N + 1
    t = phi.reshape(phi.shape[0], n1, n1, n1)       # [E][k][j][i]
    Eq = interpolation_matrix(lgl(N)[0], np.linspace(-1.0, 1.0, n1))
    for ax in (1, 2, 3):
        t = np.moveaxis(np.moveaxis(t, ax, -1) @ Eq.T, -1, ax)
    best = np.zeros(phi.shape[0])
    for ax in (1, 2, 3):
        a = np.moveaxis(t, ax, -1)
        for i in range(1, N):
            pm, p0, pp = a[..., i - 1], a[..., i], a[..., i + 1]
            num = np.abs(pp - 2.0 * p0 + pm)
            den = np.abs(pp - p0) + np.abs(p0 - pm) + f * (np.abs(pp) + 2.0 * np.abs(p0) + np.abs(pm))
            with np.errstate(divide="ignore", invalid="ignore"):
                r = np.where(den > 0.0, num / den, 0.0)
            best = np.maximum(best, r.reshape(r.shape[0], -1).max(1))
    return best


def hennemann_gassner(phi, basis):
    a = blending_factor(modal_energy_ratio(phi, basis, 3), basis.N, 1.0, 1e-4)[0]
    return a


def indicator(u, N, kind, var, gamma=1.4):
    phi = variable(u, var, gamma)
    if kind == IND_LOEHNER:
        return loehner(phi, N)
    return hennemann_gassner(phi, Basis(N))


def controller(ind, base_level, med_level, max_level, med_threshold, max_threshold):
    return np.where(ind >= max_threshold, max_level, np.where(ind >= med_threshold, med_level, base_level))


# ----------------------------------------------------------------------------
# octree
def children(c):
    L, i, j, k = c
    return [(L + 1, 2 * i + a, 2 * j + b, 2 * k + cc) for cc in (0, 1) for b in (0, 1) for a in (0, 1)]


def parent(c):
    L, i, j, k = c
    return (L - 1, i // 2, j // 2, k // 2)


class Tree:
    """Leaves of a periodic octree over base^3 level-0 cells."""

    def __init__(self, base, leaves):
        self.base = base
        self.leaves = set(tuple(int(v) for v in c) for c in leaves)

    def wrap(self, L, i, j, k):
        n = self.base * 2 ** L
        return (L, i % n, j % n, k % n)

    def leaf_at(self, L, i, j, k):
        """The leaf that contains level-L cell (i, j, k), or None when that
        cell is split further."""
        L, i, j, k = self.wrap(L, i, j, k)
        for s in range(L + 1):
            c = (L - s, i >> s, j >> s, k >> s)
            if c in self.leaves:
                return c
        return None

    def face_cells(self, c, d, sgn):
        """Level-(L+1) cells across face (d, sgn) of leaf c."""
        L, i, j, k = c
        q = [2 * i, 2 * j, 2 * k]
        q[d] = 2 * (c[1 + d]) + (2 if sgn > 0 else -1)
        t = [x for x in range(3) if x != d]
        out = []
        for b in (0, 1):
            for a in (0, 1):
                qq = list(q)
                qq[t[0]] += a
                qq[t[1]] += b
                out.append(self.wrap(L + 1, *qq))
        return out

    def finest_neighbour_level(self, c):
        """Largest level among the leaves that share a face with c."""
        L, i, j, k = c
        best = -1
        for d in range(3):
            for sgn in (-1, 1):
                ii = [i, j, k]
                ii[d] += sgn
                nb = self.leaf_at(L, *ii)
                if nb is not None:
                    best = max(best, nb[0])
                    continue
                for cc in self.face_cells(c, d, sgn):
                    lf = self.leaf_at(*cc)
                    best = max(best, L + 2 if lf is None else lf[0])
        return best


def adapt(base, leaves, target):
    """One adaptation pass.  ``target``: dict leaf -> target level.
    Returns (new leaf set, plan): plan maps every new leaf to ("keep", leaf),
    ("refine", parent, child index) or ("coarsen", [8 children])."""
    tree = Tree(base, leaves)
    old = set(tree.leaves)
    split = set()
    for c in old:
        if target[c] > c[0]:
            split.add(c)
    for c in split:
        tree.leaves.discard(c)
        tree.leaves.update(children(c))
    # 2:1 balance: split any leaf that faces a leaf two levels finer
    changed = True
    while changed:
        changed = False
        for c in sorted(tree.leaves):
            if c in tree.leaves and tree.finest_neighbour_level(c) > c[0] + 1:
                tree.leaves.discard(c)
                tree.leaves.update(children(c))
                if c in old:
                    split.add(c)
                changed = True
    # coarsening of unsplit families whose targets all lie below their level
    families = {}
    for c in old:
        if c[0] > 0 and c not in split:
            families.setdefault(parent(c), []).append(c)
    merged = {}
    for p, kids in sorted(families.items()):
        if len(kids) != 8 or not all(k in tree.leaves for k in kids):
            continue
        if not all(target[k] < k[0] for k in kids):
            continue
        trial = Tree(base, (tree.leaves - set(kids)) | {p})
        if trial.finest_neighbour_level(p) > p[0] + 1:
            continue
        tree.leaves = trial.leaves
        merged[p] = children(p)
    plan = {}
    for c in tree.leaves:
        if c in old:
            plan[c] = ("keep", c)
        elif c in merged:
            plan[c] = ("coarsen", merged[c])
        else:
            # a descendant of a split old leaf (one or two levels below)
            a = c
            path = []
            while a not in old:
                path.append(((a[1] & 1) + 2 * (a[2] & 1) + 4 * (a[3] & 1)))
                a = parent(a)
            plan[c] = ("refine", a, path[::-1])
    return tree.leaves, plan


def _morton(i, j, k, bits):
    key = 0
    for b in range(bits):
        key |= ((i >> b) & 1) << (3 * b) | ((j >> b) & 1) << (3 * b + 1) | ((k >> b) & 1) << (3 * b + 2)
    return key


def morton_order(base, leaves):
    Lmax = max(c[0] for c in leaves)
    bits = max(1, int(base * 2 ** Lmax - 1).bit_length())
    return sorted(leaves, key=lambda c: _morton(c[1] << (Lmax - c[0]), c[2] << (Lmax - c[0]),
                                                c[3] << (Lmax - c[0]), bits))


def _child_op(ops1d, c):
    a, b, cc = c & 1, (c >> 1) & 1, (c >> 2) & 1
    return np.kron(ops1d[cc], np.kron(ops1d[b], ops1d[a]))


def transfer(u, old_order, new_order, plan, N):
    """New state [nvar][len(new_order)][nn] from u on old_order."""
    (I, P) = operators(Basis(N))
    eid = {c: e for e, c in enumerate(old_order)}
    nn = (N + 1) ** 3
    out = np.empty((u.shape[0], len(new_order), nn), u.dtype)
    for e, c in enumerate(new_order):
        kind = plan[c]
        if kind[0] == "keep":
            out[:, e] = u[:, eid[kind[1]]]
        elif kind[0] == "refine":
            val = u[:, eid[kind[1]]]
            for ch in kind[2]:
                val = val @ _child_op(I, ch).T
            out[:, e] = val
        else:
            acc = 0.0
            for ch, kid in enumerate(kind[1]):
                acc = acc + u[:, eid[kid]] @ _child_op(P, ch).T
            out[:, e] = acc
    return out


def mesh(base, N, order):
    """Nodal coordinates, conforming faces, mortars and levels of the leaves
    in ``order`` (the layout of the mesh tables of the library)."""
    from .basis import lgl
    tree = Tree(base, order)
    eid = {c: e for e, c in enumerate(order)}
    xi = lgl(N)[0]
    n1 = N + 1
    nn = n1 ** 3
    node = np.arange(nn)
    idx = [node % n1, (node // n1) % n1, node // (n1 * n1)]
    E = len(order)
    x = np.empty((3, E, nn))
    level = np.empty(E, np.int32)
    for e, (L, i, j, k) in enumerate(order):
        h = 1.0 / (base * 2 ** L)
        level[e] = L
        for d, cc in enumerate((i, j, k)):
            x[d, e] = h * (cc + 0.5 * (xi[idx[d]] + 1.0))
    faces, mortars = [], []
    for e, c in enumerate(order):
        L, i, j, k = c
        for d in range(3):
            for sgn in (1, -1):
                ii = [i, j, k]
                ii[d] += sgn
                nb = tree.leaf_at(L, *ii)
                if nb is not None:
                    if nb[0] == L and sgn == 1:
                        faces.append((e, 2 * d + 1, eid[nb], 2 * d))
                    continue
                small = [eid[tree.leaf_at(*cc)] for cc in tree.face_cells(c, d, sgn)]
                fl = 2 * d + (1 if sgn == 1 else 0)
                mortars.append(tuple([e, fl] + small + [fl ^ 1]))
    return x, np.asarray(faces, np.int32).reshape(-1, 4), np.asarray(mortars, np.int32).reshape(-1, 7), level

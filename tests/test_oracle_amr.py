"""Pins of the oracle's dynamic AMR (oracle/amr.py).

* Solution transfer: splitting an element evaluates its polynomial at the
  children's nodes exactly (checked against the polynomial itself);
  merging 8 children that carry one polynomial of degree <= N returns it;
  split-then-merge is the identity; merging conserves the integral of any
  children's data (the L2 projection keeps the mean).
* Loehner's estimate: 0 for a linear field, in [0, 1) always, the closed
  form for a quadratic, large at a jump; Hennemann-Gassner: the blending coefficient (pinned elsewhere).
* Adaptation: the new leaves tile the domain without overlap, every pair of
  face neighbours differs by at most one level, every leaf whose target
  exceeded its level was split, a family merges only when all its targets
  are lower, and the total integral of the state is conserved.
* Mesh tables from leaves: the oracle's own builder gives the same faces
  and mortars as the workload generator's octree mesh for the same leaves
  (two independent constructions).
"""
import numpy as np
import pytest

from oracle import amr
from oracle.basis import Basis
from oracle.dgsem import Operator
from paper_2511_17551_amd import workloads as W


def quad(N):
    w = Basis(N).w
    return np.einsum("i,j,k->kji", w, w, w).reshape(-1)


def ref_nodes(N):
    xi = Basis(N).xi
    n1 = N + 1
    node = np.arange(n1 ** 3)
    return xi[node % n1], xi[(node // n1) % n1], xi[node // (n1 * n1)]


def poly(x, y, z, N, seed=0):
    """A random polynomial of degree <= N in each variable."""
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(N + 1, N + 1, N + 1))
    out = 0.0
    for a in range(N + 1):
        for b in range(N + 1):
            for k in range(N + 1):
                out = out + c[a, b, k] * x ** a * y ** b * z ** k
    return out


@pytest.mark.parametrize("N", [3, 4])
def test_transfer_is_exact_for_polynomials(N):
    X, Y, Z = ref_nodes(N)
    parent = (0, 0, 0, 0)
    kids = amr.children(parent)
    up = poly(X, Y, Z, N)[None, None]          # one variable, one element
    plan = {k: ("refine", parent, [ch]) for ch, k in enumerate(kids)}
    u_kids = amr.transfer(up, [parent], kids, plan, N)
    for ch, k in enumerate(kids):
        a, b, c = ch & 1, (ch >> 1) & 1, (ch >> 2) & 1
        # the child's reference nodes in the parent's reference coordinates
        ref = poly(0.5 * (X + 2 * a - 1), 0.5 * (Y + 2 * b - 1), 0.5 * (Z + 2 * c - 1), N)
        assert np.abs(u_kids[0, ch] - ref).max() < 1e-12 * np.abs(ref).max()
    back = amr.transfer(u_kids, kids, [parent], {parent: ("coarsen", kids)}, N)
    assert np.abs(back - up).max() < 1e-12 * np.abs(up).max()
    # merging arbitrary children data conserves their integral
    rng = np.random.default_rng(3)
    ur = rng.normal(size=(2, 8, (N + 1) ** 3))
    pm = amr.transfer(ur, kids, [parent], {parent: ("coarsen", kids)}, N)
    w = quad(N)
    tot_kids = (ur * w).sum((1, 2)) / 8.0        # child volume = parent volume / 8
    tot_parent = (pm * w).sum((1, 2))
    assert np.abs(tot_kids - tot_parent).max() < 1e-13 * np.abs(ur).sum()


def test_loehner_estimate():
    N = 3
    X, Y, Z = ref_nodes(N)
    lin = (1.0 + 0.3 * X - 0.2 * Y + 0.5 * Z)[None]
    assert np.abs(amr.loehner(lin, N)).max() < 1e-14
    rng = np.random.default_rng(4)
    r = amr.loehner(rng.normal(size=(50, 64)), N)
    assert np.all(r >= 0.0) and np.all(r < 1.0)
    step = np.where(X > 0.0, 2.0, 1.0)[None]
    assert amr.loehner(step, N)[0] > 0.3
    # on the equidistant samples of a quadratic the estimate is exact:
    # phi = X^2 sampled at -1, -1/3, 1/3, 1: at i = 1, |1/9 - 2/9 + 1| / (|1/9 - 1/9| + |1/9 - 1| + 0.2 (1/9 + 2/9 + 1))
    q = (X * X)[None]
    ref = (1 / 9 - 2 / 9 + 1) / (0 + (1 - 1 / 9) + 0.2 * (1 / 9 + 2 / 9 + 1))
    assert abs(amr.loehner(q, N)[0] - ref) < 1e-14


def octree_leaves(base, radii, centre):
    x, faces, mortars, level = W.octree_mesh(3, base, radii, centre)
    # recover the leaves from the nodal coordinates of every element
    h = 1.0 / (base * 2.0 ** level)
    lo = x.min(2)
    return [(int(L), int(round(lo[0, e] / h[e])), int(round(lo[1, e] / h[e])), int(round(lo[2, e] / h[e])))
            for e, L in enumerate(level)], (x, faces, mortars, level)


def test_mesh_from_leaves_matches_the_generator():
    leaves, (x, faces, mortars, level) = octree_leaves(4, (0.4, 0.25), (0.45, 0.5, 0.55))
    order = amr.morton_order(4, leaves)
    x2, f2, m2, l2 = amr.mesh(4, 3, order)
    assert len(order) == x.shape[1] and np.array_equal(level, l2)
    assert np.abs(x - x2).max() < 1e-15
    assert sorted(map(tuple, faces)) == sorted(map(tuple, f2))
    assert sorted(map(tuple, mortars)) == sorted(map(tuple, m2))


def balanced(base, order):
    tree = amr.Tree(base, order)
    return all(tree.finest_neighbour_level(c) <= c[0] + 1 for c in order)


def test_adaptation_rules_and_conservation():
    base, N = 4, 3
    leaves, _ = octree_leaves(base, (0.4, 0.25), (0.45, 0.5, 0.55))
    order = amr.morton_order(base, leaves)
    x, faces, mortars, level = amr.mesh(base, N, order)
    rng = np.random.default_rng(7)
    # targets: refine a blob off-centre, coarsen elsewhere
    ctr = np.array([0.7, 0.3, 0.5])
    xc = x.mean(2).T
    dist = np.sqrt((((xc - ctr + 0.5) % 1.0 - 0.5) ** 2).sum(1))
    tgt = np.where(dist < 0.2, 2, np.where(dist < 0.3, 1, 0))
    target = {c: int(t) for c, t in zip(order, tgt)}
    new, plan = amr.adapt(base, order, target)
    new_order = amr.morton_order(base, new)
    # tiling: volumes add to 1 and no leaf contains another
    vol = sum(1.0 / (base * 2 ** c[0]) ** 3 for c in new)
    assert abs(vol - 1.0) < 1e-12
    tree = amr.Tree(base, new)
    for c in new:
        L = c[0]
        for s in range(1, L + 1):
            assert (L - s, c[1] >> s, c[2] >> s, c[3] >> s) not in tree.leaves
    assert balanced(base, new_order)
    for c in order:
        if target[c] > c[0]:
            assert c not in new and all(k in new or any(kk in new for kk in amr.children(k))
                                        for k in amr.children(c))
    for c, p in plan.items():
        if p[0] == "coarsen":
            assert all(target[k] < k[0] for k in p[1])
    assert any(p[0] == "coarsen" for p in plan.values()) and any(p[0] == "refine" for p in plan.values())
    # conservation of the integral of a state
    u = rng.normal(size=(5, len(order), (N + 1) ** 3)) + 3.0
    u2 = amr.transfer(u, order, new_order, plan, N)
    w = quad(N)
    hv = lambda ordr: np.array([(1.0 / (base * 2 ** c[0])) ** 3 / 8.0 for c in ordr])
    tot = (u * w * hv(order)[:, None]).sum((1, 2))
    tot2 = (u2 * w * hv(new_order)[:, None]).sum((1, 2))
    assert np.abs(tot - tot2).max() < 1e-13 * np.abs(tot).max()
    # the adapted mesh runs through the operator (a density wave)
    x2, f2, m2, l2 = amr.mesh(base, N, new_order)
    cfg = W.base_cfg(3, N, W.EQ_EULER)
    rho, v, p = W.density_wave(x2)
    mesh = W.Mesh(3, N, x2, f2, np.zeros((0, 3), np.int32), m2, np.zeros(0, np.int32), np.zeros((0, 5)), level=l2)
    du = Operator(cfg, mesh).rhs(W._pg_conserved(rho, v, p, 1.4))
    assert np.isfinite(du).all()


def test_controller_levels():
    ind = np.array([0.0, 0.05, 0.1, 0.15, 0.2, 0.9])
    t = amr.controller(ind, 0, 1, 2, 0.1, 0.2)
    assert list(t) == [0, 0, 1, 1, 2, 2]

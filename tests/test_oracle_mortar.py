"""Pins of the oracle mortars: projection identities, conservation and
free-stream preservation on the non-conforming octree mesh, continuity of a
degree-N polynomial across a mortar."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle.basis import Basis
from oracle.dgsem import Operator
from oracle.mortar import operators, face_op


@pytest.mark.parametrize("N", [3, 4])
def test_projection_identities(N):
    b = Basis(N)
    (I_lo, I_hi), (P_lo, P_hi) = operators(b)
    assert np.abs(P_lo @ I_lo + P_hi @ I_hi - np.eye(N + 1)).max() < 1e-13
    # interpolation is exact for polynomials of degree <= N
    for k in range(N + 1):
        assert np.abs(I_lo @ b.xi ** k - (0.5 * (b.xi - 1)) ** k).max() < 1e-13
    # the projection of the two halves of a degree-N polynomial gives it back
    f = b.xi ** N - 0.3 * b.xi
    assert np.abs(P_lo @ (I_lo @ f) + P_hi @ (I_hi @ f) - f).max() < 1e-13
    # mean preserved: w . P_s g = 1/2 w . g
    g = np.random.default_rng(0).normal(size=N + 1)
    assert abs(b.w @ (P_lo @ g) - 0.5 * b.w @ g) < 1e-14
    # 3D tensor operators: sum_s P_s I_s = identity on a face
    I4 = sum(face_op((P_lo, P_hi), s, 3) @ face_op((I_lo, I_hi), s, 3) for s in range(4))
    assert np.abs(I4 - np.eye((N + 1) ** 2)).max() < 1e-13


@pytest.fixture(scope="module")
def amr_small():
    return W.case_amr(base=4, radii=(0.4, 0.25), centre=(0.45, 0.5, 0.55))


def test_amr_mesh_tables(amr_small):
    m = amr_small.mesh
    E = m.nelem
    count = np.zeros((E, 6), int)
    for eL, fL, eR, fR in m.faces:
        count[eL, fL] += 1
        count[eR, fR] += 1
    for row in m.mortars:
        count[row[0], row[1]] += 1
        for es in row[2:6]:
            count[es, row[6]] += 1
    assert (count == 1).all()
    assert len(m.mortars) > 0


def test_amr_conservation_and_freestream(amr_small):
    c = amr_small
    op = Operator(c.cfg, c.mesh)
    du = op.rhs(c.u0)
    w = op.b.w
    wq = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
    tot = (du * op.J[None] * wq).sum(axis=(1, 2))
    scale = np.abs(du * op.J[None] * wq).sum(axis=(1, 2))
    assert np.all(np.abs(tot) < 1e-13 * scale)
    u = np.empty_like(c.u0)
    u[0] = 1.2
    u[1:4] = np.array([0.3, -0.5, 0.7])[:, None, None] * 1.2
    u[4] = 2.0 / 0.4 + 0.5 * 1.2 * (0.09 + 0.25 + 0.49)
    du = op.rhs(u)
    S = (np.abs(op.Ja).max() / op.J.min()) * 10.0
    assert np.abs(du).max() < 1e-12 * S


def test_amr_entropy_conservation(amr_small):
    """EC volume and surface fluxes on the mortar mesh: entropy production is
    at most roundoff in the conforming part and the L2 mortar coupling is
    dissipative-or-neutral only up to the projection error (checked small)."""
    import copy
    from oracle import gas
    c = amr_small
    cfg = dict(c.cfg)
    cfg["surface_flux"] = W.SF_RANOCHA
    op = Operator(cfg, c.mesh)
    du = op.rhs(c.u0)
    w = op.b.w
    wq = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
    wv = gas.entropy_variables(gas.pg_state(c.u0, 3, 1.4))
    prod = (wv * du * op.J[None] * wq)
    assert abs(prod.sum()) < 1e-3 * np.abs(prod).sum()

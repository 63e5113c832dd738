"""Shared test utilities (comparison norms, device transfer)."""
import numpy as np


def rel_err(a, b):
    """max over variables of ||a_v - b_v||_inf / ||b_v||_inf."""
    a = np.asarray(a)
    b = np.asarray(b)
    num = np.abs(a - b).reshape(a.shape[0], -1).max(1)
    den = np.abs(b).reshape(b.shape[0], -1).max(1)
    den = np.where(den > 0, den, 1.0)
    return float((num / den).max())


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def flux_scale(op, u):
    """S_v = max_n sum_d |f_v(u_n).Ja^d_n| / J_n  (oracle physical flux)."""
    from oracle import gas
    s = op.states(u)
    tot = 0.0
    for d in range(op.dim):
        tot = tot + np.abs(gas.physical_flux(s, op.Ja[d]))
    return (tot / op.J[None]).reshape(u.shape[0], -1).max(1)


def parity_err(got, ref, scale):
    """max_v ||got_v - ref_v||_inf / max(||ref_v||_inf, S_v)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    num = np.abs(got - ref).reshape(ref.shape[0], -1).max(1)
    den = np.maximum(np.abs(ref).reshape(ref.shape[0], -1).max(1), np.asarray(scale))
    # a variable that is identically zero on both sides agrees exactly
    ratio = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return float(ratio.max())


def eps_units(got, ref, scale):
    """Per variable ||got_v - ref_v||_inf / (eps_64 S_v): the difference in
    units of float64 rounding at the flux-divergence scale."""
    got = np.asarray(got, np.longdouble)
    ref = np.asarray(ref, np.longdouble)
    num = np.abs(got - ref).reshape(ref.shape[0], -1).max(1).astype(np.float64)
    return num / (np.finfo(np.float64).eps * np.asarray(scale))


def ld_reference(case, u=None):
    """The oracle's right-hand side in extended precision (x87 80-bit long
    double, eps 1.1e-19) on the same float64 inputs: the discrete operator's
    value to far below float64 rounding."""
    from oracle.dgsem import Operator
    op = Operator(case.cfg, case.mesh, case.species, case.reactions, dtype=np.longdouble)
    return op.rhs(case.u0 if u is None else u)


def oracle_dt(op, u, cfl):
    """Time step from the oracle's own states (the CFL rule of the workloads):
    cfl * 2 / ((N+1) max_n sum_d (|v.Ja^d| + c |Ja^d|) / J_n), so that no
    input of an oracle run comes from the library."""
    from oracle import gas
    s = op.states(u)
    lam = 0.0
    for d in range(op.dim):
        Ja = op.Ja[d]
        lam = lam + np.abs(gas.dot(s["v"], Ja)) + s["c"] * np.sqrt(gas.dot(Ja, Ja))
    return float(cfl * 2.0 / ((op.N + 1) * np.max(lam / op.J)))


def oracle_dt_ns(op, u, cfl=0.5, vcfl=0.2):
    """Time step of the Navier-Stokes runs: the smaller of the advective
    rule of oracle_dt and the diffusive bound vcfl dx^2 / nu_eff, with the
    node spacing dx = 4 J_min^(1/3) / (N+1)^2 and nu_eff = mu gamma / (Pr
    rho_min)."""
    s = op.states(u)
    cfg = op.cfg
    dx = 4.0 * float(op.J.min()) ** (1.0 / 3.0) / (op.N + 1) ** 2
    nu = cfg["mu"] * cfg["gamma"] / (cfg["Pr"] * float(s["rho"].min()))
    return min(oracle_dt(op, u, cfl), vcfl * dx * dx / nu)

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

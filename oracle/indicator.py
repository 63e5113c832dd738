"""Modal shock indicator and element blending factor (oracle).

Paper: Sec. Methodology, text after Eq. finitevolumeder: alpha is constant
per element, alpha in [0, alpha_max], set from the decay of the energy held
in the highest modes of an indicator quantity, following Hennemann et al.
The paper prints none of the constants; the readings below are that
method's published defaults:

* indicator quantity eps = rho * p (or p);
* modes m = (V^-1 x ... x V^-1) eps with orthonormal Legendre modes;
* E = max((E_all - E_{<=N-1}) / E_all, (E_{<=N-1} - E_{<=N-2}) / E_{<=N-1}),
  E_{<=K} summing the modes whose largest index is <= K;
* threshold T = 0.5 * 10^(-1.8 (N+1)^(1/4)), sharpness s = ln((1-1e-4)/1e-4);
* a = 1 / (1 + exp(-(s/T)(E - T))); alpha = 0 if a < alpha_min, else
  min(a, alpha_max);
* optional smoothing alpha_k <- max(alpha_k, 1/2 max over face neighbours).
"""
import math

import numpy as np

from .geometry import tensor


def modal_energy_ratio(eps, basis, dim):
    """E per element from nodal eps (E, nn)."""
    n1 = basis.n1
    N = basis.N
    m = tensor(eps, dim, n1)
    for d in range(dim):
        ax = m.ndim - 1 - d
        m = np.moveaxis(np.moveaxis(m, ax, -1) @ basis.Vinv.T, -1, ax)
    m2 = m * m
    # largest mode index of every coefficient
    idx = np.indices((n1,) * dim).max(axis=0)
    e_all = m2.reshape(m2.shape[0], -1).sum(1)
    e1 = (m2 * (idx <= N - 1)).reshape(m2.shape[0], -1).sum(1)
    e2 = (m2 * (idx <= N - 2)).reshape(m2.shape[0], -1).sum(1)
    return np.maximum((e_all - e1) / e_all, (e1 - e2) / e1)


def blending_factor(E, N, alpha_max, alpha_min):
    """Returns (alpha, alpha_raw) per element."""
    thr = 0.5 * 10.0 ** (-1.8 * (N + 1) ** 0.25)
    s = math.log((1.0 - 1e-4) / 1e-4)
    a = 1.0 / (1.0 + np.exp(-(s / thr) * (E - thr)))
    alpha = np.where(a < alpha_min, 0.0, np.minimum(a, alpha_max))
    return alpha, a


def smooth(alpha, faces, mortars=None):
    """alpha_k <- max(alpha_k, 1/2 alpha_nbr) over conforming and mortar neighbours."""
    out = alpha.copy()
    if len(faces):
        eL, eR = faces[:, 0], faces[:, 2]
        np.maximum.at(out, eL, 0.5 * alpha[eR])
        np.maximum.at(out, eR, 0.5 * alpha[eL])
    if mortars is not None and len(mortars):
        nsub = mortars.shape[1] - 3
        big = mortars[:, 0]
        for s in range(nsub):
            sm = mortars[:, 2 + s]
            np.maximum.at(out, big, 0.5 * alpha[sm])
            np.maximum.at(out, sm, 0.5 * alpha[big])
    return out

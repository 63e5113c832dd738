"""Advective fluxes, two-point volume fluxes and Riemann fluxes (oracle).

Paper: Sec. Governing Equations, Eq. adevctive_flux (physical flux),
Sec. Methodology, Eqs. riemann_problem1-3 (interface Riemann flux, Lax-
Friedrichs and HLL named), Eqs. fluxdiff/fluxdiffcons/conssymm (symmetric,
consistent two-point fluxes: entropy-conservative, or the Ducros,
Kennedy-Gruber and Pirozzoli split forms the paper lists).

A state is a dict with 'rho' (total density), 'rs' (species densities, mixture
only), 'v' (dim, ...), 'p', 'rhoE', 'c' (sound speed) and, for the perfect
gas, 'gamma'.  Conserved layout: (rho | rho_1..rho_5, rho v_1..rho v_dim,
rho E).  Normal vectors are scaled (not unit) and have shape (dim, ...).

Readings where the paper is silent:
* the entropy-conservative flux for the perfect gas is Ranocha's
  (ln-mean of rho and rho/p, with the small-difference series of the
  logarithmic mean);
* the Lax-Friedrichs (Rusanov) dissipation uses the Davis estimate
  max(|v_L.n| + c_L|n|, |v_R.n| + c_R|n|);
* HLL uses the Davis bounds min / max of v.n -+ c|n| over both sides, and
  HLLC the same bounds with Toro's contact speed and star states;
* the split forms are written as two-point fluxes with arithmetic means
  {{a}} = (a_L + a_R)/2 of the nodal quantities named in each docstring.
"""
import numpy as np


def pg_state(u, dim, gamma):
    """Perfect-gas primitives from conserved u (nvar, ...)."""
    rho = u[0]
    v = u[1:1 + dim] / rho
    rhoE = u[1 + dim]
    p = (gamma - 1.0) * (rhoE - 0.5 * rho * np.sum(v * v, axis=0))
    c = np.sqrt(gamma * p / rho)
    return dict(rho=rho, v=v, p=p, rhoE=rhoE, c=c, gamma=gamma, mix=False)


def dot(a, b):
    return np.sum(a * b, axis=0)


def physical_flux(s, n):
    """f(u).n for the Euler equations (perfect gas or mixture)."""
    vn = dot(s["v"], n)
    rows = []
    if s["mix"]:
        rows += [rs * vn for rs in s["rs"]]
    else:
        rows.append(s["rho"] * vn)
    for c in range(s["v"].shape[0]):
        rows.append(s["rho"] * s["v"][c] * vn + s["p"] * n[c])
    rows.append((s["rhoE"] + s["p"]) * vn)
    return np.stack(rows, 0)


def conserved(s):
    rows = list(s["rs"]) if s["mix"] else [s["rho"]]
    rows += [s["rho"] * s["v"][c] for c in range(s["v"].shape[0])]
    rows.append(s["rhoE"])
    return np.stack(rows, 0)


def rusanov(sL, sR, n):
    """Local Lax-Friedrichs flux  1/2 (f_L + f_R).n - 1/2 lambda (u_R - u_L)."""
    nn = np.sqrt(dot(n, n))
    lam = np.maximum(np.abs(dot(sL["v"], n)) + sL["c"] * nn,
                     np.abs(dot(sR["v"], n)) + sR["c"] * nn)
    return 0.5 * (physical_flux(sL, n) + physical_flux(sR, n)) \
        - 0.5 * lam * (conserved(sR) - conserved(sL))


def ln_mean(x, y):
    """Logarithmic mean (y - x)/ln(y/x) with the series for nearby arguments."""
    z = (x * (x - 2.0 * y) + y * y) / (x * (x + 2.0 * y) + y * y)
    small = z < 1e-4
    with np.errstate(divide="ignore", invalid="ignore"):
        big = (y - x) / np.log(y / x)
    ser = (x + y) / (2.0 + z * (2.0 / 3.0 + z * (2.0 / 5.0 + 2.0 / 7.0 * z)))
    return np.where(small, ser, big)


def ranocha(sL, sR, n):
    """Entropy-conservative, kinetic-energy-preserving two-point flux (perfect gas)."""
    g = sL["gamma"]
    rho_hat = ln_mean(sL["rho"], sR["rho"])
    beta_hat = ln_mean(sL["rho"] / sL["p"], sR["rho"] / sR["p"])
    vbar = 0.5 * (sL["v"] + sR["v"])
    pbar = 0.5 * (sL["p"] + sR["p"])
    q = 0.5 * dot(sL["v"], sR["v"])
    f_rho = rho_hat * dot(vbar, n)
    rows = [f_rho]
    for c in range(vbar.shape[0]):
        rows.append(f_rho * vbar[c] + pbar * n[c])
    rows.append(f_rho * (q + 1.0 / ((g - 1.0) * beta_hat))
                + 0.5 * (sL["p"] * dot(sR["v"], n) + sR["p"] * dot(sL["v"], n)))
    return np.stack(rows, 0)


def ducros(sL, sR, n):
    """Ducros et al. split-form two-point flux (perfect gas or mixture)."""
    vn = dot(0.5 * (sL["v"] + sR["v"]), n)
    pbar = 0.5 * (sL["p"] + sR["p"])
    rows = []
    if sL["mix"]:
        rows += [0.5 * (a + b) * vn for a, b in zip(sL["rs"], sR["rs"])]
    else:
        rows.append(0.5 * (sL["rho"] + sR["rho"]) * vn)
    for c in range(sL["v"].shape[0]):
        mbar = 0.5 * (sL["rho"] * sL["v"][c] + sR["rho"] * sR["v"][c])
        rows.append(mbar * vn + pbar * n[c])
    rows.append((0.5 * (sL["rhoE"] + sR["rhoE"]) + pbar) * vn)
    return np.stack(rows, 0)


def _mass_rows(sL, sR, f_rho):
    """Mass rows of a split form: the total mass flux f_rho, or for a mixture
    that flux times the averaged mass fractions {{rho_s/rho}} (the species
    rows then add up to f_rho)."""
    if not sL["mix"]:
        return [f_rho]
    return [f_rho * 0.5 * (a / sL["rho"] + b / sR["rho"]) for a, b in zip(sL["rs"], sR["rs"])]


def kennedy_gruber(sL, sR, n):
    """Kennedy-Gruber split form as a two-point flux, one of the split forms
    the paper lists as interchangeable volume fluxes (Sec. Methodology, after
    Eq. conssymm): mass {{rho}}{{v.n}} (mixtures: species that times
    {{rho_s/rho}}), momentum that mass flux times {{v}} plus {{p}} n, energy
    that mass flux times {{E/rho}} plus {{p}}{{v.n}}."""
    vn = dot(0.5 * (sL["v"] + sR["v"]), n)
    pbar = 0.5 * (sL["p"] + sR["p"])
    f_rho = 0.5 * (sL["rho"] + sR["rho"]) * vn
    rows = _mass_rows(sL, sR, f_rho)
    for c in range(sL["v"].shape[0]):
        rows.append(f_rho * 0.5 * (sL["v"][c] + sR["v"][c]) + pbar * n[c])
    e_bar = 0.5 * (sL["rhoE"] / sL["rho"] + sR["rhoE"] / sR["rho"])
    rows.append(f_rho * e_bar + pbar * vn)
    return np.stack(rows, 0)


def pirozzoli(sL, sR, n):
    """Pirozzoli split form as a two-point flux, listed beside Kennedy-Gruber
    (Sec. Methodology): mass and momentum as Kennedy-Gruber, energy the mass
    flux times {{h}}, h = (E + p)/rho per node."""
    vn = dot(0.5 * (sL["v"] + sR["v"]), n)
    pbar = 0.5 * (sL["p"] + sR["p"])
    f_rho = 0.5 * (sL["rho"] + sR["rho"]) * vn
    rows = _mass_rows(sL, sR, f_rho)
    for c in range(sL["v"].shape[0]):
        rows.append(f_rho * 0.5 * (sL["v"][c] + sR["v"][c]) + pbar * n[c])
    h_bar = 0.5 * ((sL["rhoE"] + sL["p"]) / sL["rho"] + (sR["rhoE"] + sR["p"]) / sR["rho"])
    rows.append(f_rho * h_bar)
    return np.stack(rows, 0)


def morinishi(sL, sR, n):
    """Morinishi's skew-symmetric splitting as a two-point flux (perfect gas),
    named beside the other split forms (Sec. Methodology): the mass flux is
    the average of the momenta, {{rho v}}.n; momentum that flux times {{v}}
    plus {{p}} n; energy that flux times the internal energy {{p/((gamma-1)
    rho)}} plus the kinetic energy of the two velocities v_L.v_R/2, plus the
    pressure work {{p v}}.n.  Parity unpinned beyond consistency, symmetry,
    kinetic-energy preservation and the mass row: the kinetic term of the
    energy row (v_L.v_R/2 rather than, say, {{|v|^2}}/2) is a reading."""
    g = sL["gamma"]
    mL, mR = sL["rho"] * sL["v"], sR["rho"] * sR["v"]
    f_rho = dot(0.5 * (mL + mR), n)
    pbar = 0.5 * (sL["p"] + sR["p"])
    rows = [f_rho]
    for c in range(sL["v"].shape[0]):
        rows.append(f_rho * 0.5 * (sL["v"][c] + sR["v"][c]) + pbar * n[c])
    e_int = 0.5 * (sL["p"] / sL["rho"] + sR["p"] / sR["rho"]) / (g - 1.0)
    kin = 0.5 * dot(sL["v"], sR["v"])
    pv = dot(0.5 * (sL["p"] * sL["v"] + sR["p"] * sR["v"]), n)
    rows.append(f_rho * (e_int + kin) + pv)
    return np.stack(rows, 0)


def hll(sL, sR, n):
    """HLL Riemann flux (named among the interface solvers, Sec. Methodology,
    Eqs. riemann_problem1-3) with Davis bounds S_L = min(v_L.n - c_L|n|,
    v_R.n - c_R|n|), S_R = max(v_L.n + c_L|n|, v_R.n + c_R|n|) (scaled n):
    f_L where S_L >= 0, f_R where S_R <= 0, otherwise
    (S_R f_L - S_L f_R + S_L S_R (u_R - u_L)) / (S_R - S_L)."""
    nn = np.sqrt(dot(n, n))
    vL, vR = dot(sL["v"], n), dot(sR["v"], n)
    SL = np.minimum(vL - sL["c"] * nn, vR - sR["c"] * nn)
    SR = np.maximum(vL + sL["c"] * nn, vR + sR["c"] * nn)
    fL, fR = physical_flux(sL, n), physical_flux(sR, n)
    uL, uR = conserved(sL), conserved(sR)
    with np.errstate(divide="ignore", invalid="ignore"):
        mid = (SR * fL - SL * fR + SL * SR * (uR - uL)) / (SR - SL)
    return np.where(SL >= 0.0, fL, np.where(SR <= 0.0, fR, mid))


def central(sL, sR, n):
    """The standard-DG form as a two-point flux (listed beside the split forms,
    Sec. Methodology): the mean of the two physical fluxes, (f(u_L) + f(u_R)).n / 2."""
    return 0.5 * (physical_flux(sL, n) + physical_flux(sR, n))


def hllc(sL, sR, n):
    """HLLC Riemann flux (named among the interface solvers, Sec.
    Methodology), perfect gas or mixture (frozen sound speed; the species
    densities of a star state scale like its total density), Davis bounds as
    in hll, on the unit normal
    n/|n| and scaled by |n|.  Contact speed
    S* = (p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R))
         / (rho_L (S_L - u_L) - rho_R (S_R - u_R)),
    star states rho_K (S_K - u_K)/(S_K - S*) (1, v_K + (S* - u_K) n,
    E_K/rho_K + (S* - u_K)(S* + p_K/(rho_K (S_K - u_K)))); the flux is f_L,
    f_L + S_L (U*_L - U_L), f_R + S_R (U*_R - U_R) or f_R as 0 lies left of
    S_L, between S_L and S*, between S* and S_R, or right of S_R."""
    nn = np.sqrt(dot(n, n))
    nh = n / nn
    uL, uR = dot(sL["v"], nh), dot(sR["v"], nh)
    SL = np.minimum(uL - sL["c"], uR - sR["c"])
    SR = np.maximum(uL + sL["c"], uR + sR["c"])
    rL, rR = sL["rho"], sR["rho"]
    Ss = (sR["p"] - sL["p"] + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR))

    def star(st, S, u):
        fac = st["rho"] * (S - u) / (S - Ss)
        # mixtures: each species density scales like the total density
        rows = [fac * rs / st["rho"] for rs in st["rs"]] if st["mix"] else [fac]
        rows += [fac * (st["v"][c] + (Ss - u) * nh[c]) for c in range(st["v"].shape[0])]
        rows.append(fac * (st["rhoE"] / st["rho"] + (Ss - u) * (Ss + st["p"] / (st["rho"] * (S - u)))))
        return np.stack(rows, 0)

    fL, fR = physical_flux(sL, nh), physical_flux(sR, nh)
    FsL = fL + SL * (star(sL, SL, uL) - conserved(sL))
    FsR = fR + SR * (star(sR, SR, uR) - conserved(sR))
    F = np.where(SL >= 0.0, fL, np.where(Ss >= 0.0, FsL, np.where(SR > 0.0, FsR, fR)))
    return F * nn


def sinhc(z):
    """sinh(z)/z with its series near 0."""
    z = np.asarray(z, dtype=float) if np.ndim(z) == 0 else z
    small = np.abs(z) < 1e-3
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        big = np.sinh(z) / z
    z2 = z * z
    return np.where(small, 1.0 + z2 / 6.0 * (1.0 + z2 / 20.0), big)


def ec_mixture(sL, sR, n, mix):
    """Entropy-conservative two-point flux for the RRHO mixture, built from
    Tadmor's condition (Sec. Methodology, Advective Fluxes) with the mixture
    entropy -sum rho_s s_s and the entropy variables w_s = (h_s - T s_s -
    |v|^2/2)/T, w_m = v/T, w_E = -1/T; beta = 1/T.  Reading (the paper
    derives such fluxes but prints none): species mass fluxes
    F_s = rho_s^ln {{v}}.n (logarithmic means of the species densities);
    momentum F_rho {{v}} + p~ n with F_rho = sum_s F_s and
    p~ = {{sum_s rho_s R_s}} / {{beta}}; energy
    sum_s e^_s F_s + F_rho (|{{v}}|^2 - {{|v|^2}}/2) + p~ {{v}}.n, where e^_s
    is the divided difference [[e_s beta - sigma_s]]/[[beta]] of the species'
    energy and thermal entropy sigma_s(T): for e_s = e0_s + c_s T +
    R_s theta_s/(exp(theta_s beta) - 1) it is
    e0_s + c_s / beta^ln + R_s [[ln(1 - exp(-theta_s beta))]]/[[beta]], the
    last term evaluated as R_s theta_s exp(-theta_s {{beta}})
    sinhc(theta_s [[beta]]/2) / ln-mean(1 - exp(-theta_s beta)), which tends
    to e_s(T) as the states meet."""
    ns = mix.ns
    bL, bR = 1.0 / sL["T"], 1.0 / sR["T"]
    bbar = 0.5 * (bL + bR)
    dB = bR - bL
    vbar = 0.5 * (sL["v"] + sR["v"])
    vn = dot(vbar, n)
    blog = ln_mean(bL, bR)
    Rs = mix.Rs
    rows = []
    F = []
    for k in range(ns):
        a, b = sL["rs"][k], sR["rs"][k]
        with np.errstate(divide="ignore", invalid="ignore"):
            m = np.where((a == 0.0) | (b == 0.0), 0.0, ln_mean(a, b))   # the limit at a zero density
        F.append(m * vn)
    f_rho = sum(F)
    rR = lambda st: sum(st["rs"][k] * Rs[k] for k in range(ns))
    pt = 0.5 * (rR(sL) + rR(sR)) / bbar
    rows = list(F)
    for c in range(vbar.shape[0]):
        rows.append(f_rho * vbar[c] + pt * n[c])
    energy = f_rho * (dot(vbar, vbar) - 0.25 * (dot(sL["v"], sL["v"]) + dot(sR["v"], sR["v"]))) + pt * vn
    for k in range(ns):
        c_k = (2.5 if mix.mol[k] else 1.5) * Rs[k]
        eh = mix.e0[k] + c_k / blog
        if mix.mol[k]:
            th = mix.th[k]
            yL, yR = -np.expm1(-th * bL), -np.expm1(-th * bR)
            eh = eh + Rs[k] * th * np.exp(-th * bbar) * sinhc(0.5 * th * dB) / ln_mean(yL, yR)
        energy = energy + eh * F[k]
    rows.append(energy)
    return np.stack(rows, 0)


def mixture_entropy_variables(s, mix):
    """w = dU/du for U = -sum_s rho_s s_s, s_s = c_s ln T + R_s [x/(e^x - 1)
    - ln(1 - e^-x)] (molecules, x = theta_s/T) - R_s ln rho_s (the additive
    constants cancel in every jump), h_s = e_s + R_s T."""
    T = s["T"]
    e = mix.e_species(T)
    v2 = dot(s["v"], s["v"])
    rows = []
    for k in range(mix.ns):
        c_k = (2.5 if mix.mol[k] else 1.5) * mix.Rs[k]
        sk = c_k * np.log(T) - mix.Rs[k] * np.log(s["rs"][k])
        if mix.mol[k]:
            x = mix.th[k] / T
            sk = sk + mix.Rs[k] * (x / np.expm1(x) - np.log(-np.expm1(-x)))
        rows.append((e[k] + mix.Rs[k] * T - T * sk - 0.5 * v2) / T)
    for c in range(s["v"].shape[0]):
        rows.append(s["v"][c] / T)
    rows.append(-1.0 / T)
    return np.stack(rows, 0)


def mixture_entropy_potential(s, mix, n):
    """psi = sum_s rho_s R_s v.n (= p v.n / T)."""
    return sum(s["rs"][k] * mix.Rs[k] for k in range(mix.ns)) * dot(s["v"], n)


def entropy_variables(s):
    """w = dU/du for U = -rho s/(gamma-1), s = ln p - gamma ln rho."""
    g = s["gamma"]
    beta = s["rho"] / s["p"]
    ent = np.log(s["p"]) - g * np.log(s["rho"])
    v2 = dot(s["v"], s["v"])
    rows = [(g - ent) / (g - 1.0) - 0.5 * beta * v2]
    rows += [beta * s["v"][c] for c in range(s["v"].shape[0])]
    rows.append(-beta)
    return np.stack(rows, 0)


def entropy_potential(s, n):
    """psi = rho v.n, the flux potential of the Tadmor condition."""
    return s["rho"] * dot(s["v"], n)


def take(s, idx):
    """Sub-state s[..., idx] (fancy index along the trailing axes)."""
    out = {}
    for k, val in s.items():
        if isinstance(val, np.ndarray):
            out[k] = val[(Ellipsis,) + idx] if isinstance(idx, tuple) else val[..., idx]
        else:
            out[k] = val
    return out

// Device-side closures and fluxes of the DGSEM right-hand side.
//
// Physical flux: Sec. Governing Equations, Eq. adevctive_flux.
// Two-point fluxes (Sec. Methodology, Eqs. fluxdiffcons and conssymm):
//   * Ranocha's entropy-conservative, kinetic-energy-preserving flux for the
//     perfect gas (logarithmic means of rho and rho/p);
//   * the Ducros split form (perfect gas or mixture).
// Riemann flux at faces and subcell interfaces (Eqs. riemann_problem1-3,
// finitevolumeflux): local Lax-Friedrichs with the wave-speed bound
// max(|v_L.n| + c_L|n|, |v_R.n| + c_R|n|).
// Mixture closures: Appendix, Thermodynamics (RRHO energies without the
// electronic mode) and Governing Equations, Eqs. internal_energies, eos.
#pragma once

#include "dgx_internal.h"

namespace dgx {

template <int DIM>
__device__ __forceinline__ double dotn(const double *a, const double *b) {
    double s = a[0] * b[0];
#pragma unroll
    for (int c = 1; c < DIM; ++c) s = fma(a[c], b[c], s);
    return s;
}

// Primitive state of one node.  For the perfect gas rs[0] is unused.
template <int DIM, bool MIX>
struct St {
    double rho, v[DIM], p, rhoE, c;
    double rs[MIX ? kNS : 1];
};

// 1/x: hardware v_rcp_f64 estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r) (each step squares the relative error).
__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// sqrt(x) for wave-speed estimates (sound speeds, face-normal lengths) of
// positive normal-range x: hardware v_rsq_f64 estimate, one coupled
// Newton-Raphson step on (sqrt x, 1/(2 sqrt x)) and a final residual
// correction, without the range scaling and special-value handling of the
// library square root.  Both sides of an interface evaluate it on identical
// inputs, so interface fluxes stay bitwise equal.
__device__ __forceinline__ double wave_sqrt(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    double g = x * r;
    double h = 0.5 * r;
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}

// Logarithmic mean (y - x)/ln(y/x) and its reciprocal.  With f = (y-x)/(y+x)
// and z = f^2, ln(y/x) = 2 atanh f, so the mean is (x+y)/(2 A(z)) with
// A(z) = atanh(sqrt z)/sqrt z = sum_n z^n/(2n+1).  Three branches by z:
//   * z < 1e-4: A to four terms, and for the mean 1/A expanded,
//     1 - z/3 - 4z^2/45 - 44z^3/945 (remainder < 1e-17 relative), which
//     saves a reciprocal;
//   * z < 0.02 (ratios y/x up to 1.33): A, and 1/A, to ten terms; the
//     coefficients of 1/A come from the exact inversion of the series of A
//     (truncation below 1e-18 relative on this range);
//   * beyond: the logarithm.
__device__ __forceinline__ double inv_atanh_ratio10(double z) {
    // 1/A(z), degree 9
    double r = -74185965772.0 / 7795859096025.0;
    r = fma(r, z, -5472607916.0 / 488462349375.0);
    r = fma(r, z, -25865068.0 / 1915538625.0);
    r = fma(r, z, -10719068.0 / 638512875.0);
    r = fma(r, z, -10196.0 / 467775.0);
    r = fma(r, z, -428.0 / 14175.0);
    r = fma(r, z, -44.0 / 945.0);
    r = fma(r, z, -4.0 / 45.0);
    r = fma(r, z, -1.0 / 3.0);
    return fma(r, z, 1.0);
}

__device__ __forceinline__ double atanh_ratio10_x2(double z) {
    // 2 A(z), degree 9
    double r = 2.0 / 19.0;
    r = fma(r, z, 2.0 / 17.0);
    r = fma(r, z, 2.0 / 15.0);
    r = fma(r, z, 2.0 / 13.0);
    r = fma(r, z, 2.0 / 11.0);
    r = fma(r, z, 2.0 / 9.0);
    r = fma(r, z, 2.0 / 7.0);
    r = fma(r, z, 2.0 / 5.0);
    r = fma(r, z, 2.0 / 3.0);
    return fma(r, z, 2.0);
}

__device__ __forceinline__ double ln_mean(double x, double y) {
    const double s = x + y;
    const double d = y - x;
    const double d2 = d * d, s2 = s * s;
    if (d2 < 1e-4 * s2) {
        const double q = d * rcp(s);
        const double z = q * q;
        const double h = 0.5 * s;
        return fma(-h * z, 1.0 / 3.0 + z * (4.0 / 45.0 + z * (44.0 / 945.0)), h);
    }
    if (d2 < 0.02 * s2) {
        const double q = d * rcp(s);
        return 0.5 * s * inv_atanh_ratio10(q * q);
    }
    return d * rcp(log(y * rcp(x)));
}

__device__ __forceinline__ double inv_ln_mean(double x, double y) {
    const double s = x + y;
    const double d = y - x;
    const double d2 = d * d, s2 = s * s;
    if (d2 < 1e-4 * s2) {
        const double rs = rcp(s);
        const double q = d * rs;
        const double z = q * q;
        const double P = 2.0 + z * (2.0 / 3.0 + z * (2.0 / 5.0 + z * (2.0 / 7.0)));
        return P * rs;
    }
    if (d2 < 0.02 * s2) {
        const double rs = rcp(s);
        const double q = d * rs;
        return atanh_ratio10_x2(q * q) * rs;
    }
    return log(y * rcp(x)) * rcp(d);
}

// ---------------------------------------------------------------- mixture
// e^-x and 1 - e^-x from one transcendental: whichever of the two is at
// least 1 - e^-1/2 (about 0.39) comes from the other by a subtraction that
// keeps it within about 2 ulp (x below 1/2: expm1, so that 1 - e^-x keeps
// its digits as x -> 0; above: exp).
__device__ __forceinline__ void exp_pair(double x, double &em, double &om) {
    if (x < 0.5) {
        om = -expm1(-x);
        em = 1.0 - om;
    } else {
        em = exp(-x);
        om = 1.0 - em;
    }
}

__device__ __forceinline__ void mix_energy_cv(const MixC &M, const double *rs, double T,
                                              double &rhoe, double &rhocv) {
    double e = 0.0, cv = 0.0;
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
        double es = 1.5 * M.Rs[s] * T + M.e0[s];
        double cs = 1.5 * M.Rs[s];
        if (M.mol[s]) {
            const double x = M.thv[s] * rcp(T);
            double em, om;  // e^-x, 1 - e^-x
            exp_pair(x, em, om);
            // R theta/(e^x - 1) = R theta e^-x / (1 - e^-x); its T-derivative R x^2 e^-x / (1 - e^-x)^2
            const double q = em * rcp(om);
            es += M.Rs[s] * T + M.Rs[s] * M.thv[s] * q;
            cs += M.Rs[s] + M.Rs[s] * x * x * q * rcp(om);
        }
        e = fma(rs[s], es, e);
        cv = fma(rs[s], cs, cv);
    }
    rhoe = e;
    rhocv = cv;
}

// Newton iteration on sum rho_s e_s(T) = rho e, from T0; returns iterations,
// or -1 if maxit was reached.  Stops when |dT| <= tol*T, or when the residual
// is at the rounding level of the energies it is made of (8 eps times
// |rho e| + sum_s |rho_s e0_s|): where the thermal energy is itself that small
// (near-vacuum gas left by the positivity limiter, T of order 1e-10 K) no
// iterate meets a relative test, and T is as accurate as the data allow.
__device__ __forceinline__ int mix_newton(const MixC &M, const double *rs, double rhoe_target,
                                          double &T, double tol, int maxit) {
    double floor = fabs(rhoe_target);
#pragma unroll
    for (int s = 0; s < kNS; ++s) floor = fma(fabs(rs[s]), fabs(M.e0[s]), floor);
    floor *= 8.0 * 2.220446049250313e-16;
    for (int it = 1; it <= maxit; ++it) {
        double f, fp;
        mix_energy_cv(M, rs, T, f, fp);
        const double r = f - rhoe_target;
        const double dT = r / fp;
        T -= dT;
        if (fabs(dT) <= tol * fabs(T) || fabs(r) <= floor) return it;
    }
    return -1;
}

__device__ __forceinline__ double mix_rR(const MixC &M, const double *rs) {
    double r = 0.0;
#pragma unroll
    for (int s = 0; s < kNS; ++s) r = fma(rs[s], M.Rs[s], r);
    return r;
}

// Frozen sound speed sqrt(gamma_f p / rho), gamma_f = 1 + sum rho_s R_s / sum rho_s cv_s.
__device__ __forceinline__ double mix_sound(const MixC &M, const double *rs, double rho, double T) {
    double cv = 0.0;
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
        double cs = 1.5 * M.Rs[s];
        if (M.mol[s]) {
            const double x = M.thv[s] * rcp(T);
            double em, om;
            exp_pair(x, em, om);
            cs += M.Rs[s] + M.Rs[s] * x * x * em * rcp(om * om);
        }
        cv = fma(rs[s], cs, cv);
    }
    const double rR = mix_rR(M, rs);
    const double g = 1.0 + rR / cv;
    return wave_sqrt(g * rR * T / rho);
}

// State of a node from its conserved vector (and T for a mixture).
template <int DIM, bool MIX>
// (mixtures: c is the given frozen sound speed when cgiven is not null)
__device__ __forceinline__ void make_state(const double *u, double T, double gamma, const MixC &M,
                                           St<DIM, MIX> &s, const double *cgiven = nullptr) {
    if constexpr (MIX) {
        double rho = 0.0;
#pragma unroll
        for (int k = 0; k < kNS; ++k) {
            s.rs[k] = u[k];
            rho += u[k];
        }
        s.rho = rho;
        const double ir = rcp(rho);
#pragma unroll
        for (int c = 0; c < DIM; ++c) s.v[c] = u[kNS + c] * ir;
        s.rhoE = u[kNS + DIM];
        const double rR = mix_rR(M, s.rs);
        s.p = rR * T;
        s.c = cgiven ? *cgiven : mix_sound(M, s.rs, rho, T);
    } else {
        s.rho = u[0];
        const double ir = rcp(u[0]);
        double v2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            s.v[c] = u[1 + c] * ir;
            v2 = fma(s.v[c], s.v[c], v2);
        }
        s.rhoE = u[1 + DIM];
        s.p = (gamma - 1.0) * (s.rhoE - 0.5 * s.rho * v2);
        s.c = wave_sqrt(gamma * s.p * ir);
        s.rs[0] = 0.0;
    }
}

// f(u).n
template <int DIM, bool MIX>
__device__ __forceinline__ void phys_flux(const St<DIM, MIX> &s, const double *n, double *f) {
    const double vn = dotn<DIM>(s.v, n);
    constexpr int off = MIX ? kNS : 1;
    if constexpr (MIX) {
#pragma unroll
        for (int k = 0; k < kNS; ++k) f[k] = s.rs[k] * vn;
    } else {
        f[0] = s.rho * vn;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) f[off + c] = s.rho * s.v[c] * vn + s.p * n[c];
    f[off + DIM] = (s.rhoE + s.p) * vn;
}

template <int DIM, bool MIX>
__device__ __forceinline__ void cons_of(const St<DIM, MIX> &s, double *u) {
    constexpr int off = MIX ? kNS : 1;
    if constexpr (MIX) {
#pragma unroll
        for (int k = 0; k < kNS; ++k) u[k] = s.rs[k];
    } else {
        u[0] = s.rho;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) u[off + c] = s.rho * s.v[c];
    u[off + DIM] = s.rhoE;
}

// HLL flux with the Davis bounds S_L = min(v_L.n - c_L|n|, v_R.n - c_R|n|),
// S_R = max(v_L.n + c_L|n|, v_R.n + c_R|n|) (scaled n): the upwind physical
// flux when both bounds have one sign, otherwise the flux of the single
// intermediate state that conserves the integral over the wave fan.
template <int DIM, bool MIX>
__device__ __forceinline__ void hll(const St<DIM, MIX> &L, const St<DIM, MIX> &R, const double *n,
                                    double *F) {
    constexpr int NV = (MIX ? kNS : 1) + DIM + 1;
    const double nn = wave_sqrt(dotn<DIM>(n, n));
    const double vL = dotn<DIM>(L.v, n), vR = dotn<DIM>(R.v, n);
    const double sL = fmin(vL - L.c * nn, vR - R.c * nn);
    const double sR = fmax(vL + L.c * nn, vR + R.c * nn);
    if (sL >= 0.0) {
        phys_flux<DIM, MIX>(L, n, F);
    } else if (sR <= 0.0) {
        phys_flux<DIM, MIX>(R, n, F);
    } else {
        double fL[NV], fR[NV], uL[NV], uR[NV];
        phys_flux<DIM, MIX>(L, n, fL);
        phys_flux<DIM, MIX>(R, n, fR);
        cons_of<DIM, MIX>(L, uL);
        cons_of<DIM, MIX>(R, uR);
        const double iw = 1.0 / (sR - sL);
        const double sLR = sL * sR;
#pragma unroll
        for (int k = 0; k < NV; ++k) F[k] = (sR * fL[k] - sL * fR[k] + sLR * (uR[k] - uL[k])) * iw;
    }
}

// HLLC flux, the HLL bounds with Toro's contact speed
// S* = (p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R))
//      / (rho_L (S_L - u_L) - rho_R (S_R - u_R)) on the unit normal, and the
// star states rho_K (S_K - u_K)/(S_K - S*) (1, v_K + (S* - u_K) n,
// E_K/rho_K + (S* - u_K)(S* + p_K/(rho_K (S_K - u_K)))); scaled by |n|.  For
// a mixture c is the frozen sound speed and the species densities of a star
// state scale like its total density.
template <int DIM, bool MIX>
__device__ __forceinline__ void hllc(const St<DIM, MIX> &L, const St<DIM, MIX> &R, const double *n,
                                     double *F) {
    constexpr int off = MIX ? kNS : 1;
    constexpr int NV = off + DIM + 1;
    const double nn = wave_sqrt(dotn<DIM>(n, n));
    const double inn = rcp(nn);
    double nh[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) nh[c] = n[c] * inn;
    const double uL = dotn<DIM>(L.v, nh), uR = dotn<DIM>(R.v, nh);
    const double sL = fmin(uL - L.c, uR - R.c);
    const double sR = fmax(uL + L.c, uR + R.c);
    const St<DIM, MIX> &K = sL >= 0.0 ? L : R;  // the upwind state when 0 is outside the fan
    if (sL >= 0.0 || sR <= 0.0) {
        phys_flux<DIM, MIX>(K, n, F);
        return;
    }
    const double mL = L.rho * (sL - uL), mR = R.rho * (sR - uR);
    const double ss = (R.p - L.p + mL * uL - mR * uR) / (mL - mR);
    const bool left = ss >= 0.0;
    const St<DIM, MIX> &S = left ? L : R;
    const double sk = left ? sL : sR, uk = left ? uL : uR, mk = left ? mL : mR;
    double f[NV], u[NV], us[NV];
    phys_flux<DIM, MIX>(S, nh, f);
    cons_of<DIM, MIX>(S, u);
    const double fac = mk / (sk - ss);
    if constexpr (MIX) {
#pragma unroll
        for (int k = 0; k < kNS; ++k) us[k] = fac * (S.rs[k] / S.rho);
    } else {
        us[0] = fac;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) us[off + c] = fac * (S.v[c] + (ss - uk) * nh[c]);
    us[off + DIM] = fac * (S.rhoE / S.rho + (ss - uk) * (ss + S.p / mk));
#pragma unroll
    for (int k = 0; k < NV; ++k) F[k] = (f[k] + sk * (us[k] - u[k])) * nn;
}

// The standard-DG form as a two-point flux: (f(u_L) + f(u_R)).n / 2.
template <int DIM, bool MIX>
__device__ __forceinline__ void central_state(const St<DIM, MIX> &L, const St<DIM, MIX> &R, const double *n,
                                              double *F) {
    constexpr int NV = (MIX ? kNS : 1) + DIM + 1;
    double fL[NV], fR[NV];
    phys_flux<DIM, MIX>(L, n, fL);
    phys_flux<DIM, MIX>(R, n, fR);
#pragma unroll
    for (int k = 0; k < NV; ++k) F[k] = 0.5 * (fL[k] + fR[k]);
}

template <int DIM, bool MIX>
__device__ __forceinline__ void rusanov(const St<DIM, MIX> &L, const St<DIM, MIX> &R,
                                        const double *n, double *F) {
    constexpr int NV = (MIX ? kNS : 1) + DIM + 1;
    const double nn = wave_sqrt(dotn<DIM>(n, n));
    const double lam = fmax(fabs(dotn<DIM>(L.v, n)) + L.c * nn, fabs(dotn<DIM>(R.v, n)) + R.c * nn);
    double fL[NV], fR[NV], uL[NV], uR[NV];
    phys_flux<DIM, MIX>(L, n, fL);
    phys_flux<DIM, MIX>(R, n, fR);
    cons_of<DIM, MIX>(L, uL);
    cons_of<DIM, MIX>(R, uR);
#pragma unroll
    for (int k = 0; k < NV; ++k) F[k] = 0.5 * (fL[k] + fR[k]) - 0.5 * lam * (uR[k] - uL[k]);
}

// Ranocha flux from primitive values (perfect gas).
template <int DIM>
__device__ __forceinline__ void ranocha_prims(double rL, const double *vL, double pL, double bL, double rR,
                                              const double *vR, double pR, double bR, const double *n,
                                              double gm1_inv, double *F) {
    const double rho_hat = ln_mean(rL, rR);
    const double ibeta_hat = inv_ln_mean(bL, bR);
    double vbar[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) vbar[c] = 0.5 * (vL[c] + vR[c]);
    const double pbar = 0.5 * (pL + pR);
    const double q = 0.5 * dotn<DIM>(vL, vR);
    const double frho = rho_hat * dotn<DIM>(vbar, n);
    F[0] = frho;
#pragma unroll
    for (int c = 0; c < DIM; ++c) F[1 + c] = frho * vbar[c] + pbar * n[c];
    F[1 + DIM] = frho * (q + gm1_inv * ibeta_hat) + 0.5 * (pL * dotn<DIM>(vR, n) + pR * dotn<DIM>(vL, n));
}

template <int DIM, bool MIX>
__device__ __forceinline__ void ranocha_state(const St<DIM, MIX> &L, const St<DIM, MIX> &R,
                                              const double *n, double gamma, double *F) {
    const double bL = L.rho / L.p, bR = R.rho / R.p;
    ranocha_prims<DIM>(L.rho, L.v, L.p, bL, R.rho, R.v, R.p, bR, n, 1.0 / (gamma - 1.0), F);
}

// Split forms as two-point fluxes with arithmetic means {{a}} = (a_L + a_R)/2.
// FORM 0 Kennedy-Gruber and 1 Pirozzoli: mass flux f = {{rho}}{{v.n}}
// (mixtures: species rows f {{rho_s/rho}}), momentum f {{v}} + {{p}} n,
// energy f {{E/rho}} + {{p}}{{v.n}} (Kennedy-Gruber) or f {{(E + p)/rho}}
// (Pirozzoli).  FORM 2 Morinishi (perfect gas): f = {{rho v}}.n, momentum as
// above, energy f ({{p/((gamma-1) rho)}} + v_L.v_R/2) + {{p v}}.n.
template <int DIM, bool MIX, int FORM>
__device__ __forceinline__ void split_form_state(const St<DIM, MIX> &L, const St<DIM, MIX> &R,
                                                 const double *n, double gm1_inv, double *F) {
    static_assert(!(MIX && FORM == 2), "Morinishi's form is perfect-gas only");
    constexpr int off = MIX ? kNS : 1;
    double vb[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) vb[c] = 0.5 * (L.v[c] + R.v[c]);
    const double vn = dotn<DIM>(vb, n);
    const double pbar = 0.5 * (L.p + R.p);
    const double iL = 1.0 / L.rho, iR = 1.0 / R.rho;
    double fm;
    if constexpr (FORM == 2) {
        double mb[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) mb[c] = 0.5 * (L.rho * L.v[c] + R.rho * R.v[c]);
        fm = dotn<DIM>(mb, n);
    } else {
        fm = 0.5 * (L.rho + R.rho) * vn;
    }
    if constexpr (MIX) {
#pragma unroll
        for (int k = 0; k < kNS; ++k) F[k] = fm * (0.5 * (L.rs[k] * iL + R.rs[k] * iR));
    } else {
        F[0] = fm;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) F[off + c] = fm * vb[c] + pbar * n[c];
    if constexpr (FORM == 2) {
        const double eint = 0.5 * (L.p * iL + R.p * iR) * gm1_inv;
        double pv[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) pv[c] = 0.5 * (L.p * L.v[c] + R.p * R.v[c]);
        F[off + DIM] = fm * (eint + 0.5 * dotn<DIM>(L.v, R.v)) + dotn<DIM>(pv, n);
    } else if constexpr (FORM == 1) {
        F[off + DIM] = fm * (0.5 * ((L.rhoE + L.p) * iL + (R.rhoE + R.p) * iR));
    } else {
        F[off + DIM] = fm * (0.5 * (L.rhoE * iL + R.rhoE * iR)) + pbar * vn;
    }
}

// sinh(z)/z, with its series near 0
__device__ __forceinline__ double sinhc(double z) {
    const double z2 = z * z;
    if (fabs(z) < 1e-3) return fma(z2 * (1.0 / 6.0), fma(z2, 1.0 / 20.0, 1.0), 1.0);
    return sinh(z) / z;
}

// Entropy-conservative flux of the RRHO mixture (Tadmor's condition with
// the mixture entropy -sum rho_s s_s; beta = 1/T = sum rho_s R_s / p):
// species fluxes rho_s^ln {{v}}.n (0 where a density is 0, the limit),
// momentum F_rho {{v}} + p~ n with p~ = {{sum rho_s R_s}}/{{beta}}, energy
// sum_s e^_s F_s + F_rho (|{{v}}|^2 - {{|v|^2}}/2) + p~ {{v}}.n, with the
// energy means e^_s = e0_s + c_s / beta^ln (c_s = 3/2 R_s, 5/2 R_s for
// molecules) + R_s theta_s exp(-theta_s {{beta}}) sinhc(theta_s [[beta]]/2)
// / ln-mean(1 - exp(-theta_s beta)) for molecules.
template <int DIM>
__device__ __forceinline__ void ec_mixture_state(const St<DIM, true> &L, const St<DIM, true> &R, const double *n,
                                                 const MixC &M, double *F) {
    const double rRL = mix_rR(M, L.rs), rRR = mix_rR(M, R.rs);
    const double bL = rRL / L.p, bR = rRR / R.p;
    const double bbar = 0.5 * (bL + bR), dB = bR - bL;
    const double iblog = inv_ln_mean(bL, bR);
    double vb[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) vb[c] = 0.5 * (L.v[c] + R.v[c]);
    const double vn = dotn<DIM>(vb, n);
    const double pt = 0.5 * (rRL + rRR) / bbar;
    double frho = 0.0, en = 0.0;
#pragma unroll
    for (int k = 0; k < kNS; ++k) {
        const double a = L.rs[k], b = R.rs[k];
        const double m = (a == b) ? a : (a == 0.0 || b == 0.0) ? 0.0 : ln_mean(a, b);
        const double fk = m * vn;
        F[k] = fk;
        frho += fk;
        double eh = fma(M.mol[k] ? 2.5 * M.Rs[k] : 1.5 * M.Rs[k], iblog, M.e0[k]);
        if (M.mol[k]) {
            const double th = M.thv[k];
            const double yL = -expm1(-th * bL), yR = -expm1(-th * bR);
            eh += M.Rs[k] * th * exp(-th * bbar) * sinhc(0.5 * th * dB) / ln_mean(yL, yR);
        }
        en = fma(eh, fk, en);
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) F[kNS + c] = fma(frho, vb[c], pt * n[c]);
    const double k2 = dotn<DIM>(vb, vb) - 0.25 * (dotn<DIM>(L.v, L.v) + dotn<DIM>(R.v, R.v));
    F[kNS + DIM] = en + frho * k2 + pt * vn;
}

// Ducros split-form flux: {{rho_s}} {{v}}.n, {{m}} {{v}}.n + {{p}} n, ({{rhoE}} + {{p}}) {{v}}.n
template <int DIM, bool MIX>
__device__ __forceinline__ void ducros_state(const St<DIM, MIX> &L, const St<DIM, MIX> &R,
                                             const double *n, double *F) {
    double vb[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) vb[c] = 0.5 * (L.v[c] + R.v[c]);
    const double vn = dotn<DIM>(vb, n);
    const double pbar = 0.5 * (L.p + R.p);
    constexpr int off = MIX ? kNS : 1;
    if constexpr (MIX) {
#pragma unroll
        for (int k = 0; k < kNS; ++k) F[k] = 0.5 * (L.rs[k] + R.rs[k]) * vn;
    } else {
        F[0] = 0.5 * (L.rho + R.rho) * vn;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double mbar = 0.5 * (L.rho * L.v[c] + R.rho * R.v[c]);
        F[off + c] = mbar * vn + pbar * n[c];
    }
    F[off + DIM] = (0.5 * (L.rhoE + R.rhoE) + pbar) * vn;
}

}  // namespace dgx

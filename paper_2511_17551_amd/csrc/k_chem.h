// Per-node stiff chemistry: backward-Euler steps of the species sources
// (Governing Equations, Eq. source_term; Appendix, Chemical Kinetics) with
// the transport split off.  Density, momentum and total energy stay fixed,
// hence so does rho e, and one step over h from rho_s^a solves
//
//   G(rho_s) = rho_s - rho_s^a - h * omega_s(rho_s, T(rho_s, rho e)) = 0.
//
// Newton's method with the analytic Jacobian along the fixed-energy manifold,
//   d omega_s / d rho_j = W_s sum_r dnu_rs [ (dR_r/dc_j) / W_j
//                                            + (dR_r/dT) dT/drho_j ],
//   dT/drho_j = -e_j(T) / sum_k rho_k cv_k(T),
// where dR_r/dT uses d ln k_f/dT = (b + theta_a/T)/T and the van 't Hoff form
// d ln K_c/dT = -sum_s dnu_s/T + sum_s dnu_s h_s / (R_s T^2), h_s = e_s + R_s T
// (the Gibbs-Helmholtz relation of the Gibbs energies the rates use).  Each
// iterate's temperature comes from the T(e) Newton solve warm-started at the
// previous one.  The step is limited so that densities stay non-negative and
// the thermal energy rho e - sum_s rho_s e0_s stays positive; the iteration
// stops when the full Newton step is below tol * rho.
//
// Substeps.  A growing mode (atom-impact dissociation grows [X] at a rate
// k [X2]) makes I - h d omega/d rho singular as h times its growth rate
// reaches 1; past that the root near rho^a is gone, the Newton step points
// out of the admissible set and the positivity limit cuts it to nothing.  The
// iteration has failed when that limit leaves less than kChemStall of the
// step on two consecutive iterations (or after maxit iterations); the node
// then covers dt with substeps dt / 2^k: a failed substep is retried at half
// the size, and after a successful one the node goes back to the next larger
// size when its position is a multiple of it.  Positions are integers in
// units of dt / 2^kChemKmax; failing at the smallest size is
// non-convergence.
#pragma once

#include "physics.h"

namespace dgx {

// Species sources w_s and their Jacobian dw[s][j] = d w_s / d rho_j along the
// fixed-energy manifold, at the temperature T of the composition rs.
__device__ __forceinline__ void chem_sources(const KinC &K, const MixC &M, const double *rs, double T, double *w,
                                             double (*dw)[kNS]) {
    const double lnT = log(T);
    const double iT = rcp(T);
    double gRT[kNS], dgRT[kNS], conc[kNS], es[kNS];
    double rhocv = 0.0;
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
        double e = 1.5 * M.Rs[s] * T + M.e0[s];
        double cv = 1.5 * M.Rs[s];
        double g = K.gconst[s] - 2.5 * lnT + M.e0[s] * iT / M.Rs[s];
        if (M.mol[s]) {
            const double x = M.thv[s] * iT;
            double em, om;  // e^-x, 1 - e^-x
            exp_pair(x, em, om);
            const double q = em * rcp(om);
            e += M.Rs[s] * T + M.Rs[s] * M.thv[s] * q;
            cv += M.Rs[s] + M.Rs[s] * x * x * q * rcp(om);
            g += -lnT + log(om);
        }
        es[s] = e;
        rhocv = fma(rs[s], cv, rhocv);
        gRT[s] = g;                                    // g_s / (R_s T)
        dgRT[s] = -(e + M.Rs[s] * T) * iT * iT / M.Rs[s];  // d(g_s/(R_s T))/dT
        conc[s] = rs[s] / K.W[s];
        w[s] = 0.0;
#pragma unroll
        for (int j = 0; j < kNS; ++j) dw[s][j] = 0.0;
    }
    const double irc = rcp(rhocv);
    double dTdr[kNS];
#pragma unroll
    for (int j = 0; j < kNS; ++j) dTdr[j] = -es[j] * irc;
    const double lnpr = K.lnpref_Ru - lnT;
    for (int r = 0; r < K.nr; ++r) {
        double lnK = K.dnu_sum[r] * lnpr;
        double dlnK = -K.dnu_sum[r] * iT;
        double fw = 1.0, bw = 1.0;
        double dfw[kNS], dbw[kNS];
#pragma unroll
        for (int j = 0; j < kNS; ++j) {
            const int nu = K.nu[r][j], nup = K.nup[r][j];
            lnK -= (double)(nup - nu) * gRT[j];
            dlnK -= (double)(nup - nu) * dgRT[j];
            for (int q = 0; q < nu; ++q) fw *= conc[j];
            for (int q = 0; q < nup; ++q) bw *= conc[j];
        }
        // d(prod_k c_k^nu_k)/dc_j = nu_j c_j^(nu_j - 1) prod_{k != j} c_k^nu_k
#pragma unroll
        for (int j = 0; j < kNS; ++j) {
            double pf = 0.0, pb = 0.0;
            const int nuj = K.nu[r][j], nupj = K.nup[r][j];
            if (nuj > 0) {
                pf = (double)nuj;
                for (int q = 1; q < nuj; ++q) pf *= conc[j];
#pragma unroll
                for (int k = 0; k < kNS; ++k)
                    if (k != j)
                        for (int q = 0; q < K.nu[r][k]; ++q) pf *= conc[k];
            }
            if (nupj > 0) {
                pb = (double)nupj;
                for (int q = 1; q < nupj; ++q) pb *= conc[j];
#pragma unroll
                for (int k = 0; k < kNS; ++k)
                    if (k != j)
                        for (int q = 0; q < K.nup[r][k]; ++q) pb *= conc[k];
            }
            dfw[j] = pf;
            dbw[j] = pb;
        }
        const double lnkf = fma(K.b[r], lnT, K.lnA[r]) - K.tha[r] * iT;
        const double kf = exp(lnkf);
        const double kb = exp(lnkf - lnK);  // k_f / K_c without the underflow of both at low T
        const double dlnkf = (K.b[r] + K.tha[r] * iT) * iT;
        const double R = kf * fw - kb * bw;
        const double dRdT = kf * fw * dlnkf - kb * bw * (dlnkf - dlnK);
        double dRdr[kNS];
#pragma unroll
        for (int j = 0; j < kNS; ++j) dRdr[j] = (kf * dfw[j] - kb * dbw[j]) / K.W[j] + dRdT * dTdr[j];
#pragma unroll
        for (int s = 0; s < kNS; ++s) {
            const int dn = K.nup[r][s] - K.nu[r][s];
            if (dn != 0) {
                const double c = K.W[s] * (double)dn;
                w[s] = fma(c, R, w[s]);
#pragma unroll
                for (int j = 0; j < kNS; ++j) dw[s][j] = fma(c, dRdr[j], dw[s][j]);
            }
        }
    }
}

// x = A^{-1} b for the 5x5 system (Gaussian elimination, partial pivoting;
// row exchanges by selects so that the arrays stay in registers).
__device__ __forceinline__ void solve5(double (*A)[kNS], double *b, double *x) {
#pragma unroll
    for (int c = 0; c < kNS; ++c) {
        // pivot: the largest |A[k][c]|, k >= c, swapped into row c
        double best = fabs(A[c][c]);
        int piv = c;
#pragma unroll
        for (int k = c + 1; k < kNS; ++k)
            if (fabs(A[k][c]) > best) {
                best = fabs(A[k][c]);
                piv = k;
            }
#pragma unroll
        for (int k = c + 1; k < kNS; ++k) {
            const bool sw = (k == piv);
#pragma unroll
            for (int j = c; j < kNS; ++j) {
                const double t = A[c][j];
                A[c][j] = sw ? A[k][j] : A[c][j];
                A[k][j] = sw ? t : A[k][j];
            }
            const double t = b[c];
            b[c] = sw ? b[k] : b[c];
            b[k] = sw ? t : b[k];
        }
        const double ip = rcp(A[c][c]);
#pragma unroll
        for (int k = c + 1; k < kNS; ++k) {
            const double f = A[k][c] * ip;
#pragma unroll
            for (int j = c + 1; j < kNS; ++j) A[k][j] = fma(-f, A[c][j], A[k][j]);
            b[k] = fma(-f, b[c], b[k]);
        }
    }
#pragma unroll
    for (int c = kNS - 1; c >= 0; --c) {
        double s = b[c];
#pragma unroll
        for (int j = c + 1; j < kNS; ++j) s = fma(-A[c][j], x[j], s);
        x[c] = s / A[c][c];
    }
}

constexpr int kChemKmax = 20;        // smallest substep dt / 2^20
constexpr double kChemStall = 1e-3;  // a step cut below this fraction twice in a row has failed

// Damped Newton for one backward-Euler step over h from ra into rs.  Tn: the
// temperature of ra on entry, of rs on a converged exit.  Adds the
// iterations to it; returns false if the iteration failed.
__device__ __forceinline__ bool chem_newton(const KinC &K, const MixC &M, const double *ra, double *rs, double rho,
                                            double rhoe, double h, double &Tn, double tol, int maxit, double ttol,
                                            int tmaxit, int &it) {
#pragma unroll
    for (int s = 0; s < kNS; ++s) rs[s] = ra[s];
    int low = 0;
    for (int k = 0; k < maxit; ++k) {
        ++it;
        if (mix_newton(M, rs, rhoe, Tn, ttol, tmaxit) < 0 || !(Tn > 0.0)) return false;
        double w[kNS], A[kNS][kNS], G[kNS], d[kNS];
        chem_sources(K, M, rs, Tn, w, A);
#pragma unroll
        for (int s = 0; s < kNS; ++s) {
            G[s] = -(rs[s] - ra[s] - h * w[s]);
#pragma unroll
            for (int j = 0; j < kNS; ++j) A[s][j] = (s == j ? 1.0 : 0.0) - h * A[s][j];
        }
        solve5(A, G, d);
        // step limits: rho_s >= 0 and a positive thermal energy
        double theta = 1.0, thermal = rhoe, de0 = 0.0, dmax = 0.0;
#pragma unroll
        for (int s = 0; s < kNS; ++s) {
            if (rs[s] + d[s] < 0.0) theta = fmin(theta, -0.9 * rs[s] / d[s]);
            thermal -= rs[s] * M.e0[s];
            de0 = fma(d[s], M.e0[s], de0);
            dmax = fmax(dmax, fabs(d[s]));
        }
        if (de0 > 0.0) theta = fmin(theta, 0.9 * thermal / de0);
#pragma unroll
        for (int s = 0; s < kNS; ++s) rs[s] = fma(theta, d[s], rs[s]);
        if (!(dmax == dmax)) return false;
        if (dmax <= tol * rho) return mix_newton(M, rs, rhoe, Tn, ttol, tmaxit) >= 0;
        low = theta < kChemStall ? low + 1 : 0;
        if (low >= 2) return false;
    }
    return false;
}

// Chemistry over dt per node, in place on the species rows of u
// ([nvar][count], species first).  Two waves per SIMD: the Newton state,
// the 5x5 Jacobian and the per-reaction terms need about 280 registers, and
// one wave per SIMD leaves the long dependency chains (T solve, rates,
// elimination) unhidden; the compiler spills 33 VGPRs at this bound, a
// better trade (1.45x on the 131,072-node cylinder) than one wave.  T holds the incoming state's temperature
// on entry (warm start) and the new one on exit; iters (optional) the Newton
// iterations summed over the substeps, -1 if the node did not converge;
// subs (optional) the number of substeps.
template <int DIM>
__global__ void __launch_bounds__(256, 2) k_chem(double *__restrict__ u, int64_t count, double dt, const KinC *kin,
                                              MixC M, double *__restrict__ T, double tol, int maxit, double ttol,
                                              int tmaxit, int *__restrict__ iters, int *__restrict__ subs,
                                              unsigned *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const KinC &K = *kin;
    double ra[kNS];
    double rho = 0.0;
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
        ra[s] = u[s * count + i];
        rho += ra[s];
    }
    double m2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double m = u[(kNS + c) * count + i];
        m2 = fma(m, m, m2);
    }
    const double rhoe = u[(kNS + DIM) * count + i] - 0.5 * m2 / rho;
    double Ta = T[i];
    constexpr int unit = 1 << kChemKmax;
    int pos = 0, lev = 0, it = 0, nsub = 0;
    bool conv = true;
    while (pos < unit) {
        if (lev > kChemKmax) {
            conv = false;
            break;
        }
        double rs[kNS];
        double Tn = Ta;
        if (chem_newton(K, M, ra, rs, rho, rhoe, ldexp(dt, -lev), Tn, tol, maxit, ttol, tmaxit, it)) {
#pragma unroll
            for (int s = 0; s < kNS; ++s) ra[s] = rs[s];
            Ta = Tn;
            pos += unit >> lev;
            ++nsub;
            if (lev > 0 && (pos & ((unit >> (lev - 1)) - 1)) == 0) --lev;
        } else {
            ++lev;
        }
    }
#pragma unroll
    for (int s = 0; s < kNS; ++s) u[s * count + i] = ra[s];
    T[i] = Ta;
    if (iters) iters[i] = conv ? it : -1;
    if (subs) subs[i] = nsub;
    if (!conv) atomicOr(flags, FLAG_NOCONV);
}

}  // namespace dgx

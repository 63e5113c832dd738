// Per-node stiff chemistry: one backward-Euler step of the species sources
// (Governing Equations, Eq. source_term; Appendix, Chemical Kinetics) with
// the transport split off.  Density, momentum and total energy stay fixed,
// hence so does rho e, and the species densities solve
//
//   G(rho_s) = rho_s - rho_s^n - dt * omega_s(rho_s, T(rho_s, rho e)) = 0.
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
            const double em = exp(-x);
            const double om = -expm1(-x);
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
        const double kf = K.A[r] * exp(K.b[r] * lnT - K.tha[r] * iT);
        const double kb = kf * exp(-lnK);
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

// One backward-Euler chemistry step per node, in place on the species rows
// of u ([nvar][count], species first).  T holds the previous temperature on
// entry (warm start) and the new one on exit; iters (optional) the Newton
// iteration count, -1 if it did not converge.
template <int DIM>
__global__ void __launch_bounds__(256) k_chem(double *__restrict__ u, int64_t count, double dt, const KinC *kin,
                                              MixC M, double *__restrict__ T, double tol, int maxit, double ttol,
                                              int tmaxit, int *__restrict__ iters, unsigned *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const KinC &K = *kin;
    double r0[kNS], rs[kNS];
    double rho = 0.0;
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
        r0[s] = u[s * count + i];
        rs[s] = r0[s];
        rho += r0[s];
    }
    double m2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double m = u[(kNS + c) * count + i];
        m2 = fma(m, m, m2);
    }
    const double rhoe = u[(kNS + DIM) * count + i] - 0.5 * m2 / rho;
    double Tn = T[i];
    int it = 0;
    bool conv = false;
    bool fail = false;
    while (it < maxit) {
        ++it;
        if (mix_newton(M, rs, rhoe, Tn, ttol, tmaxit) < 0 || !(Tn > 0.0)) {
            fail = true;
            break;
        }
        double w[kNS], A[kNS][kNS], G[kNS], d[kNS];
        chem_sources(K, M, rs, Tn, w, A);
#pragma unroll
        for (int s = 0; s < kNS; ++s) {
            G[s] = -(rs[s] - r0[s] - dt * w[s]);
#pragma unroll
            for (int j = 0; j < kNS; ++j) A[s][j] = (s == j ? 1.0 : 0.0) - dt * A[s][j];
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
        if (!(dmax == dmax)) {
            fail = true;
            break;
        }
        if (dmax <= tol * rho) {
            conv = true;
            break;
        }
    }
    if (conv && mix_newton(M, rs, rhoe, Tn, ttol, tmaxit) < 0) conv = false;
#pragma unroll
    for (int s = 0; s < kNS; ++s) u[s * count + i] = rs[s];
    T[i] = Tn;
    if (iters) iters[i] = conv ? it : -1;
    if (!conv || fail) atomicOr(flags, FLAG_NOCONV);
}

}  // namespace dgx

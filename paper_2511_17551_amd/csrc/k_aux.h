// Auxiliary kernels of the right-hand side: BR1 gradients, mixture
// temperature, shock indicator, time-step bound.
#pragma once

#include "k_rhs.h"

namespace dgx {

// BR1 viscous terms, element-local part (Sec. Methodology, Viscous Fluxes,
// Eqs. auxil and auxstrongf; Appendix, Transport, Eq. stress; Sec. New
// Developments, gradient and viscous-flux patching across interfaces and
// mortars; Sec. Results, weak boundaries with the external state averaged
// with the interior one for the viscous terms).
//
// Per element: gradients q = (1/J) sum_d Ja^d [D_d W + lift(W* - W)] of
// W = (v, T = p/(rho R)), the nodal viscous flux F_v[c] = (tau_{.c},
// (tau v)_c + kappa dT/dx_c) and its contravariant form Ft^d = Ja^d . F_v.
// Interface values W*: (W_own + W_nbr)/2 on conforming faces; on a mortar
// face the small side's W*_s from the mortar gradient pass, the large side
// sum_s (P_a x P_b) W*_s; on a boundary face the mean with the external
// state (Dirichlet: the boundary state; outflow: W* = W; slip wall: the
// mirrored velocity), (0, T_wall) at an isothermal and (0, T) at an
// adiabatic no-slip wall.  The divergence with the interface flux F*,
//   (1/J) [ sum_d D_d Ft^d + (F* - Ft_own)/w_N |_{xi_d = 1} - (F* - Ft_own)/w_0 |_{xi_d = -1} ],
// is split into what this element knows (written to P.out, [dim+1][E][nn])
// and the face values Ft^d at its face nodes (written to P.grad as
// [E][2 dim][dim+1][nf]): on conforming and mortar faces F* is completed
// by the right-hand side kernel (the neighbour's half, or the mortar's
// averaged sub-face fluxes), on boundary faces F* = F_v(W*, q).n (viscosity
// at the temperature of W*; no heat flux at an adiabatic wall) is applied
// here.  CURV: nodal metric terms; OPEN: the mesh has boundary or mortar
// faces (the face values W* stay in LDS for the boundary fluxes).
template <int DIM, int N, bool OPEN = false>
struct GradShape {
    static constexpr int N1 = N + 1;
    static constexpr int NN = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    static constexpr int NF = NN / N1;
    static constexpr int NW = DIM + 1;
    static constexpr int NSF = 2 * DIM * NF;
    // own W and the neighbours' face traces of W (or the face values W*);
    // then the contravariant viscous fluxes of all directions, over the
    // traces, or after them when those are still needed
    static constexpr int SLOT0 = NW * NN + NW * NSF;
    static constexpr int OFF_T = OPEN ? SLOT0 : 0;
    static constexpr int SLOT = OPEN ? SLOT0 + DIM * NW * NN : (SLOT0 > DIM * NW * NN ? SLOT0 : DIM * NW * NN);
};

// Viscous flux F_v[c] (momentum, energy rows) of velocity v, gradients q,
// viscosity mu and conductivity kappa.
template <int DIM>
__device__ __forceinline__ void visc_flux(const double *v, const double (*q)[DIM + 1], double mu, double kappa,
                                          double (*Fv)[DIM + 1]) {
    double div = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) div += q[k][k];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        double en = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double t = mu * (q[c][k] + q[k][c]);
            if (k == c) t -= (2.0 / 3.0) * mu * div;
            en = fma(t, v[k], en);
            Fv[c][k] = t;
        }
        Fv[c][DIM] = en + kappa * q[c][DIM];
    }
}

// suthS > 0: Sutherland's law mu(T) = mu (T/T0)^(3/2) (T0 + S)/(T + S)
// (Eq. sutherland) at every node, the conductivity scaled alike (constant
// Pr); suthS = 0: constant mu.
template <int DIM, int N, bool CURV = false, bool OPEN = false>
__global__ void __launch_bounds__(512) k_grad(RhsParams P, double suthS, double suthT0) {
    using S = GradShape<DIM, N, OPEN>;
    constexpr int N1 = N + 1, NN = S::NN, NF = S::NF, NW = S::NW, NSF = S::NSF;
    constexpr int NV = DIM + 2;
    constexpr int GA = DIM * DIM + 1;
    constexpr int NSUB = DIM == 3 ? 4 : 2;
    extern __shared__ double smem[];
    __shared__ double sD[N1 * N1];  // read with per-lane indices
    const int tid = threadIdx.x;
    if (tid < N1 * N1) sD[tid] = P.B.D[tid];
    const int NT = P.epb * NN;
    const int e0 = (P.xcd ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x) * P.epb;
    const int nloc = min(P.epb, P.nelem - e0);
    int el = tid / NN;
    const int node = tid - el * NN;
    const bool valid = el < nloc;
    const int e = e0 + (valid ? el : 0);
    if (el >= P.epb) el = 0;
    double *sw = smem + el * S::SLOT;
    double *sn = sw + NW * NN;
    const unsigned stride = (unsigned)P.nelem * NN;
    const unsigned gi = (unsigned)e * NN + node;

    auto prim = [&](const double *u, double *W) {
        const double ir = rcp(u[0]);
        double v2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            W[c] = u[1 + c] * ir;
            v2 = fma(W[c], W[c], v2);
        }
        const double p = (P.gamma - 1.0) * (u[1 + DIM] - 0.5 * u[0] * v2);
        W[DIM] = p * ir / P.R;
    };
    auto transport = [&](double T, double &mu, double &kappa) {
        mu = P.mu;
        kappa = P.kappa;
        if (suthS > 0.0) {
            const double th = T / suthT0;
            const double f = th * sqrt(th) * (suthT0 + suthS) / (T + suthS);
            mu *= f;
            kappa *= f;
        }
    };
    // scaled normal Ja^d at node nd of element ee
    auto normal = [&](int ee, int d, int nd, double *n) {
#pragma unroll
        for (int c = 0; c < DIM; ++c)
            n[c] = CURV ? P.geo[(size_t)(d * DIM + c) * stride + (size_t)ee * NN + nd]
                        : P.geo[(size_t)ee * GA + d * DIM + c];
    };

    // Neighbour face traces (or, on an open mesh, the own trace at boundary
    // faces): one item per face node of every element of the workgroup,
    // spread over all threads; all loads are issued up front.
    constexpr int RF = (NSF + NN - 1) / NN;
    const Spread spf = spread_phase(tid, NT, P.epb * NSF, 0);
    double un[RF][NV];
    int slot[RF], code[RF], item[RF];
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        const int it = r * NT + spf.t;
        slot[r] = -1;
        code[r] = 0;
        item[r] = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) un[r][v] = 1.0;
        if (tid < NT && it < nloc * NSF) {
            const int ei = it / NSF;
            const int fi = it - ei * NSF;
            const int f = fi / NF;
            const int q = fi - f * NF;
            const int d = f >> 1, side = f & 1;
            const int nb = P.nbr[(e0 + ei) * 2 * DIM + f];
            code[r] = nb;
            item[r] = it;
            slot[r] = ei * S::SLOT + NW * NN + fi;
            unsigned gj;
            if (!OPEN || nb >= 0) {
                gj = (unsigned)nb * NN + line_node<N1, DIM>(d, side ? 0 : N, q);
            } else if (nb > kMortBase) {
                gj = (unsigned)(e0 + ei) * NN + line_node<N1, DIM>(d, side ? N : 0, q);
            } else {
                continue;  // mortar face: W* from the mortar gradient pass
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) un[r][v] = (P.u + (size_t)v * stride)[gj];
        }
    }
    double Wo[NW];
    if (valid) {
        double uo[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) uo[v] = (P.u + (size_t)v * stride)[gi];
        prim(uo, Wo);
#pragma unroll
        for (int w = 0; w < NW; ++w) sw[w * NN + node] = Wo[w];
    } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) Wo[w] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        if (slot[r] < 0) continue;
        double Wn[NW];
        const int nb = code[r];
        if (!OPEN || nb >= 0) {
            prim(un[r], Wn);
        } else {
            const int ei = item[r] / NSF;
            const int fi = item[r] - ei * NSF;
            const int f = fi / NF;
            const int q = fi - f * NF;
            const int d = f >> 1;
            if (nb > kMortBase) {
                // boundary face: W* from the own trace and the boundary kind
                const int bc = -1 - nb;
                const int kind = P.bc_kind[bc];
                double Wf[NW];
                prim(un[r], Wf);
                if (kind == 0) {
                    double ue[NV], We[NW];
#pragma unroll
                    for (int v = 0; v < NV; ++v) ue[v] = P.bc_state[bc * NV + v];
                    prim(ue, We);
#pragma unroll
                    for (int w = 0; w < NW; ++w) Wn[w] = 0.5 * (Wf[w] + We[w]);
                } else if (kind == 1) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) Wn[w] = Wf[w];
                } else if (kind == 2) {
                    double n[DIM];
                    normal(e0 + ei, d, line_node<N1, DIM>(d, (f & 1) ? N : 0, q), n);
                    const double vn = dotn<DIM>(Wf, n) / dotn<DIM>(n, n);
#pragma unroll
                    for (int c = 0; c < DIM; ++c) Wn[c] = Wf[c] - vn * n[c];
                    Wn[DIM] = Wf[DIM];
                } else {
#pragma unroll
                    for (int c = 0; c < DIM; ++c) Wn[c] = 0.0;
                    Wn[DIM] = kind == 3 ? P.bc_state[bc * NV] : Wf[DIM];
                }
            } else {
                const int mc = kMortBase - nb;
                const int m = mc >> 3, role = mc & 7;
                const double *mg = P.mgw + (size_t)m * NSUB * NW * NF;
                if (role < NSUB) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) Wn[w] = mg[(role * NW + w) * NF + q];
                } else {
                    // large side: sum_s (P_a x P_b) W*_s
#pragma unroll
                    for (int w = 0; w < NW; ++w) Wn[w] = 0.0;
                    const int qa = q % N1, qb = q / N1;
#pragma unroll 1
                    for (int sb = 0; sb < NSUB; ++sb) {
                        const int a = sb & 1, bsel = sb >> 1;
#pragma unroll 1
                        for (int j = 0; j < NF; ++j) {
                            const int ja = j % N1, jb = j / N1;
                            double wt = P.mops[50 + a * 25 + qa * N1 + ja];
                            if (DIM == 3) wt *= P.mops[50 + bsel * 25 + qb * N1 + jb];
#pragma unroll
                            for (int w = 0; w < NW; ++w) Wn[w] = fma(wt, mg[(sb * NW + w) * NF + j], Wn[w]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int w = 0; w < NW; ++w) smem[slot[r] + w * NSF] = Wn[w];
    }
    __syncthreads();
    // with a multiple of 64 nodes per element every wave holds one element:
    // its metric terms then live in scalar registers
    const int eu = (NN % 64 == 0) ? __builtin_amdgcn_readfirstlane(e) : e;
    double Ja[DIM * DIM];
    double iJ;
    if constexpr (CURV) {
#pragma unroll
        for (int k = 0; k < DIM * DIM; ++k) Ja[k] = P.geo[(size_t)k * stride + gi];
        iJ = 1.0 / P.Jn[gi];
    } else {
        const double *g = P.geo + (size_t)eu * GA;
#pragma unroll
        for (int k = 0; k < DIM * DIM; ++k) Ja[k] = g[k];
        iJ = 1.0 / g[DIM * DIM];
    }
    // face codes of this node's faces (open meshes)
    int fcode[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        fcode[d] = 0;
        if constexpr (OPEN) {
            const int a = node_pos<N1>(node, d);
            if (valid && (a == 0 || a == N)) fcode[d] = P.nbr[(size_t)e * 2 * DIM + 2 * d + (a == N ? 1 : 0)];
        }
    }
    double q[DIM][NW];
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int w = 0; w < NW; ++w) q[c][w] = 0.0;
    if (valid) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const int a = node_pos<N1>(node, d);
            const int l = node_line<N1, DIM>(node, d);
            double dW[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) dW[w] = 0.0;
#pragma unroll
            for (int j = 0; j < N1; ++j) {
                const double Dj = sD[a * N1 + j];
                const int nj = line_node<N1, DIM>(d, j, l);
#pragma unroll
                for (int w = 0; w < NW; ++w) dW[w] = fma(Dj, sw[w * NN + nj], dW[w]);
            }
            if (a == 0 || a == N) {
                const int side = (a == N) ? 1 : 0;
                const int fi = (2 * d + side) * NF + l;
                const double sc = side ? 1.0 / P.B.w[N] : -1.0 / P.B.w[0];
                const bool star = OPEN && fcode[d] < 0;  // the trace slot holds W* itself
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const double ws = star ? sn[w * NSF + fi] : 0.5 * (Wo[w] + sn[w * NSF + fi]);
                    dW[w] = fma(sc, ws - Wo[w], dW[w]);
                }
            }
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int w = 0; w < NW; ++w) q[c][w] = fma(Ja[d * DIM + c], dW[w], q[c][w]);
        }
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int w = 0; w < NW; ++w) q[c][w] *= iJ;
    // nodal viscous flux
    double Fv[DIM][NW];
    {
        double mu, kappa;
        transport(Wo[DIM], mu, kappa);
        visc_flux<DIM>(Wo, q, mu, kappa, Fv);
    }
    // divergence: volume part and the element's own half of the face terms.
    // All directions' contravariant fluxes go to LDS at once.
    double vis[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) vis[k] = 0.0;
    double *ff = P.out2;
    double *ft = smem + el * S::SLOT + S::OFF_T;  // [DIM][NW][NN]
    if (!OPEN) __syncthreads();  // the gradient's readers of sw and sn are done
    if (valid) {
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < DIM; ++c) s = fma(Ja[d * DIM + c], Fv[c][k], s);
                ft[(d * NW + k) * NN + node] = s;
            }
    }
    __syncthreads();
    if (valid) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const int a = node_pos<N1>(node, d);
            const int l = node_line<N1, DIM>(node, d);
#pragma unroll
            for (int j = 0; j < N1; ++j) {
                const double Dj = sD[a * N1 + j];
                const int nj = line_node<N1, DIM>(d, j, l);
#pragma unroll
                for (int k = 0; k < NW; ++k) vis[k] = fma(Dj, ft[(d * NW + k) * NN + nj], vis[k]);
            }
            if (a == 0 || a == N) {
                const int side = (a == N) ? 1 : 0;
                double *fo = ff + ((size_t)e * 2 * DIM + 2 * d + side) * NW * NF + l;
                if (OPEN && fcode[d] < 0 && fcode[d] > kMortBase) {
                    // boundary face: F* = F_v(W*, q).n, applied in full here
                    const int bc = -1 - fcode[d];
                    const int kind = P.bc_kind[bc];
                    const int fi = (2 * d + side) * NF + l;
                    double Wb[NW], mu, kappa, Fb[DIM][NW];
#pragma unroll
                    for (int w = 0; w < NW; ++w) Wb[w] = sn[w * NSF + fi];
                    transport(Wb[DIM], mu, kappa);
                    visc_flux<DIM>(Wb, q, mu, kind == 4 ? 0.0 : kappa, Fb);
                    const double sc = side ? 1.0 / P.B.w[N] : -1.0 / P.B.w[0];
#pragma unroll
                    for (int k = 0; k < NW; ++k) {
                        double Fs = 0.0;
#pragma unroll
                        for (int c = 0; c < DIM; ++c) Fs = fma(Ja[d * DIM + c], Fb[c][k], Fs);
                        if (kind == 4 && k == DIM) Fs = 0.0;
                        const double Ftk = ft[(d * NW + k) * NN + node];
                        vis[k] = fma(sc, Fs - Ftk, vis[k]);
                        fo[k * NF] = Ftk;
                    }
                } else {
                    const double sc = side ? -0.5 / P.B.w[N] : 0.5 / P.B.w[0];
#pragma unroll
                    for (int k = 0; k < NW; ++k) {
                        const double Ftk = ft[(d * NW + k) * NN + node];
                        vis[k] = fma(sc, Ftk, vis[k]);
                        fo[k * NF] = Ftk;
                    }
                }
            }
        }
    }
    if (valid) {
#pragma unroll
        for (int k = 0; k < NW; ++k) (P.out + (size_t)k * stride)[gi] = vis[k] * iJ;
    }
}

// Mortar gradient pass (BR1 on 2:1 meshes): one thread per small-face node
// of every mortar sub-face.  The large element's conserved trace is
// interpolated to the node (I_a x I_b), W* = (W_small + W(I u_large))/2 is
// written to P.out as [nm][2^(dim-1)][dim+1][nf] for the gradient kernel
// (the small side reads it, the large side projects it back).  Perfect gas,
// affine elements.
template <int DIM, int N>
__global__ void __launch_bounds__(256) k_mortar_grad(RhsParams P, int nmort) {
    constexpr int N1 = N + 1;
    constexpr int NN = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    constexpr int NF = NN / N1;
    constexpr int NV = DIM + 2, NW = DIM + 1;
    constexpr int NSUB = DIM == 3 ? 4 : 2;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nmort * NSUB * NF) return;
    const int m = t / (NSUB * NF);
    const int r = t - m * NSUB * NF;
    const int s = r / NF, q = r - s * NF;
    const int *row = P.mort + (size_t)m * (3 + NSUB);
    const int eL = row[0], fL = row[1], es = row[2 + s], fS = row[2 + NSUB];
    const int d = fL >> 1, sideL = fL & 1;
    const size_t stride = (size_t)P.nelem * NN;
    const int a = s & 1, bsel = s >> 1;
    const int qa = q % N1, qb = q / N1;
    double ui[NV], us[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ui[v] = 0.0;
    for (int j = 0; j < NF; ++j) {
        const int ja = j % N1, jb = j / N1;
        double w = P.mops[a * 25 + qa * N1 + ja];
        if (DIM == 3) w *= P.mops[bsel * 25 + qb * N1 + jb];
        const size_t gj = (size_t)eL * NN + line_node<N1, DIM>(d, sideL ? N : 0, j);
#pragma unroll
        for (int v = 0; v < NV; ++v) ui[v] = fma(w, P.u[v * stride + gj], ui[v]);
    }
    const size_t gs = (size_t)es * NN + line_node<N1, DIM>(d, (fS & 1) ? N : 0, q);
#pragma unroll
    for (int v = 0; v < NV; ++v) us[v] = P.u[v * stride + gs];
    double Wi[NW], Ws[NW];
    auto prim = [&](const double *u, double *W) {
        const double ir = rcp(u[0]);
        double v2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            W[c] = u[1 + c] * ir;
            v2 = fma(W[c], W[c], v2);
        }
        const double p = (P.gamma - 1.0) * (u[1 + DIM] - 0.5 * u[0] * v2);
        W[DIM] = p * ir / P.R;
    };
    prim(ui, Wi);
    prim(us, Ws);
    double *o = P.out + (size_t)m * NSUB * NW * NF;
#pragma unroll
    for (int w = 0; w < NW; ++w) o[(s * NW + w) * NF + q] = 0.5 * (Ws[w] + Wi[w]);
}

// The per-node T(e) solve (Appendix, Thermodynamics) of the conserved state
// uo of one node (species first): Newton from t (T0 when t is not a positive
// number); a failed warm start (warm != 0) is retried from T0.  Returns the
// iteration count, < 0 on failure; rs, rho for the caller.
template <int DIM>
__device__ __forceinline__ int node_temperature_state(const double *uo, double &t, double T0, double tol, int maxit,
                                                      const MixC &M, int warm, double *rs, double &rho) {
    rho = 0.0;
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
        rs[s] = uo[s];
        rho += rs[s];
    }
    double m2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) m2 = fma(uo[kNS + c], uo[kNS + c], m2);
    const double rhoe = uo[kNS + DIM] - 0.5 * m2 / rho;
    if (!(t > 0.0) || !isfinite(t)) t = T0;
    int it = mix_newton(M, rs, rhoe, t, tol, maxit);
    if (warm && (it < 0 || !isfinite(t) || !(t > 0.0))) {
        t = T0;
        it = mix_newton(M, rs, rhoe, t, tol, maxit);
    }
    return (it < 0 || !isfinite(t) || !(t > 0.0)) ? -1 : it;
}

// The same for node i of u ([nvar][count]).
template <int DIM>
__device__ __forceinline__ int node_temperature(const double *__restrict__ u, size_t count, size_t i, double &t,
                                                double T0, double tol, int maxit, const MixC &M, int warm,
                                                double *rs, double &rho) {
    double uo[kNS + DIM + 1];
#pragma unroll
    for (int v = 0; v < kNS + DIM + 1; ++v) uo[v] = u[v * count + i];
    return node_temperature_state<DIM>(uo, t, T0, tol, maxit, M, warm, rs, rho);
}

// Per-node T(e) Newton (Appendix, Thermodynamics).  Tguess may be null
// (use T0).  Writes T, optionally p, and the iteration count.
template <int DIM>
__global__ void __launch_bounds__(256) k_thermo(const double *__restrict__ u, int64_t count,
                                                const double *__restrict__ Tguess, double T0,
                                                double tol, int maxit, MixC M, double *__restrict__ T,
                                                double *__restrict__ pout, double *__restrict__ cout,
                                                int *__restrict__ iters, unsigned *flags, int warm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double rs[kNS], rho;
    // guess: the given one (a learned guess), or with warm != 0 the node's
    // previous T (the right-hand side's solves), else T0.  A failed warm
    // start, and a failed solve from a given guess, are retried from T0, so
    // the converged T never depends on how good the guess was; the
    // iteration count then includes both attempts, and the retry is marked
    // in the count (bit kItersFallback) for the statistics.
    double t = Tguess ? Tguess[i] : (warm ? T[i] : T0);
    int it = node_temperature<DIM>(u, (size_t)count, (size_t)i, t, T0, tol, maxit, M, warm, rs, rho);
    bool fell_back = false;
    if (Tguess && it < 0) {
        t = T0;
        const int it2 = node_temperature<DIM>(u, (size_t)count, (size_t)i, t, T0, tol, maxit, M, 0, rs, rho);
        it = it2 < 0 ? -1 : it2 + maxit;
        fell_back = true;
    }
    T[i] = t;
    if (pout) pout[i] = mix_rR(M, rs) * t;
    if (cout) cout[i] = mix_sound(M, rs, rho, t);
    if (iters) iters[i] = it < 0 ? -1 : (fell_back ? (it | kItersFallback) : it);
    if (it < 0) atomicOr(flags, FLAG_NOCONV);
}

// Modal shock indicator (Hennemann et al. type, as referenced in
// Sec. Methodology): eps = rho*p or p, orthonormal Legendre modes by V^-1
// along each direction, energy ratio of the top modes, logistic map to alpha.
template <int DIM, int N, bool MIX>
__global__ void __launch_bounds__(512) k_indicator(RhsParams P, int ind_var, double alpha_max,
                                                   double alpha_min, double *__restrict__ alpha,
                                                   double *__restrict__ alpha_raw, double *__restrict__ Tw,
                                                   double *__restrict__ cw, double T0, double tol, int maxit) {
    constexpr int N1 = N + 1;
    constexpr int NN = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    constexpr int NV = (MIX ? kNS : 1) + DIM + 1;
    extern __shared__ double smem[];
    __shared__ double sV[N1 * N1];  // V^-1, read with per-lane indices
    const int tid = threadIdx.x;
    if (tid < N1 * N1) sV[tid] = P.B.Vinv[tid];
    int el = tid / NN;
    const int node = tid - el * NN;
    const int e = blockIdx.x * P.epb + el;
    const bool valid = (el < P.epb) && (e < P.nelem);
    if (el >= P.epb) el = 0;
    double *x = smem + el * 3 * NN;
    double *y = x + NN;
    double *z = y + NN;
    const size_t stride = (size_t)P.nelem * NN;
    const size_t gi = (size_t)(valid ? e : 0) * NN + node;
    if (valid) {
        double uo[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) uo[v] = P.u[v * stride + gi];
        double Tn = 0.0;
        if constexpr (MIX) {
            Tn = P.T[gi];
            if (Tw) {
                // the right-hand side's T(e) solve, fused (the same steps as
                // k_thermo with a warm start): T and the frozen sound speed
                double rs[kNS], rho;
                const int it = node_temperature_state<DIM>(uo, Tn, T0, tol, maxit, P.M, 1, rs, rho);
                Tw[gi] = Tn;
                cw[gi] = mix_sound(P.M, rs, rho, Tn);
                if (it < 0) atomicOr(P.flags, FLAG_NOCONV);
            }
        }
        St<DIM, MIX> s;
        make_state<DIM, MIX>(uo, Tn, P.gamma, P.M, s);
        x[node] = ind_var == 1 ? s.p : s.rho * s.p;
    }
    __syncthreads();
#pragma unroll 1
    for (int d = 0; d < DIM; ++d) {
        double m = 0.0;
        if (valid) {
            const int a = node_pos<N1>(node, d);
            const int l = node_line<N1, DIM>(node, d);
#pragma unroll
            for (int j = 0; j < N1; ++j) m = fma(sV[a * N1 + j], x[line_node<N1, DIM>(d, j, l)], m);
        }
        __syncthreads();
        if (valid) x[node] = m;
        __syncthreads();
    }
    // modal energies: all modes, modes of degree <= N-1, <= N-2 (degree = the
    // largest one-dimensional index), summed over the element in a fixed tree
    if (valid) {
        int mx = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) mx = max(mx, node_pos<N1>(node, d));
        const double m2 = x[node] * x[node];
        x[node] = m2;
        y[node] = mx <= N - 1 ? m2 : 0.0;
        z[node] = mx <= N - 2 ? m2 : 0.0;
    }
    __syncthreads();
    constexpr int P2 = NN <= 16 ? 16 : NN <= 32 ? 32 : NN <= 64 ? 64 : 128;
#pragma unroll
    for (int h = P2 / 2; h > 0; h >>= 1) {
        if (valid && node < h && node + h < NN) {
            x[node] += x[node + h];
            y[node] += y[node + h];
            z[node] += z[node + h];
        }
        __syncthreads();
    }
    if (valid && node == 0) {
        const double eall = x[0], e1 = y[0], e2 = z[0];
        const double E = fmax((eall - e1) / eall, (e1 - e2) / e1);
        const double thr = 0.5 * pow(10.0, -1.8 * pow((double)N1, 0.25));
        const double s = log((1.0 - 1e-4) / 1e-4);
        const double a = 1.0 / (1.0 + exp(-(s / thr) * (E - thr)));
        alpha_raw[e] = a;
        alpha[e] = a < alpha_min ? 0.0 : fmin(a, alpha_max);
    }
}

// Zhang-Shu positivity-preserving scaling limiter, in place on u (see
// dgx_limit_positivity in the C ABI).  Means and minima are reduced over the
// element's nodes by one thread in a fixed order (deterministic).
template <int DIM, bool MIX>
__device__ __forceinline__ double zs_psi(const double *u, const MixC &M) {
    constexpr int off = MIX ? kNS : 1;
    double rho = 0.0, lin = u[off + DIM];
    if constexpr (MIX) {
#pragma unroll
        for (int s = 0; s < kNS; ++s) {
            rho += u[s];
            lin -= M.e0[s] * u[s];
        }
    } else {
        rho = u[0];
    }
    double m2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) m2 = fma(u[off + c], u[off + c], m2);
    return lin - 0.5 * m2 / rho;
}

template <int DIM, int N, bool MIX, bool CURV>
__global__ void __launch_bounds__(512) k_positivity(RhsParams P, double *__restrict__ u) {
    constexpr int N1 = N + 1;
    constexpr int NN = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    constexpr int NV = (MIX ? kNS : 1) + DIM + 1;
    constexpr int ND = MIX ? kNS : 1;  // density variables
    constexpr int GA = DIM * DIM + 1;
    constexpr int SL = (NV + 1) * NN + NV + ND + 2;
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    int el = tid / NN;
    const int node = tid - el * NN;
    const int e = blockIdx.x * P.epb + el;
    const bool valid = (el < P.epb) && (e < P.nelem);
    if (el >= P.epb) el = 0;
    double *sw = smem + el * SL;         // [NV+1][NN] weighted values, then scratch
    double *sbar = sw + (NV + 1) * NN;   // [NV] means
    double *sth = sbar + NV;             // [ND] density thetas, [ND] pressure theta, flag
    const size_t stride = (size_t)P.nelem * NN;
    const size_t gi = (size_t)(valid ? e : 0) * NN + node;
    double uo[NV];
    double wJ = 0.0;
    if (valid) {
#pragma unroll
        for (int v = 0; v < NV; ++v) uo[v] = u[v * stride + gi];
        double w = 1.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) w *= P.B.w[node_pos<N1>(node, d)];
        const double J = CURV ? P.Jn[gi] : P.geo[(size_t)e * GA + DIM * DIM];
        wJ = w * J;
#pragma unroll
        for (int v = 0; v < NV; ++v) sw[v * NN + node] = wJ * uo[v];
        sw[NV * NN + node] = wJ;
    }
    __syncthreads();
    if (valid && node == 0) {
        double vol = 0.0;
        for (int n = 0; n < NN; ++n) vol += sw[NV * NN + n];
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
            for (int n = 0; n < NN; ++n) s += sw[v * NN + n];
            sbar[v] = s / vol;
        }
    }
    __syncthreads();
    double ubar[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ubar[v] = sbar[v];
    // 1. densities
    if (valid) {
#pragma unroll
        for (int s = 0; s < ND; ++s) sw[s * NN + node] = uo[s];
    }
    __syncthreads();
    if (valid && node == 0) {
        for (int s = 0; s < ND; ++s) {
            double mn = sw[s * NN];
            for (int n = 1; n < NN; ++n) mn = fmin(mn, sw[s * NN + n]);
            const double eps = MIX ? 1e-14 * fmax(ubar[s], 0.0) : fmin(1e-13, ubar[s]);
            sth[s] = (mn < eps && ubar[s] > eps) ? (ubar[s] - eps) / (ubar[s] - mn) : 1.0;
        }
    }
    __syncthreads();
    bool changed = false;
#pragma unroll
    for (int s = 0; s < ND; ++s) {
        const double th = sth[s];
        if (th < 1.0) {
            uo[s] = ubar[s] + th * (uo[s] - ubar[s]);
            changed = true;
        }
    }
    // 2. pressure
    double rho_bar = 0.0;
#pragma unroll
    for (int s = 0; s < ND; ++s) rho_bar += ubar[s];
    const double pb = zs_psi<DIM, MIX>(ubar, P.M);
    const double eps_p = fmin(1e-13 * rho_bar * (MIX ? 1e5 : 1.0), pb);
    double tn = 1.0;
    if (valid && pb > 0.0 && zs_psi<DIM, MIX>(uo, P.M) < eps_p) {
        double lo = 0.0, hi = 1.0, ut[NV];
        for (int it = 0; it < 64; ++it) {
            const double mid = 0.5 * (lo + hi);
#pragma unroll
            for (int v = 0; v < NV; ++v) ut[v] = ubar[v] + mid * (uo[v] - ubar[v]);
            if (zs_psi<DIM, MIX>(ut, P.M) >= eps_p) lo = mid;
            else hi = mid;
        }
        tn = lo;
    }
    __syncthreads();
    if (valid) sw[node] = tn;
    __syncthreads();
    if (valid && node == 0) {
        double mn = 1.0;
        for (int n = 0; n < NN; ++n) mn = fmin(mn, sw[n]);
        sth[ND] = mn;
        if (pb <= 0.0) atomicOr(P.flags, FLAG_NONPHYS);
    }
    __syncthreads();
    const double thp = sth[ND];
    if (thp < 1.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) uo[v] = ubar[v] + thp * (uo[v] - ubar[v]);
        changed = true;
    }
    if (valid && changed) {
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v * stride + gi] = uo[v];
    }
}

// alpha_k <- max(alpha_k, alpha_nbr / 2) over conforming neighbours.
template <int DIM>
__global__ void k_alpha_smooth(const int *__restrict__ nbr, int nelem, const double *__restrict__ ain,
                               double *__restrict__ aout) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nelem) return;
    double a = ain[e];
#pragma unroll
    for (int f = 0; f < 2 * DIM; ++f) {
        const int nb = nbr[(size_t)e * 2 * DIM + f];
        if (nb >= 0) a = fmax(a, 0.5 * ain[nb]);
    }
    aout[e] = a;
}

// max_n sum_d (|v.Ja^d| + c |Ja^d|)/J, as an ordered uint64 of a positive double.
template <int DIM, bool MIX, bool CURV>
__global__ void k_maxrate(RhsParams P, unsigned long long *out) {
    constexpr int GA = DIM * DIM + 1;
    const int NN = P.epb;  // nodes per element passed in epb
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)P.nelem * NN;
    double rate = 0.0;
    if (i < total) {
        const int e = (int)(i / NN);
        const size_t stride = (size_t)total;
        constexpr int NV = (MIX ? kNS : 1) + DIM + 1;
        double uo[NV];
        for (int v = 0; v < NV; ++v) uo[v] = P.u[v * stride + i];
        St<DIM, MIX> s;
        make_state<DIM, MIX>(uo, MIX ? P.T[i] : 0.0, P.gamma, P.M, s, MIX ? P.csnd + i : nullptr);
        const double J = CURV ? P.Jn[i] : P.geo[(size_t)e * GA + DIM * DIM];
        for (int d = 0; d < DIM; ++d) {
            double n[DIM];
            for (int c = 0; c < DIM; ++c)
                n[c] = CURV ? P.geo[(d * DIM + c) * stride + i] : P.geo[(size_t)e * GA + d * DIM + c];
            rate += fabs(dotn<DIM>(s.v, n)) + s.c * wave_sqrt(dotn<DIM>(n, n));
        }
        rate /= fabs(J);
    }
    // wave reduction then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) rate = fmax(rate, __shfl_xor(rate, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(rate));
}

}  // namespace dgx

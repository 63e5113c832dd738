// The fused DGSEM right-hand-side kernel (one or more elements per workgroup).
//
// Per element k and node n (Sec. Methodology, Eqs. strong_form,
// fluxes_discrete_fluxdifferencing, DGvec, fluxes_discrete_with_fv):
//
//   du_n = -(1/J_n) { sum_d [ (1-alpha_k) sum_{j != n_d} 2 D_{n_d j} F#(u_n, u_j; nbar)
//                            + alpha_k (F^FV_{n_d+1} - F^FV_{n_d}) / w_{n_d} ]
//                    + F*_N / w_N (face xi_d = +1) - F*_0 / w_0 (face xi_d = -1) }
//          + viscous divergence (BR1) + species sources.
//
// The diagonal-free sum is the telescoped subcell flux difference of
// Eq. DGvec with zero end values (the end values cancel against the strong-
// form surface terms because 2 D_00 + 1/w_0 = 0).  The two-point fluxes are
// symmetric in their states, so a pair's flux feeds both of its nodes: the
// thread of a node evaluates its pairs at fixed offsets along its line and
// passes one of them to its neighbour through LDS (N = 4: offsets 1 and 2,
// every pair evaluated once; N = 3: offset 1 exchanged, offset 2 evaluated
// by both nodes with the lower one first); other tilings evaluate each pair
// (a < b) once and both nodes gather it from a pair-indexed buffer.
//
// Work layout: thread <-> node, EPB elements per workgroup, the element's
// primitives (and, for mixtures, the species densities; on curved meshes
// the metric terms) staged in LDS.  Face work (Riemann fluxes, viscous
// interface fluxes) is spread evenly over the element's threads, one item per
// face node, with one normal per face (from the element whose xi_d = +1 face
// it is) so both neighbours compute bitwise identical interface fluxes and
// no atomics are needed.
#pragma once

#include "physics.h"

namespace dgx {

template <int N1, int DIM>
__device__ __forceinline__ int line_node(int d, int a, int l) {
    if (d == 0) return a + N1 * l;
    if (d == 1) return (l % N1) + N1 * a + (DIM == 3 ? N1 * N1 * (l / N1) : 0);
    return l + N1 * N1 * a;
}
template <int N1>
__device__ __forceinline__ int node_pos(int n, int d) {
    if (d == 0) return n % N1;
    if (d == 1) return (n / N1) % N1;
    return n / (N1 * N1);
}
template <int N1, int DIM>
__device__ __forceinline__ int node_line(int n, int d) {
    if (d == 0) return n / N1;
    if (d == 1) return (n % N1) + N1 * (n / (N1 * N1));
    return n % (N1 * N1);
}
// Pairs (a < b) of a line in lexicographic order, packed as 4-bit fields:
// a of pair k is (A >> 4k) & 15, b likewise.
template <int N1>
struct PairTab {
    static constexpr unsigned long long pack(bool second) {
        unsigned long long t = 0;
        int k = 0;
        for (int a = 0; a < N1; ++a)
            for (int b = a + 1; b < N1; ++b, ++k) t |= (unsigned long long)(second ? b : a) << (4 * k);
        return t;
    }
    static constexpr unsigned long long A = pack(false), B = pack(true);
};

// The slot offset of an LDS buffer, hidden from constant folding: the
// paired LDS accesses (ds_read2/ds_write2) encode offsets of at most 2 KB, so
// a large folded constant would cost one address add per access; an opaque
// offset goes into the base register once.
__device__ __forceinline__ int opaque_offset(int x) {
    asm volatile("" : "+s"(x));
    return x;
}

// Partners of a node along its line: for offset j (1..N1-1) the node at
// position a pairs with b = (a + j) mod N1.  pidx(j) packs, in 4-bit fields
// per a, the index of the pair {a, b} in PairTab order, so that a lane finds
// its pair with one bit-field extract instead of recomputing the index.
template <int N1>
struct PartnerTab {
    static_assert(N1 <= 6, "pair indices below 16, N1 4-bit fields in 32 bits");
    static constexpr unsigned pidx(int j) {
        unsigned r = 0;
        for (int a = 0; a < N1; ++a) {
            const int b = (a + j) % N1;
            const int lo = a < b ? a : b, hi = a < b ? b : a;
            int k = 0;  // pairs before {lo, hi} in PairTab order
            for (int x = 0; x < lo; ++x) k += N1 - 1 - x;
            r |= (unsigned)(k + hi - lo - 1) << (4 * a);
        }
        return r;
    }
};

// A phase of K work items per element, spread over the NT = epb * NN threads
// of the workgroup: round r covers items r * NT + t.  The partial last round
// of consecutive phases starts where the previous one stopped (cursor), so
// the extra rounds fall on different waves instead of always the first ones.
struct Spread {
    int t;       // this thread's slot within a round
    int cursor;  // first slot of the next phase's partial round
};
__device__ __forceinline__ Spread spread_phase(int tid, int NT, int K_per_block, int cursor) {
    int t = tid - cursor;
    if (t < 0) t += NT;
    int rem = K_per_block % NT;
    int next = cursor + rem;
    if (next >= NT) next -= NT;
    return {t, next};
}

// Workgroups are dealt to the 8 XCDs round-robin (block b to XCD b mod 8),
// and each XCD has its own L2.  This renumbering gives every XCD one
// contiguous range of element groups, so that face neighbours (in particular
// the neighbours of a group's end elements) are staged under the same L2.
// It pays while the state fits the shared Infinity Cache; beyond that the
// round-robin order, one window sweeping the state, keeps the neighbours'
// data fresh there instead (the autotuner decides).  A bijection of [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int X = 8;
    const int q = nb / X, r = nb - q * X, x = b % X, i = b / X;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// CHF: work-item chunks of the pair and face phases (the LDS tiling): 0 the
// default rule below, else that many chunks for both
template <int DIM, int N, int EQ, int VF, bool CURV, int CHF = 0>
struct RhsShape {
    static constexpr int N1 = N + 1;
    static constexpr int NN = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    static constexpr int NF = NN / N1;
    static constexpr bool MIX = EQ >= 2;
    static constexpr int NV = (MIX ? kNS : 1) + DIM + 1;
    static constexpr int NW = DIM + 1;  // viscous flux components (momentum, energy)
    static constexpr bool EC = VF == 0 && !MIX;  // perfect-gas EC flux from staged (rho, v, p, beta)
    // primitives: rho, v, p, rhoE [, c (mixture)] [, beta (EC)]
    static constexpr int NQ = DIM + 3 + (MIX ? 1 : 0) + (EC ? 1 : 0);
    static constexpr int SU = MIX ? kNS * NN : 0;  // species densities
    static constexpr int NPL = N1 * N / 2;
    static constexpr int PD = NF * NPL;      // pairs per direction
    static constexpr int NFV = NF * N;       // interior subcell interfaces per direction
    static constexpr int NSF = 2 * DIM * NF; // face nodes
    // large element types handle their pair and face work items in two
    // chunks, which halves the flux buffer (LDS bounds their occupancy)
    static constexpr int NCH = CHF ? CHF : (PD * NV > 1200 ? 2 : 1);
    static constexpr int PDC = (PD + NCH - 1) / NCH;    // pairs per chunk
    // face work in one chunk where the pair phase takes one pair per thread
    // and chunk (N = 4): the larger face buffer keeps the occupancy and
    // saves the second chunk's two barriers
    static constexpr int NCHF = (CHF == 0 && NCH == 2 && PDC == NN) ? 1 : NCH;
    static constexpr int NSFC = (NSF + NCHF - 1) / NCHF;  // face nodes per chunk
    // the volume pair fluxes are stored pair-major (a pair's NV fluxes are
    // contiguous, so one base address serves all of them), with an odd row
    // stride so that rows written by consecutive lanes start on distinct LDS
    // banks; the face and subcell buffers are variable-major
    static constexpr int NVP = NV | 1;
    static constexpr int B1 = PDC * NVP;
    static constexpr int B2 = NFV * NV;
    static constexpr int B3 = NSFC * NV;
    static constexpr int M12 = B1 > B2 ? B1 : B2;
    static constexpr int BUF = M12 > B3 ? M12 : B3;
    // curved: one metric row per node (the current direction); J and the
    // face normals are read from memory
    static constexpr int GEO = CURV ? DIM * NN : 0;
    static constexpr int GEOA = CURV ? 0 : DIM * DIM + 1;  // affine: Ja rows, J
    static constexpr int SLOT = SU + NQ * NN + GEO + GEOA + BUF;
    // curved mixture elements keep their own state in registers from the
    // staging to the stage update (their working set exceeds the Infinity
    // Cache, so re-reading it costs HBM traffic; they have VGPRs to spare at
    // their LDS-bound occupancy)
    static constexpr bool KEEPU = MIX && CURV;
};

// nrm = Jaf[d][:] for a runtime direction d without dynamic indexing of a
// private array (which would live in scratch memory).
template <int DIM>
__device__ __forceinline__ void jaf_row(const double *Jaf, int d, double *nrm) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) nrm[c] = Jaf[c];
#pragma unroll
    for (int dd = 1; dd < DIM; ++dd)
        if (d == dd) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) nrm[c] = Jaf[dd * DIM + c];
        }
}

// Node state from the LDS primitives (and species densities).
template <int DIM, bool MIX>
__device__ __forceinline__ void lds_state(const double *su, const double *sq, int NN, int n, double gamma,
                                          St<DIM, MIX> &s) {
    s.rho = sq[n];
#pragma unroll
    for (int c = 0; c < DIM; ++c) s.v[c] = sq[(1 + c) * NN + n];
    s.p = sq[(1 + DIM) * NN + n];
    s.rhoE = sq[(2 + DIM) * NN + n];
    if constexpr (MIX) {
        s.c = sq[(3 + DIM) * NN + n];
#pragma unroll
        for (int k = 0; k < kNS; ++k) s.rs[k] = su[k * NN + n];
    } else {
        // perfect gas: recomputed (one LDS array less keeps five 4-element
        // workgroups per CU); bitwise equal to the value make_state gives
        s.c = wave_sqrt(gamma * s.p * rcp(s.rho));
        s.rs[0] = 0.0;
    }
}

// One workgroup's chunk of the right-hand side: elements e0 .. e0 + epb - 1.
template <int DIM, int N, int EQ, int VF, int SF, bool CURV, bool MORT, int CHF = 0>
__device__ __forceinline__ void rhs_chunk(const RhsParams &P, int mode, int e0) {
    using S = RhsShape<DIM, N, EQ, VF, CURV, CHF>;
    constexpr int N1 = S::N1, NN = S::NN, NF = S::NF, NV = S::NV, NQ = S::NQ, NW = S::NW;
    constexpr int NPL = S::NPL, PD = S::PD, NFV = S::NFV, NSF = S::NSF;
    constexpr int NCH = S::NCH, NCHF = S::NCHF, PDC = S::PDC, NSFC = S::NSFC, NVP = S::NVP;
    constexpr bool MIX = S::MIX;
    constexpr int GA = DIM * DIM + 1;
    constexpr int QB = DIM + 3 + (MIX ? 1 : 0);  // EC slot in sq
    constexpr int OFF_G = S::SU + NQ * NN;        // element geometry within a slot
    constexpr int OFF_B = OFF_G + S::GEO + S::GEOA;
    constexpr int RFC = (NSFC + NN - 1) / NN;     // face rounds per chunk
    constexpr int RF = NCHF * RFC;                // face rounds
    extern __shared__ double smem[];
    // 2 D (pair-flux coefficients) and the LGL weights: read with per-lane
    // indices, so they live in LDS rather than in the kernel arguments
    __shared__ double sDc[N1 * N1];
    __shared__ double sW[N1];
    // non-conforming variants: the L2 projection from the face halves, read
    // with per-lane indices
    __shared__ double sPm[MORT ? 2 * N1 * N1 : 1];

    const int tid = threadIdx.x;
    if (tid < N1 * N1) sDc[tid] = 2.0 * P.B.D[tid];
    if (tid < N1) sW[tid] = P.B.w[tid];
    if constexpr (MORT) {
        if (tid < 2 * N1 * N1) {
            const int h = tid / (N1 * N1);
            sPm[tid] = P.mops[50 + h * 25 + (tid - h * N1 * N1)];
        }
    }
    const int NT = P.epb * NN;  // threads that own a node
    const int nloc = min(P.epb, P.nelem - e0);
    int el = tid / NN;
    const int node = tid - el * NN;
    const bool valid = el < nloc;
    const int e = e0 + (valid ? el : 0);
    if (el >= P.epb) el = 0;
    double *su = smem + el * S::SLOT;
    double *sq = su + S::SU;
    double *sJa = su + OFF_G;  // curved: the current direction's metric row; affine: Ja, J
    const int off_b = opaque_offset(OFF_B);
    double *buf = su + off_b;
    const size_t stride = (size_t)P.nelem * NN;
    const size_t gi = (size_t)e * NN + node;
    const double gamma = P.gamma;

    // Work items (face nodes, volume pairs) of all elements of the workgroup
    // are spread over all its threads; large element types handle them in
    // NCH chunks so that one chunk's fluxes fit the LDS buffer.  The face
    // phase's neighbour indices, and then the neighbour data of its first
    // round, are fetched first so that their latency overlaps the staging.
    Spread spf[NCHF];
    int cursor = 0;
#pragma unroll
    for (int c = 0; c < NCHF; ++c) {
        spf[c] = spread_phase(tid, NT, P.epb * NSFC, cursor);
        cursor = spf[c].cursor;
    }
    // face round g = chunk * RFC + r: item of this thread (element ei, face
    // node fi), or false
    auto face_item = [&](int g, int &ei, int &fi) -> bool {
        const int c = g / RFC, r = g - c * RFC;
        const int it = r * NT + spf[c].t;
        if (tid >= NT || it >= nloc * NSFC) return false;
        ei = it / NSFC;
        fi = c * NSFC + (it - ei * NSFC);
        return fi < NSF;
    };
    int nbf[RF];
#pragma unroll
    for (int g = 0; g < RF; ++g) {
        int ei, fi;
        nbf[g] = 0;
        if (face_item(g, ei, fi)) nbf[g] = P.nbr[(e0 + ei) * 2 * DIM + fi / NF];
    }

    double une[RF][NV];   // neighbour state at the face node
    double ftr[RF][NW];   // neighbour's contravariant viscous face flux (BR1)
    double nrr[RF][DIM];  // the face normal when it comes from memory
    double Tr[RF];        // neighbour temperature (mixtures)
    double cr[RF];        // neighbour frozen sound speed (mixtures)
    // The first round's data is loaded before the staging, later rounds'
    // right before use (register pressure).  Face normals come from the
    // element whose xi_d = +1 face it is: on affine elements the own one
    // sits in LDS, the neighbour's is loaded; on curved elements both are
    // nodal and loaded.
    auto load_nbr = [&](int g) {
#pragma unroll
        for (int v = 0; v < NV; ++v) une[g][v] = 1.0;
#pragma unroll
        for (int k = 0; k < NW; ++k) ftr[g][k] = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) nrr[g][c] = 0.0;
        Tr[g] = 1.0;
        cr[g] = 1.0;
        int ei, fi;
        if (!face_item(g, ei, fi)) return;
        const int nb = nbf[g];
        const int f = fi / NF;
        const int q = fi - f * NF;
        const int d = f >> 1, side = f & 1;
        if (nb >= 0) {
            const size_t gj = (size_t)nb * NN + line_node<N1, DIM>(d, side ? 0 : N, q);
#pragma unroll
            for (int v = 0; v < NV; ++v) une[g][v] = P.u[v * stride + gj];
            if constexpr (EQ == 1) {
                const double *fn = P.grad + ((size_t)nb * 2 * DIM + (f ^ 1)) * NW * NF + q;
#pragma unroll
                for (int k = 0; k < NW; ++k) ftr[g][k] = fn[k * NF];
            }
            if constexpr (MIX) {
                Tr[g] = P.T[gj];
                cr[g] = P.csnd[gj];
            }
            if (side == 0) {
                if constexpr (CURV) {
#pragma unroll
                    for (int c = 0; c < DIM; ++c) nrr[g][c] = P.geo[(d * DIM + c) * stride + gj];
                } else {
#pragma unroll
                    for (int c = 0; c < DIM; ++c) nrr[g][c] = P.geo[(size_t)nb * GA + d * DIM + c];
                }
            }
        }
        if constexpr (CURV) {
            if (nb < 0 || side == 1) {
                const size_t go = (size_t)(e0 + ei) * NN + line_node<N1, DIM>(d, side ? N : 0, q);
#pragma unroll
                for (int c = 0; c < DIM; ++c) nrr[g][c] = P.geo[(d * DIM + c) * stride + go];
            }
        }
    };

    double ku[S::KEEPU ? NV : 1];  // the own state, kept for the stage update
    // ---- stage the element: primitives (+ species, metric terms)
    {
        double uo[NV];
        double Tn = 1.0;
        if (valid) {
#pragma unroll
            for (int v = 0; v < NV; ++v) uo[v] = P.u[v * stride + gi];
        }
        load_nbr(0);
        if (valid) {
            if constexpr (CURV) {
#pragma unroll
                for (int c = 0; c < DIM; ++c) sJa[c * NN + node] = P.geo[c * stride + gi];  // direction 0
            } else {
                if (node < GA) sJa[node] = P.geo[(size_t)e * GA + node];
            }
            if constexpr (MIX) Tn = P.T[gi];
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) uo[v] = 1.0;
        }
        if constexpr (S::KEEPU) {
#pragma unroll
            for (int v = 0; v < NV; ++v) ku[v] = uo[v];
        }
        St<DIM, MIX> own;
        make_state<DIM, MIX>(uo, Tn, gamma, P.M, own, MIX && valid ? P.csnd + gi : nullptr);
        if (valid) {
            sq[node] = own.rho;
#pragma unroll
            for (int c = 0; c < DIM; ++c) sq[(1 + c) * NN + node] = own.v[c];
            sq[(1 + DIM) * NN + node] = own.p;
            sq[(2 + DIM) * NN + node] = own.rhoE;
            if constexpr (MIX) {
                sq[(3 + DIM) * NN + node] = own.c;
#pragma unroll
                for (int k = 0; k < kNS; ++k) su[k * NN + node] = own.rs[k];
            }
            if constexpr (S::EC) {
                sq[QB * NN + node] = own.rho / own.p;
            }
            bool ok = own.rho > 0.0 && own.p > 0.0 && isfinite(own.rhoE) && isfinite(own.p);
            if constexpr (MIX) {
#pragma unroll
                for (int k = 0; k < kNS; ++k) ok = ok && own.rs[k] >= 0.0;
            }
            if (!ok) atomicOr(P.flags, FLAG_NONPHYS);
        }
    }
    __syncthreads();

    double acc[NV];  // surface terms and alpha-weighted FV terms
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;

    // ---- interface / boundary Riemann fluxes: one work item per face node
#pragma unroll
    for (int ch = 0; ch < NCHF; ++ch) {
#pragma unroll
        for (int rr = 0; rr < RFC; ++rr) {
            const int g = ch * RFC + rr;
            if (g > 0) load_nbr(g);
            int ei, fi;
            if (face_item(g, ei, fi)) {
                const int f = fi / NF;
                const int q = fi - f * NF;
                const int jb = fi - ch * NSFC;  // slot in this chunk's buffer
                const int d = f >> 1, side = f & 1;
                const double *esu = smem + ei * S::SLOT;
                const double *esq = esu + S::SU;
                const double *eg = esu + OFF_G;
                double *ebuf = smem + ei * S::SLOT + OFF_B;
                const int nd = line_node<N1, DIM>(d, side ? N : 0, q);
                St<DIM, MIX> own, ext;
                lds_state<DIM, MIX>(esu, esq, NN, nd, gamma, own);
                double nrm[DIM];
                if constexpr (CURV) {
#pragma unroll
                    for (int c = 0; c < DIM; ++c) nrm[c] = nrr[g][c];
                } else {
#pragma unroll
                    for (int c = 0; c < DIM; ++c) nrm[c] = eg[d * DIM + c];
                }
                const int nb = nbf[g];
                double F[NV];
                if (MORT && nb <= kMortBase) {
                    // non-conforming face: sub-face fluxes from the mortar items
                    constexpr int NSUB = DIM == 3 ? 4 : 2;
                    const int code = kMortBase - nb;
                    const int m = code >> 3, role = code & 7;
                    const double *mf = P.mflux + (size_t)m * NSUB * NV * NF;
                    if (role < NSUB) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) F[v] = mf[(role * NV + v) * NF + q];
                    } else {
                        // large side: 2^(dim-1) sum_s (P_a x P_b) F*_s
#pragma unroll
                        for (int v = 0; v < NV; ++v) F[v] = 0.0;
                        const int qa = q % N1, qb = q / N1;
#pragma unroll 1
                        for (int sb = 0; sb < NSUB; ++sb) {
                            const int a = sb & 1, bsel = sb >> 1;
#pragma unroll 4
                            for (int qq = 0; qq < NF; ++qq) {
                                const int ja = qq % N1, jb2 = qq / N1;
                                double w = sPm[a * N1 * N1 + qa * N1 + ja];
                                if (DIM == 3) w *= sPm[bsel * N1 * N1 + qb * N1 + jb2];
#pragma unroll
                                for (int v = 0; v < NV; ++v) F[v] = fma(w, mf[(sb * NV + v) * NF + qq], F[v]);
                            }
                        }
#pragma unroll
                        for (int v = 0; v < NV; ++v) F[v] *= (double)NSUB;
                    }
                    if constexpr (EQ == 1) {
                        // the mortar flux carries the whole viscous F*; the
                        // gradient kernel took the own half of Ft off already
                        const double *fo = P.grad + ((size_t)(e0 + ei) * 2 * DIM + f) * NW * NF + q;
#pragma unroll
                        for (int k = 0; k < NW; ++k) F[1 + k] += 0.5 * fo[k * NF];
                    }
#pragma unroll
                    for (int v = 0; v < NV; ++v) ebuf[v * NSFC + jb] = F[v];
                    continue;
                }
                if (nb >= 0) {
                    make_state<DIM, MIX>(une[g], MIX ? Tr[g] : 0.0, gamma, P.M, ext, MIX ? &cr[g] : nullptr);
                    if (side == 0) {
#pragma unroll
                        for (int c = 0; c < DIM; ++c) nrm[c] = nrr[g][c];
                    }
                } else {
                    const int bc = -1 - nb;
                    const int kind = P.bc_kind[bc];
                    if (kind == 0) {
                        double ue[NV];
#pragma unroll
                        for (int v = 0; v < NV; ++v) ue[v] = P.bc_state[bc * NV + v];
                        make_state<DIM, MIX>(ue, MIX ? P.bc_T[bc] : 0.0, gamma, P.M, ext);
                    } else if (kind == 1) {
                        ext = own;
                    } else if (kind >= 3) {
                        // no-slip wall: the whole velocity reversed
                        ext = own;
#pragma unroll
                        for (int c = 0; c < DIM; ++c) ext.v[c] = -own.v[c];
                    } else {
                        // slip wall: mirror the velocity about the face (T and p unchanged)
                        const double inn = rcp(dotn<DIM>(nrm, nrm));
                        const double vn = dotn<DIM>(own.v, nrm) * inn;
                        ext = own;
#pragma unroll
                        for (int c = 0; c < DIM; ++c) ext.v[c] = own.v[c] - 2.0 * vn * nrm[c];
                    }
                }
                if constexpr (SF == 0) {
                    if (side) rusanov<DIM, MIX>(own, ext, nrm, F);
                    else rusanov<DIM, MIX>(ext, own, nrm, F);
                } else if constexpr (SF == 2) {
                    if (side) hll<DIM, MIX>(own, ext, nrm, F);
                    else hll<DIM, MIX>(ext, own, nrm, F);
                } else if constexpr (SF == 3) {
                    if (side) hllc<DIM, MIX>(own, ext, nrm, F);
                    else hllc<DIM, MIX>(ext, own, nrm, F);
                } else if constexpr (MIX) {
                    if (side) ec_mixture_state<DIM>(own, ext, nrm, P.M, F);
                    else ec_mixture_state<DIM>(ext, own, nrm, P.M, F);
                } else {
                    if (side) ranocha_state<DIM, MIX>(own, ext, nrm, gamma, F);
                    else ranocha_state<DIM, MIX>(ext, own, nrm, gamma, F);
                }
                if constexpr (EQ == 1) {
                    // BR1 interface flux {{F_v}}: the element's own half is in
                    // the gradient kernel's output, the neighbour's half enters
                    // with the inviscid flux (F* - F_v/2 on the momentum and
                    // energy rows; at boundary faces ftr is 0: the gradient
                    // kernel applied the whole viscous boundary flux).
#pragma unroll
                    for (int k = 0; k < NW; ++k) F[1 + k] -= 0.5 * ftr[g][k];
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) ebuf[v * NSFC + jb] = F[v];
            }
        }
        __syncthreads();
        if (valid) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const int a = node_pos<N1>(node, d);
                const int l = node_line<N1, DIM>(node, d);
                if (a == N || a == 0) {
                    const int fi = (2 * d + (a == N ? 1 : 0)) * NF + l;
                    if (NCHF == 1 || (fi >= ch * NSFC && fi < (ch + 1) * NSFC)) {
                        const double sc = a == N ? 1.0 / sW[N] : -1.0 / sW[0];
#pragma unroll
                        for (int v = 0; v < NV; ++v) acc[v] = fma(sc, buf[v * NSFC + fi - ch * NSFC], acc[v]);
                    }
                }
            }
        }
        __syncthreads();
    }

    // ---- first-order subcell finite volumes (elements with alpha > 0)
    const double alpha = (P.alpha != nullptr && valid) ? P.alpha[e] : 0.0;
    if (P.alpha != nullptr && __syncthreads_or(alpha > 0.0)) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
#pragma unroll
            for (int r = 0; r < (NFV + NN - 1) / NN; ++r) {
                const int p = r * NN + node;
                if (valid && alpha > 0.0 && p < NFV) {
                    const int l = p / N;
                    const int m = p - l * N + 1;
                    const int nL = line_node<N1, DIM>(d, m - 1, l);
                    const int nR = line_node<N1, DIM>(d, m, l);
                    double nrm[DIM];
                    if constexpr (CURV) {
                        const double *ns = P.nsub + ((((size_t)e * DIM + d) * NF + l) * N + (m - 1)) * DIM;
#pragma unroll
                        for (int c = 0; c < DIM; ++c) nrm[c] = ns[c];
                    } else {
#pragma unroll
                        for (int c = 0; c < DIM; ++c) nrm[c] = sJa[d * DIM + c];
                    }
                    St<DIM, MIX> A, B;
                    lds_state<DIM, MIX>(su, sq, NN, nL, gamma, A);
                    lds_state<DIM, MIX>(su, sq, NN, nR, gamma, B);
                    double F[NV];
                    rusanov<DIM, MIX>(A, B, nrm, F);
#pragma unroll
                    for (int v = 0; v < NV; ++v) buf[v * NFV + p] = F[v];
                }
            }
            __syncthreads();
            if (valid && alpha > 0.0) {
                const int a = node_pos<N1>(node, d);
                const int l = node_line<N1, DIM>(node, d);
                const double aw = alpha / sW[a];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double hi = a < N ? buf[v * NFV + l * N + a] : 0.0;
                    const double lo = a > 0 ? buf[v * NFV + l * N + a - 1] : 0.0;
                    acc[v] = fma(aw, hi - lo, acc[v]);
                }
            }
            __syncthreads();
        }
    }

    // the epilogue's own-node loads (u, u0 of the stage form, the local
    // viscous part, curved J) are issued before the last gather, once the
    // pair fluxes no longer hold registers, so that their latency overlaps it
    double eu[NV], eu0[NV], evp[NW];
    double Jc = 1.0;  // curved: J of the node

    // ---- high-order volume term: symmetric two-point fluxes along lines
    double dg[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) dg[v] = 0.0;
    const double gm1_inv = 1.0 / (gamma - 1.0);
    // the configured two-point volume flux F#(A, B; nbar) from node states
    // (for the perfect-gas entropy-conservative flux see ec_pair)
    auto volume_flux = [&](const St<DIM, MIX> &A, const St<DIM, MIX> &B, const double *nbar, double *F) {
        if constexpr (VF == 0) {
            if constexpr (MIX) ec_mixture_state<DIM>(A, B, nbar, P.M, F);
        } else if constexpr (VF == 1) {
            ducros_state<DIM, MIX>(A, B, nbar, F);
        } else if constexpr (VF == 4) {
            central_state<DIM, MIX>(A, B, nbar, F);
        } else {
            split_form_state<DIM, MIX, VF == 5 ? 2 : VF - 2>(A, B, nbar, gm1_inv, F);
        }
    };
    // the perfect-gas entropy-conservative flux from the staged (rho, v, p,
    // beta) of nodes na and nb of the element whose primitives start at esq
    auto ec_pair = [&](const double *esq, int na, int nb, const double *nbar, double *F) {
        double vA[DIM], vB[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            vA[c] = esq[(1 + c) * NN + na];
            vB[c] = esq[(1 + c) * NN + nb];
        }
        ranocha_prims<DIM>(esq[na], vA, esq[(1 + DIM) * NN + na], esq[QB * NN + na], esq[nb], vB,
                           esq[(1 + DIM) * NN + nb], esq[QB * NN + nb], nbar, gm1_inv, F);
    };
    // circulant pairs (below): the own node's state and current metric row
    // stay in registers for the whole volume term (not with the entropy-
    // conservative mixture flux, whose registers would then cost a wave)
    constexpr bool CIRC_K = PDC == NN && (N1 % 2 == 1) && 2 * NCH == N1 - 1 && !S::EC && !(MIX && VF == 0);
    St<DIM, MIX> own_st;
    double own_row[DIM];
    if constexpr (CIRC_K) {
        if (valid) lds_state<DIM, MIX>(su, sq, NN, node, gamma, own_st);
        if constexpr (CURV) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) own_row[c] = valid ? sJa[c * NN + node] : 0.0;
        }
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        // curved elements: the next direction's metric row, loaded now and
        // stored once this direction's pair fluxes are done
        double jnext[DIM];
        if constexpr (CURV) {
#pragma unroll
            for (int c = 0; c < DIM; ++c)
                jnext[c] = (valid && d + 1 < DIM) ? P.geo[((d + 1) * DIM + c) * stride + gi] : 0.0;
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            // a chunk of exactly NN pairs per element: each thread takes the
            // pair of its own element whose slot is its node index (the
            // spread would give every thread one item as well)
            constexpr bool OWN = PDC == NN;
            // odd N1 with (N1-1)/2 such chunks (N = 4): circulant pairs, chunk
            // ch taking offset j = ch + 1.  The thread of the node at position
            // a on line l evaluates the pair {a, (a + j) mod N1}, adds its own
            // share at once and leaves the flux in its node's slot; its other
            // pair of this offset, {(a - j) mod N1, a}, is read from the slot
            // of that node.  Every pair is evaluated once, every node takes
            // all its N1 - 1 pairs, and the lanes of a wave read slots of
            // consecutive nodes (few LDS bank conflicts).
            constexpr bool CIRC = OWN && (N1 % 2 == 1) && 2 * NCH == N1 - 1;
            // four nodes per line (N = 3) in one chunk: the pair at offset 1,
            // {a, (a + 1) mod 4}, as above; the pair at offset 2 is evaluated
            // by both of its nodes (with its lower node first, so that both
            // take the same flux) and needs no exchange
            constexpr bool CIRC4 = N1 == 4 && NCH == 1;
            const int jc = ch + 1;
            if constexpr (CIRC4) {
                if (valid) {
                    const int a = node_pos<N1>(node, d);
                    const int l = node_line<N1, DIM>(node, d);
#pragma unroll
                    for (int j = 1; j <= 2; ++j) {
                        const int b = (a + j) & 3;
                        const int nb = line_node<N1, DIM>(d, b, l);
                        const int nlo = a < b ? node : nb, nhi = a < b ? nb : node;
                        double nbar[DIM];
#pragma unroll
                        for (int c = 0; c < DIM; ++c)
                            nbar[c] = CURV ? 0.5 * (sJa[c * NN + nlo] + sJa[c * NN + nhi]) : sJa[d * DIM + c];
                        double F[NV];
                        if constexpr (S::EC) {
                            ec_pair(sq, nlo, nhi, nbar, F);
                        } else {
                            St<DIM, MIX> A, B;
                            lds_state<DIM, MIX>(su, sq, NN, nlo, gamma, A);
                            lds_state<DIM, MIX>(su, sq, NN, nhi, gamma, B);
                            volume_flux(A, B, nbar, F);
                        }
                        if (j == 1) {
#pragma unroll
                            for (int v = 0; v < NV; ++v) buf[node * NVP + v] = F[v];
                        }
                        const double coef = sDc[a * N1 + b];
#pragma unroll
                        for (int v = 0; v < NV; ++v) dg[v] = fma(coef, F[v], dg[v]);
                    }
                }
            }
            Spread sp{tid, cursor};
            if constexpr (!OWN && !CIRC4) {
                sp = spread_phase(tid, NT, P.epb * PDC, cursor);
                cursor = sp.cursor;
            }
#pragma unroll
            for (int r = 0; r < (CIRC4 ? 0 : (PDC + NN - 1) / NN); ++r) {
                const int it = r * NT + sp.t;
                if (OWN ? valid : (tid < NT && it < nloc * PDC)) {
                    const int ei = OWN ? el : it / PDC;
                    const int jb = OWN ? node : it - ei * PDC;  // slot in this chunk's buffer
                    // the pair's nodes na, nb (CIRC: the own node and its
                    // partner at positions ca, cb; the volume fluxes are
                    // symmetric in their two states)
                    int na, nb, ca = 0, cb = 0;
                    if constexpr (CIRC) {
                        ca = node_pos<N1>(node, d);
                        cb = ca + jc >= N1 ? ca + jc - N1 : ca + jc;
                        na = node;
                        nb = line_node<N1, DIM>(d, cb, node_line<N1, DIM>(node, d));
                    } else {
                        const int p = ch * PDC + jb;  // pair index within the direction
                        if (NCH > 1 && p >= PD) continue;
                        const int l = p / NPL;
                        const int k = p - l * NPL;
                        na = line_node<N1, DIM>(d, (int)((PairTab<N1>::A >> (4 * k)) & 15u), l);
                        nb = line_node<N1, DIM>(d, (int)((PairTab<N1>::B >> (4 * k)) & 15u), l);
                    }
                    const double *esu = smem + ei * S::SLOT;
                    const double *esq = esu + S::SU;
                    const double *eg = esu + OFF_G;
                    double *ebuf = smem + ei * S::SLOT + off_b;
                    double nbar[DIM];
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        if constexpr (CURV && CIRC_K) nbar[c] = 0.5 * (own_row[c] + eg[c * NN + nb]);
                        else nbar[c] = CURV ? 0.5 * (eg[c * NN + na] + eg[c * NN + nb]) : eg[d * DIM + c];
                    }
                    double F[NV];
                    if constexpr (S::EC) {
                        ec_pair(esq, na, nb, nbar, F);
                    } else {
                        St<DIM, MIX> A, B;
                        if constexpr (CIRC_K) A = own_st;
                        else lds_state<DIM, MIX>(esu, esq, NN, na, gamma, A);
                        lds_state<DIM, MIX>(esu, esq, NN, nb, gamma, B);
                        volume_flux(A, B, nbar, F);
                    }
#pragma unroll
                    for (int v = 0; v < NV; ++v) ebuf[jb * NVP + v] = F[v];
                    if constexpr (CIRC) {
                        const double coef = sDc[ca * N1 + cb];
#pragma unroll
                        for (int v = 0; v < NV; ++v) dg[v] = fma(coef, F[v], dg[v]);
                    }
                }
            }
            if (d == DIM - 1 && ch == NCH - 1) {
                const bool st = valid && mode != 0;
                const bool s0 = st && P.sa != 0.0;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if constexpr (S::KEEPU) eu[v] = ku[v];
                    else eu[v] = st ? P.u[v * stride + gi] : 0.0;
                    eu0[v] = s0 ? P.u0[v * stride + gi] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < NW; ++k) evp[k] = (EQ == 1 && valid) ? P.vpart[(size_t)k * stride + gi] : 0.0;
                if constexpr (CURV) Jc = valid ? P.Jn[gi] : 1.0;
            }
            __syncthreads();
            if constexpr (CURV) {
                // every pair of this direction has read the row: replace it
                if (ch == NCH - 1 && d + 1 < DIM && valid) {
#pragma unroll
                    for (int c = 0; c < DIM; ++c) sJa[c * NN + node] = jnext[c];
                    if constexpr (CIRC_K) {
#pragma unroll
                        for (int c = 0; c < DIM; ++c) own_row[c] = jnext[c];
                    }
                }
            }
            if (CIRC4 && valid) {
                // the pair {(a + 3) mod 4, a}, left by that node
                const int a = node_pos<N1>(node, d);
                const int l = node_line<N1, DIM>(node, d);
                const int a2 = (a + 3) & 3;
                const int src = line_node<N1, DIM>(d, a2, l);
                const double coef = sDc[a * N1 + a2];
#pragma unroll
                for (int v = 0; v < NV; ++v) dg[v] = fma(coef, buf[src * NVP + v], dg[v]);
            } else if (CIRC && valid) {
                const int a = node_pos<N1>(node, d);
                const int l = node_line<N1, DIM>(node, d);
                const int a2 = a - jc < 0 ? a - jc + N1 : a - jc;
                const int src = line_node<N1, DIM>(d, a2, l);
                const double coef = sDc[a * N1 + a2];
#pragma unroll
                for (int v = 0; v < NV; ++v) dg[v] = fma(coef, buf[src * NVP + v], dg[v]);
            } else if (valid) {
                const int a = node_pos<N1>(node, d);
                const int l = node_line<N1, DIM>(node, d);
                const int sa4 = 4 * a;
                const int kl = l * NPL - ch * PDC;  // the line's first pair in this chunk's buffer
#pragma unroll
                for (int j = 1; j < N1; ++j) {
                    // partner b = (a + j) mod N1: the pair's slot and coefficient
                    const int k = kl + (int)((PartnerTab<N1>::pidx(j) >> sa4) & 15u);
                    if (NCH == 1 || (unsigned)k < (unsigned)PDC) {
                        const double coef = sDc[a * N1 + a + j - (a + j >= N1 ? N1 : 0)];
#pragma unroll
                        for (int v = 0; v < NV; ++v) dg[v] = fma(coef, buf[k * NVP + v], dg[v]);
                    }
                }
            }
            __syncthreads();
        }
    }
    const double iJ = 1.0 / (CURV ? Jc : sJa[DIM * DIM]);
    double du[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) du[v] = -fma(1.0 - alpha, dg[v], acc[v]) * iJ;

    // ---- BR1 viscous divergence (perfect-gas Navier-Stokes, affine elements).
    // The gradient kernel wrote the element-local part (volume divergence and
    // the element's own halves of the interface fluxes); the neighbours'
    // halves came in with the face fluxes above.
    if constexpr (EQ == 1) {
        if (valid) {
#pragma unroll
            for (int k = 0; k < NW; ++k) du[1 + k] += evp[k];
        }
    }

    // ---- finite-rate chemistry source
    if constexpr (EQ == 3) {
        if (valid) {
            const KinC &K = *P.kin;
            const double T = P.T[gi];
            const double lnT = log(T);
            const double iT = 1.0 / T;
            double gRT[kNS], conc[kNS];
#pragma unroll
            for (int s = 0; s < kNS; ++s) {
                double g = K.gconst[s] - (2.5 + P.M.mol[s]) * lnT + P.M.e0[s] * iT / P.M.Rs[s];
                if (P.M.mol[s]) g += log(-expm1(-P.M.thv[s] * iT));
                gRT[s] = g;
                conc[s] = su[s * NN + node] / K.W[s];
            }
            double wdot[kNS];
#pragma unroll
            for (int s = 0; s < kNS; ++s) wdot[s] = 0.0;
            const double lnpr = K.lnpref_Ru - lnT;
            for (int r = 0; r < K.nr; ++r) {
                double lnK = K.dnu_sum[r] * lnpr;
                double fw = 1.0, bw = 1.0;
#pragma unroll
                for (int s = 0; s < kNS; ++s) {
                    const int nu = K.nu[r][s], nup = K.nup[r][s];
                    lnK -= (double)(nup - nu) * gRT[s];
                    for (int q = 0; q < nu; ++q) fw *= conc[s];
                    for (int q = 0; q < nup; ++q) bw *= conc[s];
                }
                // k_b = k_f / K_c in log space: at low T both factors underflow
                const double lnkf = fma(K.b[r], lnT, K.lnA[r]) - K.tha[r] * iT;
                const double kf = exp(lnkf);
                const double kb = exp(lnkf - lnK);
                const double R = kf * fw - kb * bw;
#pragma unroll
                for (int s = 0; s < kNS; ++s) wdot[s] = fma((double)(K.nup[r][s] - K.nu[r][s]), R, wdot[s]);
            }
#pragma unroll
            for (int s = 0; s < kNS; ++s) du[s] += K.W[s] * wdot[s];
        }
    }

    if (valid) {
        if (mode == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) P.out[v * stride + gi] = du[v];
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double base = P.sa != 0.0 ? P.sa * eu0[v] : 0.0;
                P.out[v * stride + gi] = base + P.sb * (eu[v] + P.dt * du[v]);
            }
        }
    }
}

// Mortar sub-face fluxes (Sec. New Developments: interpolation to the small
// sides): one workgroup per mortar, one thread per small-face node.  The
// large element's face trace is interpolated to the node with I_a x I_b, the
// Riemann flux uses the small element's trace and scaled normal and is
// oriented along +xi_d (lower-xi state first).  Perfect gas, affine elements.
template <int DIM, int N, int SF, int EQ = 0>
__device__ __forceinline__ void mortar_item(const RhsParams &P, int m, int t) {
    constexpr int N1 = N + 1;
    constexpr int NN = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    constexpr int NF = NN / N1;
    constexpr int NV = DIM + 2;
    constexpr int NSUB = DIM == 3 ? 4 : 2;
    constexpr int GA = DIM * DIM + 1;
    if (t >= NSUB * NF) return;
    const int s = t / NF, q = t - s * NF;
    const int *row = P.mort + (size_t)m * (3 + NSUB);
    const int eL = row[0], fL = row[1], es = row[2 + s], fS = row[2 + NSUB];
    const int d = fL >> 1, sideL = fL & 1;
    const size_t stride = (size_t)P.nelem * NN;
    // interpolate the large trace to small-face node q of sub-face s
    const int a = s & 1, bsel = s >> 1;
    const int qa = q % N1, qb = q / N1;
    double ui[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ui[v] = 0.0;
    // (partly rolled: in the work-list kernel this code shares the
    // right-hand side's register budget)
#pragma unroll 4
    for (int j = 0; j < NF; ++j) {
        const int ja = j % N1, jb = j / N1;
        double w = P.mops[a * 25 + qa * N1 + ja];
        if (DIM == 3) w *= P.mops[bsel * 25 + qb * N1 + jb];
        const size_t gj = (size_t)eL * NN + line_node<N1, DIM>(d, sideL ? N : 0, j);
#pragma unroll
        for (int v = 0; v < NV; ++v) ui[v] = fma(w, P.u[v * stride + gj], ui[v]);
    }
    const size_t gs = (size_t)es * NN + line_node<N1, DIM>(d, (fS & 1) ? N : 0, q);
    double us[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) us[v] = P.u[v * stride + gs];
    St<DIM, false> A, B;
    make_state<DIM, false>(ui, 0.0, P.gamma, P.M, A);
    make_state<DIM, false>(us, 0.0, P.gamma, P.M, B);
    double nrm[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) nrm[c] = P.geo[(size_t)es * GA + d * DIM + c];
    double F[NV];
    if constexpr (SF == 0) {
        if (sideL) rusanov<DIM, false>(A, B, nrm, F);
        else rusanov<DIM, false>(B, A, nrm, F);
    } else if constexpr (SF == 2) {
        if (sideL) hll<DIM, false>(A, B, nrm, F);
        else hll<DIM, false>(B, A, nrm, F);
    } else if constexpr (SF == 3) {
        if (sideL) hllc<DIM, false>(A, B, nrm, F);
        else hllc<DIM, false>(B, A, nrm, F);
    } else {
        if (sideL) ranocha_state<DIM, false>(A, B, nrm, P.gamma, F);
        else ranocha_state<DIM, false>(B, A, nrm, P.gamma, F);
    }
    if constexpr (EQ == 1) {
        // BR1 viscous sub-face flux, the mean of the small side's Ft and the
        // large side's interpolated Ft scaled to the small normal (affine:
        // the large element's Ja^d is 2^(dim-1) times the small one's); the
        // stored flux is the advective minus the viscous one
        constexpr int NW = DIM + 1;
        const double *fs = P.grad + ((size_t)es * 2 * DIM + fS) * NW * NF + q;
        const double *fl = P.grad + ((size_t)eL * 2 * DIM + fL) * NW * NF;
        double fi[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k) fi[k] = 0.0;
#pragma unroll 4
        for (int j = 0; j < NF; ++j) {
            const int ja = j % N1, jb = j / N1;
            double w = P.mops[a * 25 + qa * N1 + ja];
            if (DIM == 3) w *= P.mops[bsel * 25 + qb * N1 + jb];
#pragma unroll
            for (int k = 0; k < NW; ++k) fi[k] = fma(w, fl[k * NF + j], fi[k]);
        }
#pragma unroll
        for (int k = 0; k < NW; ++k) F[1 + k] -= 0.5 * (fs[k * NF] + fi[k] * (1.0 / NSUB));
    }
    double *out = const_cast<double *>(P.mflux) + (size_t)m * NSUB * NV * NF;
#pragma unroll
    for (int v = 0; v < NV; ++v) out[(s * NV + v) * NF + q] = F[v];
}



template <int DIM, int N, int EQ, int VF, int SF, bool CURV, bool MORT = false, int CHF = 0>
__global__ void __launch_bounds__(512) k_rhs(RhsParams P, int mode) {
    const int e0 = (P.xcd ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x) * P.epb;
    rhs_chunk<DIM, N, EQ, VF, SF, CURV, MORT, CHF>(P, mode, e0);
}

// Work-list form: one launch over the mortars' sub-face fluxes (the mortar
// pass, non-conforming meshes) and the element chunks.  The mortar items and
// the chunks with a non-conforming face form a queue, mortar items first,
// claimed in order by the first workgroups (an atomic counter, not their
// block index); a chunk that comes up before every mortar item has finished
// waits for them.  The other chunks go to the remaining workgroups by block
// index.  The wait is bounded
// and cannot deadlock: every mortar item was claimed before the chunk by a
// workgroup that was already running and finishes it without waiting (should
// the bound ever be reached the chunk proceeds and the non-physical flag is
// raised).  Q.next and Q.done must be 0 at launch.  With Q.next null the
// kernel is the mortar pass of the grid form instead (block b: mortar item b,
// no element chunks): both forms then evaluate the sub-face fluxes with the
// same compiled code, bitwise alike.  (A persistent form, a
// grid of resident workgroups looping over the queue, was measured: the loop
// lets the compiler keep hoisted kernel-argument tables in registers, 215-256
// VGPRs, or 0.5-1.6 KB of spills per lane when held to the grid form's five
// waves; one item per workgroup keeps the grid form's registers.)
struct WorkQ {
    int *next;          // next item to claim
    int *done;          // mortar items finished
    const int *order;   // [nchunks] element chunk of queue position
    const unsigned char *waits;  // [nchunks] 1: the chunk reads mortar fluxes
    int nmort, nchunks;
    int nfree;          // chunks order[0 .. nfree-1] read no mortar fluxes
};

template <int DIM, int N, int EQ, int VF, int SF, bool CURV, bool MORT = false, int CHF = 0>
__global__ void __launch_bounds__(512) k_rhs_queue(RhsParams P, int mode, WorkQ Q) {
    __shared__ int s_item;
    if (Q.next == nullptr) {
        if constexpr (MORT) {
            if ((int)blockIdx.x < Q.nmort) mortar_item<DIM, N, SF, EQ>(P, blockIdx.x, threadIdx.x);
        }
        return;
    }
    // blocks 0 .. nq-1 claim the queue's mortar items and then the chunks
    // that read them; the blocks after take the other chunks directly (no
    // counter: a single address claimed by every block serialises them)
    const int nq = Q.nmort + Q.nchunks - Q.nfree;
    const int b = blockIdx.x;
    if (b >= nq) {
        if (b - nq < Q.nfree) rhs_chunk<DIM, N, EQ, VF, SF, CURV, MORT, CHF>(P, mode, Q.order[b - nq] * P.epb);
        return;
    }
    if (threadIdx.x == 0) s_item = atomicAdd(Q.next, 1);
    __syncthreads();
    const int item = s_item < Q.nmort ? s_item : s_item + Q.nfree;  // queue position -> item
    if (item >= Q.nmort + Q.nchunks) return;
    if (MORT && item < Q.nmort) {
        if constexpr (MORT) mortar_item<DIM, N, SF, EQ>(P, item, threadIdx.x);
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();  // the sub-face fluxes before the count
            atomicAdd(Q.done, 1);
        }
        return;
    }
    const int k = item - Q.nmort;
    if (MORT && Q.waits[k]) {
        if (threadIdx.x == 0) {
            // poll without ordering (an acquire per poll would invalidate the
            // caches every time), then one acquire fence
            int spins = 0;
            while (__hip_atomic_load(Q.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < Q.nmort &&
                   spins < (1 << 24)) {
                __builtin_amdgcn_s_sleep(2);
                ++spins;
            }
            if (spins >= (1 << 24)) atomicOr(P.flags, FLAG_NONPHYS);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
    }
    rhs_chunk<DIM, N, EQ, VF, SF, CURV, MORT, CHF>(P, mode, Q.order[k] * P.epb);
}

__global__ void k_workq_reset(int *next, int *done) {
    if (threadIdx.x == 0) {
        *next = 0;
        *done = 0;
    }
}

}  // namespace dgx

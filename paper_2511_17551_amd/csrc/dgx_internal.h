// Internal definitions shared by the host runtime and the HIP kernels of
// libdgx.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgx {

constexpr int kNS = 5;        // species of the air mixture
constexpr int kMaxR = 32;     // reactions

// Reference-element operators of one polynomial degree, passed by value
// (kernel arguments live in scalar registers / the constant cache).
struct BasisC {
    double D[25];      // D[a*(N+1)+b] = l_b'(xi_a)
    double w[5];       // LGL weights
    double Vinv[25];   // nodal -> orthonormal Legendre modes
};

// Thermodynamic data of the 5 species (RRHO, Appendix Thermodynamics).
struct MixC {
    double Rs[kNS];    // R_u / W_s
    double thv[kNS];   // vibrational temperature (0 for atoms)
    double e0[kNS];    // formation energy J/kg
    int mol[kNS];      // linear diatomic?
};

// Reaction data (device memory, read with uniform addresses).
struct KinC {
    int nr;
    double lnA[kMaxR], b[kMaxR], tha[kMaxR];  // ln of the pre-exponential factor
    double dnu_sum[kMaxR];          // sum_s (nu' - nu)
    int nu[kMaxR][kNS], nup[kMaxR][kNS];
    double W[kNS];
    double gconst[kNS];             // T-independent part of -g_s/(R_s T)
    double lnpref_Ru;               // ln(p_ref / R_u)
};

// Face codes of the element-neighbour table: >= 0 conforming neighbour,
// in (kMortBase, -1] boundary -1 - bc, <= kMortBase mortar
// kMortBase - (8 m + role), role = small position (0..3) or 7 (large side).
constexpr int kMortBase = -(1 << 24);

// Device error flags (bit mask), sticky until dgx_check.
enum : unsigned { FLAG_NONPHYS = 1u, FLAG_NOCONV = 2u };
// per-node iteration counts: this bit marks a solve from a given guess that
// failed and was redone from the freestream guess
constexpr int kItersFallback = 1 << 20;

struct RhsParams {
    int nelem;
    const double *u;        // stage input state
    double *out;            // du (mode 0) or next stage (mode 1)
    const double *u0;       // stage base (mode 1)
    double sa, sb, dt;      // out = sa*u0 + sb*(u + dt*du)
    const int *nbr;         // [E][2*dim]: >= 0 neighbour, < 0: -1-bc index
    const double *geo;      // affine: [E][dim*dim+1] (Ja rows, J); curved: Ja [dim*dim][E][nn]
    const double *Jn;       // curved: J [E][nn]
    const double *nsub;     // curved + shock: [E][dim][nf][N][dim] subcell normals
    const double *alpha;    // [E] or null
    const double *T;        // mixture temperature [E][nn]
    const double *csnd;     // mixture frozen sound speed [E][nn], from the T(e) solve
    const double *grad;     // NS: neighbours' face viscous fluxes [E][2 dim][dim+1][nf]
    const double *vpart;    // NS: element-local viscous divergence [dim+1][E][nn]
    double *out2;           // second output (k_grad: face viscous fluxes)
    const int *bc_kind;     // [nbc]
    const double *bc_state; // [nbc][nvar]
    const double *bc_T;     // [nbc] temperatures of Dirichlet states (mixture)
    const KinC *kin;        // reacting mixture
    const int *mort;        // mortar table [nm][3 + 2^(dim-1)] (eL, fL, eS.., fS)
    const double *mflux;    // mortar sub-face fluxes [nm][2^(dim-1)][nvar][nf]
    const double *mops;     // mortars: [I, P][lower, upper half][25]: interpolation to the
                            // halves of a face edge and L2 projection back ([q][j], N+1 wide)
    const double *mgw;      // NS on mortars: sub-face gradient values W*_s [nm][2^(dim-1)][dim+1][nf]
    double gamma, R, mu, kappa;
    int epb;                // elements per block
    int xcd;                // nonzero: XCD-contiguous workgroup numbering (k_rhs, k_grad)
    unsigned *flags;
    BasisC B;
    MixC M;
};

}  // namespace dgx

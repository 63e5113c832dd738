// libdgx host runtime: contexts, geometry upload, kernel dispatch and the
// C-ABI entry points declared in include/dgx.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <new>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dgx.h"
#include "host_geometry.h"
#include "host_parallel.h"
#include "host_octree.h"
#include "k_amr.h"
#include "k_aux.h"
#include "k_chem.h"
#include "surrogate.h"

using namespace dgx;

namespace {

#define HIPCHK(call)                                                              \
    do {                                                                          \
        hipError_t _e = (call);                                                   \
        if (_e != hipSuccess) {                                                   \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(_e);         \
            return DGX_E_DEVICE;                                                  \
        }                                                                         \
    } while (0)

// ------------------------------------------------------------------ dispatch
using RhsLaunch = void (*)(const RhsParams &, int, int, int, size_t, hipStream_t);
using RhsLaunchP = void (*)(const RhsParams &, int, int, size_t, hipStream_t, const WorkQ &);
using GradLaunch = void (*)(const RhsParams &, int, int, size_t, hipStream_t);
// indicator launch: ..., and for mixtures the fused T(e) solve's outputs
// (T, frozen sound speed; null: T was solved before) and its T0, tol, maxit
using IndLaunch = void (*)(const RhsParams &, int, double, double, double *, double *, int, int, size_t,
                           hipStream_t, double *, double *, double, double, int);

template <int DIM, int N, int EQ, int VF, int SF, bool CURV, bool MORT, int CHF>
void rhs_launch(const RhsParams &P, int mode, int blocks, int threads, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_rhs<DIM, N, EQ, VF, SF, CURV, MORT, CHF>), dim3(blocks), dim3(threads), lds, s, P, mode);
}
// The work-list form: one workgroup per queue item.
template <int DIM, int N, int EQ, int VF, int SF, bool CURV, bool MORT, int CHF>
void rhs_launch_p(const RhsParams &P, int mode, int threads, size_t lds, hipStream_t s, const WorkQ &Q) {
    hipLaunchKernelGGL((k_rhs_queue<DIM, N, EQ, VF, SF, CURV, MORT, CHF>), dim3(Q.nmort + Q.nchunks), dim3(threads),
                       lds, s, P, mode, Q);
}
template <int DIM, int N, bool CURV, bool OPEN>
void grad_launch(const RhsParams &P, int blocks, int threads, hipStream_t s, double suthS, double suthT0) {
    const size_t lds = (size_t)P.epb * GradShape<DIM, N, OPEN>::SLOT * sizeof(double);
    hipLaunchKernelGGL((k_grad<DIM, N, CURV, OPEN>), dim3(blocks), dim3(threads), lds, s, P, suthS, suthT0);
}
template <int DIM, int N>
void grad_launch_any(const RhsParams &P, bool curv, bool open, int blocks, int threads, hipStream_t s, double suthS,
                     double suthT0) {
    if (curv) {
        if (open) grad_launch<DIM, N, true, true>(P, blocks, threads, s, suthS, suthT0);
        else grad_launch<DIM, N, true, false>(P, blocks, threads, s, suthS, suthT0);
    } else {
        if (open) grad_launch<DIM, N, false, true>(P, blocks, threads, s, suthS, suthT0);
        else grad_launch<DIM, N, false, false>(P, blocks, threads, s, suthS, suthT0);
    }
}
template <int DIM, int N, bool MIX>
void ind_launch(const RhsParams &P, int iv, double amax, double amin, double *a, double *araw, int blocks,
                int threads, size_t lds, hipStream_t s, double *Tw, double *cw, double T0, double tol, int maxit) {
    hipLaunchKernelGGL((k_indicator<DIM, N, MIX>), dim3(blocks), dim3(threads), lds, s, P, iv, amax, amin, a,
                       araw, Tw, cw, T0, tol, maxit);
}

struct RhsEntry {
    int dim, N, eq, vf, sf, curv;
    RhsLaunch fn;
    int slot;  // doubles of LDS per element
    int mort;  // built with non-conforming (mortar) faces
    RhsLaunchP fnp;  // work-list form
    int alt;   // 1: the alternative LDS tiling (other work-item chunk count)
};

#define RHS_ENTRY(D, N, EQ, VF, SF, CV)                                                                             \
    {D, N, EQ, VF, SF, CV, &rhs_launch<D, N, EQ, VF, SF, (bool)CV, false, 0>, RhsShape<D, N, EQ, VF, (bool)CV>::SLOT, \
     0, &rhs_launch_p<D, N, EQ, VF, SF, (bool)CV, false, 0>, 0}
#define RHS_ENTRY_M(D, N, EQ, VF, SF)                                                                          \
    {D, N, EQ, VF, SF, 0, &rhs_launch<D, N, EQ, VF, SF, false, true, 0>, RhsShape<D, N, EQ, VF, false>::SLOT, 1, \
     &rhs_launch_p<D, N, EQ, VF, SF, false, true, 0>, 0}
// the alternative LDS tiling of a configuration: the pair and face work items
// in CH chunks instead of the default number (2 for the element types whose
// pair fluxes exceed 1,200 doubles, else 1)
#define RHS_ENTRY_T(D, N, EQ, VF, SF, CV, CH)                                                                 \
    {D, N, EQ, VF, SF, CV, &rhs_launch<D, N, EQ, VF, SF, (bool)CV, false, CH>,                                \
     RhsShape<D, N, EQ, VF, (bool)CV, CH>::SLOT, 0, &rhs_launch_p<D, N, EQ, VF, SF, (bool)CV, false, CH>, 1}

const RhsEntry kRhs[] = {
    // 2D perfect gas (isentropic vortex, O-grid checks)
    RHS_ENTRY(2, 3, 0, 0, 0, 0), RHS_ENTRY(2, 3, 0, 0, 1, 0), RHS_ENTRY(2, 3, 0, 0, 0, 1),
    RHS_ENTRY(2, 3, 0, 1, 0, 1), RHS_ENTRY(2, 4, 0, 0, 0, 0),
    // 3D perfect gas Euler / NS
    RHS_ENTRY(3, 3, 0, 0, 0, 0), RHS_ENTRY(3, 3, 0, 0, 1, 0), RHS_ENTRY(3, 3, 1, 0, 0, 0),
    RHS_ENTRY(3, 3, 0, 0, 0, 1), RHS_ENTRY(3, 3, 0, 0, 1, 1), RHS_ENTRY(3, 4, 0, 0, 0, 1),
    RHS_ENTRY(3, 4, 0, 0, 1, 1), RHS_ENTRY(3, 3, 0, 1, 0, 1), RHS_ENTRY(3, 4, 0, 1, 0, 1),
    // other split forms (Kennedy-Gruber, Pirozzoli) and the HLL surface flux
    RHS_ENTRY(3, 3, 0, 2, 0, 0), RHS_ENTRY(3, 3, 0, 3, 0, 0), RHS_ENTRY(3, 3, 0, 0, 2, 0),
    RHS_ENTRY(3, 3, 0, 2, 0, 1), RHS_ENTRY(3, 3, 0, 3, 0, 1), RHS_ENTRY(3, 3, 0, 1, 2, 1),
    // standard-DG volume form and the HLLC surface flux
    RHS_ENTRY(3, 3, 0, 4, 0, 0), RHS_ENTRY(3, 3, 0, 4, 0, 1), RHS_ENTRY(3, 3, 0, 0, 3, 0),
    RHS_ENTRY(3, 3, 0, 1, 3, 1),
    // and for the 2D Euler equations (affine elements)
    RHS_ENTRY(2, 3, 0, 2, 0, 0), RHS_ENTRY(2, 3, 0, 3, 0, 0), RHS_ENTRY(2, 3, 0, 4, 0, 0),
    RHS_ENTRY(2, 3, 0, 0, 2, 0), RHS_ENTRY(2, 3, 0, 0, 3, 0),
    // the same fluxes with the BR1 viscous terms (affine elements)
    RHS_ENTRY(3, 3, 1, 2, 0, 0), RHS_ENTRY(3, 3, 1, 3, 0, 0), RHS_ENTRY(3, 3, 1, 4, 0, 0),
    RHS_ENTRY(3, 3, 1, 0, 2, 0), RHS_ENTRY(3, 3, 1, 0, 3, 0),
    // and at N = 4 on curved (or affine) perfect-gas elements
    RHS_ENTRY(3, 4, 0, 2, 0, 1), RHS_ENTRY(3, 4, 0, 3, 0, 1), RHS_ENTRY(3, 4, 0, 4, 0, 1),
    RHS_ENTRY(3, 4, 0, 1, 2, 1), RHS_ENTRY(3, 4, 0, 1, 3, 1),
    // mixtures
    RHS_ENTRY(3, 4, 2, 1, 0, 1), RHS_ENTRY(3, 3, 2, 1, 0, 1), RHS_ENTRY(2, 3, 2, 1, 0, 1),
    RHS_ENTRY(3, 4, 2, 1, 2, 1),  // HLL faces on the curved 5-species shock
    // the other volume forms and HLLC faces for the curved 5-species equations
    RHS_ENTRY(3, 4, 2, 2, 0, 1), RHS_ENTRY(3, 4, 2, 3, 0, 1), RHS_ENTRY(3, 4, 2, 4, 0, 1),
    RHS_ENTRY(3, 4, 2, 1, 3, 1),
    // the entropy-conservative mixture flux (volume; also at the faces)
    RHS_ENTRY(3, 4, 2, 0, 0, 1), RHS_ENTRY(3, 4, 2, 0, 1, 1),
    // Navier-Stokes on curved elements
    RHS_ENTRY(3, 3, 1, 0, 0, 1), RHS_ENTRY(3, 4, 1, 0, 0, 1),
    // Morinishi's form (perfect gas)
    RHS_ENTRY(3, 3, 0, 5, 0, 0), RHS_ENTRY(3, 3, 0, 5, 0, 1), RHS_ENTRY(3, 4, 0, 5, 0, 1),
    RHS_ENTRY(2, 3, 0, 5, 0, 0), RHS_ENTRY(3, 3, 1, 5, 0, 0),
    RHS_ENTRY(2, 3, 3, 1, 0, 1), RHS_ENTRY(2, 3, 3, 1, 0, 0),
    // non-conforming (mortar) meshes
    RHS_ENTRY_M(3, 3, 0, 0, 0), RHS_ENTRY_M(3, 3, 0, 0, 1), RHS_ENTRY_M(3, 4, 0, 0, 0), RHS_ENTRY_M(2, 3, 0, 0, 0),
    // the other volume forms with Rusanov mortar faces
    RHS_ENTRY_M(3, 3, 0, 2, 0), RHS_ENTRY_M(3, 3, 0, 3, 0), RHS_ENTRY_M(3, 3, 0, 4, 0),
    RHS_ENTRY_M(3, 3, 0, 5, 0),
    // Navier-Stokes with viscous mortars
    RHS_ENTRY_M(3, 3, 1, 0, 0),
    // alternative tilings: the Navier-Stokes TGV kernel in two chunks, the
    // curved 5-species kernels in one
    RHS_ENTRY_T(3, 3, 1, 0, 0, 0, 2), RHS_ENTRY_T(3, 4, 2, 1, 0, 1, 1), RHS_ENTRY_T(3, 4, 2, 1, 2, 1, 1),
};

struct IndEntry {
    int dim, N, mix;
    IndLaunch fn;
};
const IndEntry kInd[] = {
    {2, 3, 0, &ind_launch<2, 3, false>}, {2, 3, 1, &ind_launch<2, 3, true>},
    {3, 3, 0, &ind_launch<3, 3, false>}, {3, 3, 1, &ind_launch<3, 3, true>},
    {3, 4, 0, &ind_launch<3, 4, false>}, {3, 4, 1, &ind_launch<3, 4, true>},
    {2, 4, 0, &ind_launch<2, 4, false>}, {2, 4, 1, &ind_launch<2, 4, true>},
};

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

}  // namespace

struct dgx_ctx {
    dgx_config cfg{};
    dgx_species sp{};
    bool has_sp = false;
    std::vector<double> rA, rb, rth;
    std::vector<int> rnu, rnup;
    int nvar = 0, N1 = 0, nn = 0, nf = 0;
    HostBasis basis;
    BasisC bc{};
    MixC mix{};
    KinC kin{};
    std::string err;
    const char *err_fixed = nullptr;  // static text of the last error (no allocation), else err
    // mesh
    int nelem = 0;
    bool curved = false;
    bool mesh_ok = false;
    int nbc = 0;
    DevBuf<double> geo, Jn, nsub, bc_state, bc_T, T, csnd, alpha, alpha_tmp, alpha_raw, grad, vpart, u1, u2, dtbuf;
    DevBuf<int> nbr, bc_kind, mort, iters, subs;
    DevBuf<double> mops;
    // work-list launches: queue counters (next item, mortar items done) and,
    // per elements-per-workgroup candidate 1, 2, 4, 8, the queue order of the
    // element chunks and which of them read mortar fluxes
    DevBuf<int> wq_ctr, wq_order[4];
    DevBuf<unsigned char> wq_waits[4];
    int wq_nchunks[4] = {}, wq_nfree[4] = {};
    DevBuf<double> tg;
    DevBuf<double> mflux;
    DevBuf<double> mgw;  // NS on mortars: sub-face gradient values W*_s
    // dynamic AMR: the octree leaves in element order, a pending adaptation
    // (new leaves and transfer rows), the transfer and sampling operators
    int oct_base = 0;
    std::vector<OctLeaf> oct, oct_new;
    std::vector<int32_t> oct_tab;
    DevBuf<int> amr_tab;
    DevBuf<double> amr_ops, amr_eq;
    bool open = false;   // the mesh has boundary or mortar faces
    int nmortar = 0;
    double Im[2][25] = {}, Pm[2][25] = {};
    DevBuf<KinC> kin_d;
    DevBuf<unsigned> flags;
    DevBuf<unsigned long long> rate;
    // launch configuration (autotuned elements per block)
    int epb = 1;
    int xcd = 0;  // launch form: 0 round-robin, 1 XCD-contiguous, 2 work list
    int tile = 0;  // 1: the alternative LDS tiling (rhs_alt)
    const RhsEntry *rhs_alt = nullptr;
    const RhsEntry *rhs = nullptr;
    // graph cache for ssprk3
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap_stream = nullptr;
    const double *g_u = nullptr;
    double g_dt = 0.0;
    // surrogate
    Surrogate sur;
};

namespace {

int set_err(dgx_ctx *ctx, int code, const std::string &msg) {
    if (ctx) {
        ctx->err = msg;
        ctx->err_fixed = nullptr;
    }
    return code;
}

// An error whose text is a string literal: records it without allocating.
int set_err_fixed(dgx_ctx *ctx, int code, const char *msg) {
    if (ctx) ctx->err_fixed = msg;
    return code;
}

// Runs f() and turns a C++ exception (a failed host allocation or thread
// start) into an error code, so that none leaves the C ABI.
template <typename F>
int guarded(dgx_ctx *ctx, F &&f) {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return set_err_fixed(ctx, DGX_E_NOMEM, "host memory allocation failed");
    } catch (...) {
        return set_err_fixed(ctx, DGX_E_NOMEM, "host resources exhausted (memory or threads)");
    }
}

template <typename T>
int dalloc(dgx_ctx *ctx, DevBuf<T> &b, size_t n) {
    if (b.n == n && b.p) return DGX_OK;
    b.release();
    if (n == 0) return DGX_OK;
    if (hipMalloc(&b.p, n * sizeof(T)) != hipSuccess) {
        b.p = nullptr;
        return set_err(ctx, DGX_E_NOMEM, "hipMalloc failed");
    }
    b.n = n;
    return DGX_OK;
}

int threads_for(int nn, int epb) { return ((nn * epb + 63) / 64) * 64; }

// the kernel variant of the current LDS tiling
const RhsEntry *cur_rhs(const dgx_ctx *ctx) { return ctx->tile && ctx->rhs_alt ? ctx->rhs_alt : ctx->rhs; }

// process-wide autotuner cache: configuration key -> elements per workgroup
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;  // key -> (epb, launch form | tiling << 2)

std::string tune_key(const dgx_ctx *ctx);
bool epb_fits(const dgx_ctx *ctx, int epb);

void clear_graph(dgx_ctx *ctx) {
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
    ctx->g_u = nullptr;
}

bool is_mix(const dgx_ctx *ctx) { return ctx->cfg.equation >= DGX_EQ_EULER_MIX; }

// Host T(e) for a single mixture state (Dirichlet boundary states).
double host_T(const dgx_ctx *ctx, const double *u) {
    const MixC &M = ctx->mix;
    const int dim = ctx->cfg.dim;
    double rho = 0.0, m2 = 0.0;
    for (int s = 0; s < kNS; ++s) rho += u[s];
    for (int c = 0; c < dim; ++c) m2 += u[kNS + c] * u[kNS + c];
    const double target = u[kNS + dim] - 0.5 * m2 / rho;
    double T = ctx->cfg.T_guess;
    for (int it = 0; it < 200; ++it) {
        double e = 0.0, cv = 0.0;
        for (int s = 0; s < kNS; ++s) {
            double es = 1.5 * M.Rs[s] * T + M.e0[s], cs = 1.5 * M.Rs[s];
            if (M.mol[s]) {
                const double x = M.thv[s] / T, em1 = std::expm1(x);
                es += M.Rs[s] * T + M.Rs[s] * M.thv[s] / em1;
                cs += M.Rs[s] + M.Rs[s] * x * x * (em1 + 1.0) / (em1 * em1);
            }
            e += u[s] * es;
            cv += u[s] * cs;
        }
        const double dT = (e - target) / cv;
        T -= dT;
        if (std::fabs(dT) <= 1e-14 * T) break;
    }
    return T;
}

RhsParams base_params(dgx_ctx *ctx) {
    RhsParams P{};
    P.nelem = ctx->nelem;
    P.nbr = ctx->nbr.p;
    P.geo = ctx->geo.p;
    P.Jn = ctx->Jn.p;
    P.nsub = ctx->nsub.p;
    P.T = ctx->T.p;
    P.csnd = ctx->csnd.p;
    P.grad = ctx->grad.p;
    P.vpart = ctx->vpart.p;
    P.bc_kind = ctx->bc_kind.p;
    P.bc_state = ctx->bc_state.p;
    P.bc_T = ctx->bc_T.p;
    P.kin = ctx->kin_d.p;
    P.mort = ctx->mort.p;
    P.mflux = ctx->mflux.p;
    P.mops = ctx->mops.p;
    P.mgw = ctx->mgw.p;
    P.gamma = ctx->cfg.gamma;
    P.R = ctx->cfg.R;
    P.mu = ctx->cfg.mu;
    P.kappa = ctx->cfg.mu * ctx->cfg.gamma * ctx->cfg.R / ((ctx->cfg.gamma - 1.0) * ctx->cfg.Pr);
    P.epb = ctx->epb;
    P.xcd = ctx->xcd == 1 ? 1 : 0;  // 2: work-list launches (queue order)
    P.flags = ctx->flags.p;
    P.B = ctx->bc;
    P.M = ctx->mix;
    return P;
}

const IndEntry *find_ind(const dgx_ctx *ctx) {
    for (const auto &e : kInd)
        if (e.dim == ctx->cfg.dim && e.N == ctx->cfg.N && e.mix == (is_mix(ctx) ? 1 : 0)) return &e;
    return nullptr;
}

// thermo for the mesh state (mixtures), T stored in ctx->T
int enqueue_thermo_mesh(dgx_ctx *ctx, const double *u, hipStream_t s) {
    const int64_t count = (int64_t)ctx->nelem * ctx->nn;
    const int th = 256;
    const int blocks = (int)((count + th - 1) / th);
    if (ctx->cfg.dim == 2)
        hipLaunchKernelGGL(k_thermo<2>, dim3(blocks), dim3(th), 0, s, u, count, (const double *)nullptr,
                           ctx->cfg.T_guess, ctx->cfg.newton_tol, ctx->cfg.newton_maxit, ctx->mix, ctx->T.p,
                           (double *)nullptr, ctx->csnd.p, (int *)nullptr, ctx->flags.p, 1);
    else
        hipLaunchKernelGGL(k_thermo<3>, dim3(blocks), dim3(th), 0, s, u, count, (const double *)nullptr,
                           ctx->cfg.T_guess, ctx->cfg.newton_tol, ctx->cfg.newton_maxit, ctx->mix, ctx->T.p,
                           (double *)nullptr, ctx->csnd.p, (int *)nullptr, ctx->flags.p, 1);
    return hipGetLastError() == hipSuccess ? DGX_OK : DGX_E_DEVICE;
}

// Everything of one right-hand-side evaluation.  mode 0: out = du;
// mode 1: out = sa*u0 + sb*(u + dt*du).
struct EventTape {
    hipEvent_t ev[9];
    const char *name[8];
    int n = 0;  // kernels recorded
};

void tape_mark(EventTape *tp, const char *name, hipStream_t s) {
    if (!tp || tp->n >= 8) return;
    tp->name[tp->n] = name;
    (void)hipEventRecord(tp->ev[++tp->n], s);
}

int enqueue_rhs(dgx_ctx *ctx, const double *u, double *out, int mode, const double *u0, double sa, double sb,
                double dt, hipStream_t s, EventTape *tp = nullptr) {
    const dgx_config &c = ctx->cfg;
    if (tp) (void)hipEventRecord(tp->ev[0], s);
    // mixtures: the T(e) solve runs inside the shock indicator when there is
    // one (the same per-node steps, one pass over the state less)
    const bool fuse_T = is_mix(ctx) && c.force_alpha < 0.0 && c.shock && find_ind(ctx);
    if (is_mix(ctx) && !fuse_T) {
        int rc = enqueue_thermo_mesh(ctx, u, s);
        if (rc) return set_err(ctx, rc, "thermo launch failed");
        tape_mark(tp, "k_thermo", s);
    }
    RhsParams P = base_params(ctx);
    P.u = u;
    const int epb = ctx->epb;
    const int th = threads_for(ctx->nn, epb);
    const int blocks = (ctx->nelem + epb - 1) / epb;
    // shock indicator / forced blending
    if (c.force_alpha >= 0.0) {
        P.alpha = ctx->alpha.p;
    } else if (c.shock) {
        const IndEntry *ie = find_ind(ctx);
        if (!ie) return set_err(ctx, DGX_E_INVAL, "no indicator kernel for this configuration");
        ie->fn(P, c.ind_var, c.alpha_max, c.alpha_min, ctx->alpha.p, ctx->alpha_raw.p, blocks, th,
               (size_t)epb * 3 * ctx->nn * sizeof(double), s, fuse_T ? ctx->T.p : nullptr,
               fuse_T ? ctx->csnd.p : nullptr, c.T_guess, c.newton_tol, c.newton_maxit);
        if (c.alpha_smooth) {
            const int tb = 256;
            if (c.dim == 2)
                hipLaunchKernelGGL(k_alpha_smooth<2>, dim3((ctx->nelem + tb - 1) / tb), dim3(tb), 0, s,
                                   ctx->nbr.p, ctx->nelem, ctx->alpha.p, ctx->alpha_tmp.p);
            else
                hipLaunchKernelGGL(k_alpha_smooth<3>, dim3((ctx->nelem + tb - 1) / tb), dim3(tb), 0, s,
                                   ctx->nbr.p, ctx->nelem, ctx->alpha.p, ctx->alpha_tmp.p);
            (void)hipMemcpyAsync(ctx->alpha.p, ctx->alpha_tmp.p, ctx->nelem * sizeof(double), hipMemcpyDeviceToDevice,
                           s);
        }
        P.alpha = ctx->alpha.p;
        tape_mark(tp, fuse_T ? "k_indicator_T" : "k_indicator", s);
    }
    if (c.equation == DGX_EQ_NS) {
        if (ctx->nmortar) {
            RhsParams M = P;
            M.out = ctx->mgw.p;
            const int nsub = c.dim == 3 ? 4 : 2;
            const int items = ctx->nmortar * nsub * ctx->nf;
            if (c.dim == 3 && c.N == 3)
                hipLaunchKernelGGL((k_mortar_grad<3, 3>), dim3((items + 255) / 256), dim3(256), 0, s, M, ctx->nmortar);
            else if (c.dim == 3 && c.N == 4)
                hipLaunchKernelGGL((k_mortar_grad<3, 4>), dim3((items + 255) / 256), dim3(256), 0, s, M, ctx->nmortar);
            else if (c.dim == 2 && c.N == 3)
                hipLaunchKernelGGL((k_mortar_grad<2, 3>), dim3((items + 255) / 256), dim3(256), 0, s, M, ctx->nmortar);
            else return set_err(ctx, DGX_E_INVAL, "NS mortar gradients not built for this dim/N");
            tape_mark(tp, "k_mortar_grad", s);
        }
        RhsParams G = P;
        G.out = ctx->vpart.p;
        G.out2 = ctx->grad.p;
        const double sS = c.sutherland_S, sT = c.sutherland_T0;
        const bool cv = ctx->curved, op = ctx->open;
        if (c.dim == 3 && c.N == 3) grad_launch_any<3, 3>(G, cv, op, blocks, th, s, sS, sT);
        else if (c.dim == 3 && c.N == 4) grad_launch_any<3, 4>(G, cv, op, blocks, th, s, sS, sT);
        else if (c.dim == 2 && c.N == 3) grad_launch_any<2, 3>(G, cv, op, blocks, th, s, sS, sT);
        else return set_err(ctx, DGX_E_INVAL, "NS gradients not built for this dim/N");
        tape_mark(tp, "k_grad", s);
    }
    const bool persist = ctx->xcd == 2;
    if (ctx->nmortar && !persist) {
        // the grid form's mortar pass: the work-list kernel with no queue
        WorkQ Q{nullptr, nullptr, nullptr, nullptr, ctx->nmortar, 0, 0};
        cur_rhs(ctx)->fnp(P, mode, th, 0, s, Q);
        tape_mark(tp, "k_mortar", s);
    }
    P.out = out;
    P.u0 = u0;
    P.sa = sa;
    P.sb = sb;
    P.dt = dt;
    if (persist) {
        const int k = epb == 1 ? 0 : epb == 2 ? 1 : epb == 4 ? 2 : 3;
        hipLaunchKernelGGL(k_workq_reset, dim3(1), dim3(64), 0, s, ctx->wq_ctr.p, ctx->wq_ctr.p + 1);
        WorkQ Q{ctx->wq_ctr.p, ctx->wq_ctr.p + 1, ctx->wq_order[k].p, ctx->wq_waits[k].p, ctx->nmortar,
                ctx->wq_nchunks[k], ctx->wq_nfree[k]};
        cur_rhs(ctx)->fnp(P, mode, th, (size_t)epb * cur_rhs(ctx)->slot * sizeof(double), s, Q);
    } else {
        cur_rhs(ctx)->fn(P, mode, blocks, th, (size_t)epb * cur_rhs(ctx)->slot * sizeof(double), s);
    }
    tape_mark(tp, "k_rhs", s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, DGX_E_DEVICE, std::string("rhs launch: ") + hipGetErrorString(e));
    return DGX_OK;
}

std::string tune_key(const dgx_ctx *ctx) {
    const dgx_config &c = ctx->cfg;
    return std::to_string(c.dim) + "," + std::to_string(c.N) + "," + std::to_string(c.equation) + "," +
           std::to_string(c.volume_flux) + "," + std::to_string(c.surface_flux) + "," + std::to_string(ctx->curved) +
           "," + std::to_string(ctx->nelem) + "," + std::to_string(ctx->nmortar > 0);
}

// default elements per workgroup: about 256 threads, within 32 KB of LDS
// (element types whose slot alone is large, the curved mixture kernels at
// N = 4, then run one element per workgroup: measured faster than two)
int default_epb(int nn, int slot) {
    int epb = std::max(1, 256 / nn);
    while (epb > 1 && (size_t)epb * slot * sizeof(double) > 32 * 1024) epb >>= 1;
    return epb;
}

bool epb_fits(const dgx_ctx *ctx, int epb) {
    if (epb < 1 || epb > 8 || (epb & (epb - 1)) || !ctx->rhs) return false;
    if (threads_for(ctx->nn, epb) > 512) return false;
    if (ctx->cfg.equation == DGX_EQ_NS) {
        // the gradient kernel's slot (GradShape): own W and face traces, then
        // the contravariant fluxes of all directions
        const int dim = ctx->cfg.dim, nw = dim + 1, nsf = 2 * dim * ctx->nf;
        const size_t g0 = (size_t)nw * ctx->nn + (size_t)nw * nsf, gt = (size_t)dim * nw * ctx->nn;
        const size_t gslot = ctx->open ? g0 + gt : std::max(g0, gt);
        if ((size_t)epb * gslot * sizeof(double) > 64 * 1024) return false;
    }
    return (size_t)epb * cur_rhs(ctx)->slot * sizeof(double) <= 64 * 1024;
}

template <int DIM, int N, bool MIX, bool CURV>
void pos_launch(const RhsParams &P, double *u, int blocks, int threads, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_positivity<DIM, N, MIX, CURV>), dim3(blocks), dim3(threads), lds, s, P, u);
}

int enqueue_positivity(dgx_ctx *ctx, double *u, hipStream_t s) {
    const dgx_config &c = ctx->cfg;
    RhsParams P = base_params(ctx);
    const int epb = ctx->epb;
    const int th = threads_for(ctx->nn, epb);
    const int blocks = (ctx->nelem + epb - 1) / epb;
    const int nv = ctx->nvar, nd = is_mix(ctx) ? 5 : 1;
    const size_t lds = (size_t)epb * ((nv + 1) * ctx->nn + nv + nd + 2) * sizeof(double);
    const int key = c.dim * 1000 + c.N * 100 + (is_mix(ctx) ? 10 : 0) + (ctx->curved ? 1 : 0);
    switch (key) {
        case 2300: pos_launch<2, 3, false, false>(P, u, blocks, th, lds, s); break;
        case 2301: pos_launch<2, 3, false, true>(P, u, blocks, th, lds, s); break;
        case 2311: pos_launch<2, 3, true, true>(P, u, blocks, th, lds, s); break;
        case 2310: pos_launch<2, 3, true, false>(P, u, blocks, th, lds, s); break;
        case 3300: pos_launch<3, 3, false, false>(P, u, blocks, th, lds, s); break;
        case 3301: pos_launch<3, 3, false, true>(P, u, blocks, th, lds, s); break;
        case 3401: pos_launch<3, 4, false, true>(P, u, blocks, th, lds, s); break;
        case 3411: pos_launch<3, 4, true, true>(P, u, blocks, th, lds, s); break;
        case 3311: pos_launch<3, 3, true, true>(P, u, blocks, th, lds, s); break;
        default: return set_err(ctx, DGX_E_INVAL, "no positivity kernel for this configuration");
    }
    return hipGetLastError() == hipSuccess ? DGX_OK : set_err(ctx, DGX_E_DEVICE, "positivity launch failed");
}

int check_ctx(dgx_ctx *ctx) {
    if (!ctx) return DGX_E_INVAL;
    if (!ctx->mesh_ok) return set_err(ctx, DGX_E_STATE, "no mesh set");
    return DGX_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

static int create_body(const dgx_config *cfg, dgx_ctx **out) {
    if (!cfg || !out) return DGX_E_INVAL;
    *out = nullptr;
    if ((cfg->dim != 2 && cfg->dim != 3) || (cfg->N != 3 && cfg->N != 4)) return DGX_E_INVAL;
    if (cfg->equation < 0 || cfg->equation > 3) return DGX_E_INVAL;
    if (!(cfg->sutherland_S >= 0.0) || (cfg->sutherland_S > 0.0 && !(cfg->sutherland_T0 > 0.0)))
        return DGX_E_INVAL;
    const bool mix = cfg->equation >= DGX_EQ_EULER_MIX;
    if (mix && (!cfg->species || cfg->species->nspecies != 5)) return DGX_E_INVAL;
    if (mix && cfg->volume_flux == DGX_VF_MORINISHI) return DGX_E_INVAL;
    if (cfg->equation == DGX_EQ_REACT_MIX && !cfg->reactions) return DGX_E_INVAL;
    if (mix && cfg->reactions) {
        const dgx_reactions *r = cfg->reactions;
        if (r->nreactions < 1 || r->nreactions > kMaxR || !r->A || !r->b || !r->theta_a || !r->nu || !r->nup)
            return DGX_E_INVAL;
        for (int i = 0; i < r->nreactions; ++i)
            if (!(r->A[i] > 0.0) || !std::isfinite(r->A[i]) || !std::isfinite(r->b[i]) ||
                !std::isfinite(r->theta_a[i]))
                return DGX_E_INVAL;
    }
    if (cfg->equation == DGX_EQ_NS && (cfg->mu < 0.0 || cfg->Pr <= 0.0)) return DGX_E_INVAL;
    if (!mix && !(cfg->gamma > 1.0)) return DGX_E_INVAL;
    dgx_ctx *ctx = new (std::nothrow) dgx_ctx();
    if (!ctx) return DGX_E_NOMEM;
    ctx->cfg = *cfg;
    ctx->cfg.species = nullptr;
    ctx->cfg.reactions = nullptr;
    ctx->N1 = cfg->N + 1;
    ctx->nn = cfg->dim == 2 ? ctx->N1 * ctx->N1 : ctx->N1 * ctx->N1 * ctx->N1;
    ctx->nf = ctx->nn / ctx->N1;
    ctx->nvar = (mix ? 5 : 1) + cfg->dim + 1;
    ctx->basis = make_basis(cfg->N);
    mortar_operators(ctx->basis, ctx->Im, ctx->Pm);
    for (int i = 0; i < ctx->N1 * ctx->N1; ++i) {
        ctx->bc.D[i] = ctx->basis.D[i];
        ctx->bc.Vinv[i] = ctx->basis.Vinv[i];
    }
    for (int i = 0; i < ctx->N1; ++i) ctx->bc.w[i] = ctx->basis.w[i];
    if (mix) {
        ctx->sp = *cfg->species;
        ctx->has_sp = true;
        for (int s = 0; s < 5; ++s) {
            ctx->mix.Rs[s] = ctx->sp.Ru / ctx->sp.W[s];
            ctx->mix.thv[s] = ctx->sp.molecule[s] ? ctx->sp.theta_v[s] : 0.0;
            ctx->mix.e0[s] = ctx->sp.e0[s];
            ctx->mix.mol[s] = ctx->sp.molecule[s] ? 1 : 0;
        }
    }
    if (mix && cfg->reactions) {
        // reaction table: sources in the right-hand side (DGX_EQ_REACT_MIX)
        // and the split stiff-chemistry step (dgx_chem_step)
        const dgx_reactions *r = cfg->reactions;
        KinC &K = ctx->kin;
        K.nr = r->nreactions;
        const dgx_species &sp = ctx->sp;
        for (int i = 0; i < K.nr; ++i) {
            K.lnA[i] = std::log(r->A[i]);
            K.b[i] = r->b[i];
            K.tha[i] = r->theta_a[i];
            double sum = 0.0;
            for (int s = 0; s < 5; ++s) {
                K.nu[i][s] = r->nu[i * 5 + s];
                K.nup[i][s] = r->nup[i * 5 + s];
                sum += K.nup[i][s] - K.nu[i][s];
            }
            K.dnu_sum[i] = sum;
        }
        for (int s = 0; s < 5; ++s) {
            K.W[s] = sp.W[s];
            // -g_s/(R_s T) = ln c_s + (5/2 + mol) ln T - mol [ln theta_r + ln sigma]
            //                - mol ln(1 - e^{-theta_v/T}) + ln Qe - e0/(R_s T);
            // gconst = -ln c_s + mol (ln theta_r + ln sigma) - ln Qe  (see k_rhs)
            const double ct = std::log(sp.Ru / (sp.NA * sp.p_ref)) +
                              1.5 * std::log(2.0 * M_PI * sp.W[s] * sp.Ru / (sp.NA * sp.NA * sp.hP * sp.hP));
            double g = -ct - std::log(sp.Qe[s]);
            if (sp.molecule[s]) g += std::log(sp.theta_r[s]) + std::log(sp.sigma[s]);
            K.gconst[s] = g;
        }
        K.lnpref_Ru = std::log(sp.p_ref / sp.Ru);
    }
    for (const auto &e : kRhs) {
        if (e.dim == cfg->dim && e.N == cfg->N && e.eq == cfg->equation && e.vf == cfg->volume_flux &&
            e.sf == cfg->surface_flux) {
            ctx->rhs = &e;  // curved flag fixed at set_mesh
            break;
        }
    }
    if (!ctx->rhs) {
        delete ctx;
        return DGX_E_INVAL;
    }
    if (hipMalloc(&ctx->flags.p, sizeof(unsigned)) != hipSuccess) {
        delete ctx;
        return DGX_E_DEVICE;
    }
    ctx->flags.n = 1;
    (void)hipMemset(ctx->flags.p, 0, sizeof(unsigned));
    if (hipMalloc(&ctx->rate.p, sizeof(unsigned long long)) != hipSuccess) {
        ctx->flags.release();
        delete ctx;
        return DGX_E_DEVICE;
    }
    ctx->rate.n = 1;
    *out = ctx;
    return DGX_OK;
}

int dgx_create(const dgx_config *cfg, dgx_ctx **out) {
    return guarded(nullptr, [&] { return create_body(cfg, out); });
}

static int set_mesh_body(dgx_ctx *ctx, const dgx_mesh *m) {
    if (!ctx || !m || !m->x || m->nelem <= 0) return set_err(ctx, DGX_E_INVAL, "bad mesh");
    const int dim = ctx->cfg.dim, N = ctx->cfg.N, n1 = ctx->N1, nn = ctx->nn, E = m->nelem;
    const int nv = ctx->nvar;
    if (m->nface < 0 || (m->nface && !m->faces) || m->nbface < 0 || (m->nbface && !m->bfaces) ||
        m->nbc < 0 || (m->nbc && (!m->bc_kind || !m->bc_state)))
        return set_err(ctx, DGX_E_INVAL, "bad mesh tables");
    if (m->nmortar < 0 || (m->nmortar && !m->mortars)) return set_err(ctx, DGX_E_INVAL, "bad mortar table");
    if (m->nmortar && ctx->cfg.equation != DGX_EQ_EULER && ctx->cfg.equation != DGX_EQ_NS)
        return set_err(ctx, DGX_E_INVAL, "mortars are supported for the perfect-gas equations");
    // connectivity (every check below runs before the context changes, so a
    // rejected mesh leaves the previous one in place)
    std::vector<int> nbr((size_t)E * 2 * dim, INT_MIN);
    for (int i = 0; i < m->nface; ++i) {
        const int eL = m->faces[4 * i], fL = m->faces[4 * i + 1], eR = m->faces[4 * i + 2], fR = m->faces[4 * i + 3];
        if (eL < 0 || eL >= E || eR < 0 || eR >= E || fL < 0 || fL >= 2 * dim || fL % 2 != 1 || fR != fL - 1)
            return set_err(ctx, DGX_E_INVAL, "face row " + std::to_string(i) + " is not a (+d, -d) pair");
        nbr[(size_t)eL * 2 * dim + fL] = eR;
        nbr[(size_t)eR * 2 * dim + fR] = eL;
    }
    for (int i = 0; i < m->nbface; ++i) {
        const int e = m->bfaces[3 * i], f = m->bfaces[3 * i + 1], b = m->bfaces[3 * i + 2];
        if (e < 0 || e >= E || f < 0 || f >= 2 * dim || b < 0 || b >= m->nbc)
            return set_err(ctx, DGX_E_INVAL, "bad boundary face " + std::to_string(i));
        nbr[(size_t)e * 2 * dim + f] = -1 - b;
    }
    const int nsub = dim == 3 ? 4 : 2;
    for (int i = 0; i < m->nmortar; ++i) {
        const int32_t *row = m->mortars + (size_t)i * (3 + nsub);
        const int eL = row[0], fL = row[1], fS = row[2 + nsub];
        if (eL < 0 || eL >= E || fL < 0 || fL >= 2 * dim || fS != (fL ^ 1))
            return set_err(ctx, DGX_E_INVAL, "bad mortar row " + std::to_string(i));
        nbr[(size_t)eL * 2 * dim + fL] = kMortBase - (8 * i + 7);
        for (int s2 = 0; s2 < nsub; ++s2) {
            const int es = row[2 + s2];
            if (es < 0 || es >= E) return set_err(ctx, DGX_E_INVAL, "bad mortar element");
            nbr[(size_t)es * 2 * dim + fS] = kMortBase - (8 * i + s2);
        }
    }
    for (size_t i = 0; i < nbr.size(); ++i)
        if (nbr[i] == INT_MIN) return set_err(ctx, DGX_E_INVAL, "element face without neighbour or boundary");
    for (int b = 0; b < m->nbc; ++b)
        if (m->bc_kind[b] < 0 || m->bc_kind[b] > 4) return set_err(ctx, DGX_E_INVAL, "bad boundary kind");
    // geometry: per-element metric terms at the first node and the affine
    // test first; the nodal arrays only when a curved variant runs
    const int GA = dim * dim + 1;
    std::vector<double> g((size_t)E * GA);
    std::vector<int> bad_J(16, INT_MAX);
    std::vector<unsigned char> curved_el(E, 0);
    host_parallel(E, [&](int e0, int e1, int t) {
        MetricScratch ws;
        std::vector<double> jae(dim * dim * nn), je(nn);
        const double *xe[3];
        for (int e = e0; e < e1; ++e) {
            for (int c = 0; c < dim; ++c) xe[c] = m->x + ((size_t)c * E + e) * nn;
            element_metrics(ctx->basis, dim, xe, jae.data(), je.data(), ws);
            double mx = 0.0, dev = 0.0;
            for (int k = 0; k < dim * dim; ++k)
                for (int n = 0; n < nn; ++n) {
                    mx = std::max(mx, std::fabs(jae[k * nn + n]));
                    dev = std::max(dev, std::fabs(jae[k * nn + n] - jae[k * nn]));
                }
            bool pos = true;
            for (int n = 0; n < nn; ++n) {
                pos = pos && je[n] > 0.0;
                dev = std::max(dev, std::fabs(je[n] - je[0]) * mx / std::fabs(je[0]));
            }
            if (!pos) {
                bad_J[t] = std::min(bad_J[t], e);
                continue;
            }
            // affine up to the rounding of the coordinates: an element of size h
            // at distance ~1 from the origin carries relative coordinate noise
            // ~1e-16/h (4e-13 at the finest octree level), which the metric
            // terms amplify; genuine curvature is many orders larger
            curved_el[e] = dev > 1e-10 * mx;
            for (int k = 0; k < dim * dim; ++k) g[(size_t)e * GA + k] = jae[k * nn];
            g[(size_t)e * GA + dim * dim] = je[0];
        }
    });
    {
        const int b = *std::min_element(bad_J.begin(), bad_J.end());
        if (b != INT_MAX) return set_err(ctx, DGX_E_INVAL, "non-positive Jacobian in element " + std::to_string(b));
    }
    bool affine = std::find(curved_el.begin(), curved_el.end(), (unsigned char)1) == curved_el.end();
    if (m->nmortar && !affine) return set_err(ctx, DGX_E_INVAL, "mortars need affine elements");
    // pick the kernel variant for this geometry
    const RhsEntry *sel = nullptr;
    const int want_m = m->nmortar ? 1 : 0;
    for (const auto &e : kRhs)
        if (e.dim == dim && e.N == N && e.eq == ctx->cfg.equation && e.vf == ctx->cfg.volume_flux &&
            e.sf == ctx->cfg.surface_flux && e.curv == (affine ? 0 : 1) && e.mort == want_m && !e.alt)
            sel = &e;
    if (!sel && affine && !want_m)  // fall back to the curved variant (valid for any mesh)
        for (const auto &e : kRhs)
            if (e.dim == dim && e.N == N && e.eq == ctx->cfg.equation && e.vf == ctx->cfg.volume_flux &&
                e.sf == ctx->cfg.surface_flux && e.curv == 1 && e.mort == 0 && !e.alt)
                sel = &e, affine = false;
    if (!sel) return set_err(ctx, DGX_E_INVAL, "no kernel variant for this configuration and mesh");
    const RhsEntry *alt = nullptr;
    for (const auto &e : kRhs)
        if (e.alt && e.dim == sel->dim && e.N == sel->N && e.eq == sel->eq && e.vf == sel->vf && e.sf == sel->sf &&
            e.curv == sel->curv && e.mort == sel->mort)
            alt = &e;
    clear_graph(ctx);
    ctx->mesh_ok = false;
    ctx->rhs = sel;
    ctx->rhs_alt = alt;
    ctx->tile = 0;
    ctx->curved = !affine;
    ctx->open = m->nbface > 0 || m->nmortar > 0;
    ctx->nelem = E;
    ctx->nbc = m->nbc;
    int rc;
    if ((rc = dalloc(ctx, ctx->nbr, nbr.size()))) return rc;
    HIPCHK(hipMemcpy(ctx->nbr.p, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice));
    // work queues: element chunks without non-conforming faces
    // first, then those that read mortar fluxes
    if ((rc = dalloc(ctx, ctx->wq_ctr, 2))) return rc;
    for (int k = 0; k < 4; ++k) {
        const int epb = 1 << k;
        const int nch = (E + epb - 1) / epb;
        std::vector<int> order;
        std::vector<unsigned char> waits(nch, 0), wq(nch);
        order.reserve(nch);
        for (int c = 0; c < nch; ++c) {
            for (int e = c * epb; e < std::min(E, (c + 1) * epb) && !waits[c]; ++e)
                for (int f = 0; f < 2 * dim; ++f)
                    if (nbr[(size_t)e * 2 * dim + f] <= kMortBase) waits[c] = 1;
            if (!waits[c]) order.push_back(c);
        }
        for (int c = 0; c < nch; ++c)
            if (waits[c]) order.push_back(c);
        for (int i = 0; i < nch; ++i) wq[i] = waits[order[i]];
        if ((rc = dalloc(ctx, ctx->wq_order[k], nch)) || (rc = dalloc(ctx, ctx->wq_waits[k], nch))) return rc;
        HIPCHK(hipMemcpy(ctx->wq_order[k].p, order.data(), nch * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(ctx->wq_waits[k].p, wq.data(), nch, hipMemcpyHostToDevice));
        ctx->wq_nchunks[k] = nch;
        ctx->wq_nfree[k] = (int)std::count(waits.begin(), waits.end(), (unsigned char)0);
    }
    if (affine) {
        if ((rc = dalloc(ctx, ctx->geo, g.size()))) return rc;
        HIPCHK(hipMemcpy(ctx->geo.p, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice));
        ctx->Jn.release();
        ctx->nsub.release();
    } else {
        std::vector<double> Ja((size_t)dim * dim * E * nn), Jv((size_t)E * nn);
        host_parallel(E, [&](int e0, int e1, int) {
            MetricScratch ws;
            std::vector<double> jae(dim * dim * nn);
            const double *xe[3];
            for (int e = e0; e < e1; ++e) {
                for (int c = 0; c < dim; ++c) xe[c] = m->x + ((size_t)c * E + e) * nn;
                element_metrics(ctx->basis, dim, xe, jae.data(), Jv.data() + (size_t)e * nn, ws);
                for (int k = 0; k < dim * dim; ++k)
                    std::memcpy(&Ja[((size_t)k * E + e) * nn], &jae[(size_t)k * nn], nn * sizeof(double));
            }
        });
        if ((rc = dalloc(ctx, ctx->geo, Ja.size()))) return rc;
        HIPCHK(hipMemcpy(ctx->geo.p, Ja.data(), Ja.size() * sizeof(double), hipMemcpyHostToDevice));
        if ((rc = dalloc(ctx, ctx->Jn, Jv.size()))) return rc;
        HIPCHK(hipMemcpy(ctx->Jn.p, Jv.data(), Jv.size() * sizeof(double), hipMemcpyHostToDevice));
        if (ctx->cfg.shock || ctx->cfg.force_alpha > 0.0) {
            // telescoped subcell normals n_m = Ja^d_0 + sum_{l<m} w_l (D_d Ja^d)_l, m = 1..N
            const int nf = ctx->nf;
            std::vector<double> ns((size_t)E * dim * nf * N * dim);
            std::vector<double> f(nn), df(nn);
            for (int e = 0; e < E; ++e)
                for (int d = 0; d < dim; ++d) {
                    const int st = d == 0 ? 1 : (d == 1 ? n1 : n1 * n1);
                    for (int c = 0; c < dim; ++c) {
                        for (int n = 0; n < nn; ++n) f[n] = Ja[((size_t)(d * dim + c) * E + e) * nn + n];
                        ref_derivative(ctx->basis, dim, d, f.data(), df.data());
                        for (int l = 0; l < nf; ++l) {
                            // node of line l at position a along d
                            int base;
                            if (d == 0) base = n1 * l;
                            else if (d == 1) base = (l % n1) + (dim == 3 ? n1 * n1 * (l / n1) : 0);
                            else base = l;
                            double acc = f[base];
                            for (int mm = 1; mm <= N; ++mm) {
                                acc += ctx->basis.w[mm - 1] * df[base + (mm - 1) * st];
                                ns[((((size_t)e * dim + d) * nf + l) * N + (mm - 1)) * dim + c] = acc;
                            }
                        }
                    }
                }
            if ((rc = dalloc(ctx, ctx->nsub, ns.size()))) return rc;
            HIPCHK(hipMemcpy(ctx->nsub.p, ns.data(), ns.size() * sizeof(double), hipMemcpyHostToDevice));
        }
    }
    // mortars
    ctx->nmortar = m->nmortar;
    if (m->nmortar) {
        if ((rc = dalloc(ctx, ctx->mort, (size_t)m->nmortar * (3 + nsub)))) return rc;
        HIPCHK(hipMemcpy(ctx->mort.p, m->mortars, (size_t)m->nmortar * (3 + nsub) * sizeof(int), hipMemcpyHostToDevice));
        double ops[100];
        std::memcpy(ops, ctx->Im, sizeof(ctx->Im));
        std::memcpy(ops + 50, ctx->Pm, sizeof(ctx->Pm));
        if ((rc = dalloc(ctx, ctx->mops, 100))) return rc;
        HIPCHK(hipMemcpy(ctx->mops.p, ops, sizeof(ops), hipMemcpyHostToDevice));
        if ((rc = dalloc(ctx, ctx->mflux, (size_t)m->nmortar * nsub * nv * ctx->nf))) return rc;
        if (ctx->cfg.equation == DGX_EQ_NS &&
            (rc = dalloc(ctx, ctx->mgw, (size_t)m->nmortar * nsub * (dim + 1) * ctx->nf)))
            return rc;
    }
    // boundary states
    if (m->nbc) {
        if ((rc = dalloc(ctx, ctx->bc_kind, m->nbc))) return rc;
        HIPCHK(hipMemcpy(ctx->bc_kind.p, m->bc_kind, m->nbc * sizeof(int), hipMemcpyHostToDevice));
        if ((rc = dalloc(ctx, ctx->bc_state, (size_t)m->nbc * nv))) return rc;
        HIPCHK(hipMemcpy(ctx->bc_state.p, m->bc_state, (size_t)m->nbc * nv * sizeof(double), hipMemcpyHostToDevice));
        std::vector<double> bT(m->nbc, 0.0);
        if (is_mix(ctx))
            for (int b = 0; b < m->nbc; ++b)
                if (m->bc_kind[b] == DGX_BC_DIRICHLET) bT[b] = host_T(ctx, m->bc_state + (size_t)b * nv);
        if ((rc = dalloc(ctx, ctx->bc_T, m->nbc))) return rc;
        HIPCHK(hipMemcpy(ctx->bc_T.p, bT.data(), m->nbc * sizeof(double), hipMemcpyHostToDevice));
    }
    // scratch
    if (is_mix(ctx)) {
        // per-node temperature, the warm start of the right-hand side's
        // T(e) solves: the freestream guess until the first solve
        if ((rc = dalloc(ctx, ctx->T, (size_t)E * nn))) return rc;
        if ((rc = dalloc(ctx, ctx->csnd, (size_t)E * nn))) return rc;
        std::vector<double> t0((size_t)E * nn, ctx->cfg.T_guess);
        HIPCHK(hipMemcpy(ctx->T.p, t0.data(), t0.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if ((rc = dalloc(ctx, ctx->alpha, E))) return rc;
    if ((rc = dalloc(ctx, ctx->alpha_tmp, E))) return rc;
    if ((rc = dalloc(ctx, ctx->alpha_raw, E))) return rc;
    {
        std::vector<double> a(E, ctx->cfg.force_alpha >= 0.0 ? ctx->cfg.force_alpha : 0.0);
        HIPCHK(hipMemcpy(ctx->alpha.p, a.data(), E * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(ctx->alpha_raw.p, a.data(), E * sizeof(double), hipMemcpyHostToDevice));
    }
    if (ctx->cfg.equation == DGX_EQ_NS) {
        if ((rc = dalloc(ctx, ctx->grad, (size_t)E * 2 * dim * (dim + 1) * ctx->nf))) return rc;
        if ((rc = dalloc(ctx, ctx->vpart, (size_t)(dim + 1) * E * nn))) return rc;
    }
    if (ctx->kin.nr > 0) {
        if ((rc = dalloc(ctx, ctx->kin_d, 1))) return rc;
        HIPCHK(hipMemcpy(ctx->kin_d.p, &ctx->kin, sizeof(KinC), hipMemcpyHostToDevice));
    }
    // default elements per block: about 256 threads, LDS <= 64 KB; a cached
    // autotuner choice for this configuration wins
    const int epb = default_epb(nn, sel->slot);
    ctx->epb = epb;
    // XCD-contiguous numbering by default while the state fits well inside
    // the 256 MB Infinity Cache
    ctx->xcd = (size_t)ctx->nvar * E * nn * sizeof(double) <= (size_t)128 << 20;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(tune_key(ctx));
        if (it != g_tune.end()) {
            const int saved_tile = ctx->tile;
            ctx->tile = (it->second.second >> 2) && ctx->rhs_alt ? 1 : 0;
            if (epb_fits(ctx, it->second.first)) {
                ctx->epb = it->second.first;
                ctx->xcd = it->second.second & 3;
            } else {
                ctx->tile = saved_tile;
            }
        }
    }
    ctx->mesh_ok = true;
    // a mesh from the caller replaces any octree (dgx_set_octree and
    // dgx_amr_apply record theirs after this call)
    ctx->oct.clear();
    ctx->oct_new.clear();
    ctx->oct_tab.clear();
    return DGX_OK;
}

int dgx_set_mesh(dgx_ctx *ctx, const dgx_mesh *m) {
    return guarded(ctx, [&] { return set_mesh_body(ctx, m); });
}

int dgx_rhs(dgx_ctx *ctx, const double *u, double t, double *du, void *stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    (void)t;
    if (!u || !du || u == du) return set_err(ctx, DGX_E_INVAL, "u/du must be distinct device pointers");
    return enqueue_rhs(ctx, u, du, 0, nullptr, 0.0, 1.0, 0.0, (hipStream_t)stream);
}

int dgx_ssprk3_step(dgx_ctx *ctx, double *u, double t, double dt, int nsteps, void *stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    (void)t;
    if (!u || nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return set_err(ctx, DGX_E_INVAL, "bad ssprk3 arguments");
    if (nsteps == 0) return DGX_OK;
    const size_t n = (size_t)ctx->nvar * ctx->nelem * ctx->nn;
    if ((rc = dalloc(ctx, ctx->u1, n))) return rc;
    if ((rc = dalloc(ctx, ctx->u2, n))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (!ctx->gexec || ctx->g_u != u || ctx->g_dt != dt) {
        clear_graph(ctx);
        if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        const bool lim = ctx->cfg.positivity != 0;
        int r1 = enqueue_rhs(ctx, u, ctx->u1.p, 1, nullptr, 0.0, 1.0, dt, ctx->cap_stream);
        if (!r1 && lim) r1 = enqueue_positivity(ctx, ctx->u1.p, ctx->cap_stream);
        int r2 = r1 ? r1 : enqueue_rhs(ctx, ctx->u1.p, ctx->u2.p, 1, u, 0.75, 0.25, dt, ctx->cap_stream);
        if (!r2 && lim) r2 = enqueue_positivity(ctx, ctx->u2.p, ctx->cap_stream);
        int r3 = r2 ? r2 : enqueue_rhs(ctx, ctx->u2.p, u, 1, u, 1.0 / 3.0, 2.0 / 3.0, dt, ctx->cap_stream);
        if (!r3 && lim) r3 = enqueue_positivity(ctx, u, ctx->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(ctx->cap_stream, &g);
        if (r3) {
            if (g) (void)hipGraphDestroy(g);
            return r3;
        }
        if (ee != hipSuccess) return set_err(ctx, DGX_E_DEVICE, std::string("capture: ") + hipGetErrorString(ee));
        ctx->graph = g;
        HIPCHK(hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
        ctx->g_u = u;
        ctx->g_dt = dt;
    }
    for (int i = 0; i < nsteps; ++i) HIPCHK(hipGraphLaunch(ctx->gexec, s));
    return DGX_OK;
}

int dgx_limit_positivity(dgx_ctx *ctx, double *u, void *stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!u) return set_err(ctx, DGX_E_INVAL, "null state");
    return enqueue_positivity(ctx, u, (hipStream_t)stream);
}

int dgx_max_dt(dgx_ctx *ctx, const double *u, double cfl, double *dt_host, void *stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!u || !dt_host || !(cfl > 0.0)) return set_err(ctx, DGX_E_INVAL, "bad max_dt arguments");
    hipStream_t s = (hipStream_t)stream;
    if (is_mix(ctx) && (rc = enqueue_thermo_mesh(ctx, u, s))) return rc;
    HIPCHK(hipMemsetAsync(ctx->rate.p, 0, sizeof(unsigned long long), s));
    RhsParams P = base_params(ctx);
    P.u = u;
    P.epb = ctx->nn;
    const int64_t total = (int64_t)ctx->nelem * ctx->nn;
    const int tb = 256;
    const int blocks = (int)((total + tb - 1) / tb);
    const int key = ctx->cfg.dim * 100 + (is_mix(ctx) ? 10 : 0) + (ctx->curved ? 1 : 0);
    switch (key) {
        case 200: hipLaunchKernelGGL((k_maxrate<2, false, false>), dim3(blocks), dim3(tb), 0, s, P, ctx->rate.p); break;
        case 201: hipLaunchKernelGGL((k_maxrate<2, false, true>), dim3(blocks), dim3(tb), 0, s, P, ctx->rate.p); break;
        case 210: hipLaunchKernelGGL((k_maxrate<2, true, false>), dim3(blocks), dim3(tb), 0, s, P, ctx->rate.p); break;
        case 211: hipLaunchKernelGGL((k_maxrate<2, true, true>), dim3(blocks), dim3(tb), 0, s, P, ctx->rate.p); break;
        case 300: hipLaunchKernelGGL((k_maxrate<3, false, false>), dim3(blocks), dim3(tb), 0, s, P, ctx->rate.p); break;
        case 301: hipLaunchKernelGGL((k_maxrate<3, false, true>), dim3(blocks), dim3(tb), 0, s, P, ctx->rate.p); break;
        case 310: hipLaunchKernelGGL((k_maxrate<3, true, false>), dim3(blocks), dim3(tb), 0, s, P, ctx->rate.p); break;
        default: hipLaunchKernelGGL((k_maxrate<3, true, true>), dim3(blocks), dim3(tb), 0, s, P, ctx->rate.p); break;
    }
    unsigned long long bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, ctx->rate.p, sizeof(bits), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double rate;
    std::memcpy(&rate, &bits, sizeof(rate));
    if (!(rate > 0.0) || !std::isfinite(rate)) return set_err(ctx, DGX_E_NONPHYSICAL, "non-finite wave speed");
    *dt_host = cfl * 2.0 / (ctx->N1 * rate);
    return DGX_OK;
}

// Per-node iteration counts in ctx->iters (-1: not converged), and substep
// counts in ctx->subs when with_subs -> stats.  Synchronises the stream.
static int collect_stats(dgx_ctx *ctx, int64_t count, int maxit, dgx_newton_stats *stats, hipStream_t s,
                         bool with_subs = false) {
    std::vector<int> h(count), hs;
    HIPCHK(hipMemcpyAsync(h.data(), ctx->iters.p, count * sizeof(int), hipMemcpyDeviceToHost, s));
    if (with_subs) {
        hs.resize(count);
        HIPCHK(hipMemcpyAsync(hs.data(), ctx->subs.p, count * sizeof(int), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    int64_t stot = 0;
    int smax = 0;
    for (int v : hs) {
        stot += v;
        smax = std::max(smax, v);
    }
    stats->substeps_total = stot;
    stats->substeps_max = smax;
    int64_t tot = 0, bad = 0, first = -1, fallbacks = 0;
    int mx = 0;
    double wsum = 0.0;
    int64_t nw = 0;
    for (int64_t i = 0; i < count; i += 64) {
        int wm = 0;
        for (int64_t j = i; j < std::min(count, i + 64); ++j) {
            int it = h[j];
            if (it >= 0 && (it & kItersFallback)) {
                ++fallbacks;
                it &= ~kItersFallback;
            }
            if (it < 0) {
                ++bad;
                if (first < 0) first = j;
                it = maxit;
            }
            tot += it;
            mx = std::max(mx, it);
            wm = std::max(wm, it);
        }
        wsum += wm;
        ++nw;
    }
    stats->nodes = count;
    stats->iters_total = tot;
    stats->iters_max = mx;
    stats->iters_wave_max_mean = nw ? wsum / nw : 0.0;
    stats->nonconverged = bad;
    stats->first_bad = first;
    stats->fallbacks = fallbacks;
    if (bad) return set_err(ctx, DGX_E_NOCONV, std::to_string(bad) + " nodes did not converge");
    return DGX_OK;
}

int dgx_thermo(dgx_ctx *ctx, const double *u, int64_t nstates, double *T, double *p, int guess_mode,
               dgx_newton_stats *stats, void *stream) {
    if (!ctx) return DGX_E_INVAL;
    if (!is_mix(ctx)) return set_err(ctx, DGX_E_INVAL, "thermo needs a mixture context");
    if (!u || !T) return set_err(ctx, DGX_E_INVAL, "null pointer");
    if (guess_mode != DGX_GUESS_FREESTREAM && guess_mode != DGX_GUESS_SURROGATE)
        return set_err(ctx, DGX_E_INVAL, "bad guess mode");
    int64_t count = nstates;
    if (count <= 0) {
        if (!ctx->mesh_ok) return set_err(ctx, DGX_E_STATE, "no mesh and no state count");
        count = (int64_t)ctx->nelem * ctx->nn;
    }
    if (guess_mode == DGX_GUESS_SURROGATE && !ctx->sur.ready) return set_err(ctx, DGX_E_STATE, "surrogate has no weights");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if (stats && (rc = dalloc(ctx, ctx->iters, (size_t)count))) return rc;
    const double *tg = nullptr;
    if (guess_mode == DGX_GUESS_SURROGATE) {
        if ((rc = dalloc(ctx, ctx->tg, (size_t)count))) return rc;
        rc = surrogate_predict(ctx->sur, ctx->cfg.dim, u, count, ctx->tg.p, s);
        if (rc) return set_err(ctx, rc, "surrogate launch failed");
        tg = ctx->tg.p;
    }
    int *iters = stats ? ctx->iters.p : nullptr;
    const int tb = 256;
    const int blocks = (int)((count + tb - 1) / tb);
    if (ctx->cfg.dim == 2)
        hipLaunchKernelGGL(k_thermo<2>, dim3(blocks), dim3(tb), 0, s, u, count, tg, ctx->cfg.T_guess,
                           ctx->cfg.newton_tol, ctx->cfg.newton_maxit, ctx->mix, T, p, (double *)nullptr, iters,
                           ctx->flags.p, 0);
    else
        hipLaunchKernelGGL(k_thermo<3>, dim3(blocks), dim3(tb), 0, s, u, count, tg, ctx->cfg.T_guess,
                           ctx->cfg.newton_tol, ctx->cfg.newton_maxit, ctx->mix, T, p, (double *)nullptr, iters,
                           ctx->flags.p, 0);
    if (hipGetLastError() != hipSuccess) return set_err(ctx, DGX_E_DEVICE, "thermo launch failed");
    if (!stats) return DGX_OK;
    return collect_stats(ctx, count, ctx->cfg.newton_maxit, stats, s);
}

int dgx_chem_step(dgx_ctx *ctx, double *u, double dt, double tol, int maxit, dgx_newton_stats *stats,
                  void *stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!is_mix(ctx) || ctx->kin.nr < 1) return set_err(ctx, DGX_E_INVAL, "chemistry needs a mixture with reactions");
    if (!u) return set_err(ctx, DGX_E_INVAL, "null pointer");
    if (!(dt >= 0.0) || !(tol > 0.0) || maxit < 1) return set_err(ctx, DGX_E_INVAL, "bad dt, tol or maxit");
    hipStream_t s = (hipStream_t)stream;
    const int64_t count = (int64_t)ctx->nelem * ctx->nn;
    if (stats && ((rc = dalloc(ctx, ctx->iters, (size_t)count)) || (rc = dalloc(ctx, ctx->subs, (size_t)count))))
        return rc;
    // temperature of the incoming state: the warm start of the inner solves
    if ((rc = enqueue_thermo_mesh(ctx, u, s))) return set_err(ctx, rc, "thermo launch failed");
    int *iters = stats ? ctx->iters.p : nullptr;
    const int tb = 256;
    const int blocks = (int)((count + tb - 1) / tb);
    const double ttol = 1e-14;
    const int tmaxit = 100;
    int *subs = stats ? ctx->subs.p : nullptr;
    if (ctx->cfg.dim == 2)
        hipLaunchKernelGGL(k_chem<2>, dim3(blocks), dim3(tb), 0, s, u, count, dt, ctx->kin_d.p, ctx->mix, ctx->T.p, tol,
                           maxit, ttol, tmaxit, iters, subs, ctx->flags.p);
    else
        hipLaunchKernelGGL(k_chem<3>, dim3(blocks), dim3(tb), 0, s, u, count, dt, ctx->kin_d.p, ctx->mix, ctx->T.p, tol,
                           maxit, ttol, tmaxit, iters, subs, ctx->flags.p);
    if (hipGetLastError() != hipSuccess) return set_err(ctx, DGX_E_DEVICE, "chemistry launch failed");
    if (!stats) return DGX_OK;
    return collect_stats(ctx, count, maxit, stats, s, true);
}

const double *dgx_last_alpha(const dgx_ctx *ctx) {
    if (!ctx || !ctx->mesh_ok) return nullptr;
    if (!ctx->cfg.shock && ctx->cfg.force_alpha < 0.0) return nullptr;
    return ctx->alpha.p;
}

int dgx_check(dgx_ctx *ctx, void *stream) {
    if (!ctx) return DGX_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    unsigned f = 0;
    HIPCHK(hipMemcpyAsync(&f, ctx->flags.p, sizeof(f), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemset(ctx->flags.p, 0, sizeof(unsigned)));
    if (f & FLAG_NOCONV) return set_err(ctx, DGX_E_NOCONV, "Newton for T(e) did not converge");
    if (f & FLAG_NONPHYS) return set_err(ctx, DGX_E_NONPHYSICAL, "non-physical state (rho_s < 0, p <= 0 or non-finite)");
    return DGX_OK;
}

int dgx_species_energy(const dgx_ctx *ctx, double T, double *e, double *cv) {
    if (!ctx || !ctx->has_sp || !e || !cv || !(T > 0.0)) return DGX_E_INVAL;
    const MixC &M = ctx->mix;
    for (int s = 0; s < kNS; ++s) {
        double es = 1.5 * M.Rs[s] * T + M.e0[s], cs = 1.5 * M.Rs[s];
        if (M.mol[s]) {
            const double x = M.thv[s] / T, em1 = std::expm1(x);
            es += M.Rs[s] * T + M.Rs[s] * M.thv[s] / em1;
            cs += M.Rs[s] + M.Rs[s] * x * x * (em1 + 1.0) / (em1 * em1);
        }
        e[s] = es;
        cv[s] = cs;
    }
    return DGX_OK;
}

int dgx_mixture_energy(const dgx_ctx *ctx, const double *rs, const double *T, int64_t n, double *rhoe,
                       double *rhocv) {
    if (!ctx || !ctx->has_sp || n < 0 || (n > 0 && (!rs || !T || (!rhoe && !rhocv)))) return DGX_E_INVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!(T[i] > 0.0)) return DGX_E_INVAL;
    for (int64_t i = 0; i < n; ++i) {
        double e[kNS], cv[kNS];
        dgx_species_energy(ctx, T[i], e, cv);
        double se = 0.0, sc = 0.0;
        for (int s = 0; s < kNS; ++s) {
            se += rs[(size_t)s * n + i] * e[s];
            sc += rs[(size_t)s * n + i] * cv[s];
        }
        if (rhoe) rhoe[i] = se;
        if (rhocv) rhocv[i] = sc;
    }
    return DGX_OK;
}

int dgx_surrogate_set(dgx_ctx *ctx, const float *params, size_t n) {
    if (!ctx || !params || n != (size_t)kSurParams + kSurNorm) return set_err(ctx, DGX_E_INVAL, "bad surrogate params");
    return surrogate_set(ctx->sur, params) ? set_err(ctx, DGX_E_DEVICE, "surrogate upload failed") : DGX_OK;
}

int dgx_surrogate_get(dgx_ctx *ctx, float *params, size_t n) {
    if (!ctx || !params || n != (size_t)kSurParams + kSurNorm) return set_err(ctx, DGX_E_INVAL, "bad surrogate params");
    if (!ctx->sur.ready) return set_err(ctx, DGX_E_STATE, "surrogate has no weights");
    return surrogate_get(ctx->sur, params) ? set_err(ctx, DGX_E_DEVICE, "surrogate download failed") : DGX_OK;
}

int dgx_surrogate_train(dgx_ctx *ctx, const double *states, const double *T, int64_t count, int epochs, int batch,
                        float lr, uint64_t seed, float *loss_host, void *stream) {
    if (!ctx || !is_mix(ctx)) return set_err(ctx, DGX_E_INVAL, "surrogate needs a mixture context");
    if (!states || !T || count < 256 || epochs < 1 || batch < 64 || batch % 64 || !(lr > 0.0f))
        return set_err(ctx, DGX_E_INVAL, "bad training arguments");
    int rc = surrogate_train(ctx->sur, ctx->cfg.dim, states, T, count, epochs, batch, lr, seed, loss_host,
                             (hipStream_t)stream);
    if (rc) return set_err(ctx, rc, "surrogate training failed: " + ctx->sur.err);
    return DGX_OK;
}

int dgx_surrogate_init(dgx_ctx *ctx, const double *states, const double *T, int64_t count, uint64_t seed,
                       void *stream) {
    if (!ctx || !is_mix(ctx)) return set_err(ctx, DGX_E_INVAL, "surrogate needs a mixture context");
    if (!states || !T || count < 2) return set_err(ctx, DGX_E_INVAL, "bad init arguments");
    int rc = surrogate_init(ctx->sur, ctx->cfg.dim, states, T, count, seed, (hipStream_t)stream);
    return rc ? set_err(ctx, rc, "surrogate init failed") : DGX_OK;
}

int dgx_surrogate_grad(dgx_ctx *ctx, const double *states, const double *T, int64_t count, float *grad_host,
                       float *loss_host, void *stream) {
    if (!ctx || !is_mix(ctx)) return set_err(ctx, DGX_E_INVAL, "surrogate needs a mixture context");
    if (!states || !T || !grad_host || count < 1) return set_err(ctx, DGX_E_INVAL, "bad grad arguments");
    if (!ctx->sur.ready) return set_err(ctx, DGX_E_STATE, "surrogate has no weights");
    int rc = surrogate_grad(ctx->sur, ctx->cfg.dim, states, T, count, grad_host, loss_host, (hipStream_t)stream);
    return rc ? set_err(ctx, rc, "surrogate gradient failed") : DGX_OK;
}

int dgx_surrogate_predict(dgx_ctx *ctx, const double *states, int64_t count, double *Tg, void *stream) {
    if (!ctx || !is_mix(ctx) || !states || !Tg || count <= 0) return set_err(ctx, DGX_E_INVAL, "bad predict arguments");
    if (!ctx->sur.ready) return set_err(ctx, DGX_E_STATE, "surrogate has no weights");
    int rc = surrogate_predict(ctx->sur, ctx->cfg.dim, states, count, Tg, (hipStream_t)stream);
    return rc ? set_err(ctx, rc, "surrogate launch failed") : DGX_OK;
}

int dgx_kernel_times(dgx_ctx *ctx, const double *u, int reps, double *ms_out, int *nk, char *names_out,
                     size_t names_len, void *stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!u || reps < 1 || !ms_out || !nk) return set_err(ctx, DGX_E_INVAL, "bad kernel_times arguments");
    const size_t n = (size_t)ctx->nvar * ctx->nelem * ctx->nn;
    if ((rc = dalloc(ctx, ctx->u1, n))) return rc;
    if ((rc = dalloc(ctx, ctx->u2, n))) return rc;
    hipStream_t s = (hipStream_t)stream;
    // a second SSPRK3 stage as in a step: u0 is its own buffer (a copy of u),
    // so its reads cost what they cost in the time loop
    HIPCHK(hipMemcpyAsync(ctx->u1.p, u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    std::vector<EventTape> tapes(reps);
    for (auto &t : tapes)
        for (auto &e : t.ev) HIPCHK(hipEventCreate(&e));
    // one untimed evaluation first: the first of a series runs several
    // percent slower than the ones after it
    rc = enqueue_rhs(ctx, u, ctx->u2.p, 1, ctx->u1.p, 0.75, 0.25, 1e-6, s);
    for (int r = 0; r < reps && !rc; ++r)
        rc = enqueue_rhs(ctx, u, ctx->u2.p, 1, ctx->u1.p, 0.75, 0.25, 1e-6, s, &tapes[r]);
    HIPCHK(hipStreamSynchronize(s));
    const int k = tapes[0].n;
    for (int i = 0; i < k; ++i) {
        double tot = 0.0;
        for (int r = 0; r < reps; ++r) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, tapes[r].ev[i], tapes[r].ev[i + 1]));
            tot += ms;
        }
        ms_out[i] = tot / reps;
    }
    *nk = k;
    if (names_out && names_len) {
        std::string all;
        for (int i = 0; i < k; ++i) all += (i ? "," : "") + std::string(tapes[0].name[i]);
        std::snprintf(names_out, names_len, "%s", all.c_str());
    }
    for (auto &t : tapes)
        for (auto &e : t.ev) (void)hipEventDestroy(e);
    return rc;
}

int dgx_set_launch(dgx_ctx *ctx, int epb, int order) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (order < -1 || (order >= 0 && ((order & 3) > 2 || (order >> 2) > 1)))
        return set_err(ctx, DGX_E_INVAL, "launch order must be -1, or 0, 1, 2 plus 4 for the alternative LDS tiling");
    const int xcd = order < 0 ? ctx->xcd : (order & 3);
    const int tile = order < 0 ? ctx->tile : (order >> 2);
    if (tile && !ctx->rhs_alt)
        return set_err(ctx, DGX_E_INVAL, "no alternative LDS tiling for this configuration");
    const int saved_tile = ctx->tile;
    ctx->tile = tile;
    if (!epb_fits(ctx, epb)) {
        ctx->tile = saved_tile;
        return set_err(ctx, DGX_E_INVAL, "elements per workgroup must be 1, 2, 4 or 8 and fit in 512 threads and 64 KB of LDS");
    }
    if (epb != ctx->epb || xcd != ctx->xcd || tile != saved_tile) clear_graph(ctx);
    ctx->epb = epb;
    ctx->xcd = xcd;
    return DGX_OK;
}

int dgx_get_launch(dgx_ctx *ctx, int *epb, int *order) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (epb) *epb = ctx->epb;
    if (order) *order = ctx->xcd | (ctx->tile << 2);
    return DGX_OK;
}

int dgx_autotune(dgx_ctx *ctx, const double *u, int reps, int *epb_out, double *ms_out, void *stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!u || reps < 1) return set_err(ctx, DGX_E_INVAL, "bad autotune arguments");
    const size_t n = (size_t)ctx->nvar * ctx->nelem * ctx->nn;
    if ((rc = dalloc(ctx, ctx->u1, n))) return rc;
    if ((rc = dalloc(ctx, ctx->u2, n))) return rc;
    hipStream_t s = (hipStream_t)stream;
    // what is timed: one SSPRK3 step as dgx_ssprk3_step runs it (three fused
    // stages with u0 in its own buffer, the limiter when configured), into
    // library scratch with dt = 0 so that u is untouched and every stage
    // state stays the valid input state
    const bool lim = ctx->cfg.positivity != 0;
    auto step = [&]() -> int {
        int r = enqueue_rhs(ctx, u, ctx->u1.p, 1, nullptr, 0.0, 1.0, 0.0, s);
        if (!r && lim) r = enqueue_positivity(ctx, ctx->u1.p, s);
        if (!r) r = enqueue_rhs(ctx, ctx->u1.p, ctx->u2.p, 1, u, 0.75, 0.25, 0.0, s);
        if (!r && lim) r = enqueue_positivity(ctx, ctx->u2.p, s);
        if (!r) r = enqueue_rhs(ctx, ctx->u2.p, ctx->u1.p, 1, u, 1.0 / 3.0, 2.0 / 3.0, 0.0, s);
        if (!r && lim) r = enqueue_positivity(ctx, ctx->u1.p, s);
        return r;
    };
    const int cand[4] = {1, 2, 4, 8};
    const int saved = ctx->epb, saved_xcd = ctx->xcd, saved_tile = ctx->tile;
    // the fastest candidate of each numbering; the default numbering (chosen
    // from the state size) is kept unless the other one is faster by more
    // than 2%: run-to-run noise is of that order, while the numberings' HBM
    // traffic can differ by much more (the round-robin order re-reads face
    // neighbours from memory when the state fits the Infinity Cache)
    const int def_xcd = (size_t)ctx->nvar * ctx->nelem * ctx->nn * sizeof(double) <= (size_t)128 << 20;
    // per launch form and tiling (index xm + 3 tile): the best time and its
    // elements per workgroup
    int best_epb[6] = {saved, saved, saved, saved, saved, saved};
    double best_ms[6] = {1e300, 1e300, 1e300, 1e300, 1e300, 1e300};
    // the default elements per workgroup, kept within a launch form unless
    // another count is faster by more than 2% (as for the numbering below)
    const int def_epb = default_epb(ctx->nn, cur_rhs(ctx)->slot);
    double def_ms[6] = {1e300, 1e300, 1e300, 1e300, 1e300, 1e300};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int i = 0; i < 4; ++i)
        if (ms_out) ms_out[i] = -1.0;
    for (int tl = 0; tl < (ctx->rhs_alt ? 2 : 1) && !rc; ++tl)
    for (int i = 0; i < 4 && !rc; ++i) {
        ctx->tile = tl;
        if (!epb_fits(ctx, cand[i])) continue;
        ctx->epb = cand[i];
        // both workgroup numberings (round-robin over the XCDs, XCD-contiguous)
        // and the work-list form
        for (int xm = 0; xm < 3 && !rc; ++xm) {
            ctx->xcd = xm;
            for (int w = 0; w < 2 && !rc; ++w) rc = step();
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps && !rc; ++r) rc = step();
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) rc = set_err(ctx, DGX_E_DEVICE, "autotune sync failed");
            if (rc) break;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double avg = ms / (3.0 * reps);  // per right-hand side
            if (ms_out && (ms_out[i] < 0.0 || avg < ms_out[i])) ms_out[i] = avg;
            if (cand[i] == def_epb) def_ms[xm + 3 * tl] = avg;
            if (avg < best_ms[xm + 3 * tl]) {
                best_ms[xm + 3 * tl] = avg;
                best_epb[xm + 3 * tl] = cand[i];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int k = 0; k < 6; ++k)
        if (def_ms[k] < 1e300 && !(best_ms[k] < 0.98 * def_ms[k])) {
            best_ms[k] = def_ms[k];
            best_epb[k] = def_epb;
        }
    // the default (numbering from the state size, default tiling) unless
    // another is faster by more than 2%
    int bi = def_xcd;
    for (int k = 0; k < 6; ++k)
        if (best_ms[k] < 0.98 * best_ms[def_xcd] && best_ms[k] < best_ms[bi]) bi = k;
    const int best = best_epb[bi], best_xcd = bi % 3, best_tile = bi / 3;
    ctx->epb = rc ? saved : best;
    ctx->xcd = rc ? saved_xcd : best_xcd;
    ctx->tile = rc ? saved_tile : best_tile;
    if (ctx->epb != saved || ctx->xcd != saved_xcd || ctx->tile != saved_tile) clear_graph(ctx);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(ctx)] = std::make_pair(best, best_xcd | (best_tile << 2));
    }
    if (epb_out) *epb_out = best;
    return DGX_OK;
}

// ---------------------------------------------------------------------------
// dgx_thermo_noalloc: dgx_thermo for callers that cannot allocate device
// memory.  Its scratch (the surrogate's guesses, the per-node iteration
// counts, the statistics accumulators) lives in one static device array of
// the library instead of buffers allocated on first use.  Each GPU holds its
// own copy of the array, at its own address, until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns on
// that device (the array's name is a host-side stand-in).  Every call on a
// GPU shares that GPU's copy: calls that overlap on one GPU race.
namespace {

constexpr int64_t kNoallocMaxStates = DGX_NOALLOC_MAX_STATES;
// guesses (double) + iteration counts (int, two per double) + accumulators
constexpr size_t kNoallocAcc = 8;
constexpr size_t kNoallocDoubles = (size_t)kNoallocMaxStates + (size_t)kNoallocMaxStates / 2 + kNoallocAcc;
static __device__ __align__(256) double scratch[kNoallocDoubles];

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
double *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_rc[kMaxDevices] = {};

// The current device's copy of `scratch` (set up once per device, with that
// device current), or nullptr.
double *noalloc_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::call_once(g_scratch_once[dev], [dev] {
        void *ptr = nullptr;
        g_scratch_rc[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_rc[dev] == hipSuccess ? static_cast<double *>(ptr) : nullptr;
    });
    return g_scratch_ptr[dev];
}

// accumulator slots (unsigned 64-bit): 0 sum of iterations, 1 non-converged,
// 2 fallbacks, 3 sum over waves of the per-wave maximum, 4 maximum, 5 first
// non-converged index (ULLONG_MAX: none)
__global__ void k_noalloc_clear(unsigned long long *acc) {
    if (threadIdx.x < kNoallocAcc) acc[threadIdx.x] = threadIdx.x == 5 ? ~0ull : 0ull;
}

// Statistics of the per-node iteration counts, the same rules as the host
// reduction of dgx_thermo: a non-converged node (-1) counts maxit
// iterations, the fallback bit is counted and removed, waves are the chunks
// of 64 consecutive nodes.
__global__ void __launch_bounds__(256) k_noalloc_stats(const int *__restrict__ iters, int64_t count, int maxit,
                                                       unsigned long long *acc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int it = 0, bad = 0, fb = 0;
    if (i < count) {
        it = iters[i];
        if (it >= 0 && (it & kItersFallback)) {
            fb = 1;
            it &= ~kItersFallback;
        }
        if (it < 0) {
            bad = 1;
            it = maxit;
        }
    }
    // wave (64 lanes = 64 consecutive nodes) reductions
    int wmax = it, wsum = it, wbad = bad, wfb = fb;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        wmax = max(wmax, __shfl_xor(wmax, off));
        wsum += __shfl_xor(wsum, off);
        wbad += __shfl_xor(wbad, off);
        wfb += __shfl_xor(wfb, off);
    }
    if (bad) atomicMin(&acc[5], (unsigned long long)i);
    const int64_t w0 = i - (threadIdx.x & 63);
    if ((threadIdx.x & 63) == 0 && w0 < count) {
        atomicAdd(&acc[0], (unsigned long long)wsum);
        atomicAdd(&acc[1], (unsigned long long)wbad);
        atomicAdd(&acc[2], (unsigned long long)wfb);
        atomicAdd(&acc[3], (unsigned long long)wmax);
        atomicMax(&acc[4], (unsigned long long)wmax);
    }
}

}  // namespace

int dgx_thermo_noalloc(dgx_ctx *ctx, const double *u, int64_t nstates, double *T, double *p, int guess_mode,
                       dgx_newton_stats *stats, void *stream) {
    if (!ctx) return DGX_E_INVAL;
    if (!is_mix(ctx)) return set_err_fixed(ctx, DGX_E_INVAL, "thermo needs a mixture context");
    if (!u || !T) return set_err_fixed(ctx, DGX_E_INVAL, "null pointer");
    if (guess_mode != DGX_GUESS_FREESTREAM && guess_mode != DGX_GUESS_SURROGATE)
        return set_err_fixed(ctx, DGX_E_INVAL, "bad guess mode");
    int64_t count = nstates;
    if (count <= 0) {
        if (!ctx->mesh_ok) return set_err_fixed(ctx, DGX_E_STATE, "no mesh and no state count");
        count = (int64_t)ctx->nelem * ctx->nn;
    }
    if (count > kNoallocMaxStates)
        return set_err_fixed(ctx, DGX_E_INVAL,
                             "dgx_thermo_noalloc: more states than DGX_NOALLOC_MAX_STATES (1048576)");
    if (guess_mode == DGX_GUESS_SURROGATE && !ctx->sur.ready)
        return set_err_fixed(ctx, DGX_E_STATE, "surrogate has no weights");
    double *base = noalloc_scratch();
    if (!base) return set_err_fixed(ctx, DGX_E_DEVICE, "no address for the static scratch on this device");
    double *tg_s = base;
    int *iters_s = reinterpret_cast<int *>(base + kNoallocMaxStates);
    auto *acc = reinterpret_cast<unsigned long long *>(base + kNoallocMaxStates + kNoallocMaxStates / 2);
    hipStream_t s = (hipStream_t)stream;
    const double *tg = nullptr;
    if (guess_mode == DGX_GUESS_SURROGATE) {
        if (surrogate_predict(ctx->sur, ctx->cfg.dim, u, count, tg_s, s))
            return set_err_fixed(ctx, DGX_E_DEVICE, "surrogate launch failed");
        tg = tg_s;
    }
    int *iters = stats ? iters_s : nullptr;
    const int tb = 256;
    const int blocks = (int)((count + tb - 1) / tb);
    if (ctx->cfg.dim == 2)
        hipLaunchKernelGGL(k_thermo<2>, dim3(blocks), dim3(tb), 0, s, u, count, tg, ctx->cfg.T_guess,
                           ctx->cfg.newton_tol, ctx->cfg.newton_maxit, ctx->mix, T, p, (double *)nullptr, iters,
                           ctx->flags.p, 0);
    else
        hipLaunchKernelGGL(k_thermo<3>, dim3(blocks), dim3(tb), 0, s, u, count, tg, ctx->cfg.T_guess,
                           ctx->cfg.newton_tol, ctx->cfg.newton_maxit, ctx->mix, T, p, (double *)nullptr, iters,
                           ctx->flags.p, 0);
    if (hipGetLastError() != hipSuccess) return set_err_fixed(ctx, DGX_E_DEVICE, "thermo launch failed");
    if (!stats) return DGX_OK;
    hipLaunchKernelGGL(k_noalloc_clear, dim3(1), dim3(64), 0, s, acc);
    hipLaunchKernelGGL(k_noalloc_stats, dim3(blocks), dim3(tb), 0, s, iters_s, count, ctx->cfg.newton_maxit, acc);
    if (hipGetLastError() != hipSuccess) return set_err_fixed(ctx, DGX_E_DEVICE, "statistics launch failed");
    unsigned long long h[kNoallocAcc];
    if (hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_err_fixed(ctx, DGX_E_DEVICE, "statistics copy failed");
    const int64_t nw = (count + 63) / 64;
    stats->nodes = count;
    stats->iters_total = (int64_t)h[0];
    stats->iters_max = (int32_t)h[4];
    stats->iters_wave_max_mean = nw ? (double)h[3] / (double)nw : 0.0;
    stats->nonconverged = (int64_t)h[1];
    stats->first_bad = h[5] == ~0ull ? -1 : (int64_t)h[5];
    stats->substeps_total = 0;
    stats->substeps_max = 0;
    stats->fallbacks = (int64_t)h[2];
    if (h[1]) return set_err_fixed(ctx, DGX_E_NOCONV, "nodes did not converge");
    return DGX_OK;
}

// ---------------------------------------------------------------------------
// dynamic AMR on a periodic octree
}  // extern "C"

namespace {

// Builds the mesh of the leaves (element order as given) on the periodic
// unit cube and uploads it.
int oct_upload(dgx_ctx *ctx, int base, const std::vector<OctLeaf> &order) {
    OctTree t;
    t.base = base;
    t.leaves.reserve(order.size() * 2);
    for (auto &c : order) t.leaves.insert(oct_key(c));
    std::vector<int32_t> faces, morts;
    oct_tables(t, order, faces, morts);
    const int n1 = ctx->N1, nn = ctx->nn, E = (int)order.size();
    std::vector<double> x((size_t)3 * E * nn);
    for (int e = 0; e < E; ++e) {
        const OctLeaf &c = order[e];
        const double h = 1.0 / (double)(base << c.L);
        const int cc[3] = {c.i, c.j, c.k};
        for (int n = 0; n < nn; ++n) {
            const int idx[3] = {n % n1, (n / n1) % n1, n / (n1 * n1)};
            for (int d = 0; d < 3; ++d)
                x[((size_t)d * E + e) * nn + n] = h * (cc[d] + 0.5 * (ctx->basis.x[idx[d]] + 1.0));
        }
    }
    dgx_mesh m{};
    m.nelem = E;
    m.x = x.data();
    m.nface = (int)(faces.size() / 4);
    m.faces = faces.data();
    m.nmortar = (int)(morts.size() / 7);
    m.mortars = morts.data();
    return dgx_set_mesh(ctx, &m);
}

// operators of the transfer (half-interval interpolation and L2 projection)
// and of Loehner's equidistant sampling
int amr_ops_upload(dgx_ctx *ctx) {
    const int n1 = ctx->N1;
    double ops[100];
    std::memcpy(ops, ctx->Im, sizeof(ctx->Im));
    std::memcpy(ops + 50, ctx->Pm, sizeof(ctx->Pm));
    std::vector<double> eq((size_t)n1 * n1);
    for (int a = 0; a < n1; ++a) {
        const double y = -1.0 + 2.0 * a / (n1 - 1);
        for (int j = 0; j < n1; ++j) {
            double l = 1.0;
            for (int m = 0; m < n1; ++m)
                if (m != j) l *= (y - ctx->basis.x[m]) / (ctx->basis.x[j] - ctx->basis.x[m]);
            eq[(size_t)a * n1 + j] = l;
        }
    }
    int rc;
    if ((rc = dalloc(ctx, ctx->amr_ops, 100))) return rc;
    if ((rc = dalloc(ctx, ctx->amr_eq, eq.size()))) return rc;
    HIPCHK(hipMemcpy(ctx->amr_ops.p, ops, sizeof(ops), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->amr_eq.p, eq.data(), eq.size() * sizeof(double), hipMemcpyHostToDevice));
    return DGX_OK;
}

}  // namespace

extern "C" {

static int set_octree_body(dgx_ctx *ctx, int base, int nleaf, const int32_t *leaves) {
    if (!ctx || nleaf <= 0 || !leaves) return set_err(ctx, DGX_E_INVAL, "bad octree");
    if (ctx->cfg.dim != 3 || ctx->cfg.equation >= DGX_EQ_EULER_MIX)
        return set_err(ctx, DGX_E_INVAL, "octree meshes are built for the 3D perfect-gas equations");
    std::vector<OctLeaf> v(nleaf);
    for (int e = 0; e < nleaf; ++e) v[e] = {leaves[4 * e], leaves[4 * e + 1], leaves[4 * e + 2], leaves[4 * e + 3]};
    OctTree t;
    const std::string err = oct_check(base, v, t);
    if (!err.empty()) return set_err(ctx, DGX_E_INVAL, err);
    morton_sort(v);
    int rc;
    if ((rc = amr_ops_upload(ctx))) return rc;
    if ((rc = oct_upload(ctx, base, v))) return rc;
    ctx->oct_base = base;
    ctx->oct = v;
    ctx->oct_new.clear();
    ctx->oct_tab.clear();
    return DGX_OK;
}

int dgx_set_octree(dgx_ctx *ctx, int base, int nleaf, const int32_t *leaves) {
    return guarded(ctx, [&] { return set_octree_body(ctx, base, nleaf, leaves); });
}

int dgx_get_octree(const dgx_ctx *ctx, int32_t *leaves_out, int nmax) {
    if (!ctx || ctx->oct.empty()) return DGX_E_STATE;
    const int n = (int)ctx->oct.size();
    if (leaves_out) {
        if (nmax < n) return DGX_E_INVAL;
        for (int e = 0; e < n; ++e) {
            leaves_out[4 * e] = ctx->oct[e].L;
            leaves_out[4 * e + 1] = ctx->oct[e].i;
            leaves_out[4 * e + 2] = ctx->oct[e].j;
            leaves_out[4 * e + 3] = ctx->oct[e].k;
        }
    }
    return n;
}

int dgx_amr_indicator(dgx_ctx *ctx, const double *u, int kind, int variable, double *ind, void *stream) {
    if (!ctx || !u || !ind) return set_err(ctx, DGX_E_INVAL, "null argument");
    if (ctx->oct.empty() || !ctx->mesh_ok) return set_err(ctx, DGX_E_STATE, "no octree mesh");
    if (kind < 0 || kind > 1 || variable < 0 || variable > 3) return set_err(ctx, DGX_E_INVAL, "bad indicator");
    hipStream_t s = (hipStream_t)stream;
    const int E = ctx->nelem;
    if (ctx->cfg.N == 3)
        hipLaunchKernelGGL(k_amr_indicator<3>, dim3(E), dim3(64), 0, s, u, E, ctx->cfg.gamma, kind, variable,
                           ctx->amr_eq.p, ctx->bc, ind);
    else
        hipLaunchKernelGGL(k_amr_indicator<4>, dim3(E), dim3(128), 0, s, u, E, ctx->cfg.gamma, kind, variable,
                           ctx->amr_eq.p, ctx->bc, ind);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, DGX_E_DEVICE, std::string("indicator launch: ") + hipGetErrorString(e));
    return DGX_OK;
}

static int amr_plan_body(dgx_ctx *ctx, const double *ind, const dgx_amr_controller *c, int *nelem_new) {
    if (!ctx || !ind || !c || !nelem_new) return set_err(ctx, DGX_E_INVAL, "null argument");
    if (ctx->oct.empty()) return set_err(ctx, DGX_E_STATE, "no octree mesh");
    if (c->base_level < 0 || c->med_level < c->base_level || c->max_level < c->med_level ||
        c->max_level > kOctMaxLevel || !(c->med_threshold <= c->max_threshold))
        return set_err(ctx, DGX_E_INVAL, "bad AMR controller");
    const int E = (int)ctx->oct.size();
    std::vector<int> target(E);
    for (int e = 0; e < E; ++e) {
        if (!std::isfinite(ind[e])) return set_err(ctx, DGX_E_INVAL, "non-finite indicator value");
        target[e] = ind[e] >= c->max_threshold ? c->max_level
                    : ind[e] >= c->med_threshold ? c->med_level
                                                 : c->base_level;
    }
    std::vector<OctLeaf> nv;
    std::vector<int32_t> tab;
    const std::string err = oct_adapt(ctx->oct_base, ctx->oct, target.data(), nv, tab);
    if (!err.empty()) return set_err(ctx, DGX_E_INVAL, err);
    ctx->oct_new = std::move(nv);
    ctx->oct_tab = std::move(tab);
    *nelem_new = (int)ctx->oct_new.size();
    return DGX_OK;
}

int dgx_amr_plan(dgx_ctx *ctx, const double *ind, const dgx_amr_controller *c, int *nelem_new) {
    return guarded(ctx, [&] { return amr_plan_body(ctx, ind, c, nelem_new); });
}

static int amr_apply_body(dgx_ctx *ctx, const double *u_old, double *u_new, void *stream) {
    if (!ctx || !u_old || !u_new) return set_err(ctx, DGX_E_INVAL, "null argument");
    if (ctx->oct_new.empty()) return set_err(ctx, DGX_E_STATE, "no pending adaptation");
    if (u_old == u_new) return set_err(ctx, DGX_E_INVAL, "u_old and u_new must not alias");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = dalloc(ctx, ctx->amr_tab, ctx->oct_tab.size()))) return rc;
    HIPCHK(hipMemcpy(ctx->amr_tab.p, ctx->oct_tab.data(), ctx->oct_tab.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice));
    const int nold = (int)ctx->oct.size(), nnew = (int)ctx->oct_new.size();
    const int items = nnew * ctx->nn;
    if (ctx->cfg.N == 3)
        hipLaunchKernelGGL(k_amr_transfer<3>, dim3((items + 255) / 256), dim3(256), 0, s, u_old, nold, u_new, nnew,
                           ctx->nvar, ctx->amr_tab.p, ctx->amr_ops.p);
    else
        hipLaunchKernelGGL(k_amr_transfer<4>, dim3((items + 255) / 256), dim3(256), 0, s, u_old, nold, u_new, nnew,
                           ctx->nvar, ctx->amr_tab.p, ctx->amr_ops.p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, DGX_E_DEVICE, std::string("transfer launch: ") + hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<OctLeaf> nv = std::move(ctx->oct_new);
    ctx->oct_new.clear();
    ctx->oct_tab.clear();
    if ((rc = oct_upload(ctx, ctx->oct_base, nv))) return rc;
    ctx->oct = std::move(nv);
    return DGX_OK;
}

int dgx_amr_apply(dgx_ctx *ctx, const double *u_old, double *u_new, void *stream) {
    return guarded(ctx, [&] { return amr_apply_body(ctx, u_old, u_new, stream); });
}

const char *dgx_last_error(const dgx_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->err_fixed ? ctx->err_fixed : ctx->err.c_str();
}

void dgx_destroy(dgx_ctx *ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    clear_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    DevBuf<double> *bufs[] = {&ctx->geo,   &ctx->Jn,        &ctx->nsub,      &ctx->bc_state, &ctx->bc_T, &ctx->T, &ctx->csnd,
                              &ctx->alpha, &ctx->alpha_tmp, &ctx->alpha_raw, &ctx->grad,     &ctx->u1,   &ctx->u2,
                              &ctx->dtbuf, &ctx->vpart};
    for (auto *b : bufs) b->release();
    ctx->nbr.release();
    ctx->mops.release();
    ctx->wq_ctr.release();
    for (int k = 0; k < 4; ++k) {
        ctx->wq_order[k].release();
        ctx->wq_waits[k].release();
    }
    ctx->bc_kind.release();
    ctx->mort.release();
    ctx->mflux.release();
    ctx->mgw.release();
    ctx->amr_tab.release();
    ctx->amr_ops.release();
    ctx->amr_eq.release();
    ctx->iters.release();
    ctx->subs.release();
    ctx->tg.release();
    ctx->kin_d.release();
    ctx->flags.release();
    ctx->rate.release();
    surrogate_free(ctx->sur);
    delete ctx;
}

}  // extern "C"

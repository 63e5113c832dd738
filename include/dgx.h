/*
 * dgx — semi-discrete entropy-stable DGSEM right-hand side on one AMD MI355X.
 *
 * C ABI of libdgx.so.  Every call takes plain pointers and sizes; no C++ or
 * PyTorch type crosses this boundary.  The operation computed is the
 * semi-discrete operator of arXiv 2511.17551 (H3PC), Sec. Methodology:
 *
 *   du/dt = -(1/J) sum_d { (1/w) Delta[(1-alpha) Fbar^d + alpha F^{FV,d}]
 *                          + surface Riemann fluxes }  + viscous terms + S
 *
 * (Eqs. strong_form, fluxes_discrete_fluxdifferencing, DGvec,
 * fluxes_discrete_with_fv, finitevolumeflux, riemann_problem1-3, auxil,
 * auxstrongf; thermochemistry from the Appendix, Eqs. Internal_energy ..
 * calc_prod).
 *
 * Conventions shared by every entry point
 *   Layout   state arrays u, du are device FP64 structure-of-arrays
 *            [nvar][nelem][(N+1)^dim], node n = i + (N+1)(j + (N+1)k), i along
 *            the first reference direction.  Variables: perfect gas
 *            (rho, rho v_1..rho v_dim, rho E); mixture (rho_N2, rho_O2,
 *            rho_NO, rho_N, rho_O, rho v_1..rho v_dim, rho E).
 *   Memory   the caller owns u, du, T, p (device memory, 8-byte aligned,
 *            contiguous).  The library owns everything it allocates (geometry,
 *            connectivity, stage buffers, graphs, surrogate weights) and frees
 *            it in dgx_destroy.
 *   Streams  calls enqueue on the caller's hipStream_t (NULL = legacy default
 *            stream).  Only calls documented as synchronising wait.
 *   Errors   0 on success or a negative DGX_E_* code.  DGX_E_INVAL is returned
 *            before anything is enqueued.  Device-side errors (non-physical
 *            states, Newton non-convergence) are sticky flags reported by the
 *            next synchronising call.  dgx_last_error() gives the text.  No
 *            call aborts the process and no C++ exception leaves the library.
 *   Threads  one context per host thread; contexts are independent.
 */
#ifndef DGX_H
#define DGX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define DGX_OK 0
#define DGX_E_INVAL (-1)        /* bad argument, checked before any launch   */
#define DGX_E_NOMEM (-2)        /* device or host allocation failed           */
#define DGX_E_DEVICE (-3)       /* a HIP runtime call failed                   */
#define DGX_E_NONPHYSICAL (-4)  /* non-finite value, rho_s < 0 or p <= 0       */
#define DGX_E_NOCONV (-5)       /* T(e) Newton exceeded its iteration limit    */
#define DGX_E_STATE (-6)        /* call out of order (e.g. rhs before mesh)    */

/* equation systems (Sec. Governing Equations) */
#define DGX_EQ_EULER 0      /* calorically perfect gas, inviscid               */
#define DGX_EQ_NS 1         /* perfect gas, BR1 viscous terms, const. mu       */
#define DGX_EQ_EULER_MIX 2  /* 5-species air, RRHO energies, frozen chemistry  */
#define DGX_EQ_REACT_MIX 3  /* 5-species air, RRHO energies, Arrhenius sources */

/* two-point volume fluxes (Eq. fluxdiffcons) */
#define DGX_VF_RANOCHA 0    /* entropy-conservative: Ranocha's (perfect gas),
                               the RRHO mixture flux below (mixtures) */
#define DGX_VF_DUCROS 1     /* Ducros split form                       */
#define DGX_VF_KENNEDY_GRUBER 2  /* Kennedy-Gruber split form          */
#define DGX_VF_PIROZZOLI 3  /* Pirozzoli split form                    */
#define DGX_VF_CENTRAL 4    /* standard-DG form, (f_L + f_R).n/2       */
#define DGX_VF_MORINISHI 5  /* Morinishi split form (perfect gas only) */
/* surface fluxes (Eqs. riemann_problem1-3) */
#define DGX_SF_RUSANOV 0    /* local Lax-Friedrichs                     */
#define DGX_SF_RANOCHA 1    /* the EC flux at faces (entropy checks)    */
#define DGX_SF_HLL 2        /* HLL, Davis wave-speed bounds             */
#define DGX_SF_HLLC 3       /* HLLC, Toro's contact speed               */
/* The split forms listed in the Methodology section as interchangeable
 * volume fluxes, with {{a}} = (a_L + a_R)/2: Kennedy-Gruber (mass flux
 * f = {{rho}}{{v.n}}, momentum f {{v}} + {{p}} n, energy f {{E/rho}} +
 * {{p}}{{v.n}}), Pirozzoli (energy f {{(E+p)/rho}}), Morinishi (f =
 * {{rho v}}.n, energy f ({{p/((gamma-1) rho)}} + v_L.v_R/2) + {{p v}}.n);
 * for mixtures the species rows of Kennedy-Gruber and Pirozzoli are
 * f {{rho_s/rho}}.  The standard-DG form is (f_L + f_R).n/2.  These and the
 * HLL and HLLC interface fluxes are built for the 3D perfect-gas Euler
 * equations at N = 3 (affine and curved elements, conforming meshes; the
 * volume forms also on 2:1 non-conforming meshes with Rusanov faces), at
 * N = 4 (curved kernels, which also take affine meshes), for 3D
 * Navier-Stokes at N = 3 (affine elements) and for the 2D Euler equations at
 * N = 3 (affine elements).  For the frozen 5-species equations at N = 4 on
 * curved elements the Kennedy-Gruber, Pirozzoli and standard-DG forms are
 * built with Rusanov faces, and HLL and HLLC faces with the Ducros form (the
 * frozen sound speed in the wave-speed bounds; the species densities of an
 * HLLC star state scale like its total density).  The entropy-conservative
 * mixture flux (Tadmor's condition with the mixture entropy; beta = 1/T):
 * species rho_s^ln {{v}}.n, momentum F_rho {{v}} + p~ n with
 * p~ = {{sum rho_s R_s}}/{{beta}}, energy sum_s e^_s F_s + F_rho (|{{v}}|^2
 * - {{|v|^2}}/2) + p~ {{v}}.n, e^_s = e0_s + c_s/beta^ln + R_s theta_s
 * exp(-theta_s {{beta}}) sinhc(theta_s [[beta]]/2) / ln-mean(1 -
 * exp(-theta_s beta)) (molecules), is built for the curved 5-species
 * kernels at N = 4 with Rusanov or EC faces.  The 3D Navier-Stokes
 * equations with the entropy-conservative volume flux and Rusanov faces are
 * also built for curved elements at N = 3 and 4 and for 2:1 non-conforming
 * affine meshes at N = 3 (viscous mortars: the gradients' interface values
 * and the viscous fluxes are averaged on each sub-face and projected back to
 * the large face like the advective flux); Navier-Stokes meshes may carry
 * boundary faces of every kind.  Every other combination of equation,
 * degree, dimension and flux that the library was not built with makes
 * dgx_create (or dgx_set_mesh, for the mesh-dependent variants) return
 * DGX_E_INVAL. */
/* boundary kinds (weak, through the surface flux with an external state) */
#define DGX_BC_DIRICHLET 0
#define DGX_BC_OUTFLOW 1
#define DGX_BC_SLIPWALL 2
/* No-slip walls (Sec. Results: adiabatic and isothermal walls).  The
 * advective flux sees the interior state with the whole velocity reversed;
 * for DGX_EQ_NS the gradients take the wall value W* = (0, T_wall) or
 * (0, T) and the viscous wall flux is F_v(W*, grad W).n, without heat flux
 * at an adiabatic wall.  T_wall is bc_state[bc][0] (the rest of the row is
 * ignored).  Other boundaries of DGX_EQ_NS take W* as the mean of the
 * interior and the external state's (v, T) and the same flux rule. */
#define DGX_BC_WALL_ISOTHERMAL 3
#define DGX_BC_WALL_ADIABATIC 4
/* shock-indicator quantity */
#define DGX_IND_RHO_P 0
#define DGX_IND_P 1
/* initial guess of the T(e) Newton solve */
#define DGX_GUESS_FREESTREAM 0
#define DGX_GUESS_SURROGATE 1

/* Species data of the 5-species mixture (Appendix, Thermodynamics and
 * Chemical Kinetics).  Order N2, O2, NO, N, O.  SI units; e0 in J/kg. */
typedef struct dgx_species {
    int nspecies;          /* must be 5 */
    int molecule[5];       /* 1 = linear diatomic (rotation + vibration)   */
    double W[5];           /* molar mass, kg/mol                            */
    double theta_v[5];     /* vibrational temperature, K                    */
    double theta_r[5];     /* rotational temperature, K                     */
    double sigma[5];       /* symmetry (steric) factor                      */
    double Qe[5];          /* electronic partition function (constant)      */
    double e0[5];          /* formation energy, J/kg                        */
    double Ru, NA, hP;     /* gas constant, Avogadro, Planck                */
    double p_ref;          /* reference pressure of K_eq, Pa                */
} dgx_species;

/* Reaction table (Eq. chemreact, forward_rate): host arrays, copied.
 * A > 0 and finite b, theta_a, else dgx_create returns DGX_E_INVAL.  The
 * rates are formed in log space, k_f = exp(ln A + b ln T - theta_a/T) and
 * k_b = exp(ln k_f - ln K_c), so that k_b stays finite where k_f and K_c
 * underflow (cold gas). */
typedef struct dgx_reactions {
    int nreactions;        /* 1..32 */
    const double *A;       /* [nr] m^3 mol^-1 s^-1 (bimolecular forward)    */
    const double *b;       /* [nr] temperature exponent                     */
    const double *theta_a; /* [nr] activation temperature E/R_u, K          */
    const int32_t *nu;     /* [nr][5] reactant stoichiometry                */
    const int32_t *nup;    /* [nr][5] product stoichiometry                 */
} dgx_reactions;

typedef struct dgx_config {
    int dim;               /* 2 or 3 */
    int N;                 /* polynomial degree: 3 or 4 */
    int equation;          /* DGX_EQ_* */
    int volume_flux;       /* DGX_VF_* */
    int surface_flux;      /* DGX_SF_* */
    double gamma, R;       /* perfect gas */
    double mu, Pr;         /* DGX_EQ_NS */
    int shock;             /* 1 = modal indicator + subcell FV blending */
    double alpha_max, alpha_min;
    int ind_var;           /* DGX_IND_* */
    int alpha_smooth;      /* 1 = alpha <- max(alpha, alpha_nbr / 2) */
    double force_alpha;    /* >= 0: use this alpha everywhere (testing) */
    double newton_tol;     /* relative step tolerance of T(e) */
    int newton_maxit;
    double T_guess;        /* freestream guess of T(e); the right-hand side's
                              per-node solves start from the node's previous
                              temperature (T_guess before the first solve, and
                              again if Newton fails from it), so a mixture
                              right-hand side depends on that history at the
                              level of the Newton tolerance's rounding */
    int positivity;        /* 1 = Zhang-Shu positivity limiter after every SSPRK3 stage */
    const dgx_species *species;      /* mixture equations, else NULL */
    const dgx_reactions *reactions;  /* DGX_EQ_REACT_MIX, else NULL  */
    /* DGX_EQ_NS viscosity law (Eq. sutherland): with sutherland_S > 0,
     * mu(T) = mu (T/T0)^(3/2) (T0 + S)/(T + S) and the conductivity follows
     * at constant Pr; sutherland_S = 0 keeps mu constant.  T0 > 0 required
     * when S > 0 (else DGX_E_INVAL). */
    double sutherland_S, sutherland_T0;
} dgx_config;

/* Mesh (host arrays, copied by dgx_set_mesh).  Conforming face row
 * (eL, fL, eR, fR): the +d face of eL (fL = 2d+1) meets the -d face of eR
 * (fR = 2d) with aligned tangential node order.  Boundary row (e, f, bc).
 * Mortar row (eL, fL, eS[0..m-1], fS) with m = 2^(dim-1): the large face fL
 * of eL meets the faces fS of the small elements; sub-face s = a + 2b covers
 * the lower/upper half of each tangential direction.  One mesh may hold
 * several independent cases (batched execution): cases never share faces. */
typedef struct dgx_mesh {
    int nelem;
    const double *x;          /* [dim][nelem][(N+1)^dim] nodal coordinates   */
    int nface;
    const int32_t *faces;     /* [nface][4]   */
    int nbface;
    const int32_t *bfaces;    /* [nbface][3]  */
    int nmortar;
    const int32_t *mortars;   /* [nmortar][3 + 2^(dim-1)] */
    int nbc;
    const int32_t *bc_kind;   /* [nbc] DGX_BC_*           */
    const double *bc_state;   /* [nbc][nvar] conserved external states
                                 (isothermal walls: T_wall in column 0) */
} dgx_mesh;

typedef struct dgx_newton_stats {
    int64_t nodes;            /* nodes solved                              */
    int64_t iters_total;      /* sum of per-node iterations                */
    int32_t iters_max;        /* max per-node iterations                   */
    double iters_wave_max_mean; /* mean over wavefronts of the per-wave max */
    int64_t nonconverged;     /* nodes that did not converge               */
    int64_t first_bad;        /* first non-converged node, or -1           */
    int64_t substeps_total;   /* dgx_chem_step: sum of per-node substeps   */
    int32_t substeps_max;     /* dgx_chem_step: max per-node substeps (0 otherwise) */
    int64_t fallbacks;        /* dgx_thermo with DGX_GUESS_SURROGATE: nodes whose
                                 solve from the learned guess failed and was
                                 redone from T_guess (their iteration counts
                                 include both attempts)                    */
} dgx_newton_stats;

typedef struct dgx_ctx dgx_ctx;  /* opaque */

/* Create a context for one discretisation (Sec. Methodology; equation type
 * of Sec. Hypersonic Equations Type).  cfg and the tables it points to are
 * copied.  Returns DGX_E_INVAL for unsupported combinations
 * (dim not 2/3, N not 3/4, EC flux with a mixture, NS with a mixture). */
int dgx_create(const dgx_config *cfg, dgx_ctx **out);

/* ---- Dynamic AMR on a periodic octree (Sec. New Developments: elements
 * split into 8, 2:1 mortars; Sec. Results, AMR Taylor-Green case: an
 * indicator on a derived variable and three levels with two thresholds). */
#define DGX_AMR_LOEHNER 0            /* Loehner's weighted second-derivative estimate */
#define DGX_AMR_HENNEMANN_GASSNER 1  /* modal-energy coefficient in [0, 1]           */
#define DGX_AMR_VAR_DENSITY 0
#define DGX_AMR_VAR_PRESSURE 1
#define DGX_AMR_VAR_DENSITY_PRESSURE 2
#define DGX_AMR_VAR_VELOCITY 3       /* velocity magnitude */

typedef struct dgx_amr_controller {
    int base_level, med_level, max_level;  /* 0 <= base <= med <= max <= 12 */
    double med_threshold, max_threshold;   /* med_threshold <= max_threshold */
} dgx_amr_controller;

/* Mesh of an octree over the periodic unit cube: base^3 level-0 cells,
 * leaves[nleaf][4] = (level, i, j, k) with 0 <= i, j, k < base 2^level
 * (base <= 64, level <= 12).  The leaves must fill the cube without overlap
 * and be 2:1 balanced (face neighbours differ by at most one level), else
 * DGX_E_INVAL.  The library orders the elements along the Z-order curve of
 * the leaves' lower corners (dgx_get_octree returns that order) and builds
 * affine elements, conforming faces and mortars.  3D perfect-gas equations
 * only.  Synchronous; replaces the current mesh like dgx_set_mesh. */
int dgx_set_octree(dgx_ctx *ctx, int base, int nleaf, const int32_t *leaves);

/* The octree leaves in element order, leaves_out[nmax][4]; returns the
 * element count (leaves_out may be NULL to query it), DGX_E_STATE without an
 * octree mesh, DGX_E_INVAL when nmax is too small. */
int dgx_get_octree(const dgx_ctx *ctx, int32_t *leaves_out, int nmax);

/* Refinement indicator per element into device ind[nelem] from the device
 * state u.  DGX_AMR_LOEHNER: the variable is sampled at N+1 equidistant
 * points per direction and the element takes the largest
 * |f+ - 2 f0 + f-| / (|f+ - f0| + |f0 - f-| + 0.2 (|f+| + 2|f0| + |f-|))
 * over the interior samples of all lines.  DGX_AMR_HENNEMANN_GASSNER: the
 * blending coefficient of the shock indicator (modal energy of the highest
 * modes) with alpha_max = 1, alpha_min = 1e-4.  Enqueued on stream. */
int dgx_amr_indicator(dgx_ctx *ctx, const double *u, int kind, int variable, double *ind, void *stream);

/* One adaptation pass from host indicator values ind[nelem]: target level
 * max_level where ind >= max_threshold, med_level where ind >=
 * med_threshold, else base_level; leaves below their target are split once,
 * leaves are split further until 2:1 balanced, families of 8 unsplit
 * siblings whose targets are all below their level merge unless the parent
 * would face a leaf two levels finer.  Writes the new element count and
 * keeps the plan until dgx_amr_apply.  Host only. */
int dgx_amr_plan(dgx_ctx *ctx, const double *ind, const dgx_amr_controller *c, int *nelem_new);

/* Applies the planned adaptation: u_new (device [nvar][nelem_new][nn], not
 * aliasing u_old) receives the state of the new elements (kept elements
 * copied, split ones interpolated from their parent, merged ones the L2
 * projection of their children), then the context switches to the new
 * mesh.  Synchronises stream.  The plan is consumed by the call.  If the new
 * mesh is rejected by the checks of dgx_set_mesh the context keeps the
 * previous mesh and octree (u_new then holds the transferred state of a mesh
 * that was not set); a device failure while setting it up leaves the context
 * without a mesh (DGX_E_STATE until one is set). */
int dgx_amr_apply(dgx_ctx *ctx, const double *u_old, double *u_new, void *stream);

/* Upload a mesh: the library computes its own LGL operators, metric terms
 * (2D cross form, 3D conservative curl form), Jacobians, face normals and
 * subcell normals (Eqs. mapp, mapped_equation, jacobian).  May be called
 * again to replace the mesh.  A mesh that fails its checks (DGX_E_INVAL:
 * no elements, a face row that is not a (+d, -d) pair, an index out of
 * range, a face without neighbour or boundary, a non-positive Jacobian, a
 * combination without a kernel variant) leaves the context's previous mesh
 * in place; a failure after the checks (device allocation or copy) leaves
 * the context without a mesh (DGX_E_STATE until one is set).  Synchronous. */
int dgx_set_mesh(dgx_ctx *ctx, const dgx_mesh *mesh);

/* du = L(u, t): the DGSEM right-hand side (Eq. strong_form with the
 * flux-differencing volume term of Eq. DGvec, the FV blend of
 * Eq. fluxes_discrete_with_fv, Riemann fluxes of Eqs. riemann_problem1-3,
 * the BR1 viscous terms of Eqs. auxil/auxstrongf and species sources of
 * Eq. calc_prod).  u and du: device [nvar][nelem][nn], must not alias.
 * Enqueued on stream; t is accepted for time-dependent data (none yet). */
int dgx_rhs(dgx_ctx *ctx, const double *u, double t, double *du, void *stream);

/* nsteps steps of SSPRK3 (Shu-Osher form) at constant dt, updating u in place.
 * The three stages are captured once into a HIP graph per u pointer and
 * replayed.  Enqueued on stream. */
int dgx_ssprk3_step(dgx_ctx *ctx, double *u, double t, double dt, int nsteps, void *stream);

/* Zhang-Shu positivity-preserving scaling limiter (Sec. Results: species
 * densities and pressure kept positive weakly), applied in place to the
 * device state u: per element, each density is scaled toward its quadrature
 * mean until its minimum is admissible, then the whole state is scaled until
 * rho E - |m|^2/(2 rho) - sum rho_s e0_s (positive iff p > 0) is admissible at
 * every node.  Elements with an inadmissible mean are left unchanged (the
 * non-physical flag is then raised).  Enqueued on stream. */
int dgx_limit_positivity(dgx_ctx *ctx, double *u, void *stream);

/* Largest stable dt estimate: cfl * 2/(N+1) / max_n sum_d (|v.Ja^d| + c|Ja^d|)/J.
 * Synchronises; result written to *dt_host. */
int dgx_max_dt(dgx_ctx *ctx, const double *u, double cfl, double *dt_host, void *stream);

/* Per-node temperature from energy (Appendix Eqs. Internal_energy and
 * eos): Newton on sum rho_s e_s(T) = rho e to |dT| <= newton_tol*T, started
 * from T_guess (DGX_GUESS_FREESTREAM) or the trained surrogate
 * (DGX_GUESS_SURROGATE); a node whose solve from the surrogate's guess fails
 * (no convergence within newton_maxit, or a non-finite or non-positive
 * iterate) is solved again from T_guess, so the converged T does not depend
 * on the network (stats->fallbacks counts such nodes).  u: device [nvar][nelem][nn] of a mixture context,
 * or nstates = count of a packed [nvar][count] state set when the mesh is not
 * used (pass nstates > 0).  T, p (p may be NULL): device [count].  With
 * stats (host) the iteration counts are gathered and the call synchronises;
 * with stats == NULL it only enqueues (for timing) and non-convergence is
 * reported by dgx_check. */
int dgx_thermo(dgx_ctx *ctx, const double *u, int64_t nstates, double *T, double *p,
               int guess_mode, dgx_newton_stats *stats, void *stream);

/* Per-node stiff chemistry, split from the transport (Governing Equations,
 * Eq. source_term; rates of Appendix, Chemical Kinetics): backward Euler over
 * dt >= 0 of the species sources at fixed density, momentum and total
 * energy, in place on the species rows of u (device [nvar][nelem][nn] of the
 * mesh).  Needs a mixture context created with a reaction table
 * (DGX_EQ_EULER_MIX with cfg->reactions, or DGX_EQ_REACT_MIX).  Each step is
 * solved by Newton with the analytic Jacobian along the fixed-energy
 * manifold; every iterate's T comes from the T(e) solve warm-started at the
 * previous one (first: the incoming state's T); steps are limited so that
 * rho_s >= 0 and the thermal energy rho e - sum rho_s e0_s stays positive;
 * the iteration stops when its full Newton step is below tol * rho; it fails
 * when the limits cut the step below 1e-3 of its length on two consecutive
 * iterations (a growing mode with dt times its growth rate near or above 1)
 * or after maxit iterations.  A node whose single step fails covers dt
 * with substeps dt/2^k (k <= 20): a failed substep is retried at half the
 * size, and after a successful one the node returns to the next larger size
 * when its position in dt is a multiple of it.  A node that fails at dt/2^20
 * keeps its last accepted substep and counts as non-converged.  (Far from
 * equilibrium a Newton iteration can wander for tens of iterations, and
 * whether it lands within maxit then depends on rounding: another
 * implementation may take a different substep sequence at such a node, a
 * result that differs by the substeps' truncation error.)  The
 * library's per-node temperature is left at the new state's T.  Enqueues on
 * stream; with stats (host) it synchronises and fills the iteration and
 * substep statistics (DGX_E_NOCONV if a node failed), with stats == NULL
 * failures are reported by dgx_check.  With a DGX_EQ_EULER_MIX context, dt/2
 * chemistry, dgx_ssprk3_step over dt and dt/2 chemistry form a Strang
 * splitting. */
int dgx_chem_step(dgx_ctx *ctx, double *u, double dt, double tol, int maxit, dgx_newton_stats *stats,
                  void *stream);

/* Shock-indicator blending factor of the last dgx_rhs call (device pointer
 * to [nelem] doubles owned by the library; NULL if shock capturing is off). */
const double *dgx_last_alpha(const dgx_ctx *ctx);

/* Surrogate T-guess network 6 -> 64 -> 64 -> 64 -> 1 (tanh), BF16 operands,
 * FP32 accumulation, FP32 master weights.  Parameter vector layout (8833
 * floats): W1[64][6], b1[64], W2[64][64], b2[64], W3[64][64], b3[64],
 * W4[1][64], b4[1]; then 14 normalisation floats: mean[6], std[6],
 * T_mean, T_std.  dgx_surrogate_set copies host params (n = 8847). */
int dgx_surrogate_set(dgx_ctx *ctx, const float *params_host, size_t n);
int dgx_surrogate_get(dgx_ctx *ctx, float *params_host, size_t n);

/* Train the surrogate on device states (packed [nvar][count], count >= 256)
 * with labels T (device [count]): epochs of Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8; learning rate decaying from lr to 0 along a cosine over the
 * call's steps) over minibatches of `batch` in a seeded order.  The loss of each
 * epoch is written to loss_host[epoch] if not NULL.  Synchronises. */
int dgx_surrogate_train(dgx_ctx *ctx, const double *states, const double *T, int64_t count,
                        int epochs, int batch, float lr, uint64_t seed, float *loss_host,
                        void *stream);

/* Initialise the surrogate for a training set (packed device states
 * [nvar][count] and labels T [count]): normalisation statistics (feature and
 * temperature means and standard deviations, FP64 on the host) and
 * Glorot-uniform weights drawn from `seed`; resets the Adam state.
 * Synchronises. */
int dgx_surrogate_init(dgx_ctx *ctx, const double *states, const double *T, int64_t count, uint64_t seed,
                       void *stream);

/* Gradient of the mean squared error of the standardised temperature over
 * all `count` samples with the current parameters (no update): grad_host
 * [8833] FP32, *loss_host (may be NULL) the loss.  Synchronises. */
int dgx_surrogate_grad(dgx_ctx *ctx, const double *states, const double *T, int64_t count, float *grad_host,
                       float *loss_host, void *stream);

/* Surrogate prediction T_guess for packed states (device [nvar][count]) into
 * Tg (device [count], FP64).  Enqueued on stream. */
int dgx_surrogate_predict(dgx_ctx *ctx, const double *states, int64_t count, double *Tg,
                          void *stream);

/* Read and clear the sticky device error flags.  Synchronises. */
int dgx_check(dgx_ctx *ctx, void *stream);

/* Per-species specific energy e_s(T) and heat capacity cv_s(T) of the
 * context's mixture at one temperature (host computation, for building
 * states).  e, cv: host [5]. */
int dgx_species_energy(const dgx_ctx *ctx, double T, double *e, double *cv);

/* Mixture thermal energy and heat capacity densities (Appendix,
 * Thermodynamics, Eq. Internal_energy; Governing Equations, Eq.
 * internal_energies): rho e = sum_s rho_s e_s(T_i) and rho cv = sum_s rho_s
 * cv_s(T_i) for n states, on the host (for building mixture states; no
 * device work).  rs: host [5][n] species densities (kg/m^3, order N2, O2,
 * NO, N, O), T: host [n] temperatures (K, > 0), rhoe, rhocv: host [n] outputs
 * (either may be NULL, not both).  DGX_E_INVAL without a mixture context,
 * for n < 0 or a non-positive T (no output written then). */
int dgx_mixture_energy(const dgx_ctx *ctx, const double *rs, const double *T, int64_t n, double *rhoe,
                       double *rhocv);

/* Kernel timing for profiling: enqueue `reps` evaluations of the
 * right-hand side in the fused form of the second SSPRK3 stage
 * (out = 3/4 u0 + 1/4 (u + dt du), u0 a library copy of u in its own
 * buffer, out into library scratch; u is not modified), bracketing every
 * kernel with HIP events on `stream`, after one untimed evaluation.
 * ms_out[k] receives
 * the average duration of kernel k in launch order, names_out (may be NULL)
 * a comma-separated list of the kernel names (buffer of names_len bytes);
 * *nk the number of kernels (<= 8).  Synchronises. */
int dgx_kernel_times(dgx_ctx *ctx, const double *u, int reps, double *ms_out, int *nk,
                     char *names_out, size_t names_len, void *stream);

/* Autotuner: for each elements-per-workgroup candidate in {1, 2, 4, 8}
 * that fits (<= 512 threads, <= 64 KB LDS), each launch form
 * (round-robin over the 8 XCDs, XCD-contiguous element ranges, or the
 * work-list form of dgx_set_launch) and each LDS tiling built, time
 * `reps` SSPRK3 steps as dgx_ssprk3_step runs them (three fused stages, u0
 * in its own buffer, the positivity limiter when configured; into library
 * scratch with dt = 0, so u is read, not modified) with HIP events on
 * `stream`, and keep the fastest; the default (numbering XCD-contiguous
 * while the state takes at most 128 MB, else round-robin; default tiling) is
 * kept unless another is more than 2% faster, since the numberings can differ
 * little in time on one run and much in HBM traffic.  The winner is cached
 * process-wide under the key (dim, N, equation, fluxes, geometry kind,
 * element count) and reused by later dgx_set_mesh calls with the same key.
 * *epb_out (may be NULL) receives the elements-per-workgroup choice, ms_out
 * (may be NULL, [4]) each candidate's best average milliseconds per
 * right-hand side over the launch forms and tilings (-1 = not run).
 * Synchronises. */
int dgx_autotune(dgx_ctx *ctx, const double *u, int reps, int *epb_out, double *ms_out, void *stream);

/* Force the launch shape: elements per workgroup (1, 2, 4 or 8; must fit as
 * above) and the workgroup numbering (order: 0 round-robin over the XCDs,
 * 1 XCD-contiguous element ranges, 2 the work-list form: one launch over a
 * queue whose items are the 2:1 faces' sub-face fluxes, then the element
 * chunks, each workgroup claiming the next item from an atomic counter, the
 * chunks that read sub-face fluxes queued last and waiting until every such
 * item is done; -1 keep the current one), plus 4 for the alternative LDS
 * tiling where one is built (the pair and face work items in another number
 * of chunks: the 3D Navier-Stokes kernel at N = 3 in two, the curved
 * 5-species kernels at N = 4 in one; DGX_E_INVAL elsewhere).  The results do
 * not depend on the elements per workgroup or the launch form (bitwise); the
 * other tiling sums each node's pair fluxes in another order (rounding). */
int dgx_set_launch(dgx_ctx *ctx, int epb, int order);

/* The current launch shape, as dgx_set_launch takes it: *epb (elements per
 * workgroup) and *order (0 round-robin over the XCDs, 1 XCD-contiguous, 2 the
 * work-list form; plus 4 with the alternative LDS tiling);
 * either pointer may be NULL.  DGX_E_STATE without a mesh. */
int dgx_get_launch(dgx_ctx *ctx, int *epb, int *order);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture when called without stats, tight serving loops, harnesses that
 * forbid hipMalloc): dgx_thermo with the same arguments, results and errors,
 * whose scratch (the surrogate's guesses, the per-node iteration counts and
 * the statistics accumulators) lives in a static device buffer of the library
 * instead of memory allocated on first use.  The call allocates nothing (no
 * hipMalloc or hipFree, no host allocation): the caller passes u, T and p.
 * Limit: at most DGX_NOALLOC_MAX_STATES states (the mesh's nodes when
 * nstates <= 0); more is DGX_E_INVAL before any launch.  The buffer (about
 * 12.6 MB) is set up on a GPU at the first call there and held until the
 * process ends; all calls on one GPU share it, so calls that overlap on one
 * GPU (other streams, other threads, other contexts) race and must be
 * ordered by the caller.  With stats it synchronises, as dgx_thermo does. */
#define DGX_NOALLOC_MAX_STATES 1048576
int dgx_thermo_noalloc(dgx_ctx *ctx, const double *u, int64_t nstates, double *T, double *p,
                       int guess_mode, dgx_newton_stats *stats, void *stream);

/* Text of the last error on this context (never NULL). */
const char *dgx_last_error(const dgx_ctx *ctx);

/* Release every resource of the context.  NULL is ignored. */
void dgx_destroy(dgx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* DGX_H */

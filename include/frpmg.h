/*
 * frpmg.h -- C ABI of the MI355X (gfx950) implementation of the nonlinear
 * p-multigrid preconditioned Jacobian-free Newton-Krylov stage solve for the
 * flux-reconstruction (FR) discretisation of the compressible Navier-Stokes
 * equations.
 *
 * Paper: L. Wang, W. Trojak, F. Witherden, A. Jameson, "Nonlinear p-multigrid
 * preconditioner for implicit time integration of compressible Navier-Stokes
 * equations", arXiv 2202.09733.  Section numbers below refer to it.
 *
 * Conventions (all entry points):
 *  - Array arguments are DEVICE pointers owned by the caller, contiguous,
 *    FP64, unless stated otherwise.  The library owns only its internal
 *    workspaces (EJ factors, Krylov basis, multigrid buffers), allocated at
 *    fr_create, at the first ej_factor of a level, at the first mbnk_factor
 *    of a level, or at the first gmres_solve_stage; no other call allocates.
 *  - State arrays hold the DEVIATION dq = q - q_inf of the conservative
 *    variables (rho, rho u, rho v, [rho w], E) from the reference state q_inf
 *    given at creation, in the layout [nvar][npts][nelem]: element index
 *    fastest, element e = ix + nx (iy + ny iz), local point
 *    i = a + P (b + P c) with P = p + 1 Gauss-Legendre points per direction.
 *    R(0) = 0 exactly.  Carrying the deviation keeps FP64 meaningful at low
 *    Mach number, where E ~ p_inf/(gamma-1) would otherwise swamp the
 *    perturbations.
 *  - An element-Jacobi block of element k uses the local DOF index
 *    j = v Np + i (Np = P^dim).
 *  - Calls are asynchronous on the given stream (a hipStream_t, NULL = the
 *    default stream), except gmres_solve_stage, which synchronises.
 *  - Every call returns an fr_status; fr_last_error() describes the last
 *    failure of a context.  A context is used by one host thread at a time.
 *  - Periodic axis-aligned meshes only; element widths may vary per axis
 *    index (stretched meshes).
 */
#ifndef FRPMG_H
#define FRPMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int fr_status;
#define FR_OK 0
#define FR_EINVAL (-1)      /* invalid argument */
#define FR_ENOMEM (-2)      /* device allocation failed */
#define FR_EDEVICE (-3)     /* HIP runtime error */
#define FR_ESINGULAR (-4)   /* exact zero pivot in an EJ block */
#define FR_ENOCONV (-5)     /* iteration cap reached before the tolerance */
#define FR_EBREAKDOWN (-6)  /* Arnoldi breakdown without convergence */
#define FR_ENONFINITE (-7)  /* NaN or Inf in a norm */

typedef struct frpmg_ctx frpmg_ctx;
typedef void *fr_stream; /* hipStream_t */

#define FR_MAX_LEVELS 4

/* Mesh, polynomial levels and physics.  h[a] points to n[a] HOST doubles
 * (element widths along axis a); the library copies them.  p[0] is the
 * finest degree; levels 1.. are the coarser p-multigrid levels
 * (Sec. 3.1, hierarchy p{p0-p1}).  Constant viscosity mu, Prandtl number Pr,
 * LDG penalty tau; qinf = reference conservative state (dim + 2 values). */
typedef struct {
    int dim;              /* 2 or 3 */
    int n[3];             /* elements per axis (n[2] ignored for dim = 2) */
    const double *h[3];   /* host arrays of element widths */
    int nlevels;          /* 1 .. FR_MAX_LEVELS */
    int p[FR_MAX_LEVELS]; /* polynomial degree per level, 0 <= p <= 4, dim 3: p <= 3 (p = 0: one point
                             per element, the cell-centred finite-volume scheme) */
    double gamma, mu, Pr, tau;
    double qinf[5];
} fr_mesh_desc;

/* Create a context on the current HIP device.  Builds the 1D operators
 * (Gauss-Legendre points, differentiation, DG-recovering correction
 * derivatives, L2-projection transfers) and the residual workspaces. */
fr_status fr_create(const fr_mesh_desc *desc, frpmg_ctx **out);
void fr_destroy(frpmg_ctx *ctx);
const char *fr_last_error(const frpmg_ctx *ctx);

/* Number of doubles in a state vector of a level: (dim+2) (p+1)^dim nelem. */
size_t fr_level_size(const frpmg_ctx *ctx, int level);

/* r = R_level(dq): FR right-hand side of dq/dt = -div f (Sec. 2.1, Eq. (1)):
 * Gauss-Legendre solution points, Huynh's DG-recovering corrections, flux-
 * polynomial traces, original Roe flux without entropy fix (Sec. 4.2.1),
 * LDG viscous flux.  dq and r: fr_level_size(level) doubles, must not alias. */
fr_status fr_residual(frpmg_ctx *ctx, int level, const double *dq, double *r, fr_stream stream);

/* fr_residual for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and bitwise the same r, with the face data that the face
 * kernel hands to the volume kernel (common fluxes and state jumps on every
 * element's + faces, 2 dim (dim + 2) (p + 1)^(dim - 1) Ne doubles) kept in a
 * fixed 64 MiB device array that the library holds on each device until the
 * process ends, instead of the context's buffers.  Allocates nothing.  A
 * level whose face data exceed 64 MiB (3D p = 3: more than ~17,000
 * elements) returns FR_EINVAL.  Every call on a device shares that device's
 * array, whose contents the next call overwrites: calls that overlap on one
 * device (other streams, host threads or contexts) race, and the caller
 * must serialise them.  Asynchronous on the stream. */
fr_status fr_residual_noalloc(frpmg_ctx *ctx, int level, const double *dq, double *r, fr_stream stream);

#define FR_EPS_ABSOLUTE 0   /* h = eps */
#define FR_EPS_NORMALIZED 1 /* h = eps / ||v||_2 (perturbation of norm eps) */
#define FR_EPS_SCALED 2     /* h = eps (1 + ||dq||_2) / ||v||_2 (Knoll-Keyes scaling) */
#define FR_FD_CENTRAL 4     /* ORed into an FR_EPS_* mode: central instead of one-sided difference */

/* Finite-difference shifted Jacobian-vector product (Sec. 2.2, the matrix-
 * free product with fixed eps = 1e-6):
 *   w = shift v - (R(dq + h v) - rq) / h,
 * rq = R(dq) supplied by the caller.  With FR_FD_CENTRAL ORed into eps_mode
 * (not in the paper, which takes the one-sided difference):
 *   w = shift v - (R(dq + h v) - R(dq - h v)) / (2 h)
 * (rq unused; two residual evaluations), whose truncation error is O(h^2)
 * instead of O(h), so that the FD operator is linear in v to rounding and a
 * Krylov solve's estimate and its recomputed residual agree.  All arrays of
 * the level's size; w must not alias the inputs. */
fr_status fr_jvp(frpmg_ctx *ctx, int level, const double *dq, const double *rq, const double *v,
                 double shift, double eps, int eps_mode, double *w, fr_stream stream);

#define FR_PREC_FP64 0      /* FP64 factor, FP64 storage */
#define FR_PREC_FP32 1      /* FP64 elimination, inverse stored in FP32 */
#define FR_PREC_FP32_BF16 2 /* blocked Gauss-Jordan: FP64 panels, panel updates on BF16-input MFMA (hi/lo
                                split, FP32 accumulate), inverse stored in FP32 */
#define FR_PREC_BF16_STORE 3 /* as FR_PREC_FP32_BF16, inverse stored in BF16 (applied with FP64 accumulation) */

/* Element-Jacobi setup (Sec. 2.2, element-Jacobi preconditioner; the
 * preconditioner matrix is evaluated once per physical time step):
 * forms B_k = sigma I - dR_k/dq_k at dq_lin for every element by one-sided
 * finite differences per block column with element k alone perturbed (step
 * 1e-7 max(1, |q_j|), taken as the representable difference), then inverts
 * every block by Gauss-Jordan elimination with partial pivoting and stores
 * the inverse in the requested precision.  Needs at least two elements per
 * axis (FR_EINVAL otherwise).
 * Returns FR_ESINGULAR if a block has an exact zero pivot, FR_ENONFINITE if a
 * pivot is NaN or infinite (a non-finite state or block).  Synchronises the
 * stream at the end (to report the pivot status). */
fr_status ej_factor(frpmg_ctx *ctx, int level, const double *dq_lin, double sigma, int precision,
                    fr_stream stream);

/* y = blockdiag(B)^{-1} r with the factors of the last ej_factor of the
 * level (FP64 in and out; internal casting per the factor precision). */
fr_status ej_solve(frpmg_ctx *ctx, int level, const double *r, double *y, fr_stream stream);

/* Copy the stored inverse blocks of a level to a host buffer of
 * nelem nb nb doubles, block k column-major (entry (row, col) at
 * k nb nb + col nb + row), converted to FP64.  Synchronous. */
fr_status ej_get_inverse(frpmg_ctx *ctx, int level, double *host_out);

/* ------------------------------------------------------------------------
 * Matrix-based Newton-Krylov (MBNK) smoother (Sec. 3.2): one sweep solves
 * the linearised pseudo-time step A delta = G, A = sigma I - dR/dq, by GMRES
 * (at most 5 iterations, relative tolerance 1e-1 by default) right-
 * preconditioned by ILU0, and sets Y <- Y - delta.  The library's reading:
 *  - A keeps, for every element k, the diagonal block and the 2 dim blocks
 *    that couple k to its face neighbours (R_k also depends on edge-diagonal
 *    neighbours through the LDG gradient; those blocks are dropped).  Each
 *    block column is a one-sided difference with the EJ step, elements of one
 *    colour (at least three apart along an axis) perturbed together.
 *  - ILU0 is taken in red-black element order (colour = parity of the
 *    element's coordinate sum).  With face couplings only this keeps D_r on
 *    red elements and U_b = D_b - sum_r O_br D_r^{-1} O_rb on black ones.
 * One factorisation per context, for one level.
 *
 * mbnk_factor: assemble A at dq_lin (that level's state) and factor it.
 *   Needs an even element count >= 4 per axis and blocks of at most 136
 *   unknowns, i.e. every 2D level and the 3D levels up to p = 2 (135)
 *   (FR_EINVAL otherwise).  Allocates its workspace at the first
 *   call for a level (the blocks take (3 + 2 dim) Ne nb^2 doubles, the
 *   formation batch up to 128 MiB per buffer).  Synchronises the stream;
 *   FR_ESINGULAR on a zero pivot, FR_ENONFINITE on a NaN or infinite one.
 * mbnk_matvec: y = A x.  mbnk_ilu_solve: z = (L U)^{-1} r.
 * mbnk_solve: delta ~ A^{-1} g by one GMRES(maxit <= 8) cycle from zero to
 *   relative tolerance tol (convergence decided on the device, no host
 *   synchronisation).  g may alias delta.
 * Vectors are that level's size; matvec and ilu_solve outputs must not alias
 * their inputs.
 * mbnk_get_blocks: copy the assembled blocks to host buffers (either may be
 *   null): D = [Ne][nb][nb], O = [Ne][2 dim][nb][nb], blocks column-major,
 *   O's slot of the face neighbour across axis a on side s = -1 / +1 being
 *   2 a + (s > 0).  Synchronous. */
fr_status mbnk_factor(frpmg_ctx *ctx, int level, const double *dq_lin, double sigma, fr_stream stream);
fr_status mbnk_matvec(frpmg_ctx *ctx, const double *x, double *y, fr_stream stream);
fr_status mbnk_ilu_solve(frpmg_ctx *ctx, const double *r, double *z, fr_stream stream);
fr_status mbnk_solve(frpmg_ctx *ctx, const double *g, double *delta, double tol, int maxit, fr_stream stream);
fr_status mbnk_get_blocks(frpmg_ctx *ctx, double *host_D, double *host_O);

/* Restriction Gamma (L2 projection, Sec. 3.1 Eq. (projection)) from level
 * `from` to the coarser level `to` = from + 1, and prolongation Pi
 * (Eq. (prolongation)) from level `from` to the finer level `to` = from - 1,
 * per element and variable as tensor products of the 1D operators. */
fr_status pmg_restrict(frpmg_ctx *ctx, int from, int to, const double *x, double *y, fr_stream stream);
fr_status pmg_prolong(frpmg_ctx *ctx, int from, int to, const double *x, double *y, fr_stream stream);

#define FR_COARSE_NONE 0    /* fine-level smoothing only (n0 pre-sweeps) */
#define FR_COARSE_EJ 1      /* two-level V-cycle with EJ smoothing on level 1 */
#define FR_COARSE_LEARNED 2 /* coarse sweeps replaced by the learned correction */
#define FR_COARSE_MBNK 3    /* as FR_COARSE_EJ, with MBNK sweeps on the coarsest level of the cycle (the
                               level of the last mbnk_factor) */

#define FR_SCALE_LITERAL 0    /* s = 1 */
#define FR_SCALE_NORMALIZED 1 /* s = eps_p sigma_D / ||X||_2 */
#define FR_SCALE_SCALED 2     /* s = eps_p sigma_D (1 + ||dq||_2) / ||X||_2, dq = the set point */

/* Nonlinear pMG preconditioner parameters (Sec. 3.2).  The V-cycle runs
 * over levels 0 .. L-1 of the context (L = levels, 0: all of them); every
 * level but the coarsest takes n_l pre- and n_l post-sweeps around the
 * correction from the level below (the two-level step of Sec. 3.1 applied
 * recursively), the coarsest n_{L-1} sweeps: n{n0-n1} for two levels,
 * n{n0-n1-n2} for three. */
typedef struct {
    double sigma_D;   /* 1/dtau + 1/(a_ii dt) (ESDIRK) or 1/(a_ii dt) (ROW) */
    int n0, n1;       /* smoothing n{n0-n1} (Sec. 3.1) */
    int coarse_mode;  /* FR_COARSE_* */
    int scale_mode;   /* FR_SCALE_* */
    double eps_p;     /* scale for FR_SCALE_NORMALIZED */
    int n2, n3;       /* sweeps on levels 2 and 3 (hierarchies of three and four levels) */
    int levels;       /* levels the cycle uses (0: every level of the context; learned: 2) */
    int mbnk_maxit;   /* FR_COARSE_MBNK: GMRES iterations per sweep, 1..8 (0: 5, Sec. 3.2) */
    double mbnk_tol;  /* FR_COARSE_MBNK: relative GMRES tolerance per sweep (0: 1e-1, Sec. 3.2) */
} pmg_params;

/* Set the linearisation point of the preconditioner: dq (level 0 state) and
 * rq = R_0(dq).  Restricts dq to every coarser level and evaluates R_l
 * there.  The pointers must stay valid until the next pmg_set_point. */
fr_status pmg_set_point(frpmg_ctx *ctx, const double *dq, const double *rq, fr_stream stream);

/* y ~ A^{-1} x by one two-level FAS V-cycle on
 *   0 = X + R(q + Y) - R(q) - sigma_D Y       (Sec. 3.2, with q_hat = q + Y)
 * smoothed by the element-Jacobi linearised pseudo-time step
 * Y <- Y - B^{-1} G(Y), G(Y) = sigma_D Y - [R(q+Y) - R(q)] - X, with the
 * factors of ej_factor on each level (their sigma is sigma_S = 1/dtau* +
 * sigma_D).  x and y are level-0 vectors and must not alias. */
fr_status pmg_precond_apply(frpmg_ctx *ctx, const pmg_params *prm, const double *x, double *y,
                            fr_stream stream);

#define FR_SCHEME_ESDIRK 0
#define FR_SCHEME_ROW 1
#define FR_PRECOND_EJ 0
#define FR_PRECOND_PMG 1
#define FR_PRECOND_PMG_LEARNED 2

typedef struct {
    int scheme;        /* FR_SCHEME_* */
    double a_ii;       /* diagonal coefficient of the stage */
    double a_i1;       /* ESDIRK: coefficient of R(q^n) in the stage (explicit first stage) */
    double dt;         /* physical time step */
    double dtau;       /* pseudo-time step of the outer PTC (ESDIRK); also dtau* of the smoother */
    int m;             /* Krylov dimension K_dim, 1 .. 120 */
    int max_restarts;  /* FGMRES restarts per linear solve */
    double eta;        /* ESDIRK: relative tolerance of each inexact Newton solve */
    double tol;        /* stage tolerance: ||F|| <= tol ||F(q^n)|| (ESDIRK), Krylov tol (ROW) */
    int max_ptc;       /* cap on pseudo-time iterations (ESDIRK) */
    int precond;       /* FR_PRECOND_* */
    int precision;     /* FR_PREC_* of the EJ factors */
    int n0, n1;        /* pMG smoothing */
    double eps;        /* FD step of the JVP */
    int eps_mode;      /* FR_EPS_*, optionally ORed with FR_FD_CENTRAL */
    int scale_mode;    /* FR_SCALE_* of the preconditioner */
    double eps_p;      /* preconditioner scale */
    int skip_setup;    /* 1: reuse the EJ factors already in the context */
    int stall_window;  /* FR_PRECOND_PMG_LEARNED: fall back to plain pMG when the FGMRES residual */
    double stall_ratio; /*   estimate exceeds stall_ratio x its value stall_window iterations earlier
                             (0: defaults 5 and 0.7); the fallback holds for the rest of the stage */
    int graphs;        /* 1: each Arnoldi step (preconditioner, JVP, orthogonalisation, normalisation) is
                          captured once as a HIP graph, cached in the context and replayed on the stream;
                          0: every kernel is launched from the host.  Both give bitwise identical results
                          (measured: no faster on MI355X).  Graphs are not used with the learned
                          preconditioner or while harvesting. */
    int n2, n3;        /* pMG sweeps on levels 2 and 3 (see pmg_params) */
    int pmg_levels;    /* levels of the pMG cycle (0: every level of the context) */
    int solver;        /* FR_SOLVER_JFNK, or FR_SOLVER_PMG: ESDIRK stages solved by pMG V-cycles alone */
    int coarse_smoother; /* FR_SMOOTHER_EJ, or FR_SMOOTHER_MBNK on the coarsest level of the pMG cycle
                            (its operator assembled by mbnk_factor at the restricted q^n) */
    int mbnk_maxit;    /* MBNK GMRES iterations per sweep (0: 5) */
    double mbnk_tol;   /* MBNK relative GMRES tolerance per sweep (0: 1e-1) */
    int smoother_refresh; /* FR_SOLVER_PMG: re-form the smoothers at the current iterate every this many
                             V-cycles (0: formed once at q^n; Sec. 4.2.2 uses 20) */
    int verify;        /* ROW: 1 = the stage is solved when ||rhs - A_h Y||, recomputed at Y with the FD
                          operator, meets tol: when the Krylov estimate meets tol, FGMRES continues from the
                          recomputed residual if it misses, as long as each further cycle at least halves
                          it; when one does not (the operator's floor: FD truncation and rounding), the
                          stage ends there, converged on its estimate, with true_rel_res above tol.
                          0 = the Krylov estimate decides.  The FD operator is linear only to its truncation
                          and rounding error, so the two can differ (~1e-7 relative at eps = 1e-6 on the 3D
                          Taylor-Green stage) */
} stage_params;

#define FR_SMOOTHER_EJ 0
#define FR_SMOOTHER_MBNK 1

/* FR_SOLVER_PMG (Sec. 3.1, pMG as the nonlinear solver; the baseline of
 * Tabs. 2 and 4): each iteration applies one FAS V-cycle to X = -F(q) with
 * sigma_D = 1/(a_ii dt) and literal scaling, so that the cycle's level-0
 * equation is F(q + Y) = 0, and sets q <- q + Y; the smoothers take the
 * pseudo-time step, blocks with sigma_S = 1/dtau + 1/(a_ii dt) formed at
 * q^n.  Stops when ||F|| <= tol ||F(q^n)|| or after max_ptc cycles
 * (ptc_iters counts the cycles, gmres_iters is 0). */
#define FR_SOLVER_JFNK 0
#define FR_SOLVER_PMG 1

#define FR_MAX_NEWTON_LOG 128
typedef struct {
    int ptc_iters;
    int gmres_iters;
    int restarts;
    int converged;
    int status;
    double res0, res, rel_res;       /* ||F(q^n)||, final ||F||, ratio (ESDIRK); ROW: Krylov estimate */
    double true_rel_res;             /* ROW: ||R - A_h Y|| / ||R|| recomputed at the end */
    double t_total, t_setup, t_solve; /* seconds, host wall clock around synchronised phases */
    long n_R_fine, n_R_coarse, n_ej_fine, n_ej_coarse;
    int fallbacks;
    int gmres_per_newton[FR_MAX_NEWTON_LOG];
    double t_precond, t_jvp, t_ortho; /* seconds of the Arnoldi steps' preconditioner, FD product and
                                         orthogonalisation (HIP events on the stream, summed over the
                                         stage; 0 when the steps replay captured graphs) */
} stage_stats;

/* One implicit stage (synchronous).
 * ESDIRK (Sec. 2.1 Eq. (ESDIRK2), second stage, explicit first stage):
 *   q_i = q^n + dt (a_i1 R(q^n) + a_ii R(q_i)), solved by pseudo-transient
 *   continuation with inexact Newton (Sec. 2.2): each step solves
 *   (I/dtau + I/(a_ii dt) - dR/dq) dq = -F by FGMRES(m) to relative
 *   tolerance eta, until ||F|| <= tol ||F(q^n)||.  out = q_i (deviation).
 * ROW (Sec. 2.1 Eq. (Rosenbrock_General), first stage):
 *   (I/(a_ii dt) - dR/dq(q^n)) Y = R(q^n) by FGMRES(m) to tol.  out = Y.
 * The EJ factors are formed at q^n (skip_setup = 0).  Returns FR_ENOCONV
 * when the caps are reached, FR_ENONFINITE on a NaN/Inf norm. */
fr_status gmres_solve_stage(frpmg_ctx *ctx, const stage_params *prm, const double *dq_n, double *out,
                            stage_stats *stats, fr_stream stream);

/* ------------------------------------------------------------------------
 * Full implicit time steps (synchronous): every stage of one step of
 * dq/dt = R(q) (Sec. 2.1), the EJ factors formed once at q^n and reused by
 * every stage (Sec. 2.2).  The paper names its schemes (ESDIRK2/ESDIRK4,
 * ROW2/ROW4) without printing their tableaux.  The ones here come in pairs of
 * one order that share the diagonal gamma, hence one shift 1/(gamma dt) and
 * one preconditioner per pair; all are L-stable:
 *   order 2, gamma = 1 - 1/sqrt(2):
 *     FR_TAB_ESDIRK2: 3 stages, c = (0, 2 gamma, 1) (ESDIRK2(1)3L[2]SA);
 *     FR_TAB_ROW2: 2 stages, alpha_21 = 1, b = (1/2, 1/2).
 *   order 3, gamma = 0.43586652150845899942:
 *     FR_TAB_ESDIRK3: 4 stages, c = (0, 2 gamma, 3/5, 1)
 *       (ESDIRK3(2)4L[2]SA);
 *     FR_TAB_ROW3: 3 stages, alpha_21 = alpha_31 = 1, alpha_32 = 0,
 *       b = (2/3, 1/6, 1/6), beta_31 = beta_21.
 *   order 4:
 *     FR_TAB_ESDIRK4: 6 stages, gamma = 1/4, the implicit tableau of
 *       ARK4(3)6L[2]SA (the ESDIRK4 of Bijl et al.);
 *     FR_TAB_ROW4: 4 stages, gamma = 0.57281606248213485, Shampine's alpha
 *       and b, gamma_31 = 0, the other beta_ij from the order-4 conditions.
 * ESDIRK schemes have an explicit first stage and are stiffly accurate
 * (Eq. (ESDIRK2) generalised to every stage): stage i solves
 *   q_i = q^n + dt (sum_{j<i} a_ij R(q_j) + gamma R(q_i))
 * as gmres_solve_stage does, from q_{i-1}, to ||F_i|| <= tol ||F_i(q_{i-1})||;
 * q^{n+1} = q_s.  ROW schemes use the transformed form of
 * Eq. (Rosenbrock_General):
 *   (I/(gamma dt) - dR/dq(q^n)) Y_i = R(q^n + sum_j a_ij Y_j)
 *                                    + (1/dt) sum_j c_ij Y_j,
 * each by FGMRES to tol relative to its right-hand side; stages whose states
 * coincide share one R evaluation.  q^{n+1} = q^n + sum_i m_i Y_i.
 * prm->stage carries dt and the solver and preconditioner settings; its
 * scheme, a_ii, a_i1 and skip_setup are ignored.  dq_n and dq_np1 are
 * level-0 device vectors and must not alias.  Returns FR_ENOCONV or
 * FR_ENONFINITE if a stage fails (stats then hold the stages so far). */
#define FR_TAB_ESDIRK3 0
#define FR_TAB_ROW3 1
#define FR_TAB_ESDIRK2 2
#define FR_TAB_ROW2 3
#define FR_TAB_ESDIRK4 4
#define FR_TAB_ROW4 5
#define FR_MAX_STEP_STAGES 5 /* implicit stages: ESDIRK4 has five */

typedef struct {
    int tableau;         /* FR_TAB_* */
    stage_params stage;  /* dt, solver and preconditioner settings */
} step_params;

typedef struct {
    int nstages;         /* implicit stages solved */
    int gmres_iters;     /* over every stage */
    int ptc_iters;       /* ESDIRK: pseudo-time steps over every stage */
    int fallbacks;
    int status;
    double t_total, t_setup, t_solve;  /* seconds, host wall clock */
    long n_R_fine, n_R_coarse, n_ej_fine, n_ej_coarse;
    stage_stats stage[FR_MAX_STEP_STAGES];
} step_stats;

fr_status fr_time_step(frpmg_ctx *ctx, const step_params *prm, const double *dq_n, double *dq_np1,
                       step_stats *stats, fr_stream stream);

/* The coefficients fr_time_step uses for a tableau (host only: no context,
 * no device).  ESDIRK: rosenbrock = 0, stages = s (the first explicit),
 * A row-major s x s in A[6][6] (b = last row, stiffly accurate).  ROW:
 * rosenbrock = 1, stages = s, the transformed a, c (strictly lower) in
 * a[4][4], c[4][4] and m in m[4].  Unused entries are zero.  Returns
 * FR_EINVAL for an unknown tableau or a null pointer. */
typedef struct {
    int rosenbrock;
    int stages;
    double gamma;
    double A[6][6];
    double a[4][4], c[4][4], m[4];
} fr_tableau;

fr_status fr_step_tableau(int tableau, fr_tableau *out);

/* ------------------------------------------------------------------------
 * Learned coarse correction (not in the paper): an element-local, bias-free
 * ReLU network in -> 256 -> 256 -> out refines the element-local coarse EJ
 * step.  With C1 = B1^{-1} Gamma d (one coarse EJ application to the
 * restricted defect), the input row of an element is C1 on the element and
 * on its 2 dim face neighbours (standardised per variable,
 * divided by the row norm s) followed by dim geometry entries
 * ln(h_a / max h_a); the coarse correction is
 *   C = C1 + tau s (N(x, g) - N(-x, g)) / 2,
 * exactly positive-homogeneous and odd in the defect.  It replaces the coarse
 * smoothing sweeps of the V-cycle (FR_COARSE_LEARNED); the training target is
 * what target_sweeps coarse EJ sweeps add to C1.  Products run on BF16 MFMA
 * with FP32 accumulation; FP32 master weights, Adam.
 * Feature row layout: [own (nv Np1, index v Np1 + i) | for each axis a:
 * the -a neighbour's values, then the +a neighbour's values (nv Np1 each,
 * index v Np1 + i) | geometry (dim)], zero padded to nin_pad.
 * Weight layout (FP32, row-major): W1 [256 x nin_pad] | W2 [256 x 256] |
 * W3 [nout_pad x 256].
 * ------------------------------------------------------------------------ */

typedef struct {
    int enable;         /* 1: record pairs in every FR_COARSE_EJ V-cycle; 0: stop */
    int max_pairs;      /* harvest buffer rows (allocated at the first enable) */
    int stride;         /* record every stride-th element of a V-cycle; the offset rotates per cycle */
    int target_sweeps;  /* coarse EJ sweeps that define the target correction (>= n1) */
    int reset;          /* 1: discard pairs harvested so far (and the input/output scales) */
} lcc_harvest_params;

/* Turn harvesting on or off.  Pairs: (features of C1, Ct - C1) with Ct the
 * coarse correction after target_sweeps EJ sweeps on the coarse FAS equation
 * (the V-cycle itself keeps using n1 sweeps).  The first harvested V-cycle
 * fixes the per-variable input and output scales (RMS over the mesh). */
fr_status lcc_harvest(frpmg_ctx *ctx, const lcc_harvest_params *prm);
int lcc_harvest_count(const frpmg_ctx *ctx);

typedef struct {
    int epochs;
    int batch;        /* multiple of 32 */
    double lr;        /* Adam step size */
    uint64_t seed;    /* shuffling (and re-initialisation) */
    double holdout;   /* fraction of the harvested rows kept out of training (the last ones) */
    int reinit;       /* 1: re-initialise the weights from seed before training */
} lcc_train_params;

typedef struct {
    int steps;
    double loss_first, loss_last, val_loss, val_loss_init, t_train;
} lcc_train_stats;

/* Train on the harvested pairs (loss 0.5 ||N(x) - t||^2 averaged over the
 * batch), synchronous. */
fr_status lcc_train(frpmg_ctx *ctx, const lcc_train_params *prm, lcc_train_stats *st, fr_stream stream);

/* Dimensions (allocates the network on first use). */
fr_status lcc_dims(frpmg_ctx *ctx, int *nin, int *nin_pad, int *nh, int *nout, int *nout_pad);
size_t lcc_num_weights(frpmg_ctx *ctx);
/* Host copies of the FP32 master weights (n = lcc_num_weights); setting them
 * also refreshes the BF16 copies and resets the Adam moments. */
fr_status lcc_get_weights(frpmg_ctx *ctx, float *host, size_t n);
fr_status lcc_set_weights(frpmg_ctx *ctx, const float *host, size_t n);
/* Per-variable input and output scales (dim + 2 floats each, host). */
fr_status lcc_get_scales(frpmg_ctx *ctx, float *in_scale, float *out_scale);
fr_status lcc_set_scales(frpmg_ctx *ctx, const float *in_scale, const float *out_scale);

/* Test hooks (device pointers).  Y = N(X) for rows (multiple of 32) of
 * normalised inputs X [rows x nin_pad] -> Y [rows x nout_pad]; loss and
 * gradient (layout as the weights) of a batch (X, T [rows x nout_pad]); the
 * feature rows [Ne x nin_pad] and norms s [Ne] of a level-1 field d1 (the
 * field itself stands in for C1). */
fr_status lcc_forward(frpmg_ctx *ctx, const float *X, int rows, float *Y, fr_stream stream);
fr_status lcc_loss_grad(frpmg_ctx *ctx, const float *X, const float *T, int rows, double *loss, float *grad,
                        fr_stream stream);
fr_status lcc_features_of(frpmg_ctx *ctx, const double *d1, float *rows_out, float *s_out, fr_stream stream);
/* One Adam step (Kingma and Ba: beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-
 * corrected moments) of the FP32 master weights with the device gradient
 * grad (FP32, layout as the weights) and step size lr; refreshes the BF16
 * copies.  The moments and the step count continue from the last training
 * step (lcc_set_weights resets them).  Asynchronous. */
fr_status lcc_adam_step(frpmg_ctx *ctx, const float *grad, double lr, fr_stream stream);

/* ------------------------------------------------------------------------
 * p-adaptive FR (Sec. 3.3, "Coupling with p-adaptation")
 *
 * A context becomes p-adaptive when fr_set_degrees gives every element of
 * the finest level its own degree.  Every level then keeps the state layout
 * of its largest degree p (the context's p[l]), padded: element k of degree
 * d_k uses local points i < (d_k + 1)^dim numbered i = a + P_k (b + P_k c),
 * P_k = d_k + 1; the remaining entries of an input are ignored where stated
 * and every output writes them as 0 (state vectors of a solve stay 0 there).
 * EJ blocks keep n_b = nvar (p + 1)^dim with the identity on unused points.
 * fr_residual, fr_jvp, ej_factor/ej_solve, pmg_restrict/pmg_prolong,
 * pmg_precond_apply (EJ smoothing on every level), gmres_solve_stage and
 * fr_time_step then act on the mixed-degree discretisation; the MBNK
 * smoother, the learned correction and fr_residual_noalloc are refused
 * (FR_EINVAL).
 *
 * Face coupling (the paper defers it to its p-adaptation reference; this is
 * the library's reading): the common solution at a face is the +axis
 * element's trace, seen by the -axis element through the L2 projection onto
 * its own face polynomials; the common flux is formed at the Gauss-Legendre
 * points of the larger of the two degrees from both traces and the -axis
 * element's gradient trace carried there by L2 projection, and returned to
 * both sides by L2 projection (so the scheme stays conservative).  Faces of
 * equal degree are unchanged, so a uniform degree map gives the uniform
 * operator.
 * ------------------------------------------------------------------------ */

/* Nested p-hierarchy (Sec. 3.3): out[l * ne + k] = the degree of element k on
 * p-sublevel l (l < nlevels, order gap 1 or 2), from its finest degree deg[k]:
 * each sublevel lowers the finest degree by the gap but keeps at least as many
 * degrees as sublevels remain below it, stays below the sublevel above and
 * stops at 0 -- for P4 with three sublevels this gives p{4-2-0}, p{3-1-0},
 * p{2-1-0}, p{1-0-0} (gap 2) and p{4-3-2}, p{3-2-1}, p{2-1-0}, p{1-0-0}
 * (gap 1), the paper's listed hierarchies.  Host arrays; no context. */
fr_status fr_pa_hierarchy(const int *deg, int ne, int nlevels, int gap, int *out);

/* Give the finest level the per-element degrees host_deg[Ne] (HOST array,
 * 0 <= deg <= p[0]) and every coarser level its nested degrees (fr_pa_hierarchy
 * with the given gap); the largest degree on each level must equal the
 * context's p[l] (FR_EINVAL otherwise).  host_deg = NULL returns to uniform
 * degrees.  Synchronises the device, drops the EJ factors of every level and
 * allocates the level's face and formation buffers.  EJ blocks of a
 * mixed-degree level are formed by coloured one-sided differences of the
 * full residual (even element counts per axis). */
fr_status fr_set_degrees(frpmg_ctx *ctx, const int *host_deg, int gap);

/* Degrees of the elements of a level (HOST array of Ne ints). */
fr_status fr_get_degrees(frpmg_ctx *ctx, int level, int *host_out);

/* Spectral-decay smoothness indicator (Sec. 3.3): eta[k] = ||s_p - s_{p-1}||
 * / ||s_p|| over element k of s = q_inf[var] + dq[var] (var = 1: rho u, the
 * paper's default), where s_p is the element's polynomial and s_{p-1} keeps
 * its Legendre modes of degree <= p - 1 in every direction (the tensor space
 * one degree lower; the library's reading).  Every element needs degree >= 1.
 * dq: padded state of the level; eta: Ne device doubles. */
fr_status fr_pa_indicator(frpmg_ctx *ctx, int level, const double *dq, int var, double *eta, fr_stream stream);

/* Degree update (Sec. 3.3): deg_out[k] = deg_in[k] + 1 where
 * eta[k] > nu_max eta_max, - 1 where eta[k] < nu_min eta_max (eta_max = the
 * largest eta), clipped to [p_min, p_max]; the paper takes nu_max = 0.2,
 * nu_min = 0.001, p_min = 1.  Device arrays of Ne entries; deg_out may alias
 * deg_in. */
fr_status fr_pa_adapt(frpmg_ctx *ctx, const double *eta, const int *deg_in, int *deg_out, int p_min, int p_max,
                      double nu_max, double nu_min, fr_stream stream);

/* y = the state x carried element by element from the degree map deg_from
 * (padded to degree p_from) to deg_to (padded to p_to) by L2 projection
 * (exact when the degree rises).  Device arrays: deg_* Ne ints, x and y
 * padded states, not aliased.  An element whose degree lies outside
 * [0, p_from] or [0, p_to] gets NaN entries. */
fr_status fr_pa_project(frpmg_ctx *ctx, const int *deg_from, int p_from, const double *x, const int *deg_to, int p_to,
                        double *y, fr_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* FRPMG_H */

/*
 * fo.h -- C ABI of the MI355X hot path of level-set shape optimisation for
 * compliance minimisation (arXiv 2601.05709).
 *
 * One iteration of the paper's level-set algorithm (Section "Main algorithm",
 * Algorithm "Level set algorithm") for the compliance model (Section
 * "Compliance minimization") is exposed as four calls:
 *
 *   fo_state_solve       state problem, eq. compli_weak: find u with
 *                        int A_Omega sigma(u) : eps(v) = int_Gamma1 g . v
 *                        (P1 elements, Jacobi-preconditioned CG, matrix free);
 *   fo_shape_derivative  compliance J (eq. compli_cost) and the right-hand side
 *                        -int S1 : D xi of the velocity equation (eq. velocity)
 *                        with S1 = S1^J + lambda S1^C (eq. S0andS1,
 *                        S1^J = A (2 Du^T sigma(u) - sigma(u):eps(u) I),
 *                        S1^C = chi_Omega I / V);
 *   fo_descent_solve     velocity problem B(theta, xi) = -dJ(Omega; xi)
 *                        (eqs. velocity_eq0, velocity) with the bilinear form of
 *                        eq. compli1_bili (mass, gradient, subdomain penalty
 *                        eq. sub_dom, boundary normal penalty eq. bd_plt);
 *   fo_levelset_update   transport of phi along theta (eq. transport without
 *                        the diffusion term), one explicit step.
 *
 * Around it: the paper's transport step and reinitialisation (fo_transport,
 * fo_reinit), Algorithm 1 as a loop on the device (fo_optimize), batched
 * multi-load solves, a serving pool, and two more models on the same
 * operators with their loops: the heat-conduction model (fo_heat_*,
 * fo_optimize_heat) and the inverse elasticity problem (fo_inverse_*,
 * fo_optimize_inverse).
 *
 * Conventions
 *   - Mesh arrays passed to fo_create are HOST pointers; the library copies
 *     (and re-tiles) them, so the caller may free them afterwards.
 *   - All per-iteration arrays (phi, b, u, rhs, theta, S1, J, ...) are DEVICE
 *     pointers owned by the caller.  They must not alias each other unless
 *     stated.  Nothing is retained after a call returns.
 *   - Unknowns are node-blocked: dof = node * dim + component.  Several right
 *     hand sides are stored RHS-contiguous: value (dof, k) at [dof * ld + k].
 *   - Element arrays are structure-of-arrays: conn[a * n_elems + e].
 *   - Every call enqueues its work on the context's stream.  Calls that must
 *     test convergence (the solves, transport, reinitialisation and loops)
 *     synchronise that stream before they return; the others return without
 *     synchronising unless stated.
 *   - Errors are status codes; arguments are validated on the host before any
 *     work is enqueued.  A context is not thread safe.
 *   - Level set: Omega = {phi < 0} (eq. subdomain).  One coefficient per
 *     element from the mean of its vertex values: A_e = 1 if the mean is < 0,
 *     else the ersatz weight (eq. compli_AOmega); a mean of exactly 0 is
 *     outside Omega.
 */
#ifndef FO_H
#define FO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FO_OK = 0,
    FO_NOT_CONVERGED = 1,    /* warning: outputs written, tolerance not met       */
    FO_ERR_ARG = -1,         /* invalid argument (null pointer, size, option)     */
    FO_ERR_MESH = -2,        /* degenerate element or invalid connectivity        */
    FO_ERR_NOMEM = -3,       /* device allocation failed                          */
    FO_ERR_HIP = -4,         /* HIP runtime error                                 */
    FO_ERR_BREAKDOWN = -5,   /* CG breakdown: p.Ap <= 0, r.z < 0 or non-finite     */
    FO_ERR_STATE = -6,       /* call order: no level set / no descent setup yet   */
    FO_ERR_BUSY = -7         /* serving pool: no free slot or HBM budget for it   */
} fo_status;

enum { FO_FP64 = 0,          /* plain FP64 conjugate gradients                     */
       FO_FP32_IR = 1 };     /* FP32 CG inner solves + FP64 iterative refinement   */

enum { FO_SCATTER_TILED = 0, /* deterministic LDS-tiled element scatter (default)  */
       FO_SCATTER_ATOMIC = 1 /* element-parallel atomics (cross-check mode)        */ };

typedef struct fo_ctx fo_ctx;

typedef struct {
    int32_t dim;               /* 2 (triangles) or 3 (tetrahedra)                  */
    int64_t n_nodes, n_elems;
    const double *coords;      /* host [n_nodes][dim]                              */
    const int32_t *conn;       /* host [dim+1][n_elems], any orientation           */
    const uint8_t *dof_fixed;  /* host [n_nodes*dim], 1 = clamped (u = 0); or NULL */
    int64_t n_bfacets;         /* boundary facets (for the normal penalty)         */
    const int32_t *bfacets;    /* host [dim][n_bfacets]                            */
    const double *bnormal;     /* host [n_bfacets][dim], unit outward normals      */
} fo_mesh;

typedef struct {
    double E, nu;              /* Young's modulus, Poisson ratio                   */
    int32_t plane_stress;      /* 2D only: 1 plane stress, 0 plane strain          */
    double ersatz;             /* A_e outside Omega (weak material), in (0, 1]     */
} fo_material;

typedef struct {
    int32_t precision;         /* FO_FP64 or FO_FP32_IR                            */
    double rtol;               /* stop when ||b - A x||_2 <= rtol ||b||_2 (FP64)   */
    int32_t max_iter;          /* cap on operator applications (all levels)        */
    double inner_rtol;         /* FO_FP32_IR: relative residual of each inner solve
                                  (phase), 0: 0.1; a phase is asked for no more than
                                  the solve still needs (half the remaining factor) */
    int32_t max_outer;         /* FO_FP32_IR: cap on refinement steps               */
    int32_t check_every;       /* iterations between host convergence polls, 0=auto*/
} fo_solve_opts;

typedef struct {
    double alpha;              /* weight of int theta . xi                         */
    double gamma_n;            /* weight of int_{boundary} (theta.n)(xi.n)         */
    double gamma_s;            /* weight of int chi_Omega0 theta . xi              */
    int32_t n_boxes;           /* Omega0 = union of open boxes (element centroid),
                                  at most 64                                       */
    const double *boxes;       /* host [n_boxes][2*dim]: lo[0..d), hi[0..d)        */
    const uint8_t *fixed;      /* NULL, or device [n_dofs]: theta = 0 where set
                                  (e.g. H^1_0 velocities); copied into the context
                                  by the first solve or apply with these options
                                  (the array may be freed afterwards); options are
                                  new when any field or this pointer differs, so
                                  new contents at the same address need a fresh
                                  set-up (another pointer, or other options first) */
} fo_descent_opts;

typedef struct {
    int32_t status;            /* fo_status of the solve                           */
    int32_t iters_inner;       /* operator applications in the working precision   */
    int32_t iters_outer;       /* FP64 refinement residuals (FO_FP32_IR), else 0   */
    double rel_res;            /* final FP64 ||b - A x|| / ||b|| (max over RHS)    */
    double seconds;            /* wall time of the call                            */
} fo_solve_stats;

/* Create a context for one mesh and material.  Validates the mesh (indices in
 * range, no degenerate element), builds the element tiles, copies everything
 * to the current HIP device and allocates the Krylov workspace for up to
 * max_rhs simultaneous right-hand sides, the velocity operator's arrays and
 * the transport and reinitialisation work buffers.  stream may be NULL
 * (default stream).  The context owns its device memory until fo_destroy.
 * After creation the per-iteration calls (fo_set_levelset, the solves,
 * derivatives, applies, fo_levelset_update, fo_transport, fo_reinit and the
 * fo_heat_* calls) allocate no device memory; fo_batch_tune, the inverse
 * problem's calls (their pair buffers, on first use or for a larger ld) and
 * the loops fo_optimize* (their work vectors, per call) do.
 * Errors: FO_ERR_ARG, FO_ERR_MESH, FO_ERR_NOMEM, FO_ERR_HIP. */
int fo_create(fo_ctx **out, const fo_mesh *mesh, const fo_material *mat, int32_t max_rhs,
              void *stream);
int fo_destroy(fo_ctx *ctx);

/* A context on a caller-owned device workspace (the library allocates no
 * device memory for it).  fo_workspace_bytes returns the bytes such a context
 * needs for this mesh, material and max_rhs on the current device: it runs
 * the host part of fo_create (validation, tiles) and adds up the device
 * arrays without touching the device; 0 for an invalid argument.
 * fo_create_in is fo_create with every device array carved from ws (device
 * pointer, 256-byte aligned, ws_bytes >= fo_workspace_bytes; FO_ERR_NOMEM if
 * smaller, FO_ERR_ARG if misaligned or NULL); it still creates a private
 * stream, events and small pinned host buffers.  The caller keeps ws
 * allocated and otherwise unused until fo_destroy, and frees it afterwards.
 * fo_footprint_bytes of such a context equals fo_workspace_bytes.  The
 * per-iteration calls behave as on a fo_create context; fo_batch_tune
 * returns FO_ERR_STATE (the batch tiles stay those built at creation), and
 * the calls that allocate per call (inverse problem, loops) still do. */
size_t fo_workspace_bytes(const fo_mesh *mesh, const fo_material *mat, int32_t max_rhs);
int fo_create_in(fo_ctx **out, const fo_mesh *mesh, const fo_material *mat, int32_t max_rhs, void *stream,
                 void *ws, size_t ws_bytes);

/* Number of device allocations (hipMalloc) the library has made in this
 * process so far, for callers and tests that check that a sequence of calls
 * allocates nothing. */
int64_t fo_device_allocations(void);

/* Device bytes owned by the context (for footprint-based admission). */
size_t fo_footprint_bytes(const fo_ctx *ctx);

/* Estimate of fo_footprint_bytes for a context created on this mesh with
 * max_rhs = 1, from the mesh sizes alone (no GPU, no tile build; 0 for an
 * invalid mesh description).  The tile and halo terms assume the node ratios
 * of structured simplicial meshes and lean high (up to about 2x on small
 * meshes); admission control uses it until the actual footprint is known. */
size_t fo_footprint_estimate(const fo_mesh *mesh);

/* Select the element scatter used by the operators (FO_SCATTER_*).  The
 * atomic mode is a cross-check of the operators and of FP64 solves; FO_FP32_IR
 * solves need the tiled mode (FO_ERR_ARG otherwise). */
int fo_set_scatter(fo_ctx *ctx, int32_t mode);

/* Set the level set phi (device [n_nodes]) and derive A_e, chi_e and the Jacobi
 * diagonal of K(phi) (FP64 and FP32).  Must precede the state solve. */
int fo_set_levelset(fo_ctx *ctx, const double *phi);

/* y = K(phi) x on the free unknowns (rows and columns of clamped unknowns are
 * zero).  precision FO_FP64: x, y are double*; FO_FP32_IR: x, y are float* and
 * the operator uses single-precision geometry.  Device pointers, [n_nodes*dim]. */
int fo_apply_elasticity(fo_ctx *ctx, const void *x, void *y, int32_t precision);

/* State solve K(phi) u = b on the free unknowns, u = 0 on clamped unknowns.
 * b, u: device [n_dofs][ld], n_rhs columns (1 <= n_rhs <= max_rhs, ld >= n_rhs).
 * n_rhs > 1: FO_FP64 solves the columns one after another; FO_FP32_IR runs the
 * batched path (all columns of a block at once, see fo_batch_tune).  stats:
 * host, may be NULL.
 * Returns FO_OK, FO_NOT_CONVERGED (u holds the last iterate) or an error. */
int fo_state_solve(fo_ctx *ctx, const double *b, double *u, int32_t n_rhs, int64_t ld,
                   const fo_solve_opts *opts, fo_solve_stats *stats);

/* Compliance and shape derivative for the solution(s) u (device [n_dofs][ld]):
 *   J[k]  = sum_e A_e |T_e| sigma(u_k) : eps(u_k)     (device [n_rhs])
 *   *vol  = sum_e chi_e |T_e|                         (device scalar)
 *   rhs   = -sum_e |T_e| S1_e grad(lambda_a), S1_e = sum_k S1^J(u_k) + lambda_vol chi_e I / V
 *           (device [n_dofs]); S1 (device [dim*dim][n_elems]) may be NULL. */
int fo_shape_derivative(fo_ctx *ctx, const double *u, int32_t n_rhs, int64_t ld,
                        double lambda_vol, double V, double *rhs, double *S1, double *J,
                        double *vol);

/* Descent (velocity) solve B theta = rhs on all unknowns (H^1, no clamp),
 * or, with dopts->fixed, theta = 0 on the masked unknowns and B theta = rhs
 * on the others (the masked rows and columns of B and entries of rhs drop
 * out).  B does not depend on phi: its diagonal is built on the first call
 * with a given opts and reused.  rhs, theta: device [n_dofs]; B_tt: device
 * scalar receiving B(theta, theta) = theta . rhs (> 0 for a descent
 * direction).  fo_apply_descent: y = B x, zero on masked rows. */
int fo_descent_solve(fo_ctx *ctx, const fo_descent_opts *dopts, const double *rhs,
                     double *theta, const fo_solve_opts *opts, fo_solve_stats *stats,
                     double *B_tt);

/* y = B x for the descent operator (device double [n_dofs]). */
int fo_apply_descent(fo_ctx *ctx, const fo_descent_opts *dopts, const double *x, double *y);

/* phi_i <- phi_i - dt theta_i . G_i with G_i the |T|-weighted mean of the
 * element gradients of phi around node i.  phi: device [n_nodes], in/out;
 * theta: device [n_dofs]. */
int fo_levelset_update(fo_ctx *ctx, const double *theta, double dt, double *phi);

/* The paper's transport step of the level set (Section "Transport
 * equation", eqs. transport, weak_transport, tau_lv): `steps` Crank-Nicolson
 * steps of length dt (> 0) of d/dt phi + theta . grad phi = h^2 lap phi
 * (Neumann) with Petrov-Galerkin test functions psi + tau theta . grad psi,
 * tau = (1/2)(dt^-2 + |theta|^2/h^2)^(-1/2); theta and tau are taken per
 * element at the element mean of theta.  smooth != 0 adds the h^2 diffusion,
 * h^2 being the paper's mesh-size expression (4|D|/(N_T sqrt 3) in 2D,
 * (6 sqrt 2 |D|/N_T)^(2/3) in 3D).  Each step solves its nonsymmetric system
 * by Jacobi-preconditioned BiCGStab in FP64 from the previous phi until the
 * recomputed residual is <= opts->rtol times the right-hand side
 * (opts->max_iter operator applications per step; precision ignored).
 * theta: device [n_dofs] (e.g. from fo_descent_solve); phi: device
 * [n_nodes], in: phi(t), out: phi(t + steps dt).  stats (host, may be NULL):
 * iters_inner = operator applications, iters_outer = steps, rel_res = the
 * largest accepted relative residual.  Requires the tiled scatter.  Returns
 * FO_OK, FO_NOT_CONVERGED (phi holds the last iterate), FO_ERR_BREAKDOWN,
 * FO_ERR_STATE (atomic scatter) or FO_ERR_ARG. */
int fo_transport(fo_ctx *ctx, const double *theta, double dt, int32_t steps, int32_t smooth, double *phi,
                 const fo_solve_opts *opts, fo_solve_stats *stats);

/* Final time and step count of the transport from B(theta, theta) (Section
 * "Other implementation aspects", eqs. tend and steps, without the optional
 * noise): t_end = dfactor / B_tt clamped to [t_min, t_max], steps = (s_max -
 * s_min) ((t_end - t_min) / (t_max - t_min))^(1/6) + s_min clamped to [s_min,
 * s_max] and rounded half to even, dt = t_end / steps (host outputs).  The
 * loops use it for every iteration; fo_levelset_update takes its dt.  The
 * paper's defaults: dfactor 1e-2, t in [1e-3, 1e-1], steps in [8, 16].
 * Errors: FO_ERR_ARG. */
int fo_time_steps(double B_tt, double dfactor, double t_min, double t_max, int32_t s_min, int32_t s_max,
                  double *t_end, int32_t *steps, double *dt);

/* Parameters of the level-set loop (fo_optimize).  The paper's defaults:
 * dfactor 1e-2, t in [1e-3, 1e-1], steps in [8, 16], smooth 0,
 * start_to_check 30, prev 10, cost/lgrn/ctrn tolerances 1e-2, and the PPL
 * parameters r 0.999, delta0 0.5, alpha 2000, beta 0.5. */
typedef struct {
    int32_t n_iter;            /* iterations at most (niter)                       */
    double V;                  /* > 0: constraint vol(Omega) / V = 1 (PPL); <= 0: none */
    double dfactor;            /* t_end = dfactor / B(theta, theta)                */
    double t_min, t_max;       /* clamp of t_end                                    */
    int32_t s_min, s_max;      /* clamp of the transport step count                */
    int32_t smooth;            /* transport with the h^2 diffusion                 */
    int32_t start_to_check;    /* the stopping test runs for i > start_to_check    */
    int32_t prev;              /* window of earlier iterates in the test            */
    double cost_tol, lgrn_tol, ctrn_tol;
    double ppl_r, ppl_delta0, ppl_alpha, ppl_beta;
    fo_solve_opts state;       /* state solve                                       */
    fo_solve_opts descent;     /* velocity solve                                    */
    fo_solve_opts transport;   /* transport and reinitialisation solves            */
    fo_descent_opts velocity;  /* the velocity bilinear form                        */
    int32_t reinit_step;       /* > 0: reinitialise after the transport of every
                                  iteration i with i % reinit_step == 0            */
    int32_t reinit_iters;      /* reinitialisation steps (the paper: 8)             */
    double reinit_t;           /* reinitialisation pseudo-time (the paper: 0.1)     */
} fo_loop_opts;

/* One iteration of fo_optimize (host). */
typedef struct {
    double J;                  /* cost: compliance b . u, heat u . K u, inverse cost */
    double vol;                /* sum_e chi_e |T_e|                                 */
    double C;                  /* vol / V (vol without a constraint)                */
    double L;                  /* Proximal-Perturbed Lagrangian (J without a constraint) */
    double lambda;             /* multiplier used in the derivative                 */
    double B_tt;               /* B(theta, theta); NaN on a stopping iteration      */
    double t_end, dt;          /* transport final time and step                     */
    int32_t steps;             /* transport steps (0 on a stopping iteration)      */
    int32_t state_iters, descent_iters, transport_iters;  /* operator applications */
    int32_t status;            /* worst status of the iteration's solves            */
    int32_t reinit_iters;      /* reinitialisation operator applications (0: none) */
} fo_loop_record;

/* The level-set loop (Algorithm 1; Sections "Lagrangian method" and "Other
 * implementation aspects"): per iteration i, set phi, state solve, cost J =
 * b . u and volume; with V > 0 the PPL update of eq. lag_method for i >= 1
 * (iteration 0 uses z = lambda = mu = 0) and the Lagrangian of eq.
 * lagrangian; the stopping test (i > start_to_check: over the previous `prev`
 * iterates, the relative change of J, or of L together with |C - 1| <
 * ctrn_tol, below its tolerance); then the descent right-hand side of S =
 * S^J + lambda S^C (eq. S0andS1), the velocity solve, t_end and the step
 * count from eqs. tend and steps (no noise), fo_transport of phi, and with
 * reinit_step > 0 fo_reinit of the transported phi at every iteration i
 * with i % reinit_step == 0.
 * b: device [n_dofs], one load case; phi: device [n_nodes], in: phi^0, out:
 * the last level set.  records: host [opts->n_iter]; *n_done receives the
 * number of iterations recorded and *stopped 1 when the stopping test ended
 * the loop.  Allocates its work vectors (4 n_dofs + 4 doubles) per call.
 * Returns FO_OK, FO_NOT_CONVERGED (a solve hit its cap; the loop went on),
 * FO_ERR_ARG, or the first error of a step (the loop stops there). */
int fo_optimize(fo_ctx *ctx, const fo_loop_opts *opts, const double *b, double *phi,
                fo_loop_record *records, int32_t *n_done, int32_t *stopped);

/* fo_optimize for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that keep the allocator out of the
 * request path): the same loop, with the same arguments and results, but its
 * work vectors (3 n_dofs + 4 doubles) live in a static device array of the
 * library (64 MiB per GPU, held from when the library is loaded on that GPU
 * until the process ends) and no device memory is allocated: chunks of the
 * solvers that have no captured graph on this context yet are launched
 * directly instead of being captured.  The context must be one of fo_create
 * (its velocity and transport arrays exist from creation).  n_dofs above
 * FO_NOALLOC_MAX_DOFS: FO_ERR_ARG.  Every call on a GPU uses that GPU's one
 * array, so calls that overlap on the same GPU (from several threads or
 * contexts) race; calls one after another are independent (the loop
 * initialises everything it reads).  Returns as fo_optimize. */
enum { FO_NOALLOC_MAX_DOFS = 2796201 };
int fo_optimize_noalloc(fo_ctx *ctx, const fo_loop_opts *opts, const double *b, double *phi,
                        fo_loop_record *records, int32_t *n_done, int32_t *stopped);

/* Reinitialisation of the level set (Section "Other implementation
 * aspects", eqs. Eikonal, HJ, grad_H, weak_HJ): `steps` pseudo-time steps up
 * to t_end (the paper's defaults: 8 steps, 0.1) of
 *   d/dt varphi + S(phi) |grad varphi| = S(phi) + h^2 lap varphi (Neumann),
 * S(phi) = phi / sqrt(phi^2 + h^2), from varphi(0) = phi, with
 * Petrov-Galerkin test functions psi + tau grad H . grad psi (grad H =
 * S g / |g| for the element gradient g of varphi(t), 0 on an element whose
 * vertex values agree to 1e-12 relative; tau = (1/2)(dt^-2 +
 * S^2/h^2)^(-1/2)); S enters per element at the mean of its nodal values,
 * h^2 is the transport step's mesh-size expression.  The first step is
 * explicit Euler, the others two-step Adams-Bashforth; each solves its
 * nonsymmetric mass system by Jacobi BiCGStab in FP64 to opts->rtol
 * (recomputed residual; opts->max_iter applications per step).  phi: device
 * [n_nodes], in: phi, out: varphi(t_end).  stats (host, may be NULL) as for
 * fo_transport.  Requires the tiled scatter.  Returns FO_OK,
 * FO_NOT_CONVERGED, FO_ERR_BREAKDOWN, FO_ERR_STATE or FO_ERR_ARG. */
int fo_reinit(fo_ctx *ctx, double *phi, int32_t steps, double t_end, const fo_solve_opts *opts,
              fo_solve_stats *stats);

/* Heat-conduction model (Section "Heat conduction": eqs. heat_cost,
 * heat_prob, heat_weak, heat_AOmega): minimise J = int A |grad u|^2 for
 * -div A grad u = f, u = 0 on Gamma_0, insulated elsewhere, A = 1 in Omega
 * and the context's ersatz value (the paper: 1e-3) outside, per element from
 * the level set of fo_set_levelset; P1 u and f (nodal).  The adjoint is
 * p = -u.  All on the tiled scatter; device pointers; N = n_nodes.
 *
 * fo_heat_load: b = int f lambda_a (exact P1 mass), b and f [N].
 * fo_heat_solve: u [N] with K u = b on the free nodes, u = 0 where gamma0
 *   [N] (uint8) is nonzero, by FP64 Jacobi-preconditioned CG (the system is
 *   SPD) to opts->rtol on the recomputed residual; stats->iters_inner counts
 *   operator applications.  Returns FO_OK, FO_NOT_CONVERGED,
 *   FO_ERR_BREAKDOWN, FO_ERR_STATE (no level set, or the atomic scatter) or
 *   FO_ERR_ARG.
 * fo_heat_derivative: the descent right-hand side rhs [n_dofs] of S0 =
 *   2 u grad f, S1 = (2 u f - A |grad u|^2) I + 2 A grad u (x) grad u +
 *   lambda_vol chi I / V (rhs_(a,i) = -(int S0_i lambda_a + int (S1 grad
 *   lambda_a)_i), exact for P1), the cost *J = u . K u and *vol = sum_e chi_e
 *   |T_e| (device scalars).  Feeds fo_descent_solve like fo_shape_derivative. */
int fo_heat_load(fo_ctx *ctx, const double *f, double *b);
int fo_heat_solve(fo_ctx *ctx, const uint8_t *gamma0, const double *b, double *u, const fo_solve_opts *opts,
                  fo_solve_stats *stats);
int fo_heat_derivative(fo_ctx *ctx, const double *u, const double *f, double lambda_vol, double V, double *rhs,
                       double *J, double *vol);

/* Inverse elasticity problem (Section "Inverse problem": eqs. cost, f-prob,
 * g-prob, AOmega, w-f, w-g, the adjoint problems of eqs. dL1 and dL2, and
 * eq. SDelast_inv) for n_pairs force-displacement pairs (f_k, g_k):
 *   J_k = alpha/2 int_D |u_k - v_k - g_k|^2 + beta/2 int_Gamma1 |u_k - g_k|^2,
 * u_k with traction f_k on Gamma_1 and u_k = 0 on Gamma_0, y_k = v_k + g_k
 * with v_k = 0 on the whole boundary, A = kappa in Omega and 1 outside
 * (element mean of phi negative: Omega); the cost of several pairs is
 * sum_k J_k.  Two contexts on the same mesh and device: ctx_f clamps Gamma_0
 * and lists the Gamma_1 facets (its boundary facets carry the beta-term),
 * ctx_g clamps every boundary unknown; both are created with ersatz =
 * 1/kappa (their operator is K/kappa; fo_create takes ersatz in (0, 1], so
 * kappa >= 1) and the tiled scatter; the pairs are
 * solved one after the other.  Contexts on different streams solve u and v
 * (then p and q) concurrently, one of them from a helper host thread (same
 * results); the call returns when all work has finished.  g_k
 * is the P1 Dirichlet data extended into D; it may be nonzero anywhere.
 * Device arrays [n_dofs][ld] (pair k in column k, ld >= n_pairs) unless
 * stated.
 *
 * fo_inverse_states: sets phi on both contexts and solves, by their state
 *   solves with opts, u (ctx_f), v with K v = -K g (ctx_g), the adjoints p
 *   with K p = -alpha M (u - v - g) - beta M_Gamma1 (u - g) (ctx_f) and q
 *   with K q = alpha M (u - v - g) (ctx_g), M the P1 mass and M_Gamma1 the
 *   P1 mass of the Gamma_1 facets; J (device [n_pairs]) the cost of each
 *   pair.  stats sum the four solves.  Returns FO_OK, FO_NOT_CONVERGED,
 *   FO_ERR_BREAKDOWN, FO_ERR_ARG (kappa inconsistent with the contexts'
 *   ersatz value, contexts of different sizes or devices, n_pairs < 1,
 *   ld < n_pairs) or FO_ERR_STATE (atomic scatter).
 * fo_inverse_derivative: the descent right-hand side rhs (device [n_dofs])
 *   of eq. SDelast_inv summed over the pairs in pair order, per pair
 *   rhs_(a,i) = -(int S0_i lambda_a + int (S1 grad lambda_a)_i) with S0 =
 *   -alpha Dg^T w and S1 = [alpha/2 |w|^2 + A (sigma(u):eps(p) +
 *   sigma(v+g):eps(q))] I - A (Du^T sigma(p) + Dp^T sigma(u) + Dv^T sigma(q)
 *   + Dq^T sigma(v+g)), w = u - v - g, (Du)_ij = d_j u_i, for the level set
 *   last set on ctx_f.  The velocity of the paper's H^1_0 setting is then
 *   fo_descent_solve on ctx_f with fixed = the boundary unknowns. */
int fo_inverse_states(fo_ctx *ctx_f, fo_ctx *ctx_g, const double *phi, int32_t n_pairs, int64_t ld,
                      const double *f, const double *g, double kappa, double alpha, double beta,
                      const fo_solve_opts *opts, double *u, double *v, double *p, double *q, double *J,
                      fo_solve_stats *stats);
int fo_inverse_derivative(fo_ctx *ctx_f, int32_t n_pairs, int64_t ld, const double *u, const double *v,
                          const double *p, const double *q, const double *g, double kappa, double alpha,
                          double *rhs);

/* Algorithm 1 on the heat-conduction model: fo_optimize's loop (the PPL
 * volume constraint when opts->V > 0, the stopping rule, the velocity with
 * opts->velocity, the adaptive time stepping, transport, reinitialisation)
 * with, per iteration, fo_set_levelset, fo_heat_solve with opts->state (its
 * rtol and max_iter), fo_heat_derivative (J = u . K u and the volume, then
 * the right-hand side of S^J + lambda S^C).  gamma0: device [n_nodes] uint8
 * (u = 0 where set); f: device [n_nodes] P1 source, its load computed once.
 * Allocates its work vectors for the call.  Returns as fo_optimize. */
int fo_optimize_heat(fo_ctx *ctx, const fo_loop_opts *opts, const uint8_t *gamma0, const double *f, double *phi,
                     fo_loop_record *records, int32_t *n_done, int32_t *stopped);

/* Algorithm 1 on the inverse problem: fo_optimize's loop with, per
 * iteration, fo_inverse_states (phi set on both contexts), the cost J =
 * sum_k J_k (pair order), the stopping test on J (no constraint: opts->V must
 * be <= 0, the PPL fields are unused), fo_inverse_derivative, the velocity
 * fo_descent_solve on ctx_f with opts->velocity (the paper's H^1_0 setting:
 * its fixed mask = the boundary unknowns), the adaptive final time and step
 * count, fo_transport on ctx_f and, every reinit_step iterations, fo_reinit.
 * Arguments as fo_inverse_states and fo_optimize; records hold J = L, vol =
 * C = 0 and lambda = 0.  Allocates its work vectors (4 ld + 2 columns) for
 * the call.  Returns as fo_optimize. */
int fo_optimize_inverse(fo_ctx *ctx_f, fo_ctx *ctx_g, const fo_loop_opts *opts, int32_t n_pairs, int64_t ld,
                        const double *f, const double *g, double kappa, double alpha, double beta, double *phi,
                        fo_loop_record *records, int32_t *n_done, int32_t *stopped);

/* Kernel timing for measurement tools.  While enabled, every launch of the
 * kernels named below is bracketed by a pair of HIP events recorded on the
 * context's stream; fo_profile_read synchronises the stream and returns the
 * summed event time (ms) and launch count since the last enable.  Enabling
 * resets the totals; timing adds a few microseconds of launch overhead. */
enum { FO_PROF_ELAS_TILE_FP64 = 0,   /* tiled elasticity element kernel, FP64  */
       FO_PROF_ELAS_TILE_FP32 = 1,   /* tiled elasticity element kernel, FP32  */
       FO_PROF_HALO_FP64 = 2,        /* shared-node (halo) reduction, FP64      */
       FO_PROF_HALO_FP32 = 3,        /* shared-node (halo) reduction, FP32      */
       FO_PROF_COUNT = 4 };
int fo_profile_enable(fo_ctx *ctx, int32_t on);
int fo_profile_read(fo_ctx *ctx, int32_t which, double *total_ms, int64_t *launches);

/* Average duration of one kernel, for measurement tools: `reps` back-to-back
 * launches of the named kernel on the context's stream between two HIP
 * events; *avg_us receives the elapsed time divided by reps.  The fused CG
 * operator kernels run on the context's CG work vectors with a private
 * scalar slot that never signals convergence, so every launch does the full
 * work; the work vectors (not the level set, coefficients or Jacobi
 * diagonal) hold undefined values afterwards and the next solve
 * reinitialises them.  Requires the tiled scatter and a level set.
 * Synchronises the stream.  reps in [1, 100000]. */
enum { FO_KERNEL_CG_OP_FP64 = 0,     /* fused CG operator: direction update + K(phi) p, FP64 */
       FO_KERNEL_CG_OP_FP32 = 1,     /* the same in FP32                                      */
       FO_KERNEL_BATCH_APPLY = 2,    /* batched FP32 apply on the matrix cores, all columns of
                                        the context's block (needs max_rhs > 1)               */
       FO_KERNEL_COUNT = 3 };
int fo_time_kernel(fo_ctx *ctx, int32_t kernel, int32_t reps, double *avg_us);

/* Batched multi-load solves (fo_state_solve with n_rhs > 1 and FO_FP32_IR,
 * on a context created with max_rhs > 1).  The load cases share K(phi); the
 * multi-load compliance problem sums their derivatives (Section "Compliance
 * minimization", several loads) and the paper solves such PDE sets in its
 * task-parallel mode (Section "Parallelization").  Columns are processed in
 * blocks of up to 64; each block is solved by the method of
 * fo_set_batch_method (CG per column by default), the element contraction K_e X_e
 * on the matrix cores in FP32, with FP64 residual replacement and the
 * single-load solve's stopping rule per column.  stats: iters_inner counts
 * block iterations (one block operator application each) plus the FP64 CG
 * iterations of columns finished in FP64, summed over blocks; rel_res is the
 * worst column.
 *
 * fo_batch_tune times the batched apply for every tile node cap that fits
 * the LDS and both element group sizes (elements with pairwise disjoint node
 * sets that a wave contracts together: 4, 8) and keeps the fastest pair
 * (tile_nodes: node cap, group: group size, apply_us: apply time for
 * min(n_rhs, 64) columns rounded up to a multiple of 16).  It rebuilds the
 * batch tiles (synchronises the stream) and needs a level set.  Errors:
 * FO_ERR_ARG without batch buffers or n_rhs out of [1, max_rhs]. */
int fo_batch_tune(fo_ctx *ctx, int32_t n_rhs, int32_t *tile_nodes, int32_t *group, double *apply_us);

/* Method of the batched solves (fo_state_solve with n_rhs > 1 and
 * FO_FP32_IR).  FO_BATCH_COLUMN_CG (default): CG per column on the shared
 * batched operator (a step length per column).  FO_BATCH_BLOCK_CG: block
 * conjugate gradients (O'Leary): every iteration applies K to a block of
 * directions, one per load case still running, and each case takes its best
 * step in the span of the whole block (K-conjugate block directions, their
 * s x s Gram matrix inverted in FP64 with numerically dependent directions
 * dropped); a case leaves the block when its residual has fallen by the
 * phase target (inner_rtol) and the block narrows 16 columns at a time.
 * Phases restart from the FP64 residuals of the unconverged cases (FP64
 * refinement, as the single-load path).  Both stop every column on the same
 * FP64 criterion, so their results agree within the solve tolerance; which
 * is faster depends on how independent the load cases are.  Errors:
 * FO_ERR_ARG. */
enum { FO_BATCH_BLOCK_CG = 0, FO_BATCH_COLUMN_CG = 1 };
int fo_set_batch_method(fo_ctx *ctx, int32_t method);

/* Operator of the batched solves and of fo_apply_elasticity_batch; both
 * compute K(phi) X in FP32 on the matrix cores for every column at once.
 * FO_BATCH_OP_NODAL (default): K(phi) assembled per level set (in
 * fo_set_levelset) into d x d blocks K_ij, one per pair of distinct nodes
 * sharing an element (FP64 sums of the element entries of Section
 * "Compliance minimization", rounded once to FP32, exactly symmetric), and
 * applied as y_i = sum_{j != i} K_ij (x_j - x_i) (rows of K(phi) sum to zero);
 * the FP64 residual replacement of the batched solves applies the same
 * blocks unrounded.  Memory: about N NB (4 + 12 d^2) bytes (ids, FP32 and FP64
 * blocks), NB the largest neighbour count rounded up to a multiple of 7 or of
 * 8, whichever is smaller.  FO_BATCH_OP_ELEMENT: the element contraction
 * K_e[:, b >= 1] (X_b - X_0) per element tile, node rows summed in LDS and a
 * halo (what fo_batch_tune tunes).  The two agree to FP32 rounding.  Takes
 * effect at the next solve or apply.  Errors: FO_ERR_ARG. */
enum { FO_BATCH_OP_NODAL = 0, FO_BATCH_OP_ELEMENT = 1 };
int fo_set_batch_operator(fo_ctx *ctx, int32_t op);

/* Shape of the assembled operator of the batched path: neighbour slots per
 * node (NB), off-diagonal blocks (ordered pairs of distinct nodes sharing an
 * element) and the device bytes of its arrays; all 0 when the context has
 * none (max_rhs = 1, or a mesh whose neighbourhoods exceed the apply's
 * staging buffer, NB d^2 > 512).  Any pointer may be NULL. */
int fo_nodal_stats(const fo_ctx *ctx, int32_t *slots, int64_t *off_diagonal_blocks, int64_t *bytes);

/* Y = K(phi) X for a block of load cases through the batched operator (FP32,
 * matrix cores): x, y device float [n_dofs][ncols], load case fastest; ncols
 * a multiple of 16 up to the context's column block width (fo_batch_stats).
 * Clamped rows of y are 0.  Synchronises the stream. */
int fo_apply_elasticity_batch(fo_ctx *ctx, const float *x, float *y, int32_t ncols);

/* Shape of the batched path: column block width (0 when max_rhs = 1), largest
 * tile (nodes), register group size, tile count and halo slots (any pointer
 * may be NULL). */
int fo_batch_stats(const fo_ctx *ctx, int32_t *columns, int32_t *tile_nodes, int32_t *group,
                   int64_t *n_tiles, int64_t *n_halo_slots);

/* Tile statistics of the deterministic scatter: tiles, largest tile (nodes),
 * tile-node pairs, shared nodes and halo slots (any pointer may be NULL). */
int fo_tile_stats(const fo_ctx *ctx, int64_t *n_tiles, int64_t *max_nodes, int64_t *n_slots,
                  int64_t *n_shared_nodes, int64_t *n_halo_slots);

/* ---------------------------------------------------------------------------
 * Serving: a pool of requests with continuous batching.  The paper solves sets
 * of PDEs with varying parameters in its task-parallel and mixed modes
 * (Section "Parallelization"); here such a set is a stream of requests, each
 * one iteration's finite-element work on its own mesh: level set, state
 * solve, compliance and shape derivative, descent solve.  A request is
 * admitted into a free slot when the device-memory budget has room for its
 * context (fo_footprint_estimate, replaced by the actual footprint once
 * created).  Every running request owns a context and a HIP stream.  The
 * requests run as cooperative fibers on the thread that calls fo_pool_step /
 * fo_pool_wait: a request makes its library calls until one of them would
 * wait for the device (a solver chunk's status, a stream drain), then the
 * next request runs.  So requests admitted while others run overlap on the
 * GPU, and every HIP object of the pool is created, used and destroyed on
 * that one thread.  The results of a request do not depend on what else runs
 * (every reduction has a fixed order).  A finished request's context stays
 * resident, keyed by mesh_key, and a later request with the same nonzero key
 * reuses it (mesh, tiles and workspace) instead of creating one; idle
 * resident contexts are evicted, least recently used first, when a new
 * context needs the memory.
 *
 * Threading: a pool belongs to the thread that created it; every call but
 * fo_pool_stats returns FO_ERR_STATE from another thread.
 *
 * Host memory: every pointer in fo_request is a host pointer; the arrays must
 * stay valid until the request is done (fo_pool_poll).  Requests with the
 * same nonzero mesh_key must have identical mesh and material. */
typedef struct fo_pool fo_pool;

typedef struct {
    fo_mesh mesh;
    fo_material mat;
    uint64_t mesh_key;             /* 0: never shared                                  */
    const double *phi;             /* [n_nodes] level set                              */
    const double *b;               /* [n_dofs] load                                    */
    fo_solve_opts state_opts;
    fo_solve_opts descent_solve_opts;
    fo_descent_opts descent;       /* fixed must be NULL here                          */
    double lambda_vol, V;          /* volume term of the derivative (V > 0)            */
    double *u_out;                 /* [n_dofs] displacement, or NULL                   */
    double *rhs_out;               /* [n_dofs] shape-derivative load, or NULL          */
    double *theta_out;             /* [n_dofs] descent direction, or NULL              */
} fo_request;

typedef struct {
    int32_t status;                /* worst fo_status of the request's calls           */
    int32_t reused_context;        /* 1 if a resident context was reused               */
    fo_solve_stats state, descent;
    double J, vol, B_tt;           /* compliance, volume, B(theta, theta)              */
    double t_admit, t_start, t_end;/* seconds since fo_pool_create                     */
} fo_pool_result;

/* budget_bytes: device memory the pool may hold (contexts and request
 * buffers); max_slots: requests running at once (1..64).  Uses the current
 * HIP device.  Errors: FO_ERR_ARG, FO_ERR_HIP. */
int fo_pool_create(fo_pool **out, size_t budget_bytes, int32_t max_slots);

/* Starts a request in a free slot (*slot receives its index).  Returns
 * FO_ERR_BUSY, starting nothing, when no slot is free or the budget cannot
 * fit its context even after evicting idle resident contexts; FO_ERR_ARG for
 * an invalid request. */
int fo_pool_admit(fo_pool *pool, const fo_request *req, int32_t *slot);

/* One scheduling round: resumes every running request until it waits for
 * the device or finishes (a request's context is created, on the calling
 * thread, in its first round).  *running (may be NULL) receives the number
 * of requests still running. */
int fo_pool_step(fo_pool *pool, int32_t *running);

/* Runs scheduling rounds (fo_pool_step) for up to timeout_us microseconds
 * (< 0: no limit) until some request is done and not yet released; *slot
 * receives its index, or -1 on timeout or when nothing runs.  Between rounds
 * in which every request still waits for the device it pauses 20 us. */
int fo_pool_wait(fo_pool *pool, int64_t timeout_us, int32_t *slot);

/* *done = 1 when the slot's request finished (then *res is filled; the
 * request's output arrays are written). */
int fo_pool_poll(fo_pool *pool, int32_t slot, int32_t *done, fo_pool_result *res);

/* Frees a finished slot for a new request (FO_ERR_STATE if still running). */
int fo_pool_release(fo_pool *pool, int32_t slot);

/* Budget accounting: bytes reserved, running requests, resident contexts. */
int fo_pool_stats(const fo_pool *pool, size_t *used_bytes, int32_t *running, int32_t *resident);

/* Runs every running request to its end, then frees all contexts (on the
 * calling thread, which is the pool's). */
int fo_pool_destroy(fo_pool *pool);

const char *fo_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* FO_H */

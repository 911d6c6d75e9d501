// Host-side launch wrappers of the kernels in fo_kernels.hip / fo_tiled.hip.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <tuple>

#include "fo_internal.h"

namespace fo {

int red_blocks(int64_t n);

template <typename T> void launch_fill(T *y, int64_t n, T v, hipStream_t s);
template <typename T> void launch_mask(T *y, const uint8_t *fixed, int64_t n, hipStream_t s);
template <typename T>
void launch_invert_diag(const double *diag, const uint8_t *fixed, int64_t n, T *dinv, hipStream_t s);
void launch_chi(const int32_t *conn, int64_t E, int dim, const double *phi, uint8_t *chi,
                hipStream_t s);
template <typename S, typename T>
void launch_gather_col(const S *src, int64_t ld, int64_t n, T *dst, const uint8_t *fixed,
                       hipStream_t s);
template <typename T>
void launch_scatter_col(const T *src, int64_t n, double *dst, int64_t ld, hipStream_t s);
template <typename T>
void launch_dots(int npair, const T *a0, const T *b0, const T *a1, const T *b1, const T *a2,
                 const T *b2, int64_t n, double *part, int nb, hipStream_t s);
void launch_finish_dots(const double *part, int nb, int npair, double *out, hipStream_t s);


// conjugate gradients (fo_cg.hip)
template <typename T>
void launch_cg_start(const T *b, const T *q, T *r, T *p, const T *dinv, int64_t n, double *part,
                     SolveScalars *sc, double rtol, double ref2, int max_it, hipStream_t s);
template <typename T>
void launch_cg_update(SolveScalars *sc, int P, T *x, T *r, const T *p, const T *q, const T *dinv,
                      int64_t n, const double *pq_part, int n_pq, double *rz_part, hipStream_t s);
template <typename T>
void launch_cg_direction(SolveScalars *sc, int P, T *p, const T *r, const T *dinv, int64_t n,
                         const double *rz_part, hipStream_t s);
void launch_ir_accumulate(double *x64, const float *x32, const double *s2, int64_t n, hipStream_t s);
void launch_add64(double *y, const double *x, int64_t n, hipStream_t s);
void launch_residual64(const double *b, const double *q, double *r, int64_t n, double *part,
                       double *out2, hipStream_t s);
// fused CG for the tiled elasticity operator
int node_blocks(int64_t N);
int upd_blocks(int64_t N);  // blocks of the fused update = r.z/r.r partials per sum
void launch_fold(const double *part, int n, int sets, double *out, hipStream_t s);
template <typename T>
void launch_cgn_start(const fo_ctx *c, const T *b, const T *q, T *r, const T *dinv, double rtol,
                      int max_it, hipStream_t s);
template <typename T>
void launch_cgn_update(const fo_ctx *c, int B, T *x, T *r, const T *p, const T *q, const T *dinv,
                       hipStream_t s);
// Transport step matrix of the level set (TransportOp): y = L x (which 0)
// or R x (which 1); the diagonal of L.  theta: device [N][D] nodal velocity;
// par: device [5] dt, -dt, h2 of the diffusion (0: none), h2 of tau, 1/dt^2.
// done (nullable): device flag that turns the launch into a no-op.
int launch_transport_apply(const fo_ctx *c, const double *theta, const double *par, int which, const double *x,
                           double *y, hipStream_t s, const int32_t *done = nullptr);
int launch_transport_diag(const fo_ctx *c, const double *theta, const double *par, double *diag, hipStream_t s);
// Reinitialisation step (ReinitOp): y = Lhat x, the diagonal of Lhat, and
// the step's right-hand side.  w: device [N][3] nodal u = varphi(t), v =
// varphi(t - dt), S(phi); par: device [4] dt, h^2, 1/dt^2, Euler flag.
int launch_reinit_apply(const fo_ctx *c, const double *w, const double *par, const double *x, double *y,
                        hipStream_t s, const int32_t *done = nullptr);
int launch_reinit_diag(const fo_ctx *c, const double *w, const double *par, double *diag, hipStream_t s);
int launch_reinit_rhs(const fo_ctx *c, const double *w, const double *par, double *rhs, hipStream_t s);
// Heat-conduction model (HeatOp, HeatDiagOp, MassOp, HeatSdOp): y = K x
// with the rows of fixed nodes zeroed; the diagonal of K (zero on fixed
// rows); y = M x (scalar P1 mass); the descent right-hand side [n_dofs] of
// the heat cost from u and the P1 source f.  Device arrays, N = nodes.
int launch_heat_apply(const fo_ctx *c, const uint8_t *fixed, const double *x, double *y, hipStream_t s,
                      const int32_t *done = nullptr);
int launch_heat_diag(const fo_ctx *c, const uint8_t *fixed, double *diag, hipStream_t s);
int launch_mass_apply(const fo_ctx *c, const double *x, double *y, hipStream_t s);
int launch_heat_rhs(const fo_ctx *c, const double *u, const double *f, double lambda_vol, double V, double *rhs,
                    hipStream_t s);
// Inverse elasticity (ElasOp without clamping, VecMassOp, InvSdOp, facet
// mass): y = K(phi) x on all unknowns; y = M x (vector P1 mass); the
// descent right-hand side [n_dofs] from u and aux [N][4D] = (v, p, q, g);
// y = M_Gamma1 x over the context's boundary facets.  Device arrays.
int launch_elas_apply_free(const fo_ctx *c, const double *x, double *y, hipStream_t s);
int launch_vec_mass(const fo_ctx *c, const double *x, double *y, hipStream_t s);
int launch_inverse_rhs(const fo_ctx *c, const double *u, const double *aux, double kappa, double alpha,
                       double *rhs, hipStream_t s);
void launch_facet_mass(const fo_ctx *c, const double *x, double *y, hipStream_t s);

// Operator of the fused CG kernels.
enum FusedKind { FUSED_ELAS = 0, FUSED_DESCENT = 1 };
// fold = false: the folded partials of a large mesh are already in c->fold
// (the launch times the tile kernel alone).
template <typename T>
int launch_tile_cg(const fo_ctx *c, int kind, const T *r, const T *dinv, const T *pin, T *pout, T *q,
                   SolveScalars *sc, int A, hipStream_t s, bool fold = true);
void launch_ir_phase(const fo_ctx *c, const double *r64, double *s2, float *r32, float *x32,
                     const float *dinv, double phase_rtol, int max_it, int fresh, hipStream_t s);
void launch_to_float(const double *a, float *b, int64_t n, hipStream_t s);

template <typename T>
void launch_elas_apply_atomic(const fo_ctx *c, const T *coords, const T *x, T *y, hipStream_t s);
void launch_elas_diag(const fo_ctx *c, double *diag, hipStream_t s);
void launch_descent_apply_atomic(const fo_ctx *c, const double *x, double *y, hipStream_t s);
void launch_descent_diag(const fo_ctx *c, double *diag, hipStream_t s);
void launch_in_boxes(const fo_ctx *c, int nbox, const double *boxes_dev, uint8_t *in0,
                     hipStream_t s);
int launch_shape_tensor(const fo_ctx *c, const double *u, int n_rhs, int64_t ld, double vol_coef,
                        double *S1, double *J, double *vol, hipStream_t s);
void launch_sd_rhs_atomic(const fo_ctx *c, double *rhs, hipStream_t s);
void launch_phigrad_atomic(const fo_ctx *c, const double *phi, double *gbuf, hipStream_t s);
void launch_phi_update(const fo_ctx *c, const double *theta, double dt, double *phi, hipStream_t s);


// tiled (deterministic) scatter
template <typename T>
int launch_elas_apply_tiled(const fo_ctx *c, const T *coords, const T *x, T *y, hipStream_t s,
                            double *dot_part = nullptr, const int32_t *done = nullptr,
                            bool skip_halo = false);
int launch_elas_diag_tiled(const fo_ctx *c, double *diag, hipStream_t s);
int launch_descent_apply_tiled(const fo_ctx *c, const double *x, double *y, hipStream_t s,
                               const int32_t *done = nullptr);
int tiled_prepare(const fo_ctx *c);
size_t tr_buffer_bytes(const fo_ctx *c);  // transport / reinitialisation work buffers
int launch_descent_diag_tiled(const fo_ctx *c, double *diag, hipStream_t s);
int launch_sd_rhs_tiled(const fo_ctx *c, double *rhs, hipStream_t s);
int launch_phigrad_tiled(const fo_ctx *c, const double *phi, double *gbuf, hipStream_t s);
void launch_facet_terms(const fo_ctx *c, const double *x, double *y, hipStream_t s);


// runtime helpers (fo_api.hip)
// Enqueues one chunk of solver kernels on the context stream: captured once
// into a HIP graph under `key` and replayed on the private stream (eager
// while kernel profiling is on).
int graph_chunk(fo_ctx *c, std::tuple<int, int, int, int> key,
                const std::function<int(hipStream_t)> &enqueue);
int elas_apply64(fo_ctx *c, const double *x, double *y, hipStream_t s);
// FP64 Jacobi-PCG of K(phi) x = b (contiguous b), solution left in c->x64.
int fp64_solve(fo_ctx *c, const double *b, const fo_solve_opts *o, fo_solve_stats *st);
// FP64 Jacobi-PCG of the scalar heat operator K x = b on the nodes where
// fixed is 0 (b and dinv zero where it is set; contiguous [n_nodes]),
// stopping on the recomputed residual; the solution is left in c->x64.
int heat_cg_solve(fo_ctx *c, const uint8_t *fixed, const double *b, const double *dinv, const fo_solve_opts *o,
                  fo_solve_stats *st);
int64_t first_phase_cap(int64_t n);

// batched multi-load path (fo_batch.hip)
int batch_setup(fo_ctx *c, int max_rhs, const double *coords, const std::vector<int32_t> &conn_t);
int batch_levelset(fo_ctx *c);
void batch_release(fo_ctx *c);
int batch_solve(fo_ctx *c, const double *b, double *u, int n_rhs, int64_t ld, const fo_solve_opts *o,
                fo_solve_stats *st);
int batch_time_apply(fo_ctx *c, int NC, int reps, double *avg_us, int op = -1);
// assembled node-block operator of the batched solves (fo_nodal.hip)
int nodal_blocks(const fo_ctx *c, int S);
int nodal_setup(fo_ctx *c, const std::vector<int32_t> &conn);
int nodal_levelset(fo_ctx *c);
// R[:, k] = B[:, k] - K(phi) X[:, k] in FP64 for the masked columns of
// [n_dofs][S] blocks (S <= 64; clamped rows 0), and per launched block and
// column the partial sum of squares of the new R (part: [*nblk][S], at most
// part_cap doubles; 0 outside the mask).  FO_ERR_ARG without blocks.
int nodal_residual64(const fo_ctx *c, int S, const double *X, const double *B, const uint8_t *mask, double *R,
                     double *part, int64_t part_cap, int *nblk, hipStream_t s);
void nodal_apply_launch(const fo_ctx *c, int NC, const float *P, float *Q, BatchCtl *ctl, const BatchCol *cols,
                        hipStream_t s);
int batch_apply_block(fo_ctx *c, int NC, const float *X, float *Y);
int batch_tune(fo_ctx *c, int n_rhs, int *best_nodes, int *best_group, double *best_us);
int batch_max_nodes(int D, int S);
void batch_apply_launch(const fo_ctx *c, int NC, const float *P, float *Q, BatchCtl *ctl, const BatchCol *cols,
                        hipStream_t s);
// block CG (fo_bcg.hip): buffers, phase-start direction, one iteration, block narrowing
size_t bcg_part_floats(int S);
int bcg_prepare();
void bcg_direction(const fo_ctx *c, const BcgBufs &B, int NP, int NS, hipStream_t s);
void bcg_iteration(const fo_ctx *c, const BcgBufs &B, int NP, int NS, hipStream_t s);
void bcg_restride(const fo_ctx *c, int sp_from, int sp_to, hipStream_t s);

}  // namespace fo

// Inverse elasticity problem (Section "Inverse problem": eqs. cost, f-prob,
// g-prob, AOmega, w-f, w-g, the adjoint problems of eqs. dL1 and dL2, and
// the shape derivative of eq. SDelast_inv) for one force-displacement pair
// (f, g).  The state u carries the traction f on Gamma_1 and is clamped on
// Gamma_0; the lifted state v (y = v + g) is clamped on the whole boundary;
// the adjoints p and q are clamped like u and v.  A = kappa in Omega and 1
// outside.  Each clamp set has its own context, and both contexts carry
// A / kappa (their ersatz value is 1 / kappa): the loads of u, p and q are
// divided by kappa, the lifted problem's load -K g is not.  All four solves
// are the contexts' state solves; the masses, the cost and the derivative
// run on the tiled scatter of the first context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "fo_internal.h"
#include "fo_launch.h"

namespace fo {

namespace {

struct InvBufs {
    double *b, *y, *w, *mw, *z, *mgz, *pack, *scal;
};

int inv_buffers(fo_ctx *c, InvBufs *o)
{
    const int64_t n = c->ndof;
    const size_t n_dbl = (size_t)(10 * n + 8);  // b, y, w, mw, z, mgz [n]; pack [4n]; scal [8]
    if (!c->inv_buf) {
        void *mem = nullptr;
        if (hipMalloc(&mem, n_dbl * sizeof(double)) != hipSuccess) return FO_ERR_NOMEM;
        c->inv_buf = mem;
        c->allocations.push_back(mem);  // released by fo_destroy
        c->bytes += n_dbl * sizeof(double);
    }
    double *m = reinterpret_cast<double *>(c->inv_buf);
    double **vec[] = {&o->b, &o->y, &o->w, &o->mw, &o->z, &o->mgz};
    for (double **q : vec) {
        *q = m;
        m += n;
    }
    o->pack = m;
    o->scal = m + 4 * n;
    return FO_OK;
}

int grid_of(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

__global__ __launch_bounds__(256) void k_scale(int64_t n, double a, const double *__restrict__ x,
                                               double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i];
}

// w = u - v - g, z = u - g.
__global__ __launch_bounds__(256) void k_inv_w(int64_t n, const double *__restrict__ u, const double *__restrict__ v,
                                               const double *__restrict__ g, double *__restrict__ w,
                                               double *__restrict__ z)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        w[i] = u[i] - v[i] - g[i];
        z[i] = u[i] - g[i];
    }
}

// Adjoint loads over kappa: bp = (-alpha M w - beta M_Gamma1 z) / kappa,
// bq = alpha M w / kappa.
__global__ __launch_bounds__(256) void k_inv_adj(int64_t n, double alpha, double beta, double rkappa,
                                                 const double *__restrict__ mw, const double *__restrict__ mgz,
                                                 double *__restrict__ bp, double *__restrict__ bq)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        bp[i] = (-alpha * mw[i] - beta * mgz[i]) * rkappa;
        bq[i] = alpha * mw[i] * rkappa;
    }
}

// J = alpha/2 w.Mw + beta/2 z.M_Gamma1 z from the two dot products.
__global__ void k_inv_cost(const double *__restrict__ dots, double alpha, double beta, double *__restrict__ J)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *J = 0.5 * alpha * dots[0] + 0.5 * beta * dots[1];
}

// pack[node][4D] = (v, p, q, g) of the node.
template <int D>
__global__ __launch_bounds__(256) void k_inv_pack(int64_t N, const double *__restrict__ v,
                                                  const double *__restrict__ p, const double *__restrict__ q,
                                                  const double *__restrict__ g, double *__restrict__ pack)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x) {
        double *o = pack + k * 4 * D;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            o[i] = v[k * D + i];
            o[D + i] = p[k * D + i];
            o[2 * D + i] = q[k * D + i];
            o[3 * D + i] = g[k * D + i];
        }
    }
}

int worse(int a, int b)
{
    if (a < 0 || b < 0) return std::min(a, b);
    return std::max(a, b);
}

bool kappa_matches(const fo_ctx *c, double kappa) { return std::fabs(kappa * c->ersatz - 1.0) <= 1e-12; }

}  // namespace

}  // namespace fo

using namespace fo;

extern "C" {

int fo_inverse_states(fo_ctx *cf, fo_ctx *cg, const double *phi, const double *f, const double *g, double kappa,
                      double alpha, double beta, const fo_solve_opts *o, double *u, double *v, double *p, double *q,
                      double *J, fo_solve_stats *st)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!cf || !cg || cf == cg || !phi || !f || !g || !o || !u || !v || !p || !q || !J) return FO_ERR_ARG;
    if (cf->dim != cg->dim || cf->N != cg->N || cf->E != cg->E || cf->device != cg->device) return FO_ERR_ARG;
    if (!(kappa > 0.0) || !(alpha >= 0.0) || !(beta >= 0.0) || !kappa_matches(cf, kappa) ||
        !kappa_matches(cg, kappa))
        return FO_ERR_ARG;
    if (cf->scatter != FO_SCATTER_TILED || cf->tiles.n_tiles <= 0) return FO_ERR_STATE;
    InvBufs B;
    FO_TRY(inv_buffers(cf, &B));
    FO_TRY(fo_set_levelset(cf, phi));
    FO_TRY(fo_set_levelset(cg, phi));
    hipStream_t s = cf->stream;
    const int64_t n = cf->ndof;
    const int ng = grid_of(n);
    fo_solve_stats acc{FO_OK, 0, 0, 0.0, 0.0};
    int status = FO_OK;
    auto solve = [&](fo_ctx *c, const double *b, double *x) -> int {
        fo_solve_stats one{};
        const int rc = fo_state_solve(c, b, x, 1, 1, o, &one);
        if (rc < 0 && rc != FO_ERR_BREAKDOWN) return rc;
        acc.iters_inner += one.iters_inner;
        acc.iters_outer += one.iters_outer;
        acc.rel_res = std::max(acc.rel_res, one.rel_res);
        status = worse(status, rc);
        return FO_OK;
    };
    // u: K u = f on the Gamma_0-free unknowns
    hipLaunchKernelGGL(k_scale, dim3(ng), dim3(256), 0, s, n, 1.0 / kappa, f, B.b);
    FO_HIP(hipStreamSynchronize(s));
    FO_TRY(solve(cf, B.b, u));
    // v: K v = -K g on the interior unknowns (the full product K g)
    FO_TRY(launch_elas_apply_free(cf, g, B.y, s));
    hipLaunchKernelGGL(k_scale, dim3(ng), dim3(256), 0, s, n, -1.0, B.y, B.b);
    FO_HIP(hipStreamSynchronize(s));
    FO_TRY(solve(cg, B.b, v));
    // cost and the adjoint loads
    hipLaunchKernelGGL(k_inv_w, dim3(ng), dim3(256), 0, s, n, u, v, g, B.w, B.z);
    FO_TRY(launch_vec_mass(cf, B.w, B.mw, s));
    launch_facet_mass(cf, B.z, B.mgz, s);
    const int nb = red_blocks(n);
    launch_dots<double>(2, B.w, B.mw, B.z, B.mgz, nullptr, nullptr, n, cf->partials, nb, s);
    launch_finish_dots(cf->partials, nb, 2, B.scal, s);
    hipLaunchKernelGGL(k_inv_cost, dim3(1), dim3(64), 0, s, B.scal, alpha, beta, J);
    hipLaunchKernelGGL(k_inv_adj, dim3(ng), dim3(256), 0, s, n, alpha, beta, 1.0 / kappa, B.mw, B.mgz, B.b, B.y);
    FO_HIP(hipStreamSynchronize(s));
    // p (clamped on Gamma_0) and q (clamped on the whole boundary)
    FO_TRY(solve(cf, B.b, p));
    FO_TRY(solve(cg, B.y, q));
    FO_HIP(hipGetLastError());
    acc.status = status;
    acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = acc;
    return status;
}

int fo_inverse_derivative(fo_ctx *cf, const double *u, const double *v, const double *p, const double *q,
                          const double *g, double kappa, double alpha, double *rhs)
{
    if (!cf || !u || !v || !p || !q || !g || !rhs || !(kappa > 0.0) || !(alpha >= 0.0) || !kappa_matches(cf, kappa))
        return FO_ERR_ARG;
    if (cf->scatter != FO_SCATTER_TILED || cf->tiles.n_tiles <= 0 || !cf->have_phi) return FO_ERR_STATE;
    InvBufs B;
    FO_TRY(inv_buffers(cf, &B));
    hipStream_t s = cf->stream;
    const int ng = grid_of(cf->N);
    if (cf->dim == 2)
        hipLaunchKernelGGL(k_inv_pack<2>, dim3(ng), dim3(256), 0, s, cf->N, v, p, q, g, B.pack);
    else
        hipLaunchKernelGGL(k_inv_pack<3>, dim3(ng), dim3(256), 0, s, cf->N, v, p, q, g, B.pack);
    FO_TRY(launch_inverse_rhs(cf, u, B.pack, kappa, alpha, rhs, s));
    FO_HIP(hipStreamSynchronize(s));
    return FO_OK;
}

}  // extern "C"

// Inverse elasticity problem (Section "Inverse problem": eqs. cost, f-prob,
// g-prob, AOmega, w-f, w-g, the adjoint problems of eqs. dL1 and dL2, and
// the shape derivative of eq. SDelast_inv) for one or several
// force-displacement pairs (f_k, g_k); the cost and the derivative of
// several pairs are the sums over the pairs.  The state u carries the
// traction f on Gamma_1 and is clamped on Gamma_0; the lifted state v
// (y = v + g) is clamped on the whole boundary; the adjoints p and q are
// clamped like u and v.  A = kappa in Omega and 1 outside.  Each clamp set
// has its own context, and both contexts carry A / kappa (their ersatz value
// is 1 / kappa): the loads of u, p and q are divided by kappa, the lifted
// problem's load -K g is not.  All four solves are the contexts' state
// solves, pair by pair (the batched multi-column path pays off only from
// several dozen columns); the masses, the cost and the derivative also run
// pair by pair, on the tiled scatter of the first context.  Pair k of an
// [n_dofs][ld] array is column k.  When the two contexts run on different
// streams, the solves of u and v (then of p and q) run at the same time, one
// of them from a helper host thread: each solve alone leaves CUs idle during
// its update kernels and the last round of its operator kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <thread>

#include "fo_internal.h"
#include "fo_launch.h"

namespace fo {

namespace {

// Strided arrays hold the pairs (b, y: [n][ld]); the others are one column.
struct InvBufs {
    double *b, *y, *t0, *t1, *t2, *t3, *pack, *scal;
};

int inv_buffers(fo_ctx *c, int64_t ld, InvBufs *o)
{
    const int64_t n = c->ndof;
    const size_t n_dbl = (size_t)(2 * n * ld + 8 * n + 8);  // b, y [n][ld]; t0..t3 [n]; pack [4n]; scal [8]
    if (!c->inv_buf || c->inv_cap < n_dbl) {
        if (c->inv_buf) {
            (void)fo::wait_stream(c->stream);
            (void)hipFree(c->inv_buf);
            auto it = std::find(c->allocations.begin(), c->allocations.end(), c->inv_buf);
            if (it != c->allocations.end()) c->allocations.erase(it);
            c->bytes -= c->inv_cap * sizeof(double);
            c->inv_buf = nullptr;
            c->inv_cap = 0;
        }
        void *mem = nullptr;
        if (fo::device_malloc(&mem, n_dbl * sizeof(double)) != hipSuccess) return FO_ERR_NOMEM;
        c->inv_buf = mem;
        c->inv_cap = n_dbl;
        c->allocations.push_back(mem);  // released by fo_destroy
        c->bytes += n_dbl * sizeof(double);
    }
    double *m = reinterpret_cast<double *>(c->inv_buf);
    o->b = m;
    o->y = m + n * ld;
    m += 2 * n * ld;
    double **vec[] = {&o->t0, &o->t1, &o->t2, &o->t3};
    for (double **q : vec) {
        *q = m;
        m += n;
    }
    o->pack = m;
    o->scal = m + 4 * n;
    return FO_OK;
}

int grid_of(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

// y[i ld + k] = a x[i ld + k] for the first np columns.
__global__ __launch_bounds__(256) void k_scale_cols(int64_t n, int64_t ld, int np, double a,
                                                    const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t tot = n * np;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = j / np, k = j - i * np;
        y[i * ld + k] = a * x[i * ld + k];
    }
}

// Column copies between a strided column (stride ld) and a contiguous vector:
// y_col = a x (k_put) or y = x_col (k_get).
__global__ __launch_bounds__(256) void k_put(int64_t n, int64_t ld, double a, const double *__restrict__ x,
                                             double *__restrict__ ycol)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        ycol[i * ld] = a * x[i];
}

__global__ __launch_bounds__(256) void k_get(int64_t n, int64_t ld, const double *__restrict__ xcol,
                                             double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = xcol[i * ld];
}

// w = u - v - g, z = u - g from one column of each (stride ld).
__global__ __launch_bounds__(256) void k_inv_w(int64_t n, int64_t ld, const double *__restrict__ u,
                                               const double *__restrict__ v, const double *__restrict__ g,
                                               double *__restrict__ w, double *__restrict__ z)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ui = u[i * ld], gi = g[i * ld];
        w[i] = ui - v[i * ld] - gi;
        z[i] = ui - gi;
    }
}

// Adjoint loads over kappa into one column of each (stride ld):
// bp = (-alpha M w - beta M_Gamma1 z) / kappa, bq = alpha M w / kappa.
__global__ __launch_bounds__(256) void k_inv_adj(int64_t n, int64_t ld, double alpha, double beta, double rkappa,
                                                 const double *__restrict__ mw, const double *__restrict__ mgz,
                                                 double *__restrict__ bp, double *__restrict__ bq)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        bp[i * ld] = (-alpha * mw[i] - beta * mgz[i]) * rkappa;
        bq[i * ld] = alpha * mw[i] * rkappa;
    }
}

// J = alpha/2 w.Mw + beta/2 z.M_Gamma1 z from the two dot products.
__global__ void k_inv_cost(const double *__restrict__ dots, double alpha, double beta, double *__restrict__ J)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *J = 0.5 * alpha * dots[0] + 0.5 * beta * dots[1];
}

// pack[node][4D] = (v, p, q, g) of the node, from one column of each.
template <int D>
__global__ __launch_bounds__(256) void k_inv_pack(int64_t N, int64_t ld, const double *__restrict__ v,
                                                  const double *__restrict__ p, const double *__restrict__ q,
                                                  const double *__restrict__ g, double *__restrict__ pack)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x) {
        double *o = pack + k * 4 * D;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t j = (k * D + i) * ld;
            o[i] = v[j];
            o[D + i] = p[j];
            o[2 * D + i] = q[j];
            o[3 * D + i] = g[j];
        }
    }
}

int worse(int a, int b)
{
    if (a < 0 || b < 0) return std::min(a, b);
    return std::max(a, b);
}

bool kappa_matches(const fo_ctx *c, double kappa) { return std::fabs(kappa * c->ersatz - 1.0) <= 1e-12; }

// The state solves of n_pairs columns (stride ld) of b on c, one after the
// other; iterations and the worst status accumulate into acc.
int solve_pairs(fo_ctx *c, const double *b, double *x, int n_pairs, int64_t ld, const fo_solve_opts *o,
                fo_solve_stats *acc)
{
    for (int k = 0; k < n_pairs; ++k) {
        fo_solve_stats one{};
        const int rc = fo_state_solve(c, b + k, x + k, 1, ld, o, &one);
        if (rc < 0 && rc != FO_ERR_BREAKDOWN) return rc;
        acc->iters_inner += one.iters_inner;
        acc->iters_outer += one.iters_outer;
        acc->rel_res = std::max(acc->rel_res, one.rel_res);
        acc->status = worse(acc->status, rc);
    }
    return FO_OK;
}

// Solves on cf (bf -> xf) and on cg (bg -> xg): concurrently from a helper
// thread when the contexts have their own streams, else in turn.
int solve_both(fo_ctx *cf, const double *bf, double *xf, fo_ctx *cg, const double *bg, double *xg, int n_pairs,
               int64_t ld, const fo_solve_opts *o, fo_solve_stats *acc)
{
    fo_solve_stats af{FO_OK, 0, 0, 0.0, 0.0}, ag{FO_OK, 0, 0, 0.0, 0.0};
    int rf = FO_OK, rg = FO_OK;
    std::thread t;
    if (cf->stream != cg->stream) {
        try {  // no exception may cross the C ABI: without a thread, solve in turn
            t = std::thread([&]() {
                if (hipSetDevice(cg->device) != hipSuccess) {
                    rg = FO_ERR_HIP;
                    return;
                }
                rg = solve_pairs(cg, bg, xg, n_pairs, ld, o, &ag);
            });
        } catch (...) {
        }
    }
    if (t.joinable()) {
        rf = solve_pairs(cf, bf, xf, n_pairs, ld, o, &af);
        t.join();
    } else {
        rf = solve_pairs(cf, bf, xf, n_pairs, ld, o, &af);
        if (rf == FO_OK) rg = solve_pairs(cg, bg, xg, n_pairs, ld, o, &ag);
    }
    if (rf != FO_OK) return rf;
    if (rg != FO_OK) return rg;
    for (const fo_solve_stats *a : {&af, &ag}) {
        acc->iters_inner += a->iters_inner;
        acc->iters_outer += a->iters_outer;
        acc->rel_res = std::max(acc->rel_res, a->rel_res);
        acc->status = worse(acc->status, a->status);
    }
    return FO_OK;
}

}  // namespace

}  // namespace fo

using namespace fo;

extern "C" {

int fo_inverse_states(fo_ctx *cf, fo_ctx *cg, const double *phi, int32_t n_pairs, int64_t ld, const double *f,
                      const double *g, double kappa, double alpha, double beta, const fo_solve_opts *o, double *u,
                      double *v, double *p, double *q, double *J, fo_solve_stats *st)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!cf || !cg || cf == cg || !phi || !f || !g || !o || !u || !v || !p || !q || !J) return FO_ERR_ARG;
    if (cf->dim != cg->dim || cf->N != cg->N || cf->E != cg->E || cf->device != cg->device) return FO_ERR_ARG;
    if (n_pairs < 1 || ld < n_pairs) return FO_ERR_ARG;
    if (!(kappa > 0.0) || !(alpha >= 0.0) || !(beta >= 0.0) || !kappa_matches(cf, kappa) ||
        !kappa_matches(cg, kappa))
        return FO_ERR_ARG;
    if (cf->scatter != FO_SCATTER_TILED || cf->tiles.n_tiles <= 0) return FO_ERR_STATE;
    InvBufs B;
    FO_TRY(inv_buffers(cf, ld, &B));
    FO_TRY(fo_set_levelset(cf, phi));
    FO_TRY(fo_set_levelset(cg, phi));
    hipStream_t s = cf->stream;
    const int64_t n = cf->ndof;
    const int ng = grid_of(n);
    fo_solve_stats acc{FO_OK, 0, 0, 0.0, 0.0};
    // loads of u (f / kappa, in b) and of v (-K g, in y; the full product K g)
    hipLaunchKernelGGL(k_scale_cols, dim3(grid_of(n * n_pairs)), dim3(256), 0, s, n, ld, (int)n_pairs, 1.0 / kappa,
                       f, B.b);
    for (int k = 0; k < n_pairs; ++k) {
        hipLaunchKernelGGL(k_get, dim3(ng), dim3(256), 0, s, n, ld, g + k, B.t0);
        FO_TRY(launch_elas_apply_free(cf, B.t0, B.t1, s));
        hipLaunchKernelGGL(k_put, dim3(ng), dim3(256), 0, s, n, ld, -1.0, B.t1, B.y + k);
    }
    FO_HIP(fo::wait_stream(s));
    // u (clamped on Gamma_0) and v (clamped on the whole boundary)
    FO_TRY(solve_both(cf, B.b, u, cg, B.y, v, n_pairs, ld, o, &acc));
    // cost and the adjoint loads, pair by pair
    const int nb = red_blocks(n);
    for (int k = 0; k < n_pairs; ++k) {
        hipLaunchKernelGGL(k_inv_w, dim3(ng), dim3(256), 0, s, n, ld, u + k, v + k, g + k, B.t0, B.t1);
        FO_TRY(launch_vec_mass(cf, B.t0, B.t2, s));
        launch_facet_mass(cf, B.t1, B.t3, s);
        launch_dots<double>(2, B.t0, B.t2, B.t1, B.t3, nullptr, nullptr, n, cf->partials, nb, s);
        launch_finish_dots(cf->partials, nb, 2, B.scal, s);
        hipLaunchKernelGGL(k_inv_cost, dim3(1), dim3(64), 0, s, B.scal, alpha, beta, J + k);
        hipLaunchKernelGGL(k_inv_adj, dim3(ng), dim3(256), 0, s, n, ld, alpha, beta, 1.0 / kappa, B.t2, B.t3,
                           B.b + k, B.y + k);
    }
    FO_HIP(fo::wait_stream(s));
    // p (clamped on Gamma_0) and q (clamped on the whole boundary)
    FO_TRY(solve_both(cf, B.b, p, cg, B.y, q, n_pairs, ld, o, &acc));
    FO_HIP(hipGetLastError());
    acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = acc;
    return acc.status;
}

int fo_inverse_derivative(fo_ctx *cf, int32_t n_pairs, int64_t ld, const double *u, const double *v,
                          const double *p, const double *q, const double *g, double kappa, double alpha, double *rhs)
{
    if (!cf || !u || !v || !p || !q || !g || !rhs || !(kappa > 0.0) || !(alpha >= 0.0) || !kappa_matches(cf, kappa))
        return FO_ERR_ARG;
    if (n_pairs < 1 || ld < n_pairs) return FO_ERR_ARG;
    if (cf->scatter != FO_SCATTER_TILED || cf->tiles.n_tiles <= 0 || !cf->have_phi) return FO_ERR_STATE;
    InvBufs B;
    FO_TRY(inv_buffers(cf, 1, &B));
    hipStream_t s = cf->stream;
    const int ng = grid_of(cf->N);
    for (int k = 0; k < n_pairs; ++k) {
        if (cf->dim == 2)
            hipLaunchKernelGGL(k_inv_pack<2>, dim3(ng), dim3(256), 0, s, cf->N, ld, v + k, p + k, q + k, g + k,
                               B.pack);
        else
            hipLaunchKernelGGL(k_inv_pack<3>, dim3(ng), dim3(256), 0, s, cf->N, ld, v + k, p + k, q + k, g + k,
                               B.pack);
        if (ld > 1) hipLaunchKernelGGL(k_get, dim3(grid_of(cf->ndof)), dim3(256), 0, s, cf->ndof, ld, u + k, B.t0);
        // the sum over the pairs in pair order
        FO_TRY(launch_inverse_rhs(cf, ld > 1 ? B.t0 : u, B.pack, kappa, alpha, k == 0 ? rhs : B.t1, s));
        if (k > 0) launch_add64(rhs, B.t1, cf->ndof, s);
    }
    FO_HIP(fo::wait_stream(s));
    return FO_OK;
}

}  // extern "C"

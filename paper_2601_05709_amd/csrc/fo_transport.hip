// Transport step of the level set (Section "Transport equation", eqs.
// transport, weak_transport, tau_lv): `steps` Crank-Nicolson steps of the
// Petrov-Galerkin form with test functions psi + tau theta . grad psi and
// optional h^2 diffusion.  Each step solves L phi' = R phi (L, R from
// TransportOp with sdt = +dt / -dt, the same for every step) by
// Jacobi-preconditioned BiCGStab in FP64, from phi, with the Krylov scalars
// on the device.  The host polls the residual every few iterations and
// checks the recomputed residual before it accepts a step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>

#include "fo_internal.h"
#include "fo_launch.h"
#include "fo_reduce.h"

namespace fo {

namespace {

// Device scalars of one BiCGStab solve.
struct TrScal {
    double rho, alpha, omega, beta;
    double rho_new, rv, ts, tt, rr, bb;
    int32_t bad;  // a division by zero or a non-finite coefficient: restart
    int32_t pad;
};

// Element-mean velocity and tau = (1/2) (dt^-2 + |theta|^2 / h^2)^(-1/2).
template <int D>
__global__ __launch_bounds__(256) void k_tr_coef(const int32_t *__restrict__ conn, int64_t E,
                                                 const double *__restrict__ theta, double dt, double h2,
                                                 double *__restrict__ coef)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
         e += (int64_t)gridDim.x * blockDim.x) {
        double th[D];
#pragma unroll
        for (int i = 0; i < D; ++i) th[i] = 0.0;
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            const int64_t node = conn[(int64_t)a * E + e];
#pragma unroll
            for (int i = 0; i < D; ++i) th[i] += theta[node * D + i];
        }
        double t2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            th[i] /= (double)(D + 1);
            t2 += th[i] * th[i];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) coef[e * 4 + i] = i < D ? th[i] : 0.0;
        coef[e * 4 + 3] = 0.5 / sqrt(1.0 / (dt * dt) + t2 / h2);
    }
}

// r = b - t; rh = r; p = v = 0
__global__ __launch_bounds__(256) void k_tr_start(const double *__restrict__ b, const double *__restrict__ t,
                                                  double *__restrict__ r, double *__restrict__ rh,
                                                  double *__restrict__ p, double *__restrict__ v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = b[i] - t[i];
        r[i] = ri;
        rh[i] = ri;
        p[i] = 0.0;
        v[i] = 0.0;
    }
}

__global__ void k_tr_reset(TrScal *sc)
{
    sc->rho = sc->alpha = sc->omega = 1.0;
    sc->bad = 0;
}

__device__ __forceinline__ bool fin(double x) { return x == x && x != INFINITY && x != -INFINITY; }

// beta = (rho_new / rho) (alpha / omega); rho = rho_new
__global__ void k_tr_beta(TrScal *sc)
{
    const double rn = sc->rho_new;
    if (!(rn != 0.0) || !fin(rn) || sc->rho == 0.0 || sc->omega == 0.0) {
        sc->bad = 1;
        sc->beta = 0.0;
        return;
    }
    sc->beta = (rn / sc->rho) * (sc->alpha / sc->omega);
    sc->rho = rn;
}

__global__ void k_tr_alpha(TrScal *sc)
{
    if (sc->bad) return;
    const double rv = sc->rv;
    if (!(rv != 0.0) || !fin(rv)) {
        sc->bad = 1;
        return;
    }
    sc->alpha = sc->rho / rv;
}

__global__ void k_tr_omega(TrScal *sc)
{
    if (sc->bad) return;
    const double tt = sc->tt;
    if (!(tt > 0.0) || !fin(tt) || !fin(sc->ts)) {
        sc->bad = 1;
        return;
    }
    sc->omega = sc->ts / tt;
}

// p = r + beta (p - omega v); y = D^-1 p
__global__ __launch_bounds__(256) void k_tr_p(const TrScal *sc, const double *__restrict__ r, double *__restrict__ p,
                                              const double *__restrict__ v, const double *__restrict__ dinv,
                                              double *__restrict__ y, int64_t n)
{
    if (sc->bad) return;
    const double beta = sc->beta, omega = sc->omega;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double pi = r[i] + beta * (p[i] - omega * v[i]);
        p[i] = pi;
        y[i] = dinv[i] * pi;
    }
}

// x += alpha y; s = r - alpha v; z = D^-1 s
__global__ __launch_bounds__(256) void k_tr_s(const TrScal *sc, double *__restrict__ x, const double *__restrict__ y,
                                              const double *__restrict__ r, const double *__restrict__ v,
                                              const double *__restrict__ dinv, double *__restrict__ s,
                                              double *__restrict__ z, int64_t n)
{
    if (sc->bad) return;
    const double alpha = sc->alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * y[i];
        const double si = r[i] - alpha * v[i];
        s[i] = si;
        z[i] = dinv[i] * si;
    }
}

// x += omega z; r = s - omega t
__global__ __launch_bounds__(256) void k_tr_xr(const TrScal *sc, double *__restrict__ x, const double *__restrict__ z,
                                               const double *__restrict__ s, const double *__restrict__ t,
                                               double *__restrict__ r, int64_t n)
{
    if (sc->bad) return;
    const double omega = sc->omega;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += omega * z[i];
        r[i] = s[i] - omega * t[i];
    }
}

int blocks_for(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096); }

}  // namespace

}  // namespace fo

using namespace fo;

namespace {

// Transport work buffers of a context, allocated on first use.
struct TrBufs {
    double *coef, *b, *x, *r, *rh, *p, *v, *y, *s, *z, *t, *dinv;
    TrScal *sc;
};

int tr_buffers(fo_ctx *c, TrBufs *o)
{
    if (!c->tr_buf) {
        const int64_t N = c->N, E = c->E;
        const size_t bytes = (size_t)(E * 4 + 11 * N) * sizeof(double) + 256;
        void *mem = nullptr;
        if (hipMalloc(&mem, bytes) != hipSuccess) return FO_ERR_NOMEM;
        c->tr_buf = mem;
        c->allocations.push_back(mem);  // released by fo_destroy
        c->bytes += bytes;
    }
    double *m = reinterpret_cast<double *>(c->tr_buf);
    const int64_t N = c->N;
    o->coef = m;
    m += c->E * 4;
    double **vec[] = {&o->b, &o->x, &o->r, &o->rh, &o->p, &o->v, &o->y, &o->s, &o->z, &o->t, &o->dinv};
    for (double **q : vec) {
        *q = m;
        m += N;
    }
    o->sc = reinterpret_cast<TrScal *>(m);
    return FO_OK;
}

}  // namespace

extern "C" {

int fo_transport(fo_ctx *c, const double *theta, double dt, int32_t steps, int32_t smooth, double *phi,
                 const fo_solve_opts *o, fo_solve_stats *st)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !theta || !phi || !o || !(dt > 0.0) || !(dt < INFINITY) || steps < 0 || !(o->rtol > 0.0) ||
        o->max_iter <= 0)
        return FO_ERR_ARG;
    if (c->scatter != FO_SCATTER_TILED || c->tiles.n_tiles <= 0) return FO_ERR_STATE;
    TrBufs B;
    FO_TRY(tr_buffers(c, &B));
    hipStream_t s = c->stream;
    const int64_t N = c->N;
    const double h2 = c->transport_h2;
    const double h2e = smooth ? h2 : 0.0;
    const int nb = blocks_for(N), red = red_blocks(N);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_tr_coef<2>, dim3(blocks_for(c->E)), dim3(256), 0, s, c->conn, c->E, theta, dt, h2,
                           B.coef);
    else
        hipLaunchKernelGGL(k_tr_coef<3>, dim3(blocks_for(c->E)), dim3(256), 0, s, c->conn, c->E, theta, dt, h2,
                           B.coef);
    FO_TRY(launch_transport_diag(c, B.coef, dt, h2e, B.dinv, s));
    launch_invert_diag<double>(B.dinv, nullptr, N, B.dinv, s);
    TrScal *sc = B.sc;
    TrScal h{};
    auto read = [&]() -> int {
        FO_HIP(hipMemcpyAsync(&h, sc, sizeof(TrScal), hipMemcpyDeviceToHost, s));
        FO_HIP(hipStreamSynchronize(s));
        return FO_OK;
    };
    auto dot = [&](int npair, const double *a0, const double *b0, const double *a1, const double *b1,
                   double *out) {
        launch_dots<double>(npair, a0, b0, a1, b1, nullptr, nullptr, N, c->partials, red, s);
        launch_finish_dots(c->partials, red, npair, out, s);
    };
    int64_t iters = 0;
    double worst = 0.0;  // largest accepted relative residual
    int status = FO_OK;
    const int poll_every = 4;
    for (int step = 0; step < steps && status == FO_OK; ++step) {
        FO_TRY(launch_transport_apply(c, B.coef, -dt, h2e, phi, B.b, s));  // b = R phi
        FO_HIP(hipMemcpyAsync(B.x, phi, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        dot(1, B.b, B.b, nullptr, nullptr, &sc->bb);
        bool ok = false;
        int64_t its = 0;  // operator applications of this step
        double rel = 0.0;
        for (int restart = 0; restart < 50 && !ok; ++restart) {
            FO_TRY(launch_transport_apply(c, B.coef, dt, h2e, B.x, B.t, s));  // t = L x
            if (restart > 0) ++its;
            hipLaunchKernelGGL(k_tr_start, dim3(nb), dim3(256), 0, s, B.b, B.t, B.r, B.rh, B.p, B.v, N);
            hipLaunchKernelGGL(k_tr_reset, dim3(1), dim3(1), 0, s, sc);
            dot(1, B.r, B.r, nullptr, nullptr, &sc->rr);
            FO_TRY(read());
            const double target = o->rtol * std::sqrt(h.bb);
            rel = h.bb > 0.0 ? std::sqrt(h.rr / h.bb) : 0.0;
            if (!(h.rr == h.rr)) {
                status = FO_ERR_BREAKDOWN;
                break;
            }
            if (std::sqrt(h.rr) <= target) {
                ok = true;
                break;
            }
            if (its >= o->max_iter) break;
            for (int k = 0; its < o->max_iter; ++k) {
                dot(1, B.rh, B.r, nullptr, nullptr, &sc->rho_new);
                hipLaunchKernelGGL(k_tr_beta, dim3(1), dim3(1), 0, s, sc);
                hipLaunchKernelGGL(k_tr_p, dim3(nb), dim3(256), 0, s, sc, B.r, B.p, B.v, B.dinv, B.y, N);
                FO_TRY(launch_transport_apply(c, B.coef, dt, h2e, B.y, B.v, s));  // v = L y
                dot(1, B.rh, B.v, nullptr, nullptr, &sc->rv);
                hipLaunchKernelGGL(k_tr_alpha, dim3(1), dim3(1), 0, s, sc);
                hipLaunchKernelGGL(k_tr_s, dim3(nb), dim3(256), 0, s, sc, B.x, B.y, B.r, B.v, B.dinv, B.s, B.z, N);
                FO_TRY(launch_transport_apply(c, B.coef, dt, h2e, B.z, B.t, s));  // t = L z
                dot(2, B.t, B.s, B.t, B.t, &sc->ts);  // t.s and t.t (adjacent fields)
                hipLaunchKernelGGL(k_tr_omega, dim3(1), dim3(1), 0, s, sc);
                hipLaunchKernelGGL(k_tr_xr, dim3(nb), dim3(256), 0, s, sc, B.x, B.z, B.s, B.t, B.r, N);
                dot(1, B.r, B.r, nullptr, nullptr, &sc->rr);
                its += 2;
                if ((k + 1) % poll_every == 0 || its >= o->max_iter) {
                    FO_TRY(read());
                    if (h.bad || !(h.rr == h.rr) || std::sqrt(h.rr) <= target) break;
                }
            }
            // the next pass recomputes b - L x and accepts the step or restarts
        }
        iters += its;
        worst = std::max(worst, rel);
        if (status == FO_OK && !ok) status = FO_NOT_CONVERGED;
        FO_HIP(hipMemcpyAsync(phi, B.x, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    FO_HIP(hipStreamSynchronize(s));
    if (st) {
        st->status = status;
        st->iters_inner = (int32_t)std::min<int64_t>(iters, INT32_MAX);
        st->iters_outer = steps;
        st->rel_res = worst;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

}  // extern "C"

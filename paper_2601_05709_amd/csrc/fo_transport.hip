// Transport step of the level set (Section "Transport equation", eqs.
// transport, weak_transport, tau_lv): `steps` Crank-Nicolson steps of the
// Petrov-Galerkin form with test functions psi + tau theta . grad psi and
// optional h^2 diffusion.  Each step solves L phi' = R phi (L, R from
// TransportOp with +dt / -dt, the same for every step).  Reinitialisation
// of the level set (Section "Other implementation aspects", eqs. HJ,
// grad_H, weak_HJ): pseudo-time steps of the diffusive Eikonal equation,
// each solving Lhat varphi' = rhs (ReinitOp, ReinitRhsOp), explicit Euler
// first and Adams-Bashforth 2 after it.  The heat-conduction model's state
// (Section "Heat conduction": scalar P1 stiffness, u = 0 on Gamma_0) is SPD
// and goes to the library's FP64 Jacobi-PCG instead; its entry points live
// here with the rest of the scalar P1 work.
//
// Both solve with Jacobi-preconditioned BiCGStab in FP64 from the previous
// iterate.  The Krylov scalars stay on the device: every block of a vector
// kernel sums the dot-product partials of the kernel before it in the same
// fixed order, so all blocks take the same coefficients and the same stop
// decision, and a device stop flag turns the rest of a launched chunk into
// no-ops.  Chunks of iterations are replayed as graphs; the host reads the
// flag once per batch of chunks (sized from the previous step's count) and
// checks the recomputed residual b - A x before it accepts a step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <tuple>

#include "fo_internal.h"
#include "fo_launch.h"
#include "fo_reduce.h"

namespace fo {

namespace {

// Device state of one BiCGStab pass.  Each field is written by block 0 of one
// kernel and read only by later kernels (rho_prev / rho_cur are separate so
// that no kernel reads a field it writes); the flag only ever goes from 0 to
// a stop code, and every block that sees it set would have set it itself.
struct TrScal {
    double rho_prev, rho_cur, alpha, omega;
    double bb;       // |b|^2
    double target2;  // (rtol |b|)^2
    double rr;       // |r|^2 at the last check
    int32_t flag;    // TR_RUN or a stop code
    int32_t its;     // operator applications of this pass
    int32_t max_its; // applications allowed in this pass
    int32_t pad;
};

enum : int32_t { TR_RUN = 0, TR_CONVERGED = 1, TR_RESTART = 2, TR_LIMIT = 3, TR_NAN = 4 };

// Step parameters of TransportOp: dt, -dt, h2 of the diffusion, h2 of tau,
// 1 / dt^2.
__global__ void k_tr_par(double *par, double dt, double h2e, double h2)
{
    par[0] = dt;
    par[1] = -dt;
    par[2] = h2e;
    par[3] = h2;
    par[4] = 1.0 / (dt * dt);
}

__device__ __forceinline__ bool fin(double x) { return x == x && x != INFINITY && x != -INFINITY; }

// Sums of one or two partial arrays [nb], the same in every thread and block.
__device__ __forceinline__ void sum_parts(const double *pa, const double *pb, int nb, double *bc, double &a,
                                          double &b)
{
    if (threadIdx.x < 64) {
        const double sa = wave0_sum_partials(pa, nb);
        const double sb = pb ? wave0_sum_partials(pb, nb) : 0.0;
        if (threadIdx.x == 0) {
            bc[0] = sa;
            bc[1] = sb;
        }
    }
    __syncthreads();
    a = bc[0];
    b = bc[1];
}

// Block sums of two per-thread values into part[blockIdx.x], part[nb + blockIdx.x].
__device__ __forceinline__ void put_parts(double a, double b, double *part, int nb, double *lds /*[32]*/)
{
    block_sum2_any(a, b, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[nb + blockIdx.x] = b;
    }
}

// r = b - t; rh = r; p = v = 0; partials r.r and rh.r (= r.r) into prr.
__global__ __launch_bounds__(256) void k_trs_start(const double *__restrict__ b, const double *__restrict__ t,
                                                   double *__restrict__ r, double *__restrict__ rh,
                                                   double *__restrict__ p, double *__restrict__ v,
                                                   double *__restrict__ prr, int nb, int64_t n)
{
    __shared__ double lds[32];
    double rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = b[i] - t[i];
        r[i] = ri;
        rh[i] = ri;
        p[i] = 0.0;
        v[i] = 0.0;
        rr += ri * ri;
    }
    put_parts(rr, rr, prr, nb, lds);
}

// Start of a pass (one block of 64 threads): rho = alpha = omega = 1, the
// residual |r|^2 from the start partials and the convergence test.
__global__ __launch_bounds__(64) void k_trs_check(TrScal *sc, const double *__restrict__ prr, int nb, double rtol,
                                                  int32_t max_its)
{
    const double rr = wave0_sum_partials(prr, nb);
    if (threadIdx.x == 0) {
        const double target2 = rtol * rtol * sc->bb;
        sc->rho_prev = sc->alpha = sc->omega = 1.0;
        sc->rho_cur = 0.0;
        sc->rr = rr;
        sc->target2 = target2;
        sc->its = 0;
        sc->max_its = max_its;
        sc->flag = !fin(rr) ? TR_NAN : rr <= target2 ? TR_CONVERGED : TR_RUN;
    }
}

// Iteration start: |r|^2 and rho = rh.r from prr; stop on convergence, the
// iteration limit or a breakdown; else beta = (rho / rho_prev)(alpha / omega),
// p = r + beta (p - omega v), y = D^-1 p.
__global__ __launch_bounds__(256) void k_trs_p(TrScal *sc, const double *__restrict__ prr, int nb,
                                               const double *__restrict__ r, double *__restrict__ p,
                                               const double *__restrict__ v, const double *__restrict__ dinv,
                                               double *__restrict__ y, int64_t n)
{
    __shared__ double bc[2];
    if (sc->flag) return;
    double rr, rho;
    sum_parts(prr, prr + nb, nb, bc, rr, rho);
    const double rho_prev = sc->rho_prev, alpha = sc->alpha, omega = sc->omega;
    int32_t flag = TR_RUN;
    if (!fin(rr))
        flag = TR_NAN;
    else if (rr <= sc->target2)
        flag = TR_CONVERGED;
    else if (sc->its >= sc->max_its)
        flag = TR_LIMIT;
    else if (!(rho != 0.0) || !fin(rho) || rho_prev == 0.0 || omega == 0.0)
        flag = TR_RESTART;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rr = rr;
        sc->rho_cur = rho;
        if (flag) sc->flag = flag;
    }
    if (flag) return;
    const double beta = (rho / rho_prev) * (alpha / omega);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double pi = r[i] + beta * (p[i] - omega * v[i]);
        p[i] = pi;
        y[i] = dinv[i] * pi;
    }
}

// Partials of a0.b0 and a1.b1 (b1 == nullptr: the second is 0).
__global__ __launch_bounds__(256) void k_trs_dot(const TrScal *sc, const double *__restrict__ a0,
                                                 const double *__restrict__ b0, const double *__restrict__ a1,
                                                 const double *__restrict__ b1, double *__restrict__ part,
                                                 int nb, int64_t n)
{
    __shared__ double lds[32];
    if (sc->flag) return;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        s0 += a0[i] * b0[i];
        if (b1) s1 += a1[i] * b1[i];
    }
    put_parts(s0, s1, part, nb, lds);
}

// alpha = rho / rh.v; x += alpha y; s = r - alpha v; z = D^-1 s.
__global__ __launch_bounds__(256) void k_trs_s(TrScal *sc, const double *__restrict__ prv, int nb,
                                               double *__restrict__ x, const double *__restrict__ y,
                                               const double *__restrict__ r, const double *__restrict__ v,
                                               const double *__restrict__ dinv, double *__restrict__ s,
                                               double *__restrict__ z, int64_t n)
{
    __shared__ double bc[2];
    if (sc->flag) return;
    double rv, unused;
    sum_parts(prv, nullptr, nb, bc, rv, unused);
    const double rho = sc->rho_cur;
    const bool bad = !(rv != 0.0) || !fin(rv);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->its += bad ? 1 : 2;
        if (bad) {
            sc->flag = TR_RESTART;
        } else {
            sc->alpha = rho / rv;
            sc->rho_prev = rho;
        }
    }
    if (bad) return;
    const double alpha = rho / rv;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * y[i];
        const double si = r[i] - alpha * v[i];
        s[i] = si;
        z[i] = dinv[i] * si;
    }
}

// omega = t.s / t.t; x += omega z; r = s - omega t; partials r.r and rh.r.
__global__ __launch_bounds__(256) void k_trs_xr(TrScal *sc, const double *__restrict__ pts, int nb,
                                                double *__restrict__ x, const double *__restrict__ z,
                                                const double *__restrict__ s, const double *__restrict__ t,
                                                double *__restrict__ r, const double *__restrict__ rh,
                                                double *__restrict__ prr, int64_t n)
{
    __shared__ double bc[2];
    __shared__ double lds[32];
    if (sc->flag) return;
    double ts, tt;
    sum_parts(pts, pts + nb, nb, bc, ts, tt);
    const bool bad = !(tt > 0.0) || !fin(tt) || !fin(ts);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (bad)
            sc->flag = TR_RESTART;
        else
            sc->omega = ts / tt;
    }
    if (bad) return;
    const double omega = ts / tt;
    double rr = 0.0, rhr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += omega * z[i];
        const double ri = s[i] - omega * t[i];
        r[i] = ri;
        rr += ri * ri;
        rhr += rh[i] * ri;
    }
    put_parts(rr, rhr, prr, nb, lds);
}

}  // namespace

}  // namespace fo

using namespace fo;

namespace {

// Work buffers of the transport and reinitialisation solves, allocated on
// first use.  The captured graphs hold these addresses, so the velocity and
// the nodal data of a reinitialisation step are copied in.
struct TrBufs {
    double *theta, *par, *w, *prev, *b, *x, *r, *rh, *p, *v, *y, *s, *z, *t, *dinv;
    double *prr, *prv, *pts;  // partials [2 nb], [nb], [2 nb]
    TrScal *sc;
    uint8_t *mask;            // [N] fixed nodes of the heat problem
};

// Which matrix the solver applies: the transport L, or the
// reinitialisation Lhat (its parameters at par + 8).
enum { SYS_TRANSPORT = 0, SYS_REINIT = 1 };

int64_t tr_doubles(const fo_ctx *c)
{
    const int64_t N = c->N;
    return N * c->dim + 16 + 3 * N + N + 11 * N + 5 * (int64_t)kRedBlocks + (N + 7) / 8;
}

int tr_buffers(fo_ctx *c, TrBufs *o)
{
    const int64_t N = c->N;
    if (!c->tr_buf) return FO_ERR_STATE;
    double *m = reinterpret_cast<double *>(c->tr_buf);
    o->theta = m;
    m += N * c->dim;
    o->par = m;
    m += 16;
    o->w = m;
    m += 3 * N;
    o->prev = m;
    m += N;
    double **vec[] = {&o->b, &o->x, &o->r, &o->rh, &o->p, &o->v, &o->y, &o->s, &o->z, &o->t, &o->dinv};
    for (double **q : vec) {
        *q = m;
        m += N;
    }
    o->prr = m;
    o->prv = m + 2 * kRedBlocks;
    o->pts = m + 3 * kRedBlocks;
    m += 5 * kRedBlocks;
    o->mask = reinterpret_cast<uint8_t *>(m);
    m += (N + 7) / 8;
    o->sc = reinterpret_cast<TrScal *>(m);
    return FO_OK;
}

}  // namespace

size_t fo::tr_buffer_bytes(const fo_ctx *c) { return (size_t)tr_doubles(c) * sizeof(double) + sizeof(TrScal) + 256; }

namespace {

int sys_apply(const fo_ctx *c, const TrBufs &B, int sys, const double *x, double *y, hipStream_t s,
              const int32_t *stop = nullptr)
{
    if (sys == SYS_REINIT) return launch_reinit_apply(c, B.w, B.par + 8, x, y, s, stop);
    return launch_transport_apply(c, B.theta, B.par, 0, x, y, s, stop);
}

// Enqueues g BiCGStab iterations (each a no-op once the stop flag is set).
int tr_iterations(const fo_ctx *c, const TrBufs &B, int sys, int g, hipStream_t s)
{
    const int64_t N = c->N;
    const int nb = red_blocks(N);
    const int32_t *stop = &B.sc->flag;
    for (int k = 0; k < g; ++k) {
        hipLaunchKernelGGL(k_trs_p, dim3(nb), dim3(kBlock), 0, s, B.sc, B.prr, nb, B.r, B.p, B.v, B.dinv, B.y, N);
        FO_TRY(sys_apply(c, B, sys, B.y, B.v, s, stop));  // v = A y
        hipLaunchKernelGGL(k_trs_dot, dim3(nb), dim3(kBlock), 0, s, B.sc, B.rh, B.v, (const double *)nullptr,
                           (const double *)nullptr, B.prv, nb, N);
        hipLaunchKernelGGL(k_trs_s, dim3(nb), dim3(kBlock), 0, s, B.sc, B.prv, nb, B.x, B.y, B.r, B.v, B.dinv,
                           B.s, B.z, N);
        FO_TRY(sys_apply(c, B, sys, B.z, B.t, s, stop));  // t = A z
        hipLaunchKernelGGL(k_trs_dot, dim3(nb), dim3(kBlock), 0, s, B.sc, B.t, B.s, B.t, B.t, B.pts, nb, N);
        hipLaunchKernelGGL(k_trs_xr, dim3(nb), dim3(kBlock), 0, s, B.sc, B.pts, nb, B.x, B.z, B.s, B.t, B.r, B.rh,
                           B.prr, N);
    }
    return FO_OK;
}

// Enqueues g iterations as graphs of 32, 16, ..., 1 iterations.
int tr_enqueue(fo_ctx *c, const TrBufs &B, int sys, int g)
{
    for (int len = 32; len >= 1; len >>= 1)
        while (g >= len) {
            auto key = std::make_tuple(300 + sys, len, (int)c->scatter, 0);
            FO_TRY(graph_chunk(c, key, [&](hipStream_t s) { return tr_iterations(c, B, sys, len, s); }));
            g -= len;
        }
    return FO_OK;
}

// One step's solve A x = b (A by `sys`; B.b, B.x = the initial guess, B.dinv
// the inverted diagonal set by the caller): passes of BiCGStab, each from
// the recomputed residual, until that residual meets rtol |b|.  pred carries
// the first batch size from step to step.  Adds operator applications to
// *iters, raises *worst to the accepted relative residual.
int solve_step(fo_ctx *c, const TrBufs &B, int sys, const fo_solve_opts *o, int *pred, int64_t *iters,
               double *worst, int *status)
{
    hipStream_t s = c->stream;
    const int64_t N = c->N;
    const int nb = red_blocks(N);
    TrScal h{};
    auto read = [&]() -> int {
        FO_HIP(hipMemcpyAsync(&h, B.sc, sizeof(TrScal), hipMemcpyDeviceToHost, s));
        FO_HIP(fo::wait_stream(s));
        return FO_OK;
    };
    launch_dots<double>(1, B.b, B.b, nullptr, nullptr, nullptr, nullptr, N, c->partials, red_blocks(N), s);
    launch_finish_dots(c->partials, red_blocks(N), 1, &B.sc->bb, s);
    bool ok = false;
    int64_t its = 0;  // operator applications of this step
    double rel = 0.0;
    for (int restart = 0; restart < 50 && !ok && *status == FO_OK; ++restart) {
        FO_TRY(sys_apply(c, B, sys, B.x, B.t, s));  // t = A x
        if (restart > 0) ++its;
        hipLaunchKernelGGL(k_trs_start, dim3(nb), dim3(kBlock), 0, s, B.b, B.t, B.r, B.rh, B.p, B.v, B.prr, nb,
                           N);
        const int64_t left = std::max<int64_t>(o->max_iter - its, 0);
        hipLaunchKernelGGL(k_trs_check, dim3(1), dim3(64), 0, s, B.sc, B.prr, nb, o->rtol,
                           (int32_t)std::min<int64_t>(left, INT32_MAX));
        FO_TRY(read());
        rel = h.bb > 0.0 ? std::sqrt(h.rr / h.bb) : 0.0;
        if (h.flag == TR_NAN) {
            *status = FO_ERR_BREAKDOWN;
            break;
        }
        if (h.flag == TR_CONVERGED) {
            ok = true;
            break;
        }
        if (its >= o->max_iter) break;
        // iterate until the device stops; the next pass recomputes b - A x
        // and accepts the step or restarts
        int batch = *pred;
        while (true) {
            FO_TRY(tr_enqueue(c, B, sys, batch));
            FO_TRY(read());
            if (h.flag != TR_RUN) break;
            batch = 2;
        }
        if (restart == 0) *pred = std::min(std::max(h.its / 2 + 1, 1), 64);
        its += h.its;
    }
    *iters += its;
    *worst = std::max(*worst, rel);
    if (*status == FO_OK && !ok) *status = FO_NOT_CONVERGED;
    return FO_OK;
}

// Reinitialisation: nodal S(phi) = phi / sqrt(phi^2 + h^2) into w[.][2].
__global__ __launch_bounds__(256) void k_rn_s(const double *__restrict__ phi, double h2, double *__restrict__ w,
                                              int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        w[i * 3 + 2] = phi[i] / sqrt(phi[i] * phi[i] + h2);
}

// w[.][0] = u = varphi(t), w[.][1] = v = varphi(t - dt).
__global__ __launch_bounds__(256) void k_rn_pack(const double *__restrict__ u, const double *__restrict__ v,
                                                 double *__restrict__ w, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        w[i * 3] = u[i];
        w[i * 3 + 1] = v[i];
    }
}

// Reinitialisation step parameters: dt, h^2, 1/dt^2, Euler flag.
__global__ void k_rn_par(double *par, double dt, double h2, int euler)
{
    par[0] = dt;
    par[1] = h2;
    par[2] = 1.0 / (dt * dt);
    par[3] = euler ? 1.0 : 0.0;
}

// Heat system set-up: b = 0 on fixed nodes.
__global__ __launch_bounds__(256) void k_heat_fix(const uint8_t *__restrict__ mask, double *__restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (mask[i]) b[i] = 0.0;
}

// Volume sum_e chi_e |T_e|: partials per block into part[blockIdx.x].
template <int D>
__global__ __launch_bounds__(256) void k_heat_vol(const int32_t *__restrict__ conn, int64_t E,
                                                  const double *__restrict__ coords, const uint8_t *__restrict__ chi,
                                                  double *__restrict__ part)
{
    __shared__ double lds[16];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        if (!chi[e]) continue;
        double P[D + 1][D];
#pragma unroll
        for (int a = 0; a <= D; ++a)
#pragma unroll
            for (int j = 0; j < D; ++j) P[a][j] = coords[(int64_t)conn[(int64_t)a * E + e] * D + j];
        double det;
        if constexpr (D == 2) {
            det = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1]);
            s += fabs(det) / 2.0;
        } else {
            double u[3], v[3], w[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                u[j] = P[1][j] - P[0][j];
                v[j] = P[2][j] - P[0][j];
                w[j] = P[3][j] - P[0][j];
            }
            det = u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
                  u[2] * (v[0] * w[1] - v[1] * w[0]);
            s += fabs(det) / 6.0;
        }
    }
    s = block_sum_last(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

int grid_for(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096); }

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
    FO_HIP(hipMemcpyAsync(B.theta, theta, (size_t)N * c->dim * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_tr_par, dim3(1), dim3(1), 0, s, B.par, dt, smooth ? h2 : 0.0, h2);
    FO_TRY(launch_transport_diag(c, B.theta, B.par, B.dinv, s));
    launch_invert_diag<double>(B.dinv, nullptr, N, B.dinv, s);
    int64_t iters = 0;
    double worst = 0.0;  // largest accepted relative residual
    int status = FO_OK;
    int pred = 4;  // iterations of the first batch: the previous step's first pass plus its stop test
    for (int step = 0; step < steps && status == FO_OK; ++step) {
        FO_TRY(launch_transport_apply(c, B.theta, B.par, 1, phi, B.b, s));  // b = R phi
        FO_HIP(hipMemcpyAsync(B.x, phi, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        FO_TRY(solve_step(c, B, SYS_TRANSPORT, o, &pred, &iters, &worst, &status));
        FO_HIP(hipMemcpyAsync(phi, B.x, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    FO_HIP(fo::wait_stream(s));
    if (st) {
        st->status = status;
        st->iters_inner = (int32_t)std::min<int64_t>(iters, INT32_MAX);
        st->iters_outer = steps;
        st->rel_res = worst;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

int fo_reinit(fo_ctx *c, double *phi, int32_t steps, double t_end, const fo_solve_opts *o, fo_solve_stats *st)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !phi || !o || !(t_end > 0.0) || !(t_end < INFINITY) || steps < 0 || !(o->rtol > 0.0) ||
        o->max_iter <= 0)
        return FO_ERR_ARG;
    if (c->scatter != FO_SCATTER_TILED || c->tiles.n_tiles <= 0) return FO_ERR_STATE;
    TrBufs B;
    FO_TRY(tr_buffers(c, &B));
    hipStream_t s = c->stream;
    const int64_t N = c->N;
    const double h2 = c->transport_h2;
    const double dt = steps > 0 ? t_end / steps : t_end;
    const int ng = grid_for(N);
    hipLaunchKernelGGL(k_rn_s, dim3(ng), dim3(256), 0, s, phi, h2, B.w, N);
    FO_HIP(hipMemcpyAsync(B.prev, phi, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    int64_t iters = 0;
    double worst = 0.0;
    int status = FO_OK;
    int pred = 4;
    for (int step = 0; step < steps && status == FO_OK; ++step) {
        hipLaunchKernelGGL(k_rn_pack, dim3(ng), dim3(256), 0, s, phi, B.prev, B.w, N);
        hipLaunchKernelGGL(k_rn_par, dim3(1), dim3(1), 0, s, B.par + 8, dt, h2, step == 0 ? 1 : 0);
        FO_TRY(launch_reinit_rhs(c, B.w, B.par + 8, B.b, s));
        FO_TRY(launch_reinit_diag(c, B.w, B.par + 8, B.dinv, s));
        launch_invert_diag<double>(B.dinv, nullptr, N, B.dinv, s);
        FO_HIP(hipMemcpyAsync(B.x, phi, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        FO_TRY(solve_step(c, B, SYS_REINIT, o, &pred, &iters, &worst, &status));
        FO_HIP(hipMemcpyAsync(B.prev, phi, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        FO_HIP(hipMemcpyAsync(phi, B.x, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    FO_HIP(fo::wait_stream(s));
    if (st) {
        st->status = status;
        st->iters_inner = (int32_t)std::min<int64_t>(iters, INT32_MAX);
        st->iters_outer = steps;
        st->rel_res = worst;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

int fo_heat_load(fo_ctx *c, const double *f, double *b)
{
    if (!c || !f || !b) return FO_ERR_ARG;
    if (c->scatter != FO_SCATTER_TILED || c->tiles.n_tiles <= 0) return FO_ERR_STATE;
    FO_TRY(launch_mass_apply(c, f, b, c->stream));
    FO_HIP(fo::wait_stream(c->stream));
    return FO_OK;
}

int fo_heat_solve(fo_ctx *c, const uint8_t *gamma0, const double *b, double *u, const fo_solve_opts *o,
                  fo_solve_stats *st)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !gamma0 || !b || !u || !o || !(o->rtol > 0.0) || o->max_iter <= 0) return FO_ERR_ARG;
    if (c->scatter != FO_SCATTER_TILED || c->tiles.n_tiles <= 0 || !c->have_phi) return FO_ERR_STATE;
    TrBufs B;
    FO_TRY(tr_buffers(c, &B));
    hipStream_t s = c->stream;
    const int64_t N = c->N;
    const int ng = grid_for(N);
    FO_HIP(hipMemcpyAsync(B.mask, gamma0, (size_t)N, hipMemcpyDeviceToDevice, s));
    FO_HIP(hipMemcpyAsync(B.b, b, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_heat_fix, dim3(ng), dim3(256), 0, s, B.mask, B.b, N);
    // Jacobi: the diagonal of K with the fixed rows zeroed, inverted with 0 there
    FO_TRY(launch_heat_diag(c, B.mask, B.dinv, s));
    launch_invert_diag<double>(B.dinv, B.mask, N, B.dinv, s);
    fo_solve_stats one{};
    const int status = heat_cg_solve(c, B.mask, B.b, B.dinv, o, &one);
    if (status < 0 && status != FO_ERR_BREAKDOWN) return status;
    const int64_t iters = one.iters_inner;
    const double worst = one.rel_res;
    FO_HIP(hipMemcpyAsync(u, c->x64, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    FO_HIP(fo::wait_stream(s));
    if (st) {
        st->status = status;
        st->iters_inner = (int32_t)std::min<int64_t>(iters, INT32_MAX);
        st->iters_outer = 0;
        st->rel_res = worst;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

int fo_heat_derivative(fo_ctx *c, const double *u, const double *f, double lambda_vol, double V, double *rhs,
                       double *J, double *vol)
{
    if (!c || !u || !f || !rhs || !J || !vol || !(V > 0.0)) return FO_ERR_ARG;
    if (c->scatter != FO_SCATTER_TILED || c->tiles.n_tiles <= 0 || !c->have_phi) return FO_ERR_STATE;
    TrBufs B;
    FO_TRY(tr_buffers(c, &B));
    hipStream_t s = c->stream;
    const int64_t N = c->N;
    FO_TRY(launch_heat_rhs(c, u, f, lambda_vol, V, rhs, s));
    // J = u . K u over all nodes (u vanishes on the fixed ones)
    FO_TRY(launch_heat_apply(c, nullptr, u, B.t, s));
    launch_dots<double>(1, u, B.t, nullptr, nullptr, nullptr, nullptr, N, c->partials, red_blocks(N), s);
    launch_finish_dots(c->partials, red_blocks(N), 1, J, s);
    const int nb = red_blocks(c->E);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_heat_vol<2>, dim3(nb), dim3(256), 0, s, c->conn, c->E, c->coords, c->chi, c->partials);
    else
        hipLaunchKernelGGL(k_heat_vol<3>, dim3(nb), dim3(256), 0, s, c->conn, c->E, c->coords, c->chi, c->partials);
    launch_finish_dots(c->partials, nb, 1, vol, s);
    FO_HIP(fo::wait_stream(s));
    return FO_OK;
}

}  // extern "C"

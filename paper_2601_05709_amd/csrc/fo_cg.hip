// Jacobi-preconditioned conjugate gradients with device-side control.
//
// The scalars of a solve live in two slots sc[0], sc[1]: the kernels of
// iteration k read slot P = k & 1 and the last kernel of the iteration writes
// slot P ^ 1, so no kernel ever writes a scalar another block of the same
// kernel may still read.  Every block recomputes alpha and beta from the same
// partial sums in the same order, so the solve needs no single-block scalar
// kernels and stays bitwise reproducible.  Once a slot says done, kernels turn
// into no-ops and the last one of each iteration copies the final state
// forward, so after an even number of iterations the result is in sc[0].
//
// One iteration = apply (q = A p, with partial sums of p.q from the operator
// kernel) -> k_cg_update (x += alpha p, r -= alpha q, partial r.z, r.r) ->
// k_cg_direction (convergence test, p = D^-1 r + beta p).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fo_internal.h"
#include "fo_launch.h"
#include "fo_reduce.h"

namespace fo {

__device__ __forceinline__ bool finite(double v) { return v == v && v != INFINITY && v != -INFINITY; }

// r = b - q (q may be null: x0 = 0), p = D^-1 r; partial rows r.z, r.r, b.b
template <typename T>
__global__ __launch_bounds__(256) void k_cg_start(const T *__restrict__ b, const T *__restrict__ q,
                                                  T *__restrict__ r, T *__restrict__ p,
                                                  const T *__restrict__ dinv, int64_t n,
                                                  double *__restrict__ part)
{
    __shared__ double lds[4];
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T bi = b[i];
        T ri = q ? bi - q[i] : bi;
        r[i] = ri;
        T zi = dinv[i] * ri;
        p[i] = zi;
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
        bb += (double)bi * (double)bi;
    }
    double s0 = block_sum(rz, lds), s1 = block_sum(rr, lds), s2 = block_sum(bb, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[gridDim.x + blockIdx.x] = s1;
        part[2 * gridDim.x + blockIdx.x] = s2;
    }
}

// Fresh state in sc[0] (and sc[1]).  The recursive residual target is
// tol2 = rtol^2 * (b.b) when ref2 < 0, else rtol^2 * ref2.
__global__ __launch_bounds__(256) void k_cg_start_finish(SolveScalars *sc,
                                                         const double *__restrict__ part, int nb,
                                                         double rtol2, double ref2, int max_it)
{
    __shared__ double lds[4];
    double rz = block_sum_partials(part, nb, lds);
    double rr = block_sum_partials(part + nb, nb, lds);
    double bb = block_sum_partials(part + 2 * nb, nb, lds);
    if (threadIdx.x == 0) {
        SolveScalars s{};
        s.rho = rz;
        s.rr = rr;
        s.bnorm2 = bb;
        s.tol2 = rtol2 * (ref2 >= 0.0 ? ref2 : bb);
        s.it = 0;
        s.max_it = max_it;
        s.status = 0;
        s.done = (rr <= s.tol2) ? 1 : 0;
        if (!(rz >= 0.0) || !finite(rz) || !finite(rr)) {
            s.status = FO_ERR_BREAKDOWN;
            s.done = 1;
        }
        sc[0] = s;
        sc[1] = s;
    }
}

// x += alpha p; r -= alpha q with alpha = rho / sum(pq_part); partials r.z, r.r
template <typename T>
__global__ __launch_bounds__(256) void k_cg_update(SolveScalars *sc, int P, T *__restrict__ x,
                                                   T *__restrict__ r, const T *__restrict__ p,
                                                   const T *__restrict__ q,
                                                   const T *__restrict__ dinv, int64_t n,
                                                   const double *__restrict__ pq_part, int n_pq,
                                                   double *__restrict__ rz_part)
{
    __shared__ double lds[4];
    __shared__ double s_alpha;
    if (sc[P].done) return;
    double pq = block_sum_partials(pq_part, n_pq, lds);
    if (threadIdx.x == 0) {
        double a = (pq > 0.0 && finite(pq)) ? sc[P].rho / pq : 0.0;
        s_alpha = a;
        if (blockIdx.x == 0) {
            sc[P].pq = pq;
            sc[P].alpha = a;
        }
    }
    __syncthreads();
    const T alpha = (T)s_alpha;
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        T ri = r[i] - alpha * q[i];
        r[i] = ri;
        T zi = dinv[i] * ri;
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    double s0 = block_sum(rz, lds), s1 = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        rz_part[blockIdx.x] = s0;
        rz_part[gridDim.x + blockIdx.x] = s1;
    }
}

// Convergence test and p = D^-1 r + beta p.  Writes slot P ^ 1.
template <typename T>
__global__ __launch_bounds__(256) void k_cg_direction(SolveScalars *sc, int P, T *__restrict__ p,
                                                      const T *__restrict__ r,
                                                      const T *__restrict__ dinv, int64_t n,
                                                      const double *__restrict__ rz_part, int nb)
{
    __shared__ double lds[4];
    __shared__ int s_go;
    __shared__ double s_beta;
    if (sc[P].done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) sc[P ^ 1] = sc[P];
        return;
    }
    double rz = block_sum_partials(rz_part, nb, lds);
    double rr = block_sum_partials(rz_part + nb, nb, lds);
    if (threadIdx.x == 0) {
        SolveScalars cur = sc[P];
        int it = cur.it + 1;
        int done = 0, status = 0;
        if (!(cur.pq > 0.0) || !finite(cur.pq) || !(rz >= 0.0) || !finite(rz) || !finite(rr)) {
            done = 1;
            status = FO_ERR_BREAKDOWN;
        } else if (rr <= cur.tol2 || it >= cur.max_it) {
            done = 1;
        }
        double beta = done ? 0.0 : rz / cur.rho;
        s_go = !done;
        s_beta = beta;
        if (blockIdx.x == 0) {
            SolveScalars nx = cur;
            nx.it = it;
            nx.done = done;
            nx.status = status;
            nx.rr = rr;
            nx.beta = beta;
            nx.rho_new = rz;
            if (!done) nx.rho = rz;  // on exit rho keeps r.z of the last direction
            sc[P ^ 1] = nx;
        }
    }
    __syncthreads();
    if (!s_go) return;
    const T beta = (T)s_beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = dinv[i] * r[i] + beta * p[i];
}

// ---------------------------------------------------------------------------
// FP32 CG with FP64 residual replacement (iterative refinement that keeps the
// Krylov direction).  The FP32 system is scaled so that ||r32|| = 1 at the
// start of each phase: r32 = r64 / s with s = ||r64||.

// x64 += s * x32 (s^2 in s2[0])
__global__ void k_ir_accumulate(double *__restrict__ x64, const float *__restrict__ x32,
                                const double *__restrict__ s2, int64_t n)
{
    double s = sqrt(s2[0]);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x64[i] += s * (double)x32[i];
}

// y += x (FP64).
__global__ void k_add64(double *__restrict__ y, const double *__restrict__ x, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

// r64 = b - q64 and partial ||r64||^2
__global__ __launch_bounds__(256) void k_residual64(const double *__restrict__ b,
                                                    const double *__restrict__ q,
                                                    double *__restrict__ r, int64_t n,
                                                    double *__restrict__ part)
{
    __shared__ double lds[4];
    double rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double ri = b[i] - q[i];
        r[i] = ri;
        rr += ri * ri;
    }
    double t = block_sum(rr, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// Fused CG for the tiled elasticity operator (see k_tile_cg): one iteration =
// k_tile_cg (beta, direction, operator, p.q partials) + k_cgn_update.  The
// r.z / r.r partials are written by node-parallel kernels on upd_blocks(N)
// blocks, the layout k_tile_cg reduces.

// out[k] = the sum of part[k n .. k n + n), k < sets, in a fixed order (one
// block): the folded partials of the fused CG on large meshes.
__global__ __launch_bounds__(1024) void k_fold_partials(const double *__restrict__ part, int n, int sets,
                                                        double *__restrict__ out)
{
    constexpr int U = 16;  // loads in flight per thread; the sum order is the plain strided one
    __shared__ double lds[16];
    const int nt = (int)blockDim.x;
    for (int k = 0; k < sets; ++k) {
        const double *p = part + (int64_t)k * n;
        double s = 0.0;
        for (int base = (int)threadIdx.x; base < n; base += U * nt) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = p[min(base + u * nt, n - 1)];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (base + u * nt < n) s += v[u];
        }
        s = block_sum_any(s, lds);
        if (threadIdx.x == 0) out[k] = s;
    }
}

void launch_fold(const double *part, int n, int sets, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold_partials, dim3(1), dim3(1024), 0, s, part, n, sets, out);
}

// out[g] = the sum of part[g 1024 .. min((g + 1) 1024, n)), one block per
// group, in a fixed order: the per-tile p.q partials of a large mesh in
// groups, whose sums the update blocks read (49,152 tiles: 48 sums, folded
// in parallel instead of by one block).
__global__ __launch_bounds__(1024) void k_fold_groups(const double *__restrict__ part, int n,
                                                      double *__restrict__ out)
{
    __shared__ double lds[16];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = i < n ? part[i] : 0.0;
    v = block_sum_any(v, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

int upd_blocks(int64_t N)
{
    int64_t b = (N + kUpdBlock - 1) / kUpdBlock;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), kRedBlocks);
}

int node_blocks(int64_t N)
{
    int64_t b = (N + kBlock - 1) / kBlock;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), kRedBlocks);
}

// r = b - q (q nullable: x = 0); partials r.z, r.r (rz_part), b.b (bb_part)
template <typename T, int D>
__global__ __launch_bounds__(256) void k_cgn_residual(const T *__restrict__ b,
                                                      const T *__restrict__ q, T *__restrict__ r,
                                                      const T *__restrict__ dinv, int64_t N,
                                                      double *__restrict__ rz_part,
                                                      double *__restrict__ bb_part)
{
    __shared__ double lds[4];
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; node < N;
         node += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int v = 0; v < D; ++v) {
            const int64_t i = node * D + v;
            const T bi = b[i];
            const T ri = q ? bi - q[i] : bi;
            r[i] = ri;
            rz += (double)ri * (double)(dinv[i] * ri);
            rr += (double)ri * (double)ri;
            bb += (double)bi * (double)bi;
        }
    }
    double s0 = block_sum(rz, lds), s1 = block_sum(rr, lds), s2 = block_sum(bb, lds);
    if (threadIdx.x == 0) {
        rz_part[blockIdx.x] = s0;
        rz_part[gridDim.x + blockIdx.x] = s1;
        bb_part[blockIdx.x] = s2;
    }
}

// Fresh state in sc[0..1]: first direction p = D^-1 r (beta0 = 0).
__global__ __launch_bounds__(256) void k_cgn_start_finish(SolveScalars *sc,
                                                          const double *__restrict__ rz_part,
                                                          const double *__restrict__ bb_part,
                                                          int nb, double rtol2, int max_it)
{
    __shared__ double lds[4];
    double rz = block_sum_partials(rz_part, nb, lds);
    double rr = block_sum_partials(rz_part + nb, nb, lds);
    double bb = block_sum_partials(bb_part, nb, lds);
    if (threadIdx.x == 0) {
        SolveScalars s{};
        s.rho = rz;
        s.rho_new = rz;
        s.rr = rr;
        s.bnorm2 = bb;
        s.tol2 = rtol2 * bb;
        s.max_it = max_it;
        s.first = 1;
        s.beta = 0.0;
        s.done = (rr <= s.tol2) ? 1 : 0;
        if (!(rz >= 0.0) || !finite(rz) || !finite(rr)) {
            s.status = FO_ERR_BREAKDOWN;
            s.done = 1;
        }
        sc[0] = s;
        sc[1] = s;
    }
}

// x += alpha p; r -= alpha q, alpha = rho / sum(pq_part) (summed by every
// block in the same fixed order, after the node loads are issued);
// q at shared nodes is the fixed-order sum of the node's halo slots; clamped
// unknowns (dinv = 0) get q = 0.  Partials r.z, r.r per block.  Reads slot B.
// Blocks of kUpdBlock threads, one node per thread (grid-stride beyond).
template <typename T, int D>
__global__ __launch_bounds__(kUpdBlock) void k_cgn_update(
    SolveScalars *sc, int B, T *__restrict__ x, T *__restrict__ r, const T *__restrict__ p,
    const T *__restrict__ q, const T *__restrict__ dinv, int64_t N,
    const double *__restrict__ pq_part, int n_pq, double *__restrict__ rz_part,
    const int2 *__restrict__ hrange, const T *__restrict__ halo)
{
    __shared__ double lds[32];
    __shared__ double s_alpha;
    // the p.q partials first (they depend on nothing), then the node data
    PartLoad<4> ppq;
    part_issue(ppq, pq_part, n_pq, threadIdx.x, blockDim.x);
    const int32_t done = sc[B].done;
    const double rho = sc[B].rho;
    int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    T di[D], qi[D], xi[D], ri[D], pi[D];
    auto load = [&](int64_t nd) {
        const int2 hr = hrange[nd];
#pragma unroll
        for (int v = 0; v < D; ++v) {
            const int64_t i = nd * D + v;
            di[v] = dinv[i];
            xi[v] = x[i];
            ri[v] = r[i];
            pi[v] = p[i];
        }
        if (hr.x < 0) {
#pragma unroll
            for (int v = 0; v < D; ++v) qi[v] = q[(int64_t)nd * D + v];
        } else {
            // the node's halo slots in order; the first KH are loaded together
            // (indices clamped into the range, so every load is in bounds)
            constexpr int KH = 4;
            const int cnt = hr.y - hr.x;
            T hv[KH][D];
#pragma unroll
            for (int k = 0; k < KH; ++k) {
                const int64_t j = hr.x + min(k, cnt - 1);
#pragma unroll
                for (int v = 0; v < D; ++v) hv[k][v] = halo[j * D + v];
            }
#pragma unroll
            for (int v = 0; v < D; ++v) qi[v] = T(0);
#pragma unroll
            for (int k = 0; k < KH; ++k)
                if (k < cnt)
#pragma unroll
                    for (int v = 0; v < D; ++v) qi[v] += hv[k][v];
            for (int j = hr.x + KH; j < hr.y; ++j)
#pragma unroll
                for (int v = 0; v < D; ++v) qi[v] += halo[(int64_t)j * D + v];
        }
    };
    if (node < N) load(node);
    if (done) return;
    {
        // p.q: wave sums, then wave 0 sums the wave totals and sets alpha
        const double v = wave_sum(part_finish(ppq, pq_part, n_pq, threadIdx.x, blockDim.x));
        const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
        if (lane == 0) lds[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x < 64) {
            const double pq = wave_sum(lane < nw ? lds[lane] : 0.0);
            if (threadIdx.x == 0) {
                const bool ok = pq > 0.0 && finite(pq);
                s_alpha = ok ? rho / pq : 0.0;
                if (blockIdx.x == 0) {
                    sc[B].pq = pq;
                    sc[B].alpha = s_alpha;
                    if (!ok) {  // not SPD or non-finite: stop (benign race with the done test above)
                        sc[B].status = FO_ERR_BREAKDOWN;
                        sc[B].done = 1;
                    }
                }
            }
        }
        __syncthreads();
    }
    const T alpha = (T)s_alpha;
    double rz = 0.0, rr = 0.0;
    while (node < N) {
#pragma unroll
        for (int v = 0; v < D; ++v) {
            const int64_t i = node * D + v;
            const T qv = di[v] == T(0) ? T(0) : qi[v];
            x[i] = xi[v] + alpha * pi[v];
            const T rv = ri[v] - alpha * qv;
            r[i] = rv;
            rz += (double)rv * (double)(di[v] * rv);
            rr += (double)rv * (double)rv;
        }
        node += (int64_t)gridDim.x * blockDim.x;
        if (node < N) load(node);
    }
    block_sum2_any(rz, rr, lds);
    if (threadIdx.x == 0) {
        rz_part[blockIdx.x] = rz;
        rz_part[gridDim.x + blockIdx.x] = rr;
    }
}

// IR phase start: r32 = r64 / s_new (s_new^2 in s2[1]), x32 = 0; partials
// r.z, r.r in the node layout.
template <int D>
__global__ __launch_bounds__(256) void k_ir_rescale(const double *__restrict__ r64,
                                                    const double *__restrict__ s2,
                                                    float *__restrict__ r32, float *__restrict__ x32,
                                                    const float *__restrict__ dinv, int64_t N,
                                                    double *__restrict__ rz_part)
{
    __shared__ double lds[4];
    const double s = sqrt(s2[1]);
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    double rz = 0.0, rr = 0.0;
    for (int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; node < N;
         node += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int v = 0; v < D; ++v) {
            const int64_t i = node * D + v;
            const float ri = (float)(r64[i] * inv);
            r32[i] = ri;
            x32[i] = 0.0f;
            rz += (double)ri * (double)(dinv[i] * ri);
            rr += (double)ri * (double)ri;
        }
    }
    double a = block_sum(rz, lds), b = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        rz_part[blockIdx.x] = a;
        rz_part[gridDim.x + blockIdx.x] = b;
    }
}

// New phase state in sc[0..1] after a residual replacement.  With the old
// scaling s_old (s2[0]) and the new one s_new (s2[1]), the unscaled
// beta = rho_new s_new^2 / (rho_old s_old^2), and the first direction of the
// phase, in the new scaling, is D^-1 r32 + beta (s_old / s_new) p32_old.  The
// coefficient goes to the slot (first = 1) for k_tile_cg.  fresh != 0 (first
// phase, or after a breakdown) restarts the direction.  s2[0] <- s2[1].
__global__ __launch_bounds__(256) void k_ir_phase(SolveScalars *sc,
                                                  const double *__restrict__ rz_part, int nb,
                                                  double *__restrict__ s2, double phase_rtol,
                                                  int max_it, int fresh)
{
    __shared__ double lds[4];
    double rz = block_sum_partials(rz_part, nb, lds);
    double rr = block_sum_partials(rz_part + nb, nb, lds);
    if (threadIdx.x == 0) {
        const SolveScalars old = sc[0];
        const double so2 = s2[0], sn2 = s2[1];
        double coef = 0.0;
        if (!fresh && old.rho > 0.0 && finite(old.rho) && so2 > 0.0 && sn2 > 0.0) {
            const double beta = (rz * sn2) / (old.rho * so2);
            coef = beta * sqrt(so2 / sn2);
        }
        SolveScalars s{};
        s.rho = rz;
        s.rho_new = rz;
        s.rr = rr;
        s.bnorm2 = 1.0;
        s.tol2 = phase_rtol * phase_rtol;
        s.beta = coef;
        s.first = 1;
        s.max_it = max_it;
        s.done = (rr <= s.tol2) ? 1 : 0;
        if (!(rz >= 0.0) || !finite(rz)) {
            s.status = FO_ERR_BREAKDOWN;
            s.done = 1;
        }
        sc[0] = s;
        sc[1] = s;
        s2[0] = sn2;
    }
}

// ---------------------------------------------------------------------------
// launchers

template <typename T>
void launch_cg_start(const T *b, const T *q, T *r, T *p, const T *dinv, int64_t n, double *part,
                     SolveScalars *sc, double rtol, double ref2, int max_it, hipStream_t s)
{
    int nb = red_blocks(n);
    hipLaunchKernelGGL(k_cg_start<T>, dim3(nb), dim3(kBlock), 0, s, b, q, r, p, dinv, n, part);
    hipLaunchKernelGGL(k_cg_start_finish, dim3(1), dim3(kBlock), 0, s, sc, part, nb, rtol * rtol,
                       ref2, max_it);
}
template void launch_cg_start<double>(const double *, const double *, double *, double *,
                                      const double *, int64_t, double *, SolveScalars *, double,
                                      double, int, hipStream_t);
template void launch_cg_start<float>(const float *, const float *, float *, float *, const float *,
                                     int64_t, double *, SolveScalars *, double, double, int,
                                     hipStream_t);

template <typename T>
void launch_cg_update(SolveScalars *sc, int P, T *x, T *r, const T *p, const T *q, const T *dinv,
                      int64_t n, const double *pq_part, int n_pq, double *rz_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_update<T>, dim3(red_blocks(n)), dim3(kBlock), 0, s, sc, P, x, r, p, q,
                       dinv, n, pq_part, n_pq, rz_part);
}
template void launch_cg_update<double>(SolveScalars *, int, double *, double *, const double *,
                                       const double *, const double *, int64_t, const double *,
                                       int, double *, hipStream_t);
template void launch_cg_update<float>(SolveScalars *, int, float *, float *, const float *,
                                      const float *, const float *, int64_t, const double *, int,
                                      double *, hipStream_t);

template <typename T>
void launch_cg_direction(SolveScalars *sc, int P, T *p, const T *r, const T *dinv, int64_t n,
                         const double *rz_part, hipStream_t s)
{
    int nb = red_blocks(n);
    hipLaunchKernelGGL(k_cg_direction<T>, dim3(nb), dim3(kBlock), 0, s, sc, P, p, r, dinv, n,
                       rz_part, nb);
}
template void launch_cg_direction<double>(SolveScalars *, int, double *, const double *,
                                          const double *, int64_t, const double *, hipStream_t);
template void launch_cg_direction<float>(SolveScalars *, int, float *, const float *, const float *,
                                         int64_t, const double *, hipStream_t);

void launch_add64(double *y, const double *x, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add64, dim3(red_blocks(n) * 4), dim3(kBlock), 0, s, y, x, n);
}

void launch_ir_accumulate(double *x64, const float *x32, const double *s2, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_accumulate, dim3(red_blocks(n) * 4), dim3(kBlock), 0, s, x64, x32, s2, n);
}

void launch_residual64(const double *b, const double *q, double *r, int64_t n, double *part,
                       double *out2, hipStream_t s)
{
    int nb = red_blocks(n);
    hipLaunchKernelGGL(k_residual64, dim3(nb), dim3(kBlock), 0, s, b, q, r, n, part);
    launch_finish_dots(part, nb, 1, out2, s);
}

template <typename T>
void launch_cgn_start(const fo_ctx *c, const T *b, const T *q, T *r, const T *dinv, double rtol,
                      int max_it, hipStream_t s)
{
    const int nb = upd_blocks(c->N);  // the partial layout k_tile_cg reads
    if (c->dim == 2)
        hipLaunchKernelGGL((k_cgn_residual<T, 2>), dim3(nb), dim3(kBlock), 0, s, b, q, r, dinv, c->N,
                           c->rz_part, c->bb_part);
    else
        hipLaunchKernelGGL((k_cgn_residual<T, 3>), dim3(nb), dim3(kBlock), 0, s, b, q, r, dinv, c->N,
                           c->rz_part, c->bb_part);
    hipLaunchKernelGGL(k_cgn_start_finish, dim3(1), dim3(kBlock), 0, s, c->scal, c->rz_part,
                       c->bb_part, nb, rtol * rtol, max_it);
}
template void launch_cgn_start<double>(const fo_ctx *, const double *, const double *, double *,
                                       const double *, double, int, hipStream_t);
template void launch_cgn_start<float>(const fo_ctx *, const float *, const float *, float *,
                                      const float *, double, int, hipStream_t);

template <typename T>
void launch_cgn_update(const fo_ctx *c, int B, T *x, T *r, const T *p, const T *q, const T *dinv,
                       hipStream_t s)
{
    const int nb = upd_blocks(c->N);
    const T *halo = reinterpret_cast<const T *>(c->halo);
    const double *pq = c->pq_part;
    int n_pq = (int)c->tiles.n_tiles;
    if (c->fold_pq) {
        const int G = (n_pq + 1023) / 1024;
        if (G <= kFoldGroups) {  // groups of 1024 folded in parallel; the update blocks read G sums
            hipLaunchKernelGGL(k_fold_groups, dim3(G), dim3(1024), 0, s, c->pq_part, n_pq, c->fold + 4);
            pq = c->fold + 4;
            n_pq = G;
        } else {  // one block folds them all; the update blocks read one value
            launch_fold(c->pq_part, n_pq, 1, c->fold + 2, s);
            pq = c->fold + 2;
            n_pq = 1;
        }
    }
    if (c->dim == 2)
        hipLaunchKernelGGL((k_cgn_update<T, 2>), dim3(nb), dim3(kUpdBlock), 0, s, c->scal, B, x, r, p, q,
                           dinv, c->N, pq, n_pq, c->rz_part,
                           reinterpret_cast<const int2 *>(c->tiles.node_hrange), halo);
    else
        hipLaunchKernelGGL((k_cgn_update<T, 3>), dim3(nb), dim3(kUpdBlock), 0, s, c->scal, B, x, r, p, q,
                           dinv, c->N, pq, n_pq, c->rz_part,
                           reinterpret_cast<const int2 *>(c->tiles.node_hrange), halo);
}
template void launch_cgn_update<double>(const fo_ctx *, int, double *, double *, const double *,
                                        const double *, const double *, hipStream_t);
template void launch_cgn_update<float>(const fo_ctx *, int, float *, float *, const float *,
                                       const float *, const float *, hipStream_t);

void launch_ir_phase(const fo_ctx *c, const double *r64, double *s2, float *r32, float *x32,
                     const float *dinv, double phase_rtol, int max_it, int fresh, hipStream_t s)
{
    const int nb = upd_blocks(c->N);  // the partial layout k_tile_cg reads
    if (c->dim == 2)
        hipLaunchKernelGGL(k_ir_rescale<2>, dim3(nb), dim3(kBlock), 0, s, r64, s2, r32, x32, dinv,
                           c->N, c->rz_part);
    else
        hipLaunchKernelGGL(k_ir_rescale<3>, dim3(nb), dim3(kBlock), 0, s, r64, s2, r32, x32, dinv,
                           c->N, c->rz_part);
    hipLaunchKernelGGL(k_ir_phase, dim3(1), dim3(kBlock), 0, s, c->scal, c->rz_part, nb, s2,
                       phase_rtol, max_it, fresh);
}

}  // namespace fo

// Host runtime of libfo: the C ABI of include/fo.h.
//
// Contexts own their device memory (hipMalloc at creation, hipFree at
// destruction).  The solvers keep all Krylov scalars on the device; the host
// only polls a small status block every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "fo_internal.h"
#include "fo_launch.h"
#include "fo_tiles.h"

using namespace fo;


namespace fo {

// Enqueues one chunk; with profiling off, a graph of it (captured once on the
// private stream, which only records) is replayed on the context stream.  In
// no-capture mode a chunk without a graph is enqueued directly.
int graph_chunk(fo_ctx *c, std::tuple<int, int, int, int> key,
                const std::function<int(hipStream_t)> &enqueue)
{
    auto it = c->graphs.find(key);
    if (c->prof || (c->no_capture && it == c->graphs.end())) return enqueue(c->stream);
    hipGraphExec_t exec = nullptr;
    if (it == c->graphs.end()) {
        hipGraph_t g = nullptr;
        FO_HIP(hipStreamBeginCapture(c->work, hipStreamCaptureModeRelaxed));
        int rc = enqueue(c->work);
        hipError_t e = hipStreamEndCapture(c->work, &g);
        if (rc != FO_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return FO_ERR_HIP;
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return FO_ERR_HIP;
        c->graphs[key] = exec;
    } else {
        exec = it->second;
    }
    FO_HIP(hipGraphLaunch(exec, c->stream));
    return FO_OK;
}

}  // namespace fo

namespace fo {

namespace {
std::atomic<int64_t> g_device_allocations{0};
}

hipError_t device_malloc(void **p, size_t bytes)
{
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) g_device_allocations.fetch_add(1, std::memory_order_relaxed);
    return e;
}

int ctx_alloc(fo_ctx *c, void **p, size_t bytes)
{
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    *p = nullptr;
    if (c->measure) {
        c->bytes += bytes;
        return FO_OK;
    }
    if (c->ws) {
        if (bytes > c->ws_cap - c->bytes) return FO_ERR_NOMEM;
        *p = c->ws + c->bytes;
        c->bytes += bytes;
        return FO_OK;
    }
    void *v = nullptr;
    if (device_malloc(&v, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return FO_ERR_NOMEM;
    }
    c->allocations.push_back(v);
    c->bytes += bytes;
    *p = v;
    return FO_OK;
}

}  // namespace fo

namespace {

template <typename T>
int dev_alloc(fo_ctx *c, T **p, size_t count)
{
    return fo::ctx_alloc_n(c, p, std::max<size_t>(count, 1));
}


double host_det(int dim, const double *X, const int32_t *conn, int64_t E, int64_t e)
{
    const double *p0 = X + (int64_t)conn[e] * dim;
    const double *p1 = X + (int64_t)conn[E + e] * dim;
    const double *p2 = X + (int64_t)conn[2 * E + e] * dim;
    if (dim == 2)
        return (p1[0] - p0[0]) * (p2[1] - p0[1]) - (p1[1] - p0[1]) * (p2[0] - p0[0]);
    const double *p3 = X + (int64_t)conn[3 * E + e] * dim;
    double a[3], b[3], d[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = p1[i] - p0[i];
        b[i] = p2[i] - p0[i];
        d[i] = p3[i] - p0[i];
    }
    return a[0] * (b[1] * d[2] - b[2] * d[1]) - a[1] * (b[0] * d[2] - b[2] * d[0]) +
           a[2] * (b[0] * d[1] - b[1] * d[0]);
}

// ---------------------------------------------------------------------------
// operators

template <typename T>
int elas_apply(fo_ctx *c, const T *x, T *y, hipStream_t s);

template <>
int elas_apply<double>(fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    if (c->scatter == FO_SCATTER_TILED && c->tiles.n_tiles > 0) {
        if (c->has_isolated) launch_fill<double>(y, c->ndof, 0.0, s);
        return launch_elas_apply_tiled<double>(c, c->coords, x, y, s);
    }
    launch_elas_apply_atomic<double>(c, c->coords, x, y, s);
    return FO_OK;
}

template <>
int elas_apply<float>(fo_ctx *c, const float *x, float *y, hipStream_t s)
{
    if (c->scatter == FO_SCATTER_TILED && c->tiles.n_tiles > 0) {
        if (c->has_isolated) launch_fill<float>(y, c->ndof, 0.0f, s);
        return launch_elas_apply_tiled<float>(c, c->coords32, x, y, s);
    }
    launch_elas_apply_atomic<float>(c, c->coords32, x, y, s);
    return FO_OK;
}

bool tiled(const fo_ctx *c) { return c->scatter == FO_SCATTER_TILED && c->tiles.n_tiles > 0; }

// y = 0 where the mask is set.
__global__ __launch_bounds__(256) void k_zero_masked(const uint8_t *__restrict__ fixed, double *__restrict__ y,
                                                     int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (fixed[i]) y[i] = 0.0;
}

void zero_masked(const fo_ctx *c, const uint8_t *fixed, double *y, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>((c->ndof + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_masked, dim3(nb), dim3(256), 0, s, fixed, y, c->ndof);
}

// y = B x; with a velocity mask, the rows of masked unknowns are zero (the
// iterates vanish there, so their columns never contribute).
int descent_apply(fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    if (tiled(c)) {
        if (c->has_isolated) launch_fill<double>(y, c->ndof, 0.0, s);
        FO_TRY(launch_descent_apply_tiled(c, x, y, s));
    } else {
        launch_descent_apply_atomic(c, x, y, s);
    }
    if (c->descent.fixed) zero_masked(c, c->descent.fixed, y, s);
    return FO_OK;
}

}  // namespace

int fo::elas_apply64(fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    return elas_apply<double>(c, x, y, s);
}

namespace {

// ---------------------------------------------------------------------------
// conjugate-gradient driver

enum OpKind { OP_ELAS64 = 0, OP_ELAS32 = 1, OP_DESCENT64 = 2, OP_HEAT64 = 3 };

// Unknowns of an operator: the scalar heat operator has one per node.
int64_t op_len(const fo_ctx *c, OpKind k) { return k == OP_HEAT64 ? c->N : c->ndof; }

template <typename T>
struct CgVecs {
    T *x, *r, *p, *q;
    const T *dinv;
};

int poll(fo_ctx *c)
{
    FO_HIP(hipMemcpyAsync(c->scal_host, c->scal, sizeof(SolveScalars), hipMemcpyDeviceToHost,
                          c->stream));
    FO_HIP(fo::wait_stream(c->stream));
    return FO_OK;
}

// q = A p inside the CG loop; the p.q partials land in c->pq_part.  done:
// device flag that turns the operator kernels into no-ops.
template <typename T>
int cg_apply(fo_ctx *c, OpKind k, const T *p, T *q, const int32_t *done, hipStream_t s, int *n_pq)
{
    const int64_t n = op_len(c, k);
    if (k != OP_DESCENT64 && k != OP_HEAT64 && tiled(c)) {
        if (c->has_isolated) launch_fill<T>(q, n, T(0), s);
        *n_pq = c->tiles.n_tiles;
        if constexpr (sizeof(T) == 8)
            return launch_elas_apply_tiled<double>(c, c->coords, (const double *)p, (double *)q, s,
                                                   c->pq_part, done);
        else
            return launch_elas_apply_tiled<float>(c, c->coords32, (const float *)p, (float *)q, s,
                                                  c->pq_part, done);
    }
    if (k == OP_DESCENT64) {
        if (tiled(c)) {
            if (c->has_isolated) launch_fill<double>((double *)q, n, 0.0, s);
            FO_TRY(launch_descent_apply_tiled(c, (const double *)p, (double *)q, s, done));
        } else {
            launch_descent_apply_atomic(c, (const double *)p, (double *)q, s);
        }
        if (c->descent.fixed) zero_masked(c, c->descent.fixed, (double *)q, s);
    } else if (k == OP_HEAT64) {
        if constexpr (sizeof(T) == 8) {
            FO_TRY(launch_heat_apply(c, c->heat_mask, (const double *)p, (double *)q, s, done));
        } else {
            return FO_ERR_ARG;
        }
    } else {
        FO_TRY(elas_apply<T>(c, p, q, s));
    }
    int nb = red_blocks(n);
    launch_dots<T>(1, p, q, nullptr, nullptr, nullptr, nullptr, n, c->pq_part, nb, s);
    *n_pq = nb;
    return FO_OK;
}

// `chunk` (even) iterations of the generic CG (any operator); the final
// state is in slot 0.
template <typename T>
int cg_chunk(fo_ctx *c, OpKind k, CgVecs<T> v, int chunk, hipStream_t s)
{
    const int64_t n = op_len(c, k);
    for (int i = 0; i < chunk; ++i) {
        const int P = i & 1;
        int n_pq = 0;
        FO_TRY(cg_apply<T>(c, k, v.p, v.q, &c->scal[P].done, s, &n_pq));
        launch_cg_update<T>(c->scal, P, v.x, v.r, v.p, v.q, v.dinv, n, c->pq_part, n_pq,
                            c->rz_part, s);
        launch_cg_direction<T>(c->scal, P, v.p, v.r, v.dinv, n, c->rz_part, s);
    }
    return FO_OK;
}

// Vectors of the fused CG (tiled elasticity): the direction alternates
// between p[0] and p[1]; iteration j reads p[j & 1] and writes p[(j+1) & 1].
template <typename T>
struct FusedVecs {
    T *x, *r, *q;
    T *p[2];
    const T *dinv;
    int kind;  // FusedKind: the operator
};

template <typename T>
int fused_chunk(fo_ctx *c, FusedVecs<T> v, int chunk, hipStream_t s)
{
    for (int j = 0; j < chunk; ++j) {
        const int A = j & 1;
        FO_TRY(launch_tile_cg<T>(c, v.kind, v.r, v.dinv, v.p[A], v.p[A ^ 1], v.q, c->scal, A, s));
        launch_cgn_update<T>(c, A ^ 1, v.x, v.r, v.p[A ^ 1], v.q, v.dinv, s);
    }
    return FO_OK;
}

template <class Enqueue>
int launch_chunk(fo_ctx *c, std::tuple<int, int, int, int> key, Enqueue enqueue)
{
    return graph_chunk(c, key, std::function<int(hipStream_t)>(enqueue));
}

// Status copy of slot 0 into scal_host[k], behind everything enqueued so far.
int status_async(fo_ctx *c, int k)
{
    FO_HIP(hipMemcpyAsync(c->scal_host + k, c->scal, sizeof(SolveScalars), hipMemcpyDeviceToHost,
                          c->stream));
    FO_HIP(hipEventRecord(c->ev_poll[k], c->stream));
    return FO_OK;
}

// Runs chunks of `chunk` iterations until the device flags done; adds
// iterations.  Normally two chunks are in flight: the next one is enqueued
// before the host waits for the status of the previous one, so the GPU does
// not idle while the host polls.  When the residual trend of the last two
// statuses says the chunk in flight will finish the solve, no further chunk
// is enqueued ahead of it (a chunk after `done` would be all no-op launches).
// Chunks have even length, so the state stays in slot 0; the final status
// ends in scal_host[0].  A status copy still in flight after the loop only
// rewrites the same final bytes (launches after `done` change nothing).
template <class Chunk>
int cg_loop(fo_ctx *c, Chunk chunk_fn, int chunk, int64_t *iters)
{
    int pending[2], inflight = 0, slot = 0;
    auto launch = [&]() -> int {
        FO_TRY(chunk_fn());
        FO_TRY(status_async(c, slot));
        pending[inflight++] = slot;
        slot ^= 1;
        return FO_OK;
    };
    FO_TRY(launch());  // the first chunk goes out without waiting for the start state
    FO_TRY(launch());
    int32_t before = -1;
    double prev_rr = -1.0;
    SolveScalars last{};
    while (true) {
        const int k = pending[0];
        pending[0] = pending[1];
        --inflight;
        FO_HIP(fo::wait_event(c->ev_poll[k]));
        last = c->scal_host[k];
        if (last.done) break;
        if (last.it == before) {  // no progress: a launch failed
            hipError_t e = hipGetLastError();
            std::fprintf(stderr, "libfo: CG chunk made no progress (%s)\n", hipGetErrorString(e));
            (void)fo::wait_stream(c->stream);
            return FO_ERR_HIP;
        }
        // iterations still needed at the rate of the last chunk
        bool near = false;
        if (prev_rr > 0.0 && last.rr > 0.0 && last.rr < prev_rr && last.tol2 > 0.0 && before >= 0) {
            const double per_it = std::log(last.rr / prev_rr) / (double)(last.it - before);
            near = std::log(last.tol2 / last.rr) / per_it <= (double)chunk;
        }
        prev_rr = last.rr;
        before = last.it;
        if (inflight == 0 || !near) FO_TRY(launch());
    }
    c->scal_host[0] = last;
    *iters += last.it;
    return FO_OK;
}

int chunk_len(const fo_solve_opts *o)
{
    int chunk = o->check_every > 0 ? o->check_every : 16;
    return chunk + (chunk & 1);  // even: the final state is in slot 0
}

template <typename T>
int cg_run(fo_ctx *c, OpKind k, CgVecs<T> v, const fo_solve_opts *o, int64_t *iters)
{
    const int chunk = chunk_len(o);
    auto key = std::make_tuple((int)k, chunk, c->scatter, k == OP_DESCENT64 ? c->descent_version : 0);
    return cg_loop(c, [&]() {
        return launch_chunk(c, key, [&](hipStream_t s) { return cg_chunk<T>(c, k, v, chunk, s); });
    }, chunk, iters);
}

template <typename T>
int fused_run(fo_ctx *c, FusedVecs<T> v, const fo_solve_opts *o, int64_t *iters)
{
    const int chunk = chunk_len(o);
    auto key = std::make_tuple((sizeof(T) == 8 ? 10 : 11) + 2 * v.kind, chunk, c->scatter,
                               v.kind == FUSED_DESCENT ? c->descent_version : 0);
    return cg_loop(c, [&]() {
        return launch_chunk(c, key, [&](hipStream_t s) { return fused_chunk<T>(c, v, chunk, s); });
    }, chunk, iters);
}

template <typename T>
int op_apply(fo_ctx *c, OpKind k, const T *x, T *y, hipStream_t s)
{
    if (k == OP_DESCENT64) return descent_apply(c, (const double *)x, (double *)y, s);
    if (k == OP_HEAT64) {
        if constexpr (sizeof(T) == 8) return launch_heat_apply(c, c->heat_mask, (const double *)x, (double *)y, s);
        return FO_ERR_ARG;
    }
    return elas_apply<T>(c, x, y, s);
}

// Fused CG kernels: elasticity on tiles; the descent operator too when every
// boundary facet lies in a tile.
bool fused_path(const fo_ctx *c, OpKind k)
{
    if (k == OP_HEAT64) return false;
    return tiled(c) && (k != OP_DESCENT64 || c->tiles.facets_ok);
}

int fused_kind(OpKind k) { return k == OP_DESCENT64 ? FUSED_DESCENT : FUSED_ELAS; }

// FP64 Jacobi-PCG on A x = b (b contiguous), stopping on the recomputed
// residual ||b - A x|| <= rtol ||b||.  The solution is left in c->x64.
int solve_fp64(fo_ctx *c, OpKind k, const double *b, const double *dinv, const fo_solve_opts *o,
               fo_solve_stats *st)
{
    const int64_t n = op_len(c, k);
    hipStream_t s = c->stream;
    const bool fused = fused_path(c, k);
    CgVecs<double> v{c->x64, c->r64, c->p64, c->q64, dinv};
    FusedVecs<double> fv{c->x64, c->r64, c->q64, {c->p64, c->p64b}, dinv, fused_kind(k)};
    int64_t iters = 0;
    launch_fill<double>(v.x, n, 0.0, s);
    if (fused) {
        if (c->has_isolated) {
            launch_fill<double>(c->q64, n, 0.0, s);
            launch_fill<double>(c->p64, n, 0.0, s);
            launch_fill<double>(c->p64b, n, 0.0, s);
        }
        launch_cgn_start<double>(c, b, nullptr, v.r, dinv, o->rtol, o->max_iter, s);
    } else {
        launch_cg_start<double>(b, nullptr, v.r, v.p, dinv, n, c->partials, c->scal, o->rtol, -1.0,
                                o->max_iter, s);
    }
    int status = FO_NOT_CONVERGED;
    double relres = 1.0;
    for (int restart = 0; restart < 20; ++restart) {
        FO_TRY(fused ? fused_run<double>(c, fv, o, &iters) : cg_run<double>(c, k, v, o, &iters));
        if (c->scal_host->status == FO_ERR_BREAKDOWN) {
            status = FO_ERR_BREAKDOWN;
            break;
        }
        // recompute the residual in FP64; restart from it if needed
        FO_TRY(op_apply<double>(c, k, v.x, v.q, s));
        ++iters;
        int left = (int)std::max<int64_t>(1, (int64_t)o->max_iter - iters);
        if (fused)
            launch_cgn_start<double>(c, b, v.q, v.r, dinv, o->rtol, left, s);
        else
            launch_cg_start<double>(b, v.q, v.r, v.p, dinv, n, c->partials, c->scal, o->rtol, -1.0,
                                    left, s);
        FO_TRY(poll(c));
        const SolveScalars h = *c->scal_host;
        relres = h.bnorm2 > 0 ? std::sqrt(h.rr / h.bnorm2) : 0.0;
        if (h.bnorm2 == 0.0 || relres <= o->rtol) {
            status = FO_OK;
            break;
        }
        if (iters >= o->max_iter) break;
    }
    if (st) {
        st->status = status;
        st->iters_inner = (int32_t)iters;
        st->iters_outer = 0;
        st->rel_res = relres;
    }
    return status;
}

// Iteration cap of a first FP32 phase (no completed phase to compare with):
// Jacobi-PCG iteration counts of the elasticity operator grow like the mesh
// width, i.e. like sqrt(n) in 2D and n^(1/3) in 3D; 8 sqrt(n) is far above what
// a well-resolved first phase needs on both.
}  // namespace

int64_t fo::first_phase_cap(int64_t n) { return std::max<int64_t>(512, (int64_t)(8.0 * std::sqrt((double)n))); }

namespace {

// FP32 CG with FP64 residual replacement.  Phases of FP32 CG each lower the
// (rescaled) residual by inner_rtol; between phases x64 += s x32, the FP64
// residual b - K x64 is recomputed, the FP32 residual is replaced by it and
// the search direction is kept (rescaled), so the Krylov process continues
// instead of restarting.  Stops when ||b - K x64|| <= rtol ||b|| (FP64).
// A phase running four times as long as the longest completed one (at
// least 256 iterations; the first phase: first_phase_cap) is stopped and the
// next one restarts its direction; after two such phases in a row (FP32
// cannot resolve the operator: kappa * eps_32 near 1) the solve finishes with
// FP64 CG on the residual equation.
int solve_ir(fo_ctx *c, OpKind k, const double *b, const fo_solve_opts *o, fo_solve_stats *st)
{
    const bool desc = k == OP_DESCENT64;
    const double *dinv64 = desc ? c->descent.dinv : c->dinv64;
    const int64_t n = c->ndof;
    hipStream_t s = c->stream;
    const int nb = red_blocks(n);
    int64_t inner = 0;
    int outer = 0;
    double *s2 = c->dscratch;  // [0] current scale^2, [1] new residual^2
    launch_fill<double>(c->x64, n, 0.0, s);
    FO_HIP(hipMemcpyAsync(c->r64, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_dots<double>(1, b, b, nullptr, nullptr, nullptr, nullptr, n, c->partials, nb, s);
    launch_finish_dots(c->partials, nb, 1, s2 + 1, s);
    FO_HIP(hipMemcpyAsync(c->red_host, s2 + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    FO_HIP(fo::wait_stream(s));
    const double bnorm = std::sqrt(c->red_host[0]);
    double rn = bnorm;
    int status = FO_NOT_CONVERGED;
    const int max_outer = o->max_outer > 0 ? o->max_outer : 60;
    const double phase_rtol = o->inner_rtol > 0 ? o->inner_rtol : 0.1;
    int fresh = 1;
    int64_t longest = 0;  // iterations of the longest phase that reached its target
    int capped_run = 0;   // consecutive phases stopped at their cap
    const int64_t first_cap = first_phase_cap(n);
    const bool trace = std::getenv("FO_TRACE_IR") != nullptr;  // per-phase log on stderr
    FusedVecs<float> v{c->x32, c->r32, c->q32, {c->p32, c->p32b}, desc ? c->descent.dinv32 : c->dinv32,
                       fused_kind(k)};
    if (c->has_isolated) {
        launch_fill<float>(c->q32, n, 0.0f, s);
        launch_fill<float>(c->p32, n, 0.0f, s);
        launch_fill<float>(c->p32b, n, 0.0f, s);
    }
    while (true) {
        if (bnorm == 0.0 || rn <= o->rtol * bnorm) {
            status = FO_OK;
            break;
        }
        if (outer >= max_outer || inner >= o->max_iter) break;
        const int left = (int)std::max<int64_t>(1, (int64_t)o->max_iter - inner);
        // a phase that runs twice as long as the longest completed one has
        // stagnated (the FP32 recursion lost conjugacy): end it, replace the
        // residual and restart the direction
        const int cap = (int)std::min<int64_t>(left, longest > 0 ? std::max<int64_t>(4 * longest, 256) : first_cap);
        launch_ir_phase(c, c->r64, s2, v.r, v.x, v.dinv, phase_target(phase_rtol, o->rtol, bnorm, rn), cap, fresh,
                        s);
        const int64_t before = inner;
        FO_TRY(fused_run<float>(c, v, o, &inner));
        const bool capped = c->scal_host->it >= cap && c->scal_host->status != FO_ERR_BREAKDOWN;
        if (!capped) longest = std::max<int64_t>(longest, inner - before);
        capped_run = capped ? capped_run + 1 : 0;
        fresh = (c->scal_host->status == FO_ERR_BREAKDOWN || capped) ? 1 : 0;
        if (c->scal_host->it & 1)  // the last direction is in p[1]; phases start from p[0]
            FO_HIP(hipMemcpyAsync(v.p[0], v.p[1], n * sizeof(float), hipMemcpyDeviceToDevice, s));
        launch_ir_accumulate(c->x64, v.x, s2, n, s);
        FO_TRY(op_apply<double>(c, k, c->x64, c->q64, s));
        ++outer;
        launch_residual64(b, c->q64, c->r64, n, c->partials, s2 + 1, s);
        FO_HIP(hipMemcpyAsync(c->red_host, s2 + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        FO_HIP(fo::wait_stream(s));
        const double rn_new = std::sqrt(c->red_host[0]);
        if (!(rn_new == rn_new)) {
            status = FO_ERR_BREAKDOWN;
            break;
        }
        if (fresh && rn_new >= rn) {  // FP32 cannot make progress from here
            rn = rn_new;
            break;
        }
        if (trace)
            std::fprintf(stderr, "libfo: IR phase %d: %lld FP32 its (cap %d%s), |r| %.3e -> %.3e\n", outer,
                         (long long)(inner - before), cap, capped ? ", capped" : "", rn, rn_new);
        rn = rn_new;
        if (capped_run >= 2) break;  // FP32 stagnates (kappa * eps_32 too large): finish in FP64
    }
    if (status == FO_NOT_CONVERGED && capped_run >= 2 && !(rn <= o->rtol * bnorm) && inner < o->max_iter) {
        // FP64 CG on the residual equation K d = r64 to the same absolute
        // target, then x64 += d
        FO_HIP(hipMemcpyAsync(c->x64b, c->x64, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        FO_HIP(hipMemcpyAsync(c->t64, c->r64, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        fo_solve_opts o2 = *o;
        o2.rtol = o->rtol * bnorm / rn;
        o2.max_iter = (int32_t)std::max<int64_t>(1, (int64_t)o->max_iter - inner);
        fo_solve_stats s2st{};
        int rc = solve_fp64(c, k, c->t64, dinv64, &o2, &s2st);
        if (rc < 0 && rc != FO_ERR_BREAKDOWN) return rc;
        inner += s2st.iters_inner;
        launch_add64(c->x64, c->x64b, n, s);
        FO_TRY(op_apply<double>(c, k, c->x64, c->q64, s));
        ++outer;
        launch_residual64(b, c->q64, c->r64, n, c->partials, s2 + 1, s);
        FO_HIP(hipMemcpyAsync(c->red_host, s2 + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        FO_HIP(fo::wait_stream(s));
        rn = std::sqrt(c->red_host[0]);
        status = rc == FO_ERR_BREAKDOWN ? FO_ERR_BREAKDOWN : (rn <= o->rtol * bnorm ? FO_OK : FO_NOT_CONVERGED);
    }
    if (st) {
        st->status = status;
        st->iters_inner = (int32_t)inner;
        st->iters_outer = outer;
        st->rel_res = bnorm > 0 ? rn / bnorm : 0.0;
    }
    return status;
}

}  // namespace

int fo::heat_cg_solve(fo_ctx *c, const uint8_t *fixed, const double *b, const double *dinv, const fo_solve_opts *o,
                      fo_solve_stats *st)
{
    c->heat_mask = fixed;
    return solve_fp64(c, OP_HEAT64, b, dinv, o, st);
}

int fo::fp64_solve(fo_ctx *c, const double *b, const fo_solve_opts *o, fo_solve_stats *st)
{
    return solve_fp64(c, OP_ELAS64, b, c->dinv64, o, st);
}

namespace {

bool descent_same(const fo_ctx *c, const fo_descent_opts *d)
{
    const DescentSetup &s = c->descent;
    if (!s.valid || s.alpha != d->alpha || s.gamma_n != d->gamma_n || s.gamma_s != d->gamma_s ||
        s.fixed_src != d->fixed)
        return false;
    size_t nb = (size_t)std::max(0, d->n_boxes) * 2 * c->dim;
    if (s.boxes.size() != nb) return false;
    for (size_t i = 0; i < nb; ++i)
        if (s.boxes[i] != d->boxes[i]) return false;
    return true;
}

int descent_prepare(fo_ctx *c, const fo_descent_opts *d)
{
    if (descent_same(c, d)) return FO_OK;
    hipStream_t s = c->stream;
    DescentSetup &ds = c->descent;
    if (d->n_boxes > kMaxBoxes) return FO_ERR_ARG;
    ++c->descent_version;
    ds.alpha = d->alpha;
    ds.gamma_n = d->gamma_n;
    ds.gamma_s = d->gamma_s;
    // the mask is copied: the caller's array is not read after this call
    ds.fixed_src = d->fixed;
    ds.fixed = d->fixed ? ds.mask_copy : nullptr;
    if (d->fixed) FO_HIP(hipMemcpyAsync(ds.mask_copy, d->fixed, c->ndof, hipMemcpyDeviceToDevice, s));
    int nbx = std::max(0, d->n_boxes);
    ds.boxes.assign(d->boxes, d->boxes + (size_t)nbx * 2 * c->dim);
    if (nbx > 0) {
        // the host copy stays valid until the transfer has run
        FO_HIP(hipMemcpyAsync(ds.boxes_dev, ds.boxes.data(), ds.boxes.size() * sizeof(double),
                              hipMemcpyHostToDevice, s));
        launch_in_boxes(c, nbx, ds.boxes_dev, ds.in0, s);
        FO_HIP(fo::wait_stream(s));
    } else {
        launch_fill<uint8_t>(ds.in0, c->E, 0, s);
    }
    if (tiled(c)) {
        launch_fill<double>(ds.diag, c->ndof, 0.0, s);
        FO_TRY(launch_descent_diag_tiled(c, ds.diag, s));
    } else {
        launch_descent_diag(c, ds.diag, s);
    }
    launch_invert_diag<double>(ds.diag, ds.fixed, c->ndof, ds.dinv, s);
    launch_invert_diag<float>(ds.diag, ds.fixed, c->ndof, ds.dinv32, s);
    ds.valid = true;
    return FO_OK;
}

bool opts_ok(const fo_solve_opts *o)
{
    return o && (o->precision == FO_FP64 || o->precision == FO_FP32_IR) && o->rtol > 0 &&
           o->max_iter > 0;
}

template <typename T>
int time_cg_op(fo_ctx *c, FusedVecs<T> v, int reps, double *avg_us)
{
    hipStream_t s = c->stream;
    const int64_t n = c->ndof;
    // slot 2: never converges (tol2 < 0, unbounded iteration count) and
    // reuses beta = 1/2 on every launch, so each launch reads p_old.
    SolveScalars h{};
    h.tol2 = -1.0;
    h.beta = 0.5;
    h.first = 1;
    h.max_it = INT32_MAX;
    FO_HIP(hipMemcpyAsync(c->scal + 2, &h, sizeof(h), hipMemcpyHostToDevice, s));
    launch_fill<double>(c->rz_part, 2 * kRedBlocks, 0.0, s);
    launch_fill<T>(v.r, n, T(1), s);
    launch_fill<T>(v.p[0], n, T(1), s);
    FO_TRY(launch_tile_cg<T>(c, v.kind, v.r, v.dinv, v.p[0], v.p[1], v.q, c->scal, 2, s));  // warm-up
    hipEvent_t e0, e1;
    FO_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FO_ERR_HIP;
    }
    int rc = FO_OK;
    (void)hipEventRecord(e0, s);
    for (int k = 0; k < reps && rc == FO_OK; ++k)  // the warm-up folded the partials: the kernel alone
        rc = launch_tile_cg<T>(c, v.kind, v.r, v.dinv, v.p[0], v.p[1], v.q, c->scal, 2, s, false);
    (void)hipEventRecord(e1, s);
    float ms = 0.0f;
    if (rc == FO_OK && (fo::wait_event(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = FO_ERR_HIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == FO_OK && hipGetLastError() != hipSuccess) rc = FO_ERR_HIP;
    if (rc == FO_OK) *avg_us = 1e3 * (double)ms / reps;
    return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char *fo_status_string(int s)
{
    switch (s) {
    case FO_OK: return "ok";
    case FO_NOT_CONVERGED: return "not converged";
    case FO_ERR_ARG: return "invalid argument";
    case FO_ERR_MESH: return "invalid mesh";
    case FO_ERR_NOMEM: return "out of device memory";
    case FO_ERR_HIP: return "HIP runtime error";
    case FO_ERR_BREAKDOWN: return "CG breakdown";
    case FO_ERR_STATE: return "call order (level set or setup missing)";
    case FO_ERR_BUSY: return "no free slot or device-memory budget";
    default: return "unknown status";
    }
}

int64_t fo_device_allocations(void) { return g_device_allocations.load(std::memory_order_relaxed); }

int fo_destroy(fo_ctx *c)
{
    if (!c) return FO_ERR_ARG;
    if (c->stream) (void)fo::wait_stream(c->stream);
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    if (c->work) (void)hipStreamDestroy(c->work);
    for (hipEvent_t e : c->ev_poll)
        if (e) (void)hipEventDestroy(e);
    for (auto &v : c->prof_events)
        for (auto &pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    batch_release(c);
    for (void *p : c->allocations) (void)hipFree(p);
    if (c->scal_host) (void)hipHostFree(c->scal_host);
    if (c->red_host) (void)hipHostFree(c->red_host);
    delete c;
    return FO_OK;
}

namespace {

// fo_create, fo_create_in (ws: the caller's device workspace) and the dry run
// of fo_workspace_bytes (measure: the same host work and allocation sequence,
// no device call; *measured receives the bytes).
int create_context(fo_ctx **out, const fo_mesh *m, const fo_material *mat, int32_t max_rhs, void *stream,
                   void *ws, size_t ws_bytes, size_t *measured)
{
    if (!out || !m || !mat) return FO_ERR_ARG;
    *out = nullptr;
    if (m->dim != 2 && m->dim != 3) return FO_ERR_ARG;
    if (m->n_nodes <= 0 || m->n_elems <= 0 || !m->coords || !m->conn) return FO_ERR_ARG;
    if (m->n_nodes > INT32_MAX || m->n_elems > INT32_MAX) return FO_ERR_ARG;
    if (m->n_bfacets < 0 || (m->n_bfacets > 0 && (!m->bfacets || !m->bnormal))) return FO_ERR_ARG;
    if (max_rhs < 1 || max_rhs > 256) return FO_ERR_ARG;
    if (!(mat->E > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->ersatz > 0 && mat->ersatz <= 1))
        return FO_ERR_ARG;
    const int D = m->dim;
    const int64_t N = m->n_nodes, E = m->n_elems;
    for (int64_t k = 0; k < (int64_t)(D + 1) * E; ++k)
        if (m->conn[k] < 0 || m->conn[k] >= N) return FO_ERR_MESH;
    for (int64_t e = 0; e < E; ++e) {
        double det = host_det(D, m->coords, m->conn, E, e);
        if (!(std::fabs(det) > 0.0) || det != det) return FO_ERR_MESH;
    }
    for (int64_t k = 0; k < (int64_t)D * m->n_bfacets; ++k)
        if (m->bfacets[k] < 0 || m->bfacets[k] >= N) return FO_ERR_MESH;

    fo_ctx *c = new fo_ctx();
    c->measure = measured != nullptr;
    c->ws = static_cast<char *>(ws);
    c->ws_cap = ws ? ws_bytes : 0;
    c->dim = D;
    c->N = N;
    c->E = E;
    c->ndof = N * D;
    c->max_rhs = max_rhs;
    c->stream = (hipStream_t)stream;
    c->ersatz = mat->ersatz;
    c->mu = mat->E / (2.0 * (1.0 + mat->nu));
    c->lam = (D == 2 && mat->plane_stress) ? mat->E * mat->nu / (1.0 - mat->nu * mat->nu)
                                           : mat->E * mat->nu / ((1.0 + mat->nu) * (1.0 - 2.0 * mat->nu));
    if (!c->measure) (void)hipGetDevice(&c->device);
    int rc = FO_OK;
    auto fail = [&](int code) {
        fo_destroy(c);
        return code;
    };
    const bool live = !c->measure;  // device work (uploads, launches, streams)

    // element order: tiles along a Morton curve (identity if tiling is off)
    HostTiles ht;
    int cus = 256;
    {
        hipDeviceProp_t prop;
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
            prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    int tile_elems = tile_target_elems(D, E, cus);
    if (const char *env = std::getenv("FO_TILE_ELEMS")) {  // tuning override
        int v = std::atoi(env);
        if (v > 0) tile_elems = std::min(v, tile_max_elems(D));
    }
    build_tiles(D, N, E, m->coords, m->conn, tile_elems, &ht);
    // the fused CG kernel packs (halo slot + 1) << 3 into 32 bits
    if (!ht.halo_ptr.empty() && ht.halo_ptr.back() >= (1 << 28)) return fail(FO_ERR_MESH);
    std::vector<int32_t> conn_t((size_t)(D + 1) * E);
    for (int a = 0; a <= D; ++a)
        for (int64_t e = 0; e < E; ++e)
            conn_t[(size_t)a * E + e] = m->conn[(int64_t)a * E + ht.perm[e]];

    // h^2 of the transport diffusion: the paper's mesh-size expression
    // (Section "Transport equation"), 4|D|/(N_T sqrt 3) in 2D and
    // (6 sqrt 2 |D|/N_T)^(2/3) in 3D, which is the squared edge of N_T
    // equilateral triangles / regular tetrahedra filling D; |D| = sum of |T|
    {
        double area = 0.0;
        for (int64_t e = 0; e < E; ++e) area += std::fabs(host_det(D, m->coords, m->conn, E, e));
        area /= (D == 2 ? 2.0 : 6.0);
        c->transport_h2 = D == 2 ? 4.0 * area / ((double)E * std::sqrt(3.0))
                                 : std::pow(6.0 * std::sqrt(2.0) * area / (double)E, 2.0 / 3.0);
    }
    std::vector<float> c32((size_t)N * D);
    for (int64_t i = 0; i < N * D; ++i) c32[i] = (float)m->coords[i];
    std::vector<uint8_t> fx((size_t)N * D, 0);
    if (m->dof_fixed)
        for (int64_t i = 0; i < N * D; ++i) fx[i] = m->dof_fixed[i] ? 1 : 0;

    const int64_t n = c->ndof;
    if ((rc = dev_alloc(c, &c->coords, N * D)) || (rc = dev_alloc(c, &c->coords32, N * D)) ||
        (rc = dev_alloc(c, &c->conn, (D + 1) * E)) || (rc = dev_alloc(c, &c->elem_perm, E)) ||
        (rc = dev_alloc(c, &c->fixed, n)) || (rc = dev_alloc(c, &c->chi, E)) ||
        (rc = dev_alloc(c, &c->diag64, n)) || (rc = dev_alloc(c, &c->dinv64, n)) ||
        (rc = dev_alloc(c, &c->dinv32, n)) || (rc = dev_alloc(c, &c->x64, n)) ||
        (rc = dev_alloc(c, &c->r64, n)) || (rc = dev_alloc(c, &c->p64, n)) ||
        (rc = dev_alloc(c, &c->q64, n)) || (rc = dev_alloc(c, &c->b64, n)) ||
        (rc = dev_alloc(c, &c->t64, n)) || (rc = dev_alloc(c, &c->x32, n)) ||
        (rc = dev_alloc(c, &c->r32, n)) || (rc = dev_alloc(c, &c->p32, n)) ||
        (rc = dev_alloc(c, &c->q32, n)) || (rc = dev_alloc(c, &c->b32, n)) ||
        (rc = dev_alloc(c, &c->p64b, n)) || (rc = dev_alloc(c, &c->p32b, n)) ||
        (rc = dev_alloc(c, &c->x64b, n)) ||
        (rc = dev_alloc(c, &c->bb_part, (size_t)kRedBlocks)) ||
        (rc = dev_alloc(c, &c->partials, (size_t)kRedBlocks * 4)) ||
        (rc = dev_alloc(c, &c->pq_part, (size_t)std::max<int64_t>(ht.n_tiles, kRedBlocks))) ||
        (rc = dev_alloc(c, &c->rz_part, (size_t)kRedBlocks * 2)) || (rc = dev_alloc(c, &c->fold, 4 + kFoldGroups)) ||
        (rc = dev_alloc(c, &c->scal, 4)) || (rc = dev_alloc(c, &c->dscratch, 16)) ||
        (rc = dev_alloc(c, &c->gbuf, N * (D + 1))))
        return fail(rc);
    if ((rc = dev_alloc(c, &c->s1buf, (size_t)E * D * D))) return fail(rc);
    // velocity operator (its diagonal is built by the first velocity solve)
    // and the transport / reinitialisation work buffers
    {
        DescentSetup &ds = c->descent;
        if ((rc = dev_alloc(c, &ds.in0, E)) || (rc = dev_alloc(c, &ds.diag, n)) ||
            (rc = dev_alloc(c, &ds.dinv, n)) || (rc = dev_alloc(c, &ds.dinv32, n)) ||
            (rc = dev_alloc(c, &ds.rhs, n)) || (rc = dev_alloc(c, &ds.boxes_dev, (size_t)kMaxBoxes * 2 * D)) ||
            (rc = dev_alloc(c, &ds.mask_copy, n)) ||
            (rc = fo::ctx_alloc(c, &c->tr_buf, tr_buffer_bytes(c))))
            return fail(rc);
    }
    {
        std::vector<uint8_t> used(N, 0);
        for (int64_t k = 0; k < (int64_t)(D + 1) * E; ++k) used[m->conn[k]] = 1;
        c->has_isolated = std::find(used.begin(), used.end(), 0) != used.end();
    }
    // shape-derivative partial sums: one row per RHS (+ volume)
    c->sd_part_cap = (int)std::min<int64_t>(((E + kBlock - 1) / kBlock) * (max_rhs + 1), INT32_MAX);
    if ((rc = dev_alloc(c, &c->sd_part, c->sd_part_cap))) return fail(rc);
    if (live && (hipHostMalloc((void **)&c->scal_host, 2 * sizeof(SolveScalars)) != hipSuccess ||
                 hipHostMalloc((void **)&c->red_host, 16 * sizeof(double)) != hipSuccess))
        return fail(FO_ERR_NOMEM);
    std::vector<int32_t> bnode, bptr, bfac;
    if (m->n_bfacets > 0) {
        c->nbf = m->n_bfacets;
        if ((rc = dev_alloc(c, &c->bfacets, D * c->nbf)) || (rc = dev_alloc(c, &c->bnormal, D * c->nbf)))
            return fail(rc);
        // boundary node -> incident facets, nodes and facets in increasing order
        std::vector<int32_t> cnt(N, 0);
        for (int64_t f = 0; f < c->nbf; ++f)
            for (int a = 0; a < D; ++a) ++cnt[m->bfacets[(int64_t)a * c->nbf + f]];
        std::vector<int32_t> idx(N, -1);
        bptr.push_back(0);
        for (int64_t n2 = 0; n2 < N; ++n2)
            if (cnt[n2]) {
                idx[n2] = (int32_t)bnode.size();
                bnode.push_back((int32_t)n2);
                bptr.push_back(bptr.back() + cnt[n2]);
            }
        bfac.assign(bptr.back(), 0);
        std::vector<int32_t> fillp(bptr.begin(), bptr.end() - 1);
        for (int64_t f = 0; f < c->nbf; ++f)
            for (int a = 0; a < D; ++a) {
                int32_t n2 = m->bfacets[(int64_t)a * c->nbf + f];
                bfac[fillp[idx[n2]]++] = (int32_t)f;
            }
        c->n_bnodes = (int64_t)bnode.size();
        if ((rc = dev_alloc(c, &c->bnodes, bnode.size())) || (rc = dev_alloc(c, &c->bnode_ptr, bptr.size())) ||
            (rc = dev_alloc(c, &c->bnode_fac, bfac.size())))
            return fail(rc);
    }
    hipStream_t s = c->stream;
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return live ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    if (up(c->coords, m->coords, N * D * sizeof(double)) ||
        up(c->coords32, c32.data(), N * D * sizeof(float)) ||
        up(c->conn, conn_t.data(), conn_t.size() * sizeof(int32_t)) ||
        up(c->elem_perm, ht.perm.data(), E * sizeof(int32_t)) ||
        up(c->fixed, fx.data(), n) ||
        (c->nbf && (up(c->bfacets, m->bfacets, D * c->nbf * sizeof(int32_t)) ||
                    up(c->bnormal, m->bnormal, D * c->nbf * sizeof(double)) ||
                    up(c->bnodes, bnode.data(), bnode.size() * sizeof(int32_t)) ||
                    up(c->bnode_ptr, bptr.data(), bptr.size() * sizeof(int32_t)) ||
                    up(c->bnode_fac, bfac.data(), bfac.size() * sizeof(int32_t)))))
        return fail(FO_ERR_HIP);
    if ((rc = upload_tiles(c, ht))) return fail(rc);
    // large meshes fold the fused CG's partials first: the r.z / r.r ones
    // beyond one pass of the loads of the tile kernel's wave 0; the per-tile
    // p.q ones, which every update block reads, beyond 8,192 tiles (120x60x60
    // with 5,063 tiles solves in 131.8 ms reading them directly against 140.0
    // with the fold; 256x128x128 with 49,152 tiles needs it)
    c->fold_rz = upd_blocks(c->N) > 4 * 64;
    c->fold_pq = ht.n_tiles > 8 * kUpdBlock;
    // FP32 operator geometry: tile-node coordinates relative to the tile's
    // first node, formed in FP64 (kept alive until the stream sync below)
    std::vector<float> tx((size_t)std::max<int64_t>((int64_t)ht.n_tiles * ht.max_nodes * D, 1), 0.0f);
    {
        const int64_t T = ht.n_tiles, MN = ht.max_nodes;
        for (int64_t t = 0; t < T; ++t) {
            const int32_t nn = ht.info[(size_t)t * kTileInfo + kTileNN];
            const double *o = m->coords + (int64_t)ht.nodes[(size_t)t * MN] * D;
            for (int32_t l = 0; l < nn; ++l) {
                const double *x = m->coords + (int64_t)ht.nodes[(size_t)(t * MN + l)] * D;
                for (int q = 0; q < D; ++q) tx[(size_t)(t * MN + l) * D + q] = (float)(x[q] - o[q]);
            }
        }
        if ((rc = dev_alloc(c, &c->tiles.tx32, tx.size())) || up(c->tiles.tx32, tx.data(), tx.size() * sizeof(float)))
            return fail(rc ? rc : FO_ERR_HIP);
    }
    // Boundary facets of the descent operator per tile node: a facet goes to
    // the tile of an element that has it as a face (so all its vertices are
    // nodes of that tile); each of its vertices gets an incidence holding the
    // facet's local vertex ids and a = sqrt(|F| / (d (d+1))) n, so that the
    // facet adds gamma_n a (a . (x_vertex + sum over the facet's vertices x))
    // at the vertex.  Kept alive until the stream sync below.
    std::vector<int32_t> fptr_h;
    std::vector<uint64_t> fconn_h;
    std::vector<double> fa64_h;
    std::vector<float> fa32_h;
    c->tiles.facets_ok = true;
    if (c->nbf > 0 && ht.n_tiles > 0) {
        const int64_t F = c->nbf, T = ht.n_tiles, MN = ht.max_nodes;
        std::vector<int32_t> nptr((size_t)N + 1, 0), nel((size_t)(D + 1) * E);
        for (int64_t k = 0; k < (int64_t)(D + 1) * E; ++k) ++nptr[(size_t)conn_t[k] + 1];
        for (int64_t i = 0; i < N; ++i) nptr[i + 1] += nptr[i];
        {
            std::vector<int32_t> fill(nptr.begin(), nptr.end() - 1);
            for (int64_t e = 0; e < E; ++e)
                for (int a = 0; a <= D; ++a) nel[fill[conn_t[(size_t)a * E + e]]++] = (int32_t)e;
        }
        std::vector<int32_t> etile((size_t)E);
        for (int64_t t = 0; t < T; ++t) {
            const int32_t e0 = ht.info[(size_t)t * kTileInfo + kTileE0];
            const int32_t ne = ht.info[(size_t)t * kTileInfo + kTileNE];
            for (int32_t i = 0; i < ne; ++i) etile[(size_t)e0 + i] = (int32_t)t;
        }
        std::vector<int32_t> ftile((size_t)F, -1);
        for (int64_t f = 0; f < F && c->tiles.facets_ok; ++f) {
            const int32_t v0 = m->bfacets[f];
            for (int32_t k = nptr[v0]; k < nptr[v0 + 1] && ftile[f] < 0; ++k) {
                const int64_t e = nel[k];
                bool all = true;
                for (int b = 1; b < D && all; ++b) {
                    const int32_t vb = m->bfacets[(int64_t)b * F + f];
                    bool in = false;
                    for (int a = 0; a <= D; ++a) in = in || conn_t[(size_t)a * E + e] == vb;
                    all = in;
                }
                if (all) ftile[f] = etile[e];
            }
            if (ftile[f] < 0) c->tiles.facets_ok = false;
        }
        if (c->tiles.facets_ok) {
            // facets grouped by tile (increasing facet id within a tile)
            std::vector<int64_t> tptr((size_t)T + 1, 0), tfac((size_t)F);
            for (int64_t f = 0; f < F; ++f) ++tptr[(size_t)ftile[f] + 1];
            for (int64_t t = 0; t < T; ++t) tptr[t + 1] += tptr[t];
            {
                std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
                for (int64_t f = 0; f < F; ++f) tfac[fill[ftile[f]]++] = f;
            }
            std::vector<int32_t> loc((size_t)N, -1);
            fptr_h.assign((size_t)T * (MN + 1), 0);
            struct Inc {
                int32_t l;
                int64_t f;
                uint64_t conn;
            };
            std::vector<Inc> inc;
            for (int64_t t = 0; t < T; ++t) {
                const int32_t nn = ht.info[(size_t)t * kTileInfo + kTileNN];
                for (int32_t l = 0; l < nn; ++l) loc[ht.nodes[(size_t)t * MN + l]] = l;
                inc.clear();
                for (int64_t k = tptr[t]; k < tptr[t + 1]; ++k) {
                    const int64_t f = tfac[k];
                    uint64_t cw = 0;
                    int32_t lid[3] = {0, 0, 0};
                    for (int b = 0; b < D; ++b) {
                        lid[b] = loc[m->bfacets[(int64_t)b * F + f]];
                        cw |= (uint64_t)(uint16_t)lid[b] << (16 * b);
                    }
                    for (int b = 0; b < D; ++b) inc.push_back(Inc{lid[b], f, cw});
                }
                std::stable_sort(inc.begin(), inc.end(), [](const Inc &x, const Inc &y) { return x.l < y.l; });
                const int64_t base = (int64_t)fconn_h.size();
                size_t j = 0;
                for (int32_t l = 0; l <= MN; ++l) {
                    fptr_h[(size_t)t * (MN + 1) + l] = (int32_t)(base + (int64_t)j);
                    while (j < inc.size() && inc[j].l == l) ++j;
                }
                for (const Inc &x : inc) {
                    const int64_t f = x.f;
                    double P[3][3] = {};
                    for (int b = 0; b < D; ++b)
                        for (int q = 0; q < D; ++q) P[b][q] = m->coords[(int64_t)m->bfacets[(int64_t)b * F + f] * D + q];
                    double area;
                    if (D == 2) {
                        area = std::hypot(P[1][0] - P[0][0], P[1][1] - P[0][1]);
                    } else {
                        const double u0 = P[1][0] - P[0][0], u1 = P[1][1] - P[0][1], u2 = P[1][2] - P[0][2];
                        const double v0 = P[2][0] - P[0][0], v1 = P[2][1] - P[0][1], v2 = P[2][2] - P[0][2];
                        const double c0 = u1 * v2 - u2 * v1, c1 = u2 * v0 - u0 * v2, c2 = u0 * v1 - u1 * v0;
                        area = 0.5 * std::sqrt(c0 * c0 + c1 * c1 + c2 * c2);
                    }
                    const double sw = std::sqrt(area / (double)(D * (D + 1)));
                    fconn_h.push_back(x.conn);
                    for (int q = 0; q < 4; ++q) {
                        const double a = q < D ? sw * m->bnormal[f * D + q] : 0.0;
                        fa64_h.push_back(a);
                        fa32_h.push_back((float)a);
                    }
                }
                for (int32_t l = 0; l < nn; ++l) loc[ht.nodes[(size_t)t * MN + l]] = -1;
            }
            c->tiles.n_fent = (int64_t)fconn_h.size();
            if (c->tiles.n_fent > INT32_MAX) return fail(FO_ERR_MESH);
            if ((rc = dev_alloc(c, &c->tiles.fptr, fptr_h.size())) ||
                (rc = dev_alloc(c, &c->tiles.fconn, std::max<size_t>(fconn_h.size(), 1))) ||
                (rc = dev_alloc(c, &c->tiles.fa64, std::max<size_t>(fa64_h.size(), 4))) ||
                (rc = dev_alloc(c, &c->tiles.fa32, std::max<size_t>(fa32_h.size(), 4))))
                return fail(rc);
            if (up(c->tiles.fptr, fptr_h.data(), fptr_h.size() * sizeof(int32_t)) ||
                (c->tiles.n_fent > 0 &&
                 (up(c->tiles.fconn, fconn_h.data(), fconn_h.size() * sizeof(uint64_t)) ||
                  up(c->tiles.fa64, fa64_h.data(), fa64_h.size() * sizeof(double)) ||
                  up(c->tiles.fa32, fa32_h.data(), fa32_h.size() * sizeof(float)))))
                return fail(FO_ERR_HIP);
        }
    }
    if (live && (rc = tiled_prepare(c))) return fail(rc);
    if (live && (hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking) != hipSuccess ||
                 hipEventCreateWithFlags(&c->ev_poll[0], hipEventDisableTiming) != hipSuccess ||
                 hipEventCreateWithFlags(&c->ev_poll[1], hipEventDisableTiming) != hipSuccess))
        return fail(FO_ERR_HIP);
    if (max_rhs > 1 && tiled(c) && (rc = batch_setup(c, max_rhs, m->coords, conn_t))) return fail(rc);
    if (live && fo::wait_stream(s) != hipSuccess) return fail(FO_ERR_HIP);
    if (measured) {
        *measured = c->bytes;
        fo_destroy(c);
        return FO_OK;
    }
    *out = c;
    return FO_OK;
}

}  // namespace

int fo_create(fo_ctx **out, const fo_mesh *m, const fo_material *mat, int32_t max_rhs, void *stream)
{
    return create_context(out, m, mat, max_rhs, stream, nullptr, 0, nullptr);
}

size_t fo_workspace_bytes(const fo_mesh *m, const fo_material *mat, int32_t max_rhs)
{
    fo_ctx *c = nullptr;
    size_t bytes = 0;
    if (create_context(&c, m, mat, max_rhs, nullptr, nullptr, 0, &bytes) != FO_OK) return 0;
    return bytes;
}

int fo_create_in(fo_ctx **out, const fo_mesh *m, const fo_material *mat, int32_t max_rhs, void *stream, void *ws,
                 size_t ws_bytes)
{
    if (!out) return FO_ERR_ARG;
    *out = nullptr;
    if (!ws || ((uintptr_t)ws & 255) != 0 || ws_bytes == 0) return FO_ERR_ARG;
    return create_context(out, m, mat, max_rhs, stream, ws, ws_bytes, nullptr);
}

size_t fo_footprint_bytes(const fo_ctx *c) { return c ? c->bytes : 0; }
size_t fo_footprint_estimate(const fo_mesh *m)
{
    if (!m || (m->dim != 2 && m->dim != 3) || m->n_nodes <= 0 || m->n_elems <= 0) return 0;
    const size_t D = (size_t)m->dim, N = (size_t)m->n_nodes, E = (size_t)m->n_elems, n = N * D;
    const size_t F = m->n_bfacets > 0 ? (size_t)m->n_bfacets : 0;
    size_t b = 0;
    b += N * D * 12 + (D + 1) * E * 4 + E * 4 + n + E;   // coordinates, connectivity, perm, clamp, chi
    b += n * 8 * 2 + n * 4;                               // diagonal, Jacobi FP64/FP32
    b += n * 8 * 7 + n * 4 * 6;                           // Krylov vectors FP64 / FP32
    b += (size_t)kRedBlocks * 8 * 8 + 8192;               // partial sums, scalars
    b += N * (D + 1) * 8 + E * D * D * 8;                 // level-set recovery, S1 tensors
    b += ((E + kBlock - 1) / kBlock) * 2 * 8;             // derivative partials
    b += F * D * 12 + F * 8 + N * 8;                      // facets, normals, boundary nodes
    // tiles of the target size for 256 CUs (a quarter more for tiles that the
    // node cap closes early), nodes per tile at 2.5x the mesh's node/element
    // ratio (the tile surface), padded per-tile arrays, tile-node pairs and
    // halo slots, halo partials of d+1 values per slot
    const size_t target = (size_t)tile_target_elems((int)D, (int64_t)E, 256);
    const size_t T = (E + target - 1) / target * 5 / 4 + 1;
    const size_t ME = std::min<size_t>(E, target);
    const size_t MN = std::min<size_t>((size_t)tile_max_nodes((int)D), (ME * N * 5) / (2 * E) + 16);
    b += T * (32 + ME * 16 + MN * 10) + N * 8 + N * 3 * 4;
    b += std::min(T * MN, (D + 1) * E) * (D + 1) * 8;
    b += E + 3 * n * 8 + n * 4 + n + (size_t)kMaxBoxes * 2 * D * 8;  // velocity operator arrays
    b += (N * D + 16 * N + 16 + 5 * (size_t)kRedBlocks + N / 8 + 1) * 8 + 512;  // transport buffers
    b += 80 * 256;                                        // allocation rounding
    return b;
}

int fo_profile_enable(fo_ctx *c, int32_t on)
{
    if (!c) return FO_ERR_ARG;
    FO_HIP(fo::wait_stream(c->stream));
    c->prof = on != 0;
    for (int k = 0; k < FO_PROF_COUNT; ++k) c->prof_used[k] = 0;
    return FO_OK;
}

int fo_profile_read(fo_ctx *c, int32_t which, double *total_ms, int64_t *launches)
{
    if (!c || which < 0 || which >= FO_PROF_COUNT) return FO_ERR_ARG;
    FO_HIP(fo::wait_stream(c->stream));
    double tot = 0.0;
    for (size_t i = 0; i < c->prof_used[which]; ++i) {
        float ms = 0.0f;
        FO_HIP(hipEventElapsedTime(&ms, c->prof_events[which][i].first, c->prof_events[which][i].second));
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)c->prof_used[which];
    return FO_OK;
}

int fo_time_kernel(fo_ctx *c, int32_t kernel, int32_t reps, double *avg_us)
{
    if (!c || !avg_us || reps < 1 || reps > 100000 || kernel < 0 || kernel >= FO_KERNEL_COUNT)
        return FO_ERR_ARG;
    if (c->scatter != FO_SCATTER_TILED) return FO_ERR_ARG;
    if (!c->have_phi) return FO_ERR_STATE;
    if (kernel == FO_KERNEL_BATCH_APPLY) {
        if (c->batch.S == 0) return FO_ERR_ARG;
        return batch_time_apply(c, c->batch.S / 16, reps, avg_us);
    }
    if (kernel == FO_KERNEL_CG_OP_FP64)
        return time_cg_op<double>(c, FusedVecs<double>{c->x64, c->r64, c->q64, {c->p64, c->p64b}, c->dinv64, FUSED_ELAS},
                                  reps, avg_us);
    return time_cg_op<float>(c, FusedVecs<float>{c->x32, c->r32, c->q32, {c->p32, c->p32b}, c->dinv32, FUSED_ELAS},
                             reps, avg_us);
}

int fo_set_batch_method(fo_ctx *c, int32_t method)
{
    if (!c || (method != FO_BATCH_BLOCK_CG && method != FO_BATCH_COLUMN_CG)) return FO_ERR_ARG;
    c->batch.method = method;
    return FO_OK;
}

int fo_set_batch_operator(fo_ctx *c, int32_t op)
{
    if (!c || (op != FO_BATCH_OP_NODAL && op != FO_BATCH_OP_ELEMENT)) return FO_ERR_ARG;
    if (op == FO_BATCH_OP_NODAL && c->batch.S > 0 && !c->batch.kb) return FO_ERR_ARG;  // mesh too irregular
    c->batch.op = op;
    return FO_OK;
}

int fo_nodal_stats(const fo_ctx *c, int32_t *slots, int64_t *off_diagonal_blocks, int64_t *bytes)
{
    if (!c) return FO_ERR_ARG;
    const bool have = c->batch.kb != nullptr;
    if (slots) *slots = have ? c->batch.nb : 0;
    if (off_diagonal_blocks) *off_diagonal_blocks = have ? c->batch.n_offdiag : 0;
    if (bytes) *bytes = have ? c->batch.nodal_bytes : 0;
    return FO_OK;
}

int fo_batch_tune(fo_ctx *c, int32_t n_rhs, int32_t *tile_nodes, int32_t *group, double *apply_us)
{
    if (!c || n_rhs < 1 || n_rhs > c->max_rhs) return FO_ERR_ARG;
    if (c->batch.S == 0) return FO_ERR_ARG;
    if (!c->have_phi) return FO_ERR_STATE;
    int best = 0, kc = 0;
    double us = 0.0;
    FO_TRY(batch_tune(c, std::min<int>(n_rhs, c->batch.S), &best, &kc, &us));
    if (tile_nodes) *tile_nodes = best;
    if (group) *group = kc;
    if (apply_us) *apply_us = us;
    return FO_OK;
}

int fo_apply_elasticity_batch(fo_ctx *c, const float *x, float *y, int32_t ncols)
{
    if (!c || !x || !y || ncols < 16 || ncols % 16 != 0 || ncols > c->batch.S) return FO_ERR_ARG;
    if (!c->have_phi) return FO_ERR_STATE;
    return batch_apply_block(c, ncols / 16, x, y);
}

int fo_batch_stats(const fo_ctx *c, int32_t *columns, int32_t *tile_nodes, int32_t *group,
                   int64_t *n_tiles, int64_t *n_halo_slots)
{
    if (!c) return FO_ERR_ARG;
    const BatchState &b = c->batch;
    if (columns) *columns = b.S;
    if (tile_nodes) *tile_nodes = b.tiles.max_nodes;
    if (group) *group = b.group;
    if (n_tiles) *n_tiles = b.tiles.n_tiles;
    if (n_halo_slots) *n_halo_slots = b.tiles.n_shared_slots;
    return FO_OK;
}

int fo_tile_stats(const fo_ctx *c, int64_t *n_tiles, int64_t *max_nodes, int64_t *n_slots,
                  int64_t *n_shared_nodes, int64_t *n_halo_slots)
{
    if (!c) return FO_ERR_ARG;
    if (n_tiles) *n_tiles = c->tiles.n_tiles;
    if (max_nodes) *max_nodes = c->tiles.max_nodes;
    if (n_slots) *n_slots = c->tiles.n_slots;
    if (n_shared_nodes) *n_shared_nodes = c->tiles.n_shared_nodes;
    if (n_halo_slots) *n_halo_slots = c->tiles.n_shared_slots;
    return FO_OK;
}

int fo_set_scatter(fo_ctx *c, int32_t mode)
{
    if (!c || (mode != FO_SCATTER_TILED && mode != FO_SCATTER_ATOMIC)) return FO_ERR_ARG;
    c->scatter = mode;
    return FO_OK;
}

int fo_set_levelset(fo_ctx *c, const double *phi)
{
    if (!c || !phi) return FO_ERR_ARG;
    hipStream_t s = c->stream;
    launch_chi(c->conn, c->E, c->dim, phi, c->chi, s);
    if (tiled(c)) {
        launch_fill<double>(c->diag64, c->ndof, 0.0, s);
        FO_TRY(launch_elas_diag_tiled(c, c->diag64, s));
    } else {
        launch_elas_diag(c, c->diag64, s);
    }
    launch_invert_diag<double>(c->diag64, c->fixed, c->ndof, c->dinv64, s);
    launch_invert_diag<float>(c->diag64, c->fixed, c->ndof, c->dinv32, s);
    FO_TRY(batch_levelset(c));
    FO_HIP(hipGetLastError());
    c->have_phi = true;
    return FO_OK;
}

int fo_apply_elasticity(fo_ctx *c, const void *x, void *y, int32_t precision)
{
    if (!c || !x || !y) return FO_ERR_ARG;
    if (!c->have_phi) return FO_ERR_STATE;
    int rc;
    if (precision == FO_FP64) rc = elas_apply<double>(c, (const double *)x, (double *)y, c->stream);
    else if (precision == FO_FP32_IR) rc = elas_apply<float>(c, (const float *)x, (float *)y, c->stream);
    else return FO_ERR_ARG;
    FO_HIP(hipGetLastError());
    return rc;
}

int fo_state_solve(fo_ctx *c, const double *b, double *u, int32_t n_rhs, int64_t ld,
                   const fo_solve_opts *o, fo_solve_stats *st)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !b || !u || !opts_ok(o) || n_rhs < 1 || n_rhs > c->max_rhs || ld < n_rhs)
        return FO_ERR_ARG;
    if (!c->have_phi) return FO_ERR_STATE;
    if (o->precision == FO_FP32_IR && !tiled(c)) return FO_ERR_ARG;  // IR runs on the tiled operator
    hipStream_t s = c->stream;
    int worst = FO_OK;
    fo_solve_stats acc{FO_OK, 0, 0, 0.0, 0.0};
    if (o->precision == FO_FP32_IR && n_rhs > 1 && c->batch.S > 0) {
        worst = batch_solve(c, b, u, n_rhs, ld, o, &acc);
        if (worst < 0 && worst != FO_ERR_BREAKDOWN) return worst;
        acc.status = worst;
        acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (st) *st = acc;
        return worst;
    }
    for (int k = 0; k < n_rhs; ++k) {
        launch_gather_col<double, double>(b + k, ld, c->ndof, c->b64, c->fixed, s);
        fo_solve_stats one{};
        int rc = o->precision == FO_FP64 ? solve_fp64(c, OP_ELAS64, c->b64, c->dinv64, o, &one)
                                         : solve_ir(c, OP_ELAS64, c->b64, o, &one);
        if (rc < 0 && rc != FO_ERR_BREAKDOWN) return rc;
        launch_scatter_col<double>(c->x64, c->ndof, u + k, ld, s);
        acc.iters_inner += one.iters_inner;
        acc.iters_outer += one.iters_outer;
        acc.rel_res = std::max(acc.rel_res, one.rel_res);
        if (rc != FO_OK && (worst == FO_OK || rc < worst)) worst = rc;
    }
    FO_HIP(fo::wait_stream(s));
    acc.status = worst;
    acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = acc;
    return worst;
}

int fo_shape_derivative(fo_ctx *c, const double *u, int32_t n_rhs, int64_t ld, double lambda_vol,
                        double V, double *rhs, double *S1, double *J, double *vol)
{
    if (!c || !u || !rhs || !J || !vol || n_rhs < 1 || n_rhs > c->max_rhs || ld < n_rhs || !(V > 0))
        return FO_ERR_ARG;
    if (!c->have_phi) return FO_ERR_STATE;
    if (launch_shape_tensor(c, u, n_rhs, ld, lambda_vol / V, S1, J, vol, c->stream)) return FO_ERR_ARG;
    if (tiled(c)) {
        if (c->has_isolated) launch_fill<double>(rhs, c->ndof, 0.0, c->stream);
        FO_TRY(launch_sd_rhs_tiled(c, rhs, c->stream));
    } else {
        launch_sd_rhs_atomic(c, rhs, c->stream);
    }
    FO_HIP(hipGetLastError());
    return FO_OK;
}

int fo_apply_descent(fo_ctx *c, const fo_descent_opts *d, const double *x, double *y)
{
    if (!c || !d || !x || !y || d->n_boxes < 0 || (d->n_boxes > 0 && !d->boxes)) return FO_ERR_ARG;
    FO_TRY(descent_prepare(c, d));
    FO_TRY(descent_apply(c, x, y, c->stream));
    FO_HIP(hipGetLastError());
    return FO_OK;
}

int fo_descent_solve(fo_ctx *c, const fo_descent_opts *d, const double *rhs, double *theta,
                     const fo_solve_opts *o, fo_solve_stats *st, double *B_tt)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !d || !rhs || !theta || !opts_ok(o) || d->n_boxes < 0 || (d->n_boxes > 0 && !d->boxes))
        return FO_ERR_ARG;
    if (!(d->alpha > 0) || d->gamma_n < 0 || d->gamma_s < 0) return FO_ERR_ARG;
    FO_TRY(descent_prepare(c, d));
    hipStream_t s = c->stream;
    fo_solve_stats one{};
    const double *b = rhs;
    if (c->descent.fixed) {  // theta = 0 on the mask: solve with those entries of rhs zeroed
        FO_HIP(hipMemcpyAsync(c->descent.rhs, rhs, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
        zero_masked(c, c->descent.fixed, c->descent.rhs, s);
        b = c->descent.rhs;
    }
    int rc = o->precision == FO_FP32_IR && fused_path(c, OP_DESCENT64)
                 ? solve_ir(c, OP_DESCENT64, b, o, &one)
                 : solve_fp64(c, OP_DESCENT64, b, c->descent.dinv, o, &one);
    if (rc < 0 && rc != FO_ERR_BREAKDOWN) return rc;
    FO_HIP(hipMemcpyAsync(theta, c->x64, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (B_tt) {
        int nb = red_blocks(c->ndof);
        launch_dots<double>(1, theta, rhs, nullptr, nullptr, nullptr, nullptr, c->ndof, c->partials,
                            nb, s);
        launch_finish_dots(c->partials, nb, 1, B_tt, s);
    }
    FO_HIP(fo::wait_stream(s));
    one.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = one;
    return rc;
}

int fo_levelset_update(fo_ctx *c, const double *theta, double dt, double *phi)
{
    if (!c || !theta || !phi || !(dt == dt)) return FO_ERR_ARG;
    if (tiled(c)) {
        if (c->has_isolated) launch_fill<double>(c->gbuf, c->N * (c->dim + 1), 0.0, c->stream);
        FO_TRY(launch_phigrad_tiled(c, phi, c->gbuf, c->stream));
    } else {
        launch_phigrad_atomic(c, phi, c->gbuf, c->stream);
    }
    launch_phi_update(c, theta, dt, phi, c->stream);
    FO_HIP(hipGetLastError());
    return FO_OK;
}

}  // extern "C"

// Device kernels of libfo: element operators, Krylov vector updates and
// deterministic reductions.  Launch wrappers are declared in fo_launch.h.
#include <hip/hip_runtime.h>

#include "fo_element.h"
#include "fo_ops.h"
#include "fo_reduce.h"
#include "fo_internal.h"
#include "fo_launch.h"

namespace fo {

int red_blocks(int64_t n)
{
    int64_t b = (n + kBlock * 4 - 1) / (kBlock * 4);
    if (b < 1) b = 1;
    if (b > kRedBlocks) b = kRedBlocks;
    return (int)b;
}

// ---------------------------------------------------------------------------
// element-parallel scatter (atomic mode)

template <typename T>
__device__ __forceinline__ void atomic_add(T *p, T v)
{
    atomicAdd(p, v);
}

template <int D, typename T, class Op>
__global__ __launch_bounds__(256) void k_scatter_atomic(Op op, const int32_t *__restrict__ conn,
                                                        int64_t E, const T *__restrict__ coords,
                                                        const T *__restrict__ xin,
                                                        T *__restrict__ out)
{
    constexpr int NX = Op::NX, NV = Op::NV;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int32_t nodes[D + 1];
    T Xv[D + 1][D];
    T Uv[D + 1][NX > 0 ? NX : 1];
    const T *Xp[D + 1];
    const T *Up[D + 1];
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        nodes[a] = conn[(int64_t)a * E + e];
#pragma unroll
        for (int i = 0; i < D; ++i) Xv[a][i] = coords[(int64_t)nodes[a] * D + i];
#pragma unroll
        for (int k = 0; k < NX; ++k) Uv[a][k] = xin[(int64_t)nodes[a] * NX + k];
        Xp[a] = Xv[a];
        Up[a] = Uv[a];
    }
    T res[D + 1][NV];
    op(op.load(e), Xp, Up, res);
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
        for (int v = 0; v < NV; ++v) atomic_add(&out[(int64_t)nodes[a] * NV + v], res[a][v]);
}

// ---------------------------------------------------------------------------
// simple vector kernels

template <typename T>
__global__ void k_fill(T *__restrict__ y, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = v;
}

template <typename T>
__global__ void k_mask(T *__restrict__ y, const uint8_t *__restrict__ fixed, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (fixed[i]) y[i] = T(0);
}

// dinv = 1/diag on free unknowns, 0 on clamped ones (or where diag == 0).
template <typename T>
__global__ void k_invert_diag(const double *__restrict__ diag, const uint8_t *__restrict__ fixed,
                              int64_t n, T *__restrict__ dinv)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double d = diag[i];
        bool f = fixed ? fixed[i] != 0 : false;
        dinv[i] = (T)((f || d == 0.0) ? 0.0 : 1.0 / d);
    }
}

__global__ void k_chi(const int32_t *__restrict__ conn, int64_t E, int dim,
                      const double *__restrict__ phi, uint8_t *__restrict__ chi)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int a = 0; a <= dim; ++a) s += phi[conn[(int64_t)a * E + e]];
        chi[e] = (s / (double)(dim + 1)) < 0.0 ? 1 : 0;
    }
}

// Strided column <-> contiguous vector copies (with precision change).
template <typename S, typename T>
__global__ void k_gather_col(const S *__restrict__ src, int64_t ld, int64_t n, T *__restrict__ dst,
                             const uint8_t *__restrict__ fixed)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T v = (T)src[i * ld];
        dst[i] = (fixed && fixed[i]) ? T(0) : v;
    }
}

template <typename T>
__global__ void k_scatter_col(const T *__restrict__ src, int64_t n, double *__restrict__ dst,
                              int64_t ld)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i * ld] = (double)src[i];
}

// ---------------------------------------------------------------------------
// dot products into fixed-size partial arrays

// part[k * nb + block] for k < npair: sum_i a_k[i] * b_k[i]
template <typename T>
__global__ __launch_bounds__(256) void k_dots(int npair, const T *__restrict__ a0,
                                              const T *__restrict__ b0, const T *__restrict__ a1,
                                              const T *__restrict__ b1, const T *__restrict__ a2,
                                              const T *__restrict__ b2, int64_t n,
                                              double *__restrict__ part)
{
    __shared__ double lds[4];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        s0 += (double)a0[i] * (double)b0[i];
        if (npair > 1) s1 += (double)a1[i] * (double)b1[i];
        if (npair > 2) s2 += (double)a2[i] * (double)b2[i];
    }
    double r0 = block_sum(s0, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = r0;
    if (npair > 1) {
        double r1 = block_sum(s1, lds);
        if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = r1;
    }
    if (npair > 2) {
        double r2 = block_sum(s2, lds);
        if (threadIdx.x == 0) part[2 * gridDim.x + blockIdx.x] = r2;
    }
}

// out[k] = sum of partial row k (k < npair), one block.
__global__ __launch_bounds__(256) void k_finish_dots(const double *__restrict__ part, int nb,
                                                     int npair, double *__restrict__ out)
{
    __shared__ double lds[4];
    for (int k = 0; k < npair; ++k) {
        double s = block_sum_partials(part + (int64_t)k * nb, nb, lds);
        if (threadIdx.x == 0) out[k] = s;
    }
}

// ---------------------------------------------------------------------------
// mixed precision helpers

__global__ void k_to_float(const double *__restrict__ a, float *__restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------
// shape derivative, element pass: S1_e (tile order) and the J / volume partials

template <int D>
__global__ __launch_bounds__(256) void k_shape_tensor(
    const int32_t *__restrict__ conn, const int32_t *__restrict__ perm, int64_t E,
    const double *__restrict__ coords, const uint8_t *__restrict__ chi, double ersatz,
    double lam, double mu, const double *__restrict__ u, int n_rhs, int64_t ld,
    double vol_coef, double *__restrict__ s1buf, double *__restrict__ S1,
    double *__restrict__ part /*[(n_rhs+1)][nb]*/)
{
    __shared__ double lds[4];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = e < E;
    double vol = 0.0;
    Geom<D, double> g;
    int32_t nodes[D + 1];
    double A = 0.0;
    double S[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) S[i][j] = 0.0;
    if (act) {
        double Xv[D + 1][D];
        const double *Xp[D + 1];
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            nodes[a] = conn[(int64_t)a * E + e];
#pragma unroll
            for (int i = 0; i < D; ++i) Xv[a][i] = coords[(int64_t)nodes[a] * D + i];
            Xp[a] = Xv[a];
        }
        g = geom<D, double>(Xp);
        A = chi[e] ? 1.0 : ersatz;
        vol = fabs(g.det) / (D == 2 ? 2.0 : 6.0);
    }
    for (int k = 0; k < n_rhs; ++k) {
        double Jk = 0.0;
        if (act) {
            double Uv[D + 1][D];
            const double *Up[D + 1];
#pragma unroll
            for (int a = 0; a <= D; ++a) {
#pragma unroll
                for (int i = 0; i < D; ++i) Uv[a][i] = u[((int64_t)nodes[a] * D + i) * ld + k];
                Up[a] = Uv[a];
            }
            double Dt[D][D], se;
            grad_scaled<D, double>(g, Up, Dt);
            // with Dt = det Du:  A (2 Du^T sigma - sigma:eps I) = (A / det^2) (2 Dt^T St - St:Dt I)
            double s2 = A / (g.det * g.det);
            shape_tensor_scaled<D, double>(Dt, lam, mu, S, s2, &se);
            Jk = A * inv_measure_det2<D, double>(g.det) * se;  // A |T| sigma : eps
        }
        double t = block_sum(Jk, lds);
        if (threadIdx.x == 0) part[(int64_t)k * gridDim.x + blockIdx.x] = t;
    }
    double vs = block_sum(act && chi[e] ? vol : 0.0, lds);
    if (threadIdx.x == 0) part[(int64_t)n_rhs * gridDim.x + blockIdx.x] = vs;
    if (!act) return;
    if (chi[e]) {
#pragma unroll
        for (int i = 0; i < D; ++i) S[i][i] += vol_coef;
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) s1buf[e * D * D + i * D + j] = S[i][j];
    if (S1) {
        int64_t eo = perm[e];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) S1[(int64_t)(i * D + j) * E + eo] = S[i][j];
    }
}

// J[k] and vol from the partial rows of k_shape_tensor.
__global__ __launch_bounds__(256) void k_finish_sd(const double *__restrict__ part, int nb,
                                                   int n_rhs, double *__restrict__ J,
                                                   double *__restrict__ vol)
{
    __shared__ double lds[4];
    for (int k = 0; k <= n_rhs; ++k) {
        double s = block_sum_partials(part + (int64_t)k * nb, nb, lds);
        if (threadIdx.x == 0) {
            if (k < n_rhs) J[k] = s;
            else *vol = s;
        }
    }
}

// element centroid inside one of the open boxes
__global__ void k_in_boxes(const int32_t *__restrict__ conn, int64_t E, int dim,
                           const double *__restrict__ coords, int nbox,
                           const double *__restrict__ boxes, uint8_t *__restrict__ in0)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
         e += (int64_t)gridDim.x * blockDim.x) {
        double c[3] = {0, 0, 0};
        for (int a = 0; a <= dim; ++a)
            for (int i = 0; i < dim; ++i) c[i] += coords[(int64_t)conn[(int64_t)a * E + e] * dim + i];
        for (int i = 0; i < dim; ++i) c[i] /= (double)(dim + 1);
        uint8_t in = 0;
        for (int k = 0; k < nbox && !in; ++k) {
            bool ok = true;
            for (int i = 0; i < dim; ++i)
                ok = ok && c[i] > boxes[k * 2 * dim + i] && c[i] < boxes[k * 2 * dim + dim + i];
            in = ok ? 1 : 0;
        }
        in0[e] = in;
    }
}

// phi_i -= dt theta_i . G_i / W_i   (gbuf rows: G_i (D values), W_i)
template <int D>
__global__ void k_phi_update(const double *__restrict__ gbuf, const double *__restrict__ theta,
                             double dt, double *__restrict__ phi, int64_t N)
{
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * blockDim.x) {
        double w = gbuf[n * (D + 1) + D];
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) s += theta[n * D + i] * gbuf[n * (D + 1) + i];
        phi[n] -= dt * (w > 0.0 ? s / w : 0.0);
    }
}


// ---------------------------------------------------------------------------
// launch wrappers

static inline int grid_for(int64_t n, int per = 1)
{
    int64_t b = (n + (int64_t)kBlock * per - 1) / ((int64_t)kBlock * per);
    if (b < 1) b = 1;
    if (b > (1 << 23)) b = 1 << 23;  // covers n <= INT32_MAX at one item per thread
    return (int)b;
}

template <typename T>
void launch_fill(T *y, int64_t n, T v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n, 4)), dim3(kBlock), 0, s, y, n, v);
}
template void launch_fill<double>(double *, int64_t, double, hipStream_t);
template void launch_fill<float>(float *, int64_t, float, hipStream_t);
template void launch_fill<uint8_t>(uint8_t *, int64_t, uint8_t, hipStream_t);

template <typename T>
void launch_mask(T *y, const uint8_t *fixed, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_mask<T>, dim3(grid_for(n, 4)), dim3(kBlock), 0, s, y, fixed, n);
}
template void launch_mask<double>(double *, const uint8_t *, int64_t, hipStream_t);
template void launch_mask<float>(float *, const uint8_t *, int64_t, hipStream_t);

template <typename T>
void launch_invert_diag(const double *diag, const uint8_t *fixed, int64_t n, T *dinv, hipStream_t s)
{
    hipLaunchKernelGGL(k_invert_diag<T>, dim3(grid_for(n, 4)), dim3(kBlock), 0, s, diag, fixed, n,
                       dinv);
}
template void launch_invert_diag<double>(const double *, const uint8_t *, int64_t, double *,
                                         hipStream_t);
template void launch_invert_diag<float>(const double *, const uint8_t *, int64_t, float *,
                                        hipStream_t);

void launch_chi(const int32_t *conn, int64_t E, int dim, const double *phi, uint8_t *chi,
                hipStream_t s)
{
    hipLaunchKernelGGL(k_chi, dim3(grid_for(E, 4)), dim3(kBlock), 0, s, conn, E, dim, phi, chi);
}

template <typename S, typename T>
void launch_gather_col(const S *src, int64_t ld, int64_t n, T *dst, const uint8_t *fixed,
                       hipStream_t s)
{
    hipLaunchKernelGGL((k_gather_col<S, T>), dim3(grid_for(n, 4)), dim3(kBlock), 0, s, src, ld, n,
                       dst, fixed);
}
template void launch_gather_col<double, double>(const double *, int64_t, int64_t, double *,
                                                const uint8_t *, hipStream_t);

template <typename T>
void launch_scatter_col(const T *src, int64_t n, double *dst, int64_t ld, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter_col<T>, dim3(grid_for(n, 4)), dim3(kBlock), 0, s, src, n, dst, ld);
}
template void launch_scatter_col<double>(const double *, int64_t, double *, int64_t, hipStream_t);

template <typename T>
void launch_dots(int npair, const T *a0, const T *b0, const T *a1, const T *b1, const T *a2,
                 const T *b2, int64_t n, double *part, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_dots<T>, dim3(nb), dim3(kBlock), 0, s, npair, a0, b0, a1, b1, a2, b2, n,
                       part);
}
template void launch_dots<double>(int, const double *, const double *, const double *,
                                  const double *, const double *, const double *, int64_t,
                                  double *, int, hipStream_t);
template void launch_dots<float>(int, const float *, const float *, const float *, const float *,
                                 const float *, const float *, int64_t, double *, int, hipStream_t);

void launch_finish_dots(const double *part, int nb, int npair, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_dots, dim3(1), dim3(kBlock), 0, s, part, nb, npair, out);
}

void launch_to_float(const double *a, float *b, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_float, dim3(grid_for(n, 4)), dim3(kBlock), 0, s, a, b, n);
}

// ---- element operators, atomic mode

template <int D, typename T>
static void elas_apply_atomic_d(const fo_ctx *c, const T *coords, const T *x, T *y, hipStream_t s)
{
    ElasOp<D, T> op{c->chi, (T)c->ersatz, (T)c->lam, (T)c->mu};
    hipLaunchKernelGGL((k_scatter_atomic<D, T, ElasOp<D, T>>), dim3(grid_for(c->E)), dim3(kBlock),
                       0, s, op, c->conn, c->E, coords, x, y);
}

template <typename T>
void launch_elas_apply_atomic(const fo_ctx *c, const T *coords, const T *x, T *y, hipStream_t s)
{
    launch_fill<T>(y, c->ndof, T(0), s);
    if (c->dim == 2) elas_apply_atomic_d<2, T>(c, coords, x, y, s);
    else elas_apply_atomic_d<3, T>(c, coords, x, y, s);
    launch_mask<T>(y, c->fixed, c->ndof, s);
}
template void launch_elas_apply_atomic<double>(const fo_ctx *, const double *, const double *,
                                               double *, hipStream_t);
template void launch_elas_apply_atomic<float>(const fo_ctx *, const float *, const float *,
                                              float *, hipStream_t);

void launch_elas_diag(const fo_ctx *c, double *diag, hipStream_t s)
{
    launch_fill<double>(diag, c->ndof, 0.0, s);
    if (c->dim == 2) {
        ElasDiagOp<2, double> op{c->chi, c->ersatz, c->lam, c->mu};
        hipLaunchKernelGGL((k_scatter_atomic<2, double, ElasDiagOp<2, double>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, op, c->conn, c->E, c->coords, (const double *)nullptr,
                           diag);
    } else {
        ElasDiagOp<3, double> op{c->chi, c->ersatz, c->lam, c->mu};
        hipLaunchKernelGGL((k_scatter_atomic<3, double, ElasDiagOp<3, double>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, op, c->conn, c->E, c->coords, (const double *)nullptr,
                           diag);
    }
}

void launch_descent_apply_atomic(const fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    launch_fill<double>(y, c->ndof, 0.0, s);
    const fo::DescentSetup &d = c->descent;
    if (c->dim == 2) {
        DescentOp<2> op{d.in0, d.alpha, d.gamma_s};
        hipLaunchKernelGGL((k_scatter_atomic<2, double, DescentOp<2>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, op, c->conn, c->E, c->coords, x, y);
    } else {
        DescentOp<3> op{d.in0, d.alpha, d.gamma_s};
        hipLaunchKernelGGL((k_scatter_atomic<3, double, DescentOp<3>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, op, c->conn, c->E, c->coords, x, y);
    }
    launch_facet_terms(c, x, y, s);
}

void launch_descent_diag(const fo_ctx *c, double *diag, hipStream_t s)
{
    launch_fill<double>(diag, c->ndof, 0.0, s);
    const fo::DescentSetup &d = c->descent;
    if (c->dim == 2) {
        DescentDiagOp<2> op{d.in0, d.alpha, d.gamma_s};
        hipLaunchKernelGGL((k_scatter_atomic<2, double, DescentDiagOp<2>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, op, c->conn, c->E, c->coords, (const double *)nullptr,
                           diag);
    } else {
        DescentDiagOp<3> op{d.in0, d.alpha, d.gamma_s};
        hipLaunchKernelGGL((k_scatter_atomic<3, double, DescentDiagOp<3>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, op, c->conn, c->E, c->coords, (const double *)nullptr,
                           diag);
    }
    launch_facet_terms(c, nullptr, diag, s);
}

void launch_in_boxes(const fo_ctx *c, int nbox, const double *boxes_dev, uint8_t *in0,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_in_boxes, dim3(grid_for(c->E, 4)), dim3(kBlock), 0, s, c->conn, c->E,
                       c->dim, c->coords, nbox, boxes_dev, in0);
}

int launch_shape_tensor(const fo_ctx *c, const double *u, int n_rhs, int64_t ld, double vol_coef,
                        double *S1, double *J, double *vol, hipStream_t s)
{
    int nb = grid_for(c->E);
    if ((int64_t)nb * (n_rhs + 1) > c->sd_part_cap) return -1;
    if (c->dim == 2)
        hipLaunchKernelGGL(k_shape_tensor<2>, dim3(nb), dim3(kBlock), 0, s, c->conn, c->elem_perm,
                           c->E, c->coords, c->chi, c->ersatz, c->lam, c->mu, u, n_rhs, ld,
                           vol_coef, c->s1buf, S1, c->sd_part);
    else
        hipLaunchKernelGGL(k_shape_tensor<3>, dim3(nb), dim3(kBlock), 0, s, c->conn, c->elem_perm,
                           c->E, c->coords, c->chi, c->ersatz, c->lam, c->mu, u, n_rhs, ld,
                           vol_coef, c->s1buf, S1, c->sd_part);
    hipLaunchKernelGGL(k_finish_sd, dim3(1), dim3(kBlock), 0, s, c->sd_part, nb, n_rhs, J, vol);
    return 0;
}

void launch_sd_rhs_atomic(const fo_ctx *c, double *rhs, hipStream_t s)
{
    launch_fill<double>(rhs, c->ndof, 0.0, s);
    if (c->dim == 2)
        hipLaunchKernelGGL((k_scatter_atomic<2, double, SdRhsOp<2>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, SdRhsOp<2>{c->s1buf}, c->conn, c->E, c->coords,
                           (const double *)nullptr, rhs);
    else
        hipLaunchKernelGGL((k_scatter_atomic<3, double, SdRhsOp<3>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, SdRhsOp<3>{c->s1buf}, c->conn, c->E, c->coords,
                           (const double *)nullptr, rhs);
}

void launch_phigrad_atomic(const fo_ctx *c, const double *phi, double *gbuf, hipStream_t s)
{
    launch_fill<double>(gbuf, c->N * (c->dim + 1), 0.0, s);
    if (c->dim == 2)
        hipLaunchKernelGGL((k_scatter_atomic<2, double, PhiGradOp<2>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, PhiGradOp<2>{}, c->conn, c->E, c->coords, phi, gbuf);
    else
        hipLaunchKernelGGL((k_scatter_atomic<3, double, PhiGradOp<3>>), dim3(grid_for(c->E)),
                           dim3(kBlock), 0, s, PhiGradOp<3>{}, c->conn, c->E, c->coords, phi, gbuf);
}

void launch_phi_update(const fo_ctx *c, const double *theta, double dt, double *phi, hipStream_t s)
{
    if (c->dim == 2)
        hipLaunchKernelGGL(k_phi_update<2>, dim3(grid_for(c->N, 4)), dim3(kBlock), 0, s, c->gbuf,
                           theta, dt, phi, c->N);
    else
        hipLaunchKernelGGL(k_phi_update<3>, dim3(grid_for(c->N, 4)), dim3(kBlock), 0, s, c->gbuf,
                           theta, dt, phi, c->N);
}


}  // namespace fo

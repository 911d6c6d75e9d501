// Kernels of the block conjugate gradient method for many load cases on one
// level set (O'Leary's block CG with Jacobi preconditioning).
//
// The load cases share K(phi), so the search space of all of them can be
// shared: every iteration applies K to a block P of directions (one per load
// case still running) and takes, for every residual column, the best step in
// the span of the whole block.  The directions are kept K-conjugate as a
// block:
//
//   Q = K P,  G = P^T Q = L L^T (Cholesky),
//   Gamma = G^-1 (P^T R),   X += P Gamma,   R -= Q Gamma,   Z = D^-1 R,
//   Delta = G^-1 (Q^T Z_a), P <- Z_a - P Delta,
//
// with Z_a the columns of Z whose residual has not yet reached its target (a
// converged column leaves the block, so the block narrows as the cases
// converge).  G is inverted by Gauss-Jordan elimination; a direction whose
// pivot is below a small fraction (kBcgDrop) of its diagonal is linearly dependent on the
// earlier ones to the precision of the FP32 block and is dropped for that
// step (its row of Gamma and Delta is zero).
//
// Block vectors are FP32 [n_dofs][S] (load case fastest); P and Q use the
// stride SP = 16 NP of the current block width.  The s x s products run on
// the matrix cores (v_mfma_f32_16x16x4f32): the Gram products P^T Q, P^T R,
// Q^T Z contract over the unknowns (each 256-thread block sums its rows and
// writes one partial; the partials are added in FP64 in a fixed order), the
// updates P Gamma, Q Gamma, P Delta contract over the block.  The small
// s x s algebra runs in FP64 in one workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "fo_internal.h"
#include "fo_launch.h"

namespace fo {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row tiles of 16 rows: block b owns tiles [b tpb, (b+1) tpb), its wave w
// every 4th of them from w.
__device__ __forceinline__ int64_t tiles_per_block(int64_t ndof)
{
    const int64_t nt = (ndof + 15) / 16;
    return (nt + gridDim.x - 1) / gridDim.x;
}

// Q's shared rows from the apply's halo (the slots of a shared node summed in
// tile order), clamped shared rows zero; one thread per (shared node,
// component, column).  Interior rows are the apply's own.
template <int D>
__global__ __launch_bounds__(256) void k_bcg_collect(const BatchCtl *__restrict__ ctl, const int32_t *__restrict__ hnode,
                                                     const int32_t *__restrict__ hptr, int64_t n_shared,
                                                     const float *__restrict__ halo, const uint8_t *__restrict__ fixed,
                                                     float *__restrict__ Q, int sp)
{
    if (ctl->done) return;
    const int64_t total = n_shared * D * sp;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t sn = e / (D * sp);
        const int r = (int)(e - sn * D * sp), i = r / sp, q = r - i * sp;
        const int64_t row = (int64_t)hnode[sn] * D + i;
        float v = 0.f;
        for (int j = hptr[sn]; j < hptr[sn + 1]; ++j) v += halo[((int64_t)j * D + i) * sp + q];
        Q[row * sp + q] = fixed[row] ? 0.f : v;
    }
}

// G = P^T Q (tiles on and above the diagonal) and W = P^T R, one partial per
// block: G [SP][SP] (upper tiles) then W [SP][S], row-major.
template <int NP, int NS>
__global__ __launch_bounds__(256) void k_bcg_gram(const BatchCtl *__restrict__ ctl, const float *__restrict__ P,
                                                  const float *__restrict__ Q, const float *__restrict__ R,
                                                  int64_t ndof, float *__restrict__ part)
{
    constexpr int SP = 16 * NP, S = 16 * NS, NG = NP * (NP + 1) / 2, NT = NG + NP * NS;
    __shared__ f32x4 red[NT][64];
    if (ctl->done) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r4 = lane >> 4, c = lane & 15;
    f32x4 acc[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int64_t tpb = tiles_per_block(ndof);
    const int64_t t0 = (int64_t)blockIdx.x * tpb, t1 = t0 + tpb;
    for (int64_t t = t0 + wave; t < t1; t += 4) {
        if (t * 16 >= ndof) break;
#pragma unroll 1
        for (int ks = 0; ks < 4; ++ks) {
            const int64_t row = t * 16 + ks * 4 + r4;
            const bool ok = row < ndof;
            float pv[NP], qv[NP], rv[NS];
#pragma unroll
            for (int m = 0; m < NP; ++m) {
                pv[m] = ok ? P[row * SP + 16 * m + c] : 0.f;
                qv[m] = ok ? Q[row * SP + 16 * m + c] : 0.f;
            }
#pragma unroll
            for (int m = 0; m < NS; ++m) rv[m] = ok ? R[row * S + 16 * m + c] : 0.f;
            int k = 0;
#pragma unroll
            for (int a = 0; a < NP; ++a)
#pragma unroll
                for (int b = a; b < NP; ++b, ++k) acc[k] = mfma4(pv[a], qv[b], acc[k]);
#pragma unroll
            for (int a = 0; a < NP; ++a)
#pragma unroll
                for (int b = 0; b < NS; ++b) acc[NG + a * NS + b] = mfma4(pv[a], rv[b], acc[NG + a * NS + b]);
        }
    }
    for (int w = 0; w < 4; ++w) {  // the four waves' sums in a fixed order
        if (wave == w) {
#pragma unroll
            for (int k = 0; k < NT; ++k) red[k][lane] = w == 0 ? acc[k] : red[k][lane] + acc[k];
        }
        __syncthreads();
    }
    // tile entry (16 a + 4 r4 + i, 16 b + c) sits in lane (r4, c), component i
    float *out = part + (int64_t)blockIdx.x * (SP * SP + SP * S);
    for (int k = wave; k < NT; k += 4) {
        const f32x4 v = red[k][lane];
        int a, b, ld;
        float *o;
        if (k < NG) {
            a = 0;
            int kk = k;
            while (kk >= NP - a) {
                kk -= NP - a;
                ++a;
            }
            b = a + kk;
            ld = SP;
            o = out;
        } else {
            a = (k - NG) / NS;
            b = (k - NG) - a * NS;
            ld = S;
            o = out + SP * SP;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) o[(16 * a + 4 * r4 + i) * ld + 16 * b + c] = v[i];
    }
}

// out[e] = sum over the nb partials of entry e in FP64: four threads per
// entry take every 4th partial, then add their sums in order.
__global__ __launch_bounds__(256) void k_bcg_reduce(const BatchCtl *__restrict__ ctl, const float *__restrict__ part,
                                                    int nb, int E, double *__restrict__ out)
{
    __shared__ double red[4][64];
    if (ctl->done) return;
    const int el = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + el;
    double s = 0.0;
    if (e < E) {
#pragma unroll 8
        for (int p = q; p < nb; p += 4) s += (double)part[(int64_t)p * E + e];
    }
    red[q][el] = s;
    __syncthreads();
    if (q == 0 && e < E) out[e] = (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]);
}

// ---------------------------------------------------------------------------
// Small algebra (one workgroup of 256 threads, FP64 in LDS).  Thread
// (ti, tj) = (tid / 16, tid % 16) owns the entries (ti + 16 r, tj + 16 t).

// Ginv = G^-1 on the numerically independent directions: Gauss-Jordan
// elimination in place (no pivoting: G is symmetric positive semidefinite, so
// the pivots are the squared Cholesky pivots) over the first np directions
// in order; a direction whose pivot is at most `drop` times its diagonal is
// dependent on the earlier ones to working precision and is dropped (its
// row and column of Ginv are zero).  gsum: [sp][sp] Gram sums, of which the
// entries on and above the diagonal are used.  A: [sp][sp] in LDS.
__device__ void bcg_inverse(const double *__restrict__ gsum, int sp, int np, double drop, double *A, int *nlive)
{
    // wave w updates the rows i = w (mod 4), lane j the column j: every LDS
    // access of a wave is one contiguous row
    __shared__ double d0[64], rk[64], ck[64];
    __shared__ double inv_s;
    const int tid = threadIdx.x, w = tid >> 6, j = tid & 63;
    for (int i = w; i < sp; i += 4)
        if (j < sp) A[i * sp + j] = (i < np && j < np) ? gsum[min(i, j) * sp + max(i, j)] : 0.0;
    __syncthreads();
    if (tid < sp) d0[tid] = A[tid * sp + tid];
    if (tid == 0) *nlive = 0;
    __syncthreads();
    for (int k = 0; k < np; ++k) {
        const double p = A[k * sp + k];
        const bool live = p > 0.0 && p > drop * d0[k] && isfinite(p);
        if (tid == 0) inv_s = live ? 1.0 / p : 0.0;
        __syncthreads();
        const double inv = inv_s;
        if (live && tid < sp) {
            rk[tid] = tid == k ? inv : A[k * sp + tid] * inv;
            ck[tid] = A[tid * sp + k];
        }
        __syncthreads();
        if (j < sp) {
            // the wave's 16 rows: all loads first, then the updates, then the stores
            const double rj = live ? rk[j] : 0.0;
            double v[16], cv[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = w + 4 * r;
                v[r] = i < sp ? A[i * sp + j] : 0.0;
                cv[r] = (live && i < sp) ? ck[i] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = w + 4 * r;
                if (!live) {
                    if (i == k || j == k) v[r] = 0.0;
                } else if (i == k) {
                    v[r] = rj;
                } else if (j == k) {
                    v[r] = -cv[r] * inv;
                } else {
                    v[r] -= cv[r] * rj;
                }
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = w + 4 * r;
                if (i < sp) A[i * sp + j] = v[r];
            }
        }
        if (tid == 0 && live) *nlive += 1;
        __syncthreads();
    }
}

// out[i][q] = sum_k Ginv[i][k] IN[k][cols[q]] for q < nc, 0 for nc <= q < ldout;
// IN: [sp][ldin] (global), staged in LDS (T: [sp][64]).
__device__ void bcg_product(const double *Gi, int sp, const double *__restrict__ in, int ldin, const int *cols,
                            int nc, double *T, float *__restrict__ out, int ldout)
{
    const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
    for (int k = ti; k < sp; k += 16)
        for (int q = tj; q < 64; q += 16) T[k * 64 + q] = q < nc ? in[k * ldin + cols[q]] : 0.0;
    __syncthreads();
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[r][t] = 0.0;
    for (int k = 0; k < sp; ++k) {
        double g[4], v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) g[r] = ti + 16 * r < sp ? Gi[(ti + 16 * r) * sp + k] : 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = T[k * 64 + tj + 16 * t];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[r][t] += g[r] * v[t];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int i = ti + 16 * r, q = tj + 16 * t;
            if (i < sp && q < ldout) out[i * ldout + q] = q < nc ? (float)acc[r][t] : 0.f;
        }
    __syncthreads();
}

// After the Gram sums: Ginv, and Gamma = Ginv P^T R for every column.
__global__ __launch_bounds__(256) void k_bcg_step(BatchCtl *__restrict__ ctl, BcgState *__restrict__ st,
                                                  const double *__restrict__ sums, int sp, int S)
{
    extern __shared__ double sm[];
    if (ctl->done) return;
    __shared__ int cols[64];
    __shared__ int nlive;
    double *Gi = sm, *T = sm + sp * sp;
    const int np = st->np;
    bcg_inverse(sums, sp, np, st->drop, Gi, &nlive);
    for (int i = threadIdx.x; i < sp * sp; i += 256) st->Gi[i] = Gi[i];
    if (threadIdx.x < 64) cols[threadIdx.x] = threadIdx.x;
    __syncthreads();
    bcg_product(Gi, sp, sums + sp * sp, S, cols, S, T, st->gam, S);
    if (threadIdx.x == 0 && nlive == 0 && np > 0) {  // no usable direction
        st->status = FO_ERR_BREAKDOWN;
        ctl->done = 1;
    }
}

// After the update: r.r of every column, convergence, the coefficients
// Delta = Ginv Q^T Z_a of the next block, and the iteration count.
__global__ __launch_bounds__(256) void k_bcg_next(BatchCtl *__restrict__ ctl, BcgState *__restrict__ st,
                                                  const double *__restrict__ sums, int sp, int S)
{
    extern __shared__ double sm[];
    if (ctl->done) return;
    double *Gi = sm, *T = sm + sp * sp;
    __shared__ int act[64];
    __shared__ int na_s, stop_s;
    const int tid = threadIdx.x;
    for (int i = tid; i < sp * sp; i += 256) Gi[i] = st->Gi[i];
    const double *rr = sums + sp * S;
    if (tid == 0) {
        int na = 0, bad = 0;
        for (int j = 0; j < S; ++j) {
            st->rr[j] = rr[j];
            if (!st->run[j]) continue;
            if (!isfinite(rr[j])) bad = 1;
            if (rr[j] <= st->tol2) st->run[j] = 0;
            else act[na++] = j;
        }
        for (int q = na; q < 64; ++q) act[q] = 0;
        na_s = na;
        st->it_phase += 1;
        ctl->it += 1;
        if (bad) st->status = FO_ERR_BREAKDOWN;
        const int stop = bad || na == 0 || ctl->it >= ctl->max_it || st->it_phase >= st->cap;
        if (stop) {
            ctl->done = 1;
            st->capped = (!bad && na > 0 && st->it_phase >= st->cap) ? 1 : 0;
        }
        ctl->pad = na;
        stop_s = stop;
    }
    __syncthreads();
    const int na = na_s;
    if (stop_s) return;
    // Delta [sp][sp]: column q for residual column act[q], zero beyond na
    bcg_product(Gi, sp, sums, S, act, na, T, st->del, sp);
    if (tid < 64) st->act[tid] = tid < na ? act[tid] : -1;
    if (tid == 0) {
        st->np = na;
        st->first = 0;
    }
}

// ---------------------------------------------------------------------------
// Row tiles through LDS: a wave loads 16 rows of a block of stride SP with
// coalesced 16-byte loads (NP per lane, into registers, so the next tile's
// loads overlap the current tile's matrix products) and stores them in its
// LDS rows of stride SP + 4, from where the MFMA A operand
// A[m][k] = V[row m][4 s + k] is read without bank conflicts.
template <int NP>
__device__ __forceinline__ void load_rows(const float *__restrict__ V, int64_t rb, int64_t ndof, f32x4 (&v)[NP],
                                          int lane)
{
    constexpr int SP = 16 * NP, C4 = SP / 4;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e = lane + 64 * k, r = e / C4, q = e - r * C4;
        v[k] = rb + r < ndof ? *reinterpret_cast<const f32x4 *>(V + (rb + r) * SP + 4 * q)
                             : f32x4{0.f, 0.f, 0.f, 0.f};
    }
}

template <int NP>
__device__ __forceinline__ void put_rows(float *L, const f32x4 (&v)[NP], int lane)
{
    constexpr int SP = 16 * NP, C4 = SP / 4, LD = SP + 4;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e = lane + 64 * k, r = e / C4, q = e - r * C4;
        *reinterpret_cast<f32x4 *>(L + r * LD + 4 * q) = v[k];
    }
}

// X += P Gamma, R -= Q Gamma; partials of Y = Q^T Z (Z = D^-1 R new) and of
// r.r per column.
template <int NP, int NS>
__global__ __launch_bounds__(256) void k_bcg_update(const BatchCtl *__restrict__ ctl, const BcgState *__restrict__ st,
                                                    const float *__restrict__ P, const float *__restrict__ Q,
                                                    float *__restrict__ X, float *__restrict__ R,
                                                    const float *__restrict__ dinv, int64_t ndof,
                                                    float *__restrict__ part)
{
    constexpr int SP = 16 * NP, S = 16 * NS, LD = SP + 4;
    __shared__ float gam[SP * S];
    __shared__ __align__(16) float tile[4][2][16 * LD];
    __shared__ f32x4 red[NP * NS][64];
    __shared__ double rred[4][S];
    if (ctl->done) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    for (int e = tid; e < SP * S; e += 256) gam[e] = st->gam[e];
    __syncthreads();
    float *Pt = tile[wave][0], *Qt = tile[wave][1];
    f32x4 yacc[NP * NS];
#pragma unroll
    for (int k = 0; k < NP * NS; ++k) yacc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    double rr[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) rr[k] = 0.0;
    const int64_t tpb = tiles_per_block(ndof);
    const int64_t t0 = (int64_t)blockIdx.x * tpb, t1 = min(t0 + tpb, (ndof + 15) / 16);
    f32x4 pv[NP], qv[NP];
    if (t0 + wave < t1) {
        load_rows<NP>(P, (t0 + wave) * 16, ndof, pv, lane);
        load_rows<NP>(Q, (t0 + wave) * 16, ndof, qv, lane);
    }
    for (int64_t t = t0 + wave; t < t1; t += 4) {
        const int64_t rb = t * 16;
        put_rows<NP>(Pt, pv, lane);
        put_rows<NP>(Qt, qv, lane);
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        // this tile's X and R (output layout: rows rb + 4 g + i, column 16 b + c)
        float xo[NS][4], ro[NS][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = rb + 4 * g + i;
#pragma unroll
            for (int b = 0; b < NS; ++b) {
                const bool ok = row < ndof;
                xo[b][i] = ok ? X[row * S + 16 * b + c] : 0.f;
                ro[b][i] = ok ? R[row * S + 16 * b + c] : 0.f;
            }
        }
        if (t + 4 < t1) {  // the next tile's rows, in flight during the products
            load_rows<NP>(P, rb + 64, ndof, pv, lane);
            load_rows<NP>(Q, rb + 64, ndof, qv, lane);
        }
        f32x4 ax[NS], ar[NS];
#pragma unroll
        for (int b = 0; b < NS; ++b) ax[b] = ar[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4 * NP; ++s) {
            const float pa = Pt[c * LD + 4 * s + g], qa = Qt[c * LD + 4 * s + g];
#pragma unroll
            for (int b = 0; b < NS; ++b) {
                const float gv = gam[(4 * s + g) * S + 16 * b + c];
                ax[b] = mfma4(pa, gv, ax[b]);
                ar[b] = mfma4(qa, gv, ar[b]);
            }
        }
        float zv[NS][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = rb + 4 * g + i;
            const bool ok = row < ndof;
            const float di = ok ? dinv[row] : 0.f;
#pragma unroll
            for (int b = 0; b < NS; ++b) {
                const float r = ro[b][i] - ar[b][i];
                if (ok) {
                    const int64_t ix = row * S + 16 * b + c;
                    X[ix] = xo[b][i] + ax[b][i];
                    R[ix] = r;
                }
                rr[b] += (double)r * (double)r;
                zv[b][i] = di * r;
            }
        }
        // Y += Q^T Z over these 16 rows: k-step u takes rows 4 u + g; lane
        // (g, c) needs Z(row 4 u + g, column c), held by lane (u, c) as its
        // component g
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            float qt[NP];
#pragma unroll
            for (int a = 0; a < NP; ++a) qt[a] = Qt[(4 * u + g) * LD + 16 * a + c];
#pragma unroll
            for (int b = 0; b < NS; ++b) {
                float zb = 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = __shfl(zv[b][i], u * 16 + c);
                    if (g == i) zb = v;
                }
#pragma unroll
                for (int a = 0; a < NP; ++a) yacc[a * NS + b] = mfma4(qt[a], zb, yacc[a * NS + b]);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // r.r: lanes of one column (4 row groups), then the waves, in order
#pragma unroll
    for (int b = 0; b < NS; ++b) {
        double v = rr[b];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (g == 0) rred[wave][16 * b + c] = v;
    }
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int k = 0; k < NP * NS; ++k) red[k][lane] = w == 0 ? yacc[k] : red[k][lane] + yacc[k];
        }
        __syncthreads();
    }
    float *out = part + (int64_t)blockIdx.x * (SP * S + S);
    for (int k = wave; k < NP * NS; k += 4) {
        const f32x4 v = red[k][lane];
        const int a = k / NS, b = k - a * NS;
#pragma unroll
        for (int i = 0; i < 4; ++i) out[(16 * a + 4 * g + i) * S + 16 * b + c] = v[i];
    }
    for (int j = tid; j < S; j += 256)
        out[SP * S + j] = (float)((rred[0][j] + rred[1][j]) + (rred[2][j] + rred[3][j]));
}

// P <- Z_a - P Delta (in place, each wave on its own 16-row tiles); on the
// first iteration of a phase P <- Z_a.  Z_a column q = D^-1 R column act[q];
// columns q >= np are zero.
template <int NP, int NS>
__global__ __launch_bounds__(256) void k_bcg_direction(const BatchCtl *__restrict__ ctl,
                                                       const BcgState *__restrict__ st, float *__restrict__ P,
                                                       const float *__restrict__ R, const float *__restrict__ dinv,
                                                       int64_t ndof)
{
    constexpr int SP = 16 * NP, S = 16 * NS, LD = SP + 4;
    __shared__ float del[SP * SP];
    __shared__ __align__(16) float tile[4][16 * LD];
    __shared__ int act[SP];
    if (ctl->done) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    const bool first = st->first != 0;
    for (int e = tid; e < SP * SP; e += 256) del[e] = first ? 0.f : st->del[e];
    for (int e = tid; e < SP; e += 256) act[e] = st->act[e];
    __syncthreads();
    float *Pt = tile[wave];
    const int64_t tpb = tiles_per_block(ndof);
    const int64_t t0 = (int64_t)blockIdx.x * tpb, t1 = min(t0 + tpb, (ndof + 15) / 16);
    f32x4 pv[NP];
    if (!first && t0 + wave < t1) load_rows<NP>(P, (t0 + wave) * 16, ndof, pv, lane);
    for (int64_t t = t0 + wave; t < t1; t += 4) {
        const int64_t rb = t * 16;
        if (!first) {
            // the old rows are in registers before any lane of the wave stores
            put_rows<NP>(Pt, pv, lane);
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
        }
        // Z_a of this tile (output layout)
        float zo[NP][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = rb + 4 * g + i;
            const bool ok = row < ndof;
            const float di = ok ? dinv[row] : 0.f;
#pragma unroll
            for (int b = 0; b < NP; ++b) {
                const int j = act[16 * b + c];
                zo[b][i] = (ok && j >= 0) ? di * R[row * S + j] : 0.f;
            }
        }
        f32x4 acc[NP];
#pragma unroll
        for (int b = 0; b < NP; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (!first) {
            if (t + 4 < t1) load_rows<NP>(P, rb + 64, ndof, pv, lane);  // next tile, in flight
#pragma unroll
            for (int s = 0; s < 4 * NP; ++s) {
                const float pa = Pt[c * LD + 4 * s + g];
#pragma unroll
                for (int b = 0; b < NP; ++b) acc[b] = mfma4(pa, del[(4 * s + g) * SP + 16 * b + c], acc[b]);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = rb + 4 * g + i;
            if (row >= ndof) continue;
#pragma unroll
            for (int b = 0; b < NP; ++b) {
                const int q = 16 * b + c;
                P[row * SP + q] = act[q] >= 0 ? zo[b][i] - acc[b][i] : 0.f;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// P (stride SP) -> Y (stride SN <= SP): the first SN columns.
__global__ __launch_bounds__(256) void k_bcg_restride(const float *__restrict__ P, int sp, float *__restrict__ Y,
                                                      int sn, int64_t ndof)
{
    const int64_t total = ndof * sn;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t row = e / sn;
        const int q = (int)(e - row * sn);
        Y[e] = P[row * sp + q];
    }
}

template <int NP, int NS>
void gram_t(const fo_ctx *c, const BcgBufs &B, hipStream_t s)
{
    const BatchState &b = c->batch;
    hipLaunchKernelGGL((k_bcg_gram<NP, NS>), dim3(kBcgBlocks), dim3(256), 0, s, b.ctl, b.p32, b.q32, b.r32, c->ndof,
                       B.part);
}

template <int NP, int NS>
void update_t(const fo_ctx *c, const BcgBufs &B, hipStream_t s)
{
    const BatchState &b = c->batch;
    hipLaunchKernelGGL((k_bcg_update<NP, NS>), dim3(kBcgBlocks), dim3(256), 0, s, b.ctl, B.st, b.p32, b.q32, b.x32,
                       b.r32, c->dinv32, c->ndof, B.part);
}

template <int NP, int NS>
void direction_t(const fo_ctx *c, const BcgBufs &B, hipStream_t s)
{
    const BatchState &b = c->batch;
    hipLaunchKernelGGL((k_bcg_direction<NP, NS>), dim3(kBcgBlocks), dim3(256), 0, s, b.ctl, B.st, b.p32, b.r32,
                       c->dinv32, c->ndof);
}

// Dispatch over the (NP, NS) pairs with NP <= NS <= 4.
template <template <int, int> class F, class... A>
void by_ps(int NP, int NS, A... a)
{
#define FO_BCG_CASE(p, q)              \
    if (NP == p && NS == q) {          \
        F<p, q>::run(a...);            \
        return;                        \
    }
    FO_BCG_CASE(1, 1) FO_BCG_CASE(1, 2) FO_BCG_CASE(2, 2) FO_BCG_CASE(1, 3) FO_BCG_CASE(2, 3)
    FO_BCG_CASE(3, 3) FO_BCG_CASE(1, 4) FO_BCG_CASE(2, 4) FO_BCG_CASE(3, 4) FO_BCG_CASE(4, 4)
#undef FO_BCG_CASE
}

template <int NP, int NS>
struct GramL {
    static void run(const fo_ctx *c, const BcgBufs &B, hipStream_t s) { gram_t<NP, NS>(c, B, s); }
};
template <int NP, int NS>
struct UpdateL {
    static void run(const fo_ctx *c, const BcgBufs &B, hipStream_t s) { update_t<NP, NS>(c, B, s); }
};
template <int NP, int NS>
struct DirectionL {
    static void run(const fo_ctx *c, const BcgBufs &B, hipStream_t s) { direction_t<NP, NS>(c, B, s); }
};

size_t step_lds(int sp) { return (size_t)(sp * sp + sp * 64) * sizeof(double); }
size_t next_lds(int sp) { return (size_t)(sp * sp + sp * 64) * sizeof(double); }

}  // namespace

// The small kernels take up to 64 KB of dynamic LDS (outside graph capture).
int bcg_prepare()
{
    static int done = 0;
    if (done) return 0;
    if (hipFuncSetAttribute((const void *)k_bcg_step, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)step_lds(64)) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_bcg_next, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)next_lds(64)) != hipSuccess)
        return -1;
    done = 1;
    return 0;
}

size_t bcg_part_floats(int S) { return (size_t)kBcgBlocks * (size_t)(S * S + S * S + S); }

void bcg_direction(const fo_ctx *c, const BcgBufs &B, int NP, int NS, hipStream_t s)
{
    by_ps<DirectionL>(NP, NS, c, B, s);
}

void bcg_iteration(const fo_ctx *c, const BcgBufs &B, int NP, int NS, hipStream_t s)
{
    const BatchState &b = c->batch;
    const int S = 16 * NS, sp = 16 * NP;
    batch_apply_launch(c, NP, b.p32, b.q32, b.ctl, b.cols, s);
    if (b.op == FO_BATCH_OP_ELEMENT && b.tiles.n_shared_nodes > 0) {  // the nodal operator writes every row
        const int64_t tot = b.tiles.n_shared_nodes * c->dim * sp;
        const int grid = (int)std::min<int64_t>((tot + 255) / 256, 8192);
        if (c->dim == 2)
            hipLaunchKernelGGL(k_bcg_collect<2>, dim3(grid), dim3(256), 0, s, b.ctl, b.tiles.halo_node,
                               b.tiles.halo_ptr, b.tiles.n_shared_nodes, b.halo, c->fixed, b.q32, sp);
        else
            hipLaunchKernelGGL(k_bcg_collect<3>, dim3(grid), dim3(256), 0, s, b.ctl, b.tiles.halo_node,
                               b.tiles.halo_ptr, b.tiles.n_shared_nodes, b.halo, c->fixed, b.q32, sp);
    }
    by_ps<GramL>(NP, NS, c, B, s);
    const int E1 = sp * sp + sp * S;
    hipLaunchKernelGGL(k_bcg_reduce, dim3((E1 + 63) / 64), dim3(256), 0, s, b.ctl, B.part, kBcgBlocks, E1, B.sums);
    hipLaunchKernelGGL(k_bcg_step, dim3(1), dim3(256), step_lds(sp), s, b.ctl, B.st, B.sums, sp, S);
    by_ps<UpdateL>(NP, NS, c, B, s);
    const int E2 = sp * S + S;
    hipLaunchKernelGGL(k_bcg_reduce, dim3((E2 + 63) / 64), dim3(256), 0, s, b.ctl, B.part, kBcgBlocks, E2, B.sums);
    hipLaunchKernelGGL(k_bcg_next, dim3(1), dim3(256), next_lds(sp), s, b.ctl, B.st, B.sums, sp, S);
    by_ps<DirectionL>(NP, NS, c, B, s);
}

void bcg_restride(const fo_ctx *c, int sp_from, int sp_to, hipStream_t s)
{
    const BatchState &b = c->batch;
    const int grid = (int)std::min<int64_t>((c->ndof * sp_to + 255) / 256, 4096);
    hipLaunchKernelGGL(k_bcg_restride, dim3(grid), dim3(256), 0, s, b.p32, sp_from, b.q32, sp_to, c->ndof);
    (void)hipMemcpyAsync(b.p32, b.q32, (size_t)c->ndof * sp_to * sizeof(float), hipMemcpyDeviceToDevice, s);
}

}  // namespace fo

// Assembled node-block operator of the batched multi-load solves.
//
// The load cases of a batched solve share K(phi) (the element stiffness of
// the elasticity state equation, Section "Compliance minimization", with the
// ersatz coefficient A_e of the level set).  With tens of right-hand sides
// per application the element matrices are worth assembling: once per level
// set, K(phi) is summed into d x d blocks K_ij, one per ordered pair of
// distinct nodes that share an element -- FP64 sums of the element entries,
// rounded once to FP32.  Every row of an element matrix sums to zero (it
// annihilates rigid translations), so K_ii = -sum_{j != i} K_ij and
//     y_i = sum_{j != i} K_ij (x_j - x_i),
// which needs no diagonal block and, like the element form's vertex
// differences, removes the common part of smooth fields before the FP32
// products.  The blocks are exactly symmetric: both nodes of a pair sum the
// same element entries, written in a transposition-invariant form, in the
// same (ascending element) order.
//
// Apply: one wave owns 64/SP nodes and their S columns (SP = S rounded up to
// a power of two; lane l serves column l mod SP of node l / SP).  Per
// neighbour j and component k, one v_mfma_f32_4x4x1f32 (16 blocks of 4
// columns) adds K_ij[:, k] (x_j - x_i)[k, :] to the node's rows: lane 4b + r
// supplies row r of the block column as the A operand, lane l its column of
// (x_j - x_i)[k] as the B operand, and register r of the result holds row r
// of the node for the lane's column.  Every output row is written once, by
// the wave that owns its node: no scatter, no halo, no atomics, and the sums
// run in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "fo_batch_dev.h"
#include "fo_element.h"
#include "fo_internal.h"
#include "fo_launch.h"
#include "fo_xcd.h"

namespace fo {

constexpr int kNodalWaves = 4;          // waves per block of the apply
constexpr int kNodalMaxBlocks = 2048;   // blocks of the apply (p.q partials per block)
constexpr int kNodalStage = 512;        // largest block floats per node (NB d^2, rounded up to 4)

// Node groups of the apply: a wave takes 64 / SP nodes at a time.
static int nodal_lanes(int S) { return S <= 16 ? 16 : (S <= 32 ? 32 : 64); }

// Upper bound of the apply's blocks at S columns (sizes the p.q partials);
// a multiple of 8 (one share per XCD).
static int nodal_block_cap(int64_t N, int S)
{
    const int64_t groups = (N + 64 / nodal_lanes(S) - 1) / (64 / nodal_lanes(S));
    const int64_t b = (groups + kNodalWaves - 1) / kNodalWaves;
    return xcd_grid((int)std::max<int64_t>(1, std::min<int64_t>(b, kNodalMaxBlocks)));
}

// Blocks of the apply at S columns: as many as are resident at once (one
// round, the waves' node runs balanced), within the cap; a multiple of 8.
int nodal_blocks(const fo_ctx *c, int S)
{
    const int cap = nodal_block_cap(c->N, S);
    const int occ = c->batch.nodal_occ[S / 16 - 1] / 8 * 8;
    return occ > 0 ? std::min(cap, occ) : cap;
}

// Dynamic LDS of the apply: two staging buffers of KW floats (a node's
// blocks) per wave.
static size_t nodal_lds(int KW) { return (size_t)kNodalWaves * 2 * KW * sizeof(float); }

// Rounds of loads per node compiled into the apply at S columns: NB / C when
// one node per wave (S > 32) and it is 1 or 2, else 0 (a loop over NB).
static int nodal_rounds(const BatchState &b, int S)
{
    const int r = b.nb_chunk > 0 ? b.nb / b.nb_chunk : 0;
    return S > 32 && (r == 1 || r == 2) ? r : 0;
}

// K_ij for every (node i, neighbour slot s): the sum over the elements that
// contain both nodes, in ascending element order, of
//   w_e (lam c_ar c_bk + mu c_ak c_br + mu delta_rk c_a . c_b),
// a, b the local indices of i, j in e, c the cofactor vectors and
// w_e = A_e / (d! |det|) (A_e = 1 in the material, the ersatz value
// outside).  Padding slots (j = i) get zero blocks, and so do the KW - NB d^2
// floats after a node's last block.  kb gets the blocks rounded to FP32, kb64
// (nullable; [N][NB][d][d]) the FP64 sums.
template <int D>
__global__ __launch_bounds__(256) void k_nodal_assemble(const int32_t *__restrict__ nbr, int NB, int KW, int64_t N,
                                                        const int32_t *__restrict__ inc_ptr,
                                                        const int32_t *__restrict__ inc_elem,
                                                        const int32_t *__restrict__ conn, int64_t E,
                                                        const double *__restrict__ coords,
                                                        const uint8_t *__restrict__ chi, double ersatz,
                                                        double lam, double mu, float *__restrict__ kb,
                                                        double *__restrict__ kb64)
{
    constexpr int NV = D + 1;
    const int64_t total = N * NB;
    for (int64_t task = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; task < total;
         task += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = task / NB;
        const int32_t j = nbr[task];
        double K[D][D];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int k = 0; k < D; ++k) K[r][k] = 0.0;
        if (j != i) {
            for (int32_t q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q) {
                const int64_t e = inc_elem[q];
                int32_t v[NV];
                int a = -1, b = -1;
#pragma unroll
                for (int t = 0; t < NV; ++t) {
                    v[t] = conn[(int64_t)t * E + e];
                    if (v[t] == i) a = t;
                    if (v[t] == j) b = t;
                }
                if (b < 0 || a < 0) continue;
                double X[NV][D];
                const double *Xp[NV];
#pragma unroll
                for (int t = 0; t < NV; ++t) {
#pragma unroll
                    for (int m = 0; m < D; ++m) X[t][m] = coords[(int64_t)v[t] * D + m];
                    Xp[t] = X[t];
                }
                const Geom<D, double> g = geom<D, double>(Xp);
                double C[NV][D];
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    double c0 = 0.0;
#pragma unroll
                    for (int t = 1; t < NV; ++t) {
                        C[t][m] = g.c[t - 1][m];
                        c0 -= g.c[t - 1][m];
                    }
                    C[0][m] = c0;
                }
                const double w = (chi[e] ? 1.0 : ersatz) * inv_measure_det2<D, double>(g.det);
                double ca[D], cb[D];
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    ca[m] = a == 0 ? C[0][m] : a == 1 ? C[1][m] : a == 2 ? C[2][m] : C[NV - 1][m];
                    cb[m] = b == 0 ? C[0][m] : b == 1 ? C[1][m] : b == 2 ? C[2][m] : C[NV - 1][m];
                }
                double dot = 0.0;
#pragma unroll
                for (int m = 0; m < D; ++m) dot += ca[m] * cb[m];
                // each product is formed so that the (j, i) block is the exact
                // transpose: (ca[r] cb[k]) and (ca[k] cb[r]) swap roles
#pragma unroll
                for (int r = 0; r < D; ++r)
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        K[r][k] += w * (lam * (ca[r] * cb[k]) + mu * (ca[k] * cb[r]) + (r == k ? mu * dot : 0.0));
            }
        }
        const int s = (int)(task - i * NB);
        float *out = kb + i * KW + s * (D * D);
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int k = 0; k < D; ++k) out[r * D + k] = (float)K[r][k];
        if (s == NB - 1)
            for (int t = NB * D * D; t < KW; ++t) kb[i * KW + t] = 0.f;
        if (kb64) {
            double *o64 = kb64 + task * (D * D);
#pragma unroll
            for (int r = 0; r < D; ++r)
#pragma unroll
                for (int k = 0; k < D; ++k) o64[r * D + k] = K[r][k];
        }
    }
}

// Q = K(phi) P on S columns (block vectors [n_dofs][S]); clamped rows of Q
// are 0.  p.q partials per block and column (gridDim.x of them, a multiple
// of 8).  NB is a multiple of C, the neighbours taken per round of loads (7
// or 8, whichever pads the largest neighbourhood less); a node's blocks start
// every KW floats (KW a multiple of 4).  NCH > 0: NB = NCH C, known when
// compiling, so the one-node-per-wave loop is unrolled and every round's
// neighbour ids and rows can be issued ahead of the matrix work (0: NB at
// run time).
template <int D, int S, int C, int NCH>
__global__ __launch_bounds__(64 * kNodalWaves) void k_nodal_apply(
    const int32_t *__restrict__ nbr, const float *__restrict__ kb, int NB, int KW, int64_t N,
    const float *__restrict__ P, float *__restrict__ Q, const uint8_t *__restrict__ fixed,
    double *__restrict__ pq_part, BatchCtl *ctl, const BatchCol *__restrict__ cols)
{
    constexpr int SP = S <= 16 ? 16 : (S <= 32 ? 32 : 64), NPW = 64 / SP, DD = D * D;
    __shared__ int s_stop;
    __shared__ double red[64 * kNodalWaves];
    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int cl = lane % SP, col = cl < S ? cl : S - 1;
    const bool live_col = cl < S;
    const int r = lane & 3, rr = r < D ? r : D - 1;  // rows >= D: any valid row, result unused
    const int64_t groups = (N + NPW - 1) / NPW;
    // XCD x (blocks dealt round-robin: blockIdx mod 8) takes the x-th eighth
    // of the node groups, and its W resident waves sweep it together: wave
    // (b, w) takes groups g0 + 4 b + w + t W, t = 0, 1, ..., so at any time
    // the XCD works on one contiguous window of W groups and the neighbour
    // rows it gathers stay in its L2 between uses.
    const int64_t per_x = (groups + 7) / 8;
    const int nb_x = (int)(gridDim.x >> 3), W = nb_x * kNodalWaves;
    const int64_t xs = (int64_t)(blk & 7) * per_x, g1 = std::min<int64_t>(groups, xs + per_x);
    const int64_t g0 = xs + (int64_t)(blk >> 3) * kNodalWaves;
    // one node per wave: the first node's blocks are loaded before the stop
    // test (the grid is one round of blocks, so the test's dependent loads
    // would otherwise stand in front of every block's first data)
    const int KQ = KW / 4;
    f32x4 pre[kNodalStage / 256];
    auto fetch = [&](int64_t n) {
        const f32x4 *src = reinterpret_cast<const f32x4 *>(kb + n * KW);
#pragma unroll
        for (int q = 0; q < kNodalStage / 256; ++q)
            if (lane + 64 * q < KQ) pre[q] = src[lane + 64 * q];
    };
    if constexpr (NPW == 1)
        if (g0 + wave < g1) fetch(g0 + wave);
    if (tid == 0) s_stop = batch_stop(ctl, cols, S);
    __syncthreads();
    if (s_stop) return;
    double pq = 0.0;
    if constexpr (NPW == 1) {
        // one node per wave: the node, its neighbour ids and their row
        // addresses are wave-uniform (scalar loads); C neighbours per round
        // of loads (padding slots add zero).  The node's blocks (KW floats, at
        // most kNodalStage) are copied to the wave's LDS buffer in 16-byte
        // pieces, the next node's while this one is contracted, and every
        // lane reads its A operands from there (four distinct addresses per
        // read): one coalesced load per node instead of a 12-byte load per
        // lane and block.
        extern __shared__ __align__(16) float s_kb[];  // [waves][2][KW]
        float *kbuf = s_kb + wave * 2 * KW;
        auto stash = [&](int half) {
            f32x4 *dst = reinterpret_cast<f32x4 *>(kbuf + half * KW);
#pragma unroll
            for (int q = 0; q < kNodalStage / 256; ++q)
                if (lane + 64 * q < KQ) dst[lane + 64 * q] = pre[q];
            // the wave's LDS operations run in order; keep the compiler from
            // moving the reads of this buffer above these writes
            __builtin_amdgcn_wave_barrier();
            asm volatile("" ::: "memory");
        };
        int cur = 0;
        if (g0 + wave < g1) stash(0);
        for (int64_t n = g0 + wave; n < g1; n += W) {
            const int64_t nn = n + W;
            if (nn < g1) fetch(nn);
            float xi[D];
#pragma unroll
            for (int k = 0; k < D; ++k) xi[k] = P[(n * D + k) * S + col];
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const int32_t *nb = nbr + n * NB;
            const float *ka = kbuf + cur * KW + rr * D;
            auto round = [&](int s0) {
                float xv[C][D];
#pragma unroll
                for (int u = 0; u < C; ++u) {
                    const int64_t j = nb[s0 + u];
#pragma unroll
                    for (int k = 0; k < D; ++k) xv[u][k] = P[(j * D + k) * S + col];
                }
#pragma unroll
                for (int u = 0; u < C; ++u)
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        acc = __builtin_amdgcn_mfma_f32_4x4x1f32(ka[(s0 + u) * DD + k], xv[u][k] - xi[k], acc, 0, 0,
                                                                 0);
            };
            if constexpr (NCH > 0) {
#pragma unroll
                for (int s0 = 0; s0 < NCH * C; s0 += C) round(s0);
            } else {
                for (int s0 = 0; s0 < NB; s0 += C) round(s0);
            }
            if (nn < g1) stash(cur ^ 1);
            cur ^= 1;
            if (live_col) {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const int64_t row = n * D + i;
                    const float q = fixed[row] ? 0.f : acc[i];
                    Q[row * S + col] = q;
                    pq += (double)xi[i] * (double)q;
                }
            }
        }
    } else
    for (int64_t grp = g0 + wave; grp < g1; grp += W) {
        const int64_t n0 = grp * NPW + lane / SP;
        const bool live = n0 < N;
        const int64_t n = live ? n0 : N - 1;
        float xi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) xi[k] = P[(n * D + k) * S + col];
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const int32_t *nb = nbr + n * NB;
        const float *kr = kb + n * KW + rr * D;
        // rounds of R neighbours: four (one 16-byte id load) when C = 8
        constexpr int R = C % 4 == 0 ? 4 : C;
        for (int s0 = 0; s0 < NB; s0 += R) {
            int jj[R];
            if constexpr (R == 4) {
                const int4 j4 = *reinterpret_cast<const int4 *>(nb + s0);
                jj[0] = j4.x;
                jj[1] = j4.y;
                jj[2] = j4.z;
                jj[3] = j4.w;
            } else {
#pragma unroll
                for (int u = 0; u < R; ++u) jj[u] = nb[s0 + u];
            }
            float xv[R][D], kv[R][D];
#pragma unroll
            for (int u = 0; u < R; ++u)
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    xv[u][k] = P[((int64_t)jj[u] * D + k) * S + col];
                    kv[u][k] = kr[(s0 + u) * DD + k];
                }
#pragma unroll
            for (int u = 0; u < R; ++u)
#pragma unroll
                for (int k = 0; k < D; ++k)
                    acc = __builtin_amdgcn_mfma_f32_4x4x1f32(kv[u][k], xv[u][k] - xi[k], acc, 0, 0, 0);
        }
        if (live && live_col) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int64_t row = n * D + i;
                const float q = fixed[row] ? 0.f : acc[i];
                Q[row * S + col] = q;
                pq += (double)xi[i] * (double)q;
            }
        }
    }
    red[tid] = pq;
    __syncthreads();
    if (tid < S) {
        double sum = 0.0;
        for (int w = 0; w < kNodalWaves; ++w)
            for (int g = 0; g < NPW; ++g) sum += red[w * 64 + g * SP + tid];
        pq_part[(int64_t)blk * S + tid] = sum;
    }
}

// R[:, k] = B[:, k] - K(phi) X[:, k] in FP64 (block vectors [n_dofs][S],
// S <= 64) for the columns k with mask[k] set, clamped rows 0: the residual
// of the FP64 refinement, from the unrounded blocks, in the same difference
// form y_i = sum_{j != i} K_ij (x_j - x_i), and per block and column the
// partial sum of the squares of the new residual (part [gridDim.x][S]; 0 for
// the columns outside the mask).  One node per wave at a time, lane k its
// column: the node's neighbour ids and blocks are wave-uniform (scalar
// loads), C neighbours' rows in flight per round.
template <int D, int C>
__global__ __launch_bounds__(256) void k_nodal_residual64(const int32_t *__restrict__ nbr,
                                                          const double *__restrict__ kb64, int NB, int64_t N,
                                                          const double *__restrict__ X,
                                                          const double *__restrict__ B,
                                                          const uint8_t *__restrict__ fixed,
                                                          const uint8_t *__restrict__ mask,
                                                          double *__restrict__ R, int S,
                                                          double *__restrict__ part)
{
    constexpr int DD = D * D;
    __shared__ double red[256];
    const int lane = threadIdx.x & 63;
    const bool act = lane < S && mask[lane];
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    double ss = 0.0;
    // the node loop stays wave-uniform (ids and blocks through scalar loads);
    // a wave with no column in the mask skips it, other lanes are predicated
    const bool any = __any(act);
    for (int64_t i = any ? wave : N; i < N; i += nw) {
        if (!act) continue;
        double xi[D], acc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            xi[k] = X[(i * D + k) * S + lane];
            acc[k] = 0.0;
        }
        const int32_t *nb = nbr + i * NB;
        const double *kr = kb64 + i * NB * DD;
        for (int s0 = 0; s0 < NB; s0 += C) {
            double dx[C][D];
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const int64_t j = nb[s0 + u];
#pragma unroll
                for (int k = 0; k < D; ++k) dx[u][k] = X[(j * D + k) * S + lane] - xi[k];
            }
#pragma unroll
            for (int u = 0; u < C; ++u)
#pragma unroll
                for (int k = 0; k < D; ++k)
#pragma unroll
                    for (int r = 0; r < D; ++r) acc[r] = fma(kr[(s0 + u) * DD + r * D + k], dx[u][k], acc[r]);
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            const int64_t row = i * D + r;
            const double v = fixed[row] ? 0.0 : B[row * S + lane] - acc[r];
            R[row * S + lane] = v;
            ss += v * v;
        }
    }
    red[threadIdx.x] = ss;
    __syncthreads();
    if ((int)threadIdx.x < S) {
        double a = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) a += red[w * 64 + threadIdx.x];
        part[(int64_t)blockIdx.x * S + threadIdx.x] = a;
    }
}

// ---------------------------------------------------------------------------
// host side

template <int D>
static int nodal_occupancy(fo_ctx *c);

// Node -> element incidence (ascending element ids) and the neighbour lists
// (ascending, padded with the node itself to NB, the largest neighbour count
// rounded up to a multiple of 7 or of 8, whichever is smaller; 8 on a tie),
// from the host mesh in the context's element order.  Allocates the device arrays in
// the context (measure mode: counts them only).  A mesh whose largest
// neighbourhood exceeds the apply's staging buffer gets no nodal arrays and
// keeps the element operator.
int nodal_setup(fo_ctx *c, const std::vector<int32_t> &conn)
{
    BatchState &b = c->batch;
    const int D = c->dim, NV = D + 1;
    const int64_t N = c->N, E = c->E;
    std::vector<int32_t> inc_ptr(N + 1, 0), inc_elem((size_t)NV * E);
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < NV; ++a) ++inc_ptr[conn[(size_t)a * E + e] + 1];
    for (int64_t i = 0; i < N; ++i) inc_ptr[i + 1] += inc_ptr[i];
    {
        std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < NV; ++a) inc_elem[fill[conn[(size_t)a * E + e]]++] = (int32_t)e;
    }
    std::vector<int32_t> nb_cnt(N);
    std::vector<std::vector<int32_t>> lists(N);
    int maxdeg = 1;
    for (int64_t i = 0; i < N; ++i) {
        std::vector<int32_t> &l = lists[i];
        for (int32_t q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q)
            for (int a = 0; a < NV; ++a) {
                const int32_t v = conn[(size_t)a * E + inc_elem[q]];
                if (v != i) l.push_back(v);
            }
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
        maxdeg = std::max(maxdeg, (int)l.size());
    }
    const int chunk = (maxdeg + 6) / 7 * 7 < (maxdeg + 7) / 8 * 8 ? 7 : 8;
    const int NB = (maxdeg + chunk - 1) / chunk * chunk, KW = (NB * D * D + 3) / 4 * 4;
    std::vector<int32_t> nbr((size_t)N * NB);
    int64_t offdiag = 0;
    for (int64_t i = 0; i < N; ++i) {
        const std::vector<int32_t> &l = lists[i];
        offdiag += (int64_t)l.size();
        for (int s = 0; s < NB; ++s) nbr[(size_t)i * NB + s] = s < (int)l.size() ? l[s] : (int32_t)i;
    }
    if (KW > kNodalStage) {  // neighbourhoods too large: element operator only
        b.op = FO_BATCH_OP_ELEMENT;
        return FO_OK;
    }
    b.nb = NB;
    b.nb_chunk = chunk;
    b.kw = KW;
    b.n_offdiag = offdiag;
    b.n_apply = nodal_block_cap(N, b.S);
    const size_t before = c->bytes;
    FO_TRY(ctx_alloc_n(c, &b.nbr, nbr.size()));
    FO_TRY(ctx_alloc_n(c, &b.inc_ptr, inc_ptr.size()));
    FO_TRY(ctx_alloc_n(c, &b.inc_elem, inc_elem.size()));
    FO_TRY(ctx_alloc_n(c, &b.kb, (size_t)N * KW));
    FO_TRY(ctx_alloc_n(c, &b.kb64, (size_t)N * NB * D * D));
    FO_TRY(ctx_alloc_n(c, &b.pq_nodal, (size_t)b.n_apply * b.S));
    b.nodal_bytes = (int64_t)(c->bytes - before);
    if (c->measure) return FO_OK;
    FO_TRY(D == 2 ? nodal_occupancy<2>(c) : nodal_occupancy<3>(c));
    if (hipMemcpyAsync(b.nbr, nbr.data(), nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(b.inc_ptr, inc_ptr.data(), inc_ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        hipMemcpyAsync(b.inc_elem, inc_elem.data(), inc_elem.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        fo::wait_stream(c->stream) != hipSuccess)
        return FO_ERR_HIP;
    return FO_OK;
}

// The blocks K_ij of the current level set (A_e from c->chi).
int nodal_levelset(fo_ctx *c)
{
    const BatchState &b = c->batch;
    if (!b.kb) return FO_OK;
    const int64_t total = c->N * b.nb;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_nodal_assemble<2>, dim3(grid), dim3(256), 0, c->stream, b.nbr, b.nb, b.kw, c->N, b.inc_ptr,
                           b.inc_elem, c->conn, c->E, c->coords, c->chi, c->ersatz, c->lam, c->mu, b.kb, b.kb64);
    else
        hipLaunchKernelGGL(k_nodal_assemble<3>, dim3(grid), dim3(256), 0, c->stream, b.nbr, b.nb, b.kw, c->N, b.inc_ptr,
                           b.inc_elem, c->conn, c->E, c->coords, c->chi, c->ersatz, c->lam, c->mu, b.kb, b.kb64);
    FO_HIP(hipGetLastError());
    return FO_OK;
}

template <int D, int S>
static void nodal_apply_t(const fo_ctx *c, const float *P, float *Q, BatchCtl *ctl, const BatchCol *cols,
                          hipStream_t s)
{
    const BatchState &b = c->batch;
    const int nblk = nodal_blocks(c, S);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nblk), dim3(64 * kNodalWaves), nodal_lds(b.kw), s, b.nbr, b.kb, b.nb, b.kw, c->N,
                           P, Q, c->fixed, b.pq_nodal, ctl, cols);
    };
    const int nch = nodal_rounds(b, S);
    if (b.nb_chunk == 7)
        nch == 1 ? go(k_nodal_apply<D, S, 7, 1>) : nch == 2 ? go(k_nodal_apply<D, S, 7, 2>) : go(k_nodal_apply<D, S, 7, 0>);
    else
        nch == 1 ? go(k_nodal_apply<D, S, 8, 1>) : nch == 2 ? go(k_nodal_apply<D, S, 8, 2>) : go(k_nodal_apply<D, S, 8, 0>);
}

int nodal_residual64(const fo_ctx *c, int S, const double *X, const double *B, const uint8_t *mask, double *R,
                     double *part, int64_t part_cap, int *nblk, hipStream_t s)
{
    const BatchState &b = c->batch;
    if (!b.kb64 || S > 64 || part_cap < S) return FO_ERR_ARG;
    const int grid = (int)std::min<int64_t>(std::min<int64_t>((c->N + 3) / 4, 2048), part_cap / S);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, b.nbr, (const double *)b.kb64, b.nb, c->N, X, B,
                           c->fixed, mask, R, S, part);
    };
    if (c->dim == 2)
        b.nb_chunk == 7 ? go(k_nodal_residual64<2, 7>) : go(k_nodal_residual64<2, 8>);
    else
        b.nb_chunk == 7 ? go(k_nodal_residual64<3, 7>) : go(k_nodal_residual64<3, 8>);
    FO_HIP(hipGetLastError());
    *nblk = grid;
    return FO_OK;
}

// Resident blocks of every column-width instance (outside graph capture).
template <int D>
static int nodal_occupancy(fo_ctx *c)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) return FO_ERR_HIP;
    // the instance each width launches (nodal_apply_t), for its occupancy
    const BatchState &bs = c->batch;
    const bool c7 = bs.nb_chunk == 7;
    auto pick = [&](int S, auto k70, auto k71, auto k72, auto k80, auto k81, auto k82) {
        const int nch = nodal_rounds(bs, S);
        if (c7) return nch == 1 ? (const void *)k71 : nch == 2 ? (const void *)k72 : (const void *)k70;
        return nch == 1 ? (const void *)k81 : nch == 2 ? (const void *)k82 : (const void *)k80;
    };
#define FO_NODAL_INST(S_)                                                                                          \
    pick(S_, k_nodal_apply<D, S_, 7, 0>, k_nodal_apply<D, S_, 7, 1>, k_nodal_apply<D, S_, 7, 2>,                     \
         k_nodal_apply<D, S_, 8, 0>, k_nodal_apply<D, S_, 8, 1>, k_nodal_apply<D, S_, 8, 2>)
    const void *fn[4] = {FO_NODAL_INST(16), FO_NODAL_INST(32), FO_NODAL_INST(48), FO_NODAL_INST(64)};
#undef FO_NODAL_INST
    for (int k = 0; k < 4; ++k) {
        int per = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn[k], 64 * kNodalWaves, nodal_lds(c->batch.kw)) !=
            hipSuccess)
            return FO_ERR_HIP;
        c->batch.nodal_occ[k] = std::max(1, per) * cus;
    }
    return FO_OK;
}

template <int D>
static void nodal_apply_d(const fo_ctx *c, int NC, const float *P, float *Q, BatchCtl *ctl,
                          const BatchCol *cols, hipStream_t s)
{
    switch (NC) {
    case 1: nodal_apply_t<D, 16>(c, P, Q, ctl, cols, s); break;
    case 2: nodal_apply_t<D, 32>(c, P, Q, ctl, cols, s); break;
    case 3: nodal_apply_t<D, 48>(c, P, Q, ctl, cols, s); break;
    default: nodal_apply_t<D, 64>(c, P, Q, ctl, cols, s); break;
    }
}

void nodal_apply_launch(const fo_ctx *c, int NC, const float *P, float *Q, BatchCtl *ctl, const BatchCol *cols,
                        hipStream_t s)
{
    if (c->dim == 2)
        nodal_apply_d<2>(c, NC, P, Q, ctl, cols, s);
    else
        nodal_apply_d<3>(c, NC, P, Q, ctl, cols, s);
}

}  // namespace fo

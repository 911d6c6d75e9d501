// Batched multi-load elasticity solves on one level set.
//
// Many load cases share the operator K(phi) (the multi-load compliance
// problem sums the derivative over the cases; the paper solves such PDE sets
// in its task-parallel mode, Numerics, Parallelization).  With s right-hand
// sides the element contraction Y_e = K_e X_e -- K_e the d(d+1)-square
// element stiffness, X_e one row per (vertex, component) and one column per
// load case -- is a dense product, and it runs on the matrix cores:
// v_mfma_f32_16x16x4f32 with K_e as the A operand and a 16-column slice of
// X_e as the B operand.  K_e annihilates rigid translations, so the product
// is formed as K_e[:, b>=1] (X_b - X_0): the differences remove the large
// common part of smooth fields before the FP32 products (the explicit
// product of X_e itself loses about two digits on a displacement field),
// and the contraction length drops from d(d+1) to d^2 (one MFMA per element
// in 2D, three in 3D).
//
// Block vectors are [n_dofs][S], load case fastest, S = 16 NC (NC = 1..4).
// One block per element tile; wave w owns columns 16w..16w+15 and walks the
// tile's elements in order, accumulating into its own columns of the tile's
// node rows in LDS, so the sum is deterministic and needs no atomics.  K_e is
// built once per element (in batches of kBatchKB elements, in the MFMA
// fragment order) and shared by the waves.  Interior nodes are written
// directly; shared nodes go to a node-major halo that the update kernel sums
// in tile order.
//
// The solver is CG on every column at once (per-column alpha, beta and
// convergence) inside the same FP64 residual-replacement scheme as the
// single-load path: FP32 phases, x64 += s x32, r64 = b - K x64 in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <vector>

#include "fo_batch_dev.h"
#include "fo_element.h"
#include "fo_internal.h"
#include "fo_launch.h"
#include "fo_reduce.h"
#include "fo_tiles.h"
#include "fo_xcd.h"

namespace fo {

constexpr int kBatchKB = 32;          // elements per K_e batch held in LDS
constexpr int kBatchLds = 163840;     // LDS per workgroup on gfx950
constexpr int kBatchStaticLds = 64;   // static LDS of the apply kernel (rounded up)

// Batch tiles: element slots in node-disjoint groups of G (padding slots
// have local ids 0xFFFF and weight 0), per-tile fixed strides MN (nodes) and
// MS (slots).
struct BatchTileArgs {
    const int32_t *info;      // [n_tiles][8]: kTileNE = slots, kTileNN, kTileNInt
    const int32_t *nodes;     // [n_tiles][MN] global node of each tile node
    const int32_t *hpos;      // [n_tiles][MN] halo slot of a shared tile node
    const uint64_t *slconn;   // [n_tiles][MS] 4 x uint16 local vertex ids
    const int4 *sgconn;       // [n_tiles][MS] global vertex ids
    int MN, MS, n_tiles;
};

static BatchTileArgs batch_tile_args(const fo_ctx *c)
{
    const BatchState &b = c->batch;
    return BatchTileArgs{b.tiles.info, b.tiles.nodes, b.tiles.hpos, b.slconn, b.sgconn, b.tiles.max_nodes,
                         b.slot_stride, b.tiles.n_tiles};
}

size_t batch_lds_bytes(int D, int S, int MN)
{
    const int KS = (D * D + 3) / 4;
    return (size_t)MN * D * S * 4 + (size_t)S * 16 + (size_t)kBatchKB * KS * 64 * 4 + (size_t)kBatchKB * (D + 1) * D * 4 +
           (size_t)kBatchKB * 4 + (size_t)2 * kBatchKB * 16 + (size_t)MN * 8 + (((size_t)MN * D + 15) / 16) * 16;
}

__device__ __forceinline__ int pick4(const int4 v, int k)
{
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

// Sum of a shared row's halo entries (slots hr.x .. hr.y-1 in order, entry
// off of each slot of `stride` floats); the first KH slots are loaded
// together (indices clamped into the range, every load in bounds).
__device__ __forceinline__ float halo_row_sum(const float *__restrict__ halo, int2 hr, int64_t off,
                                              int64_t stride)
{
    constexpr int KH = 4;
    const int cnt = hr.y - hr.x;
    float hv[KH];
#pragma unroll
    for (int k = 0; k < KH; ++k) hv[k] = halo[(int64_t)(hr.x + min(k, cnt - 1)) * stride + off];
    float q = 0.f;
#pragma unroll
    for (int k = 0; k < KH; ++k)
        if (k < cnt) q += hv[k];
    for (int j = hr.x + KH; j < hr.y; ++j) q += halo[(int64_t)j * stride + off];
    return q;
}

// Element data of the batched operator, once per level set and per slot:
// the cofactor vectors c_a (c_0 = -sum) and w = A_e / (d! |det|), so that
// K_e[(a,i),(b,j)] = w (lam c_ai c_bj + mu c_aj c_bi + mu delta_ij c_a.c_b).
// [slots][16] floats: c at a*D+i, w at 12; padding slots are all zero.
template <int D>
__global__ __launch_bounds__(256) void k_batch_geom(const int32_t *__restrict__ selem,
                                                    const int4 *__restrict__ sgconn, int64_t n_slots,
                                                    const double *__restrict__ coords,
                                                    const uint8_t *__restrict__ chi, double ersatz,
                                                    float *__restrict__ geo)
{
    constexpr int NV = D + 1;
    for (int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < n_slots;
         sl += (int64_t)gridDim.x * blockDim.x) {
        float out[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) out[k] = 0.f;
        const int32_t e = selem[sl];
        if (e >= 0) {
            const int4 gv = sgconn[sl];
            const int gid[4] = {gv.x, gv.y, gv.z, gv.w};
            // geometry in FP64, stored in FP32
            double X[NV][D];
            const double *Xp[NV];
#pragma unroll
            for (int a = 0; a < NV; ++a) {
#pragma unroll
                for (int i = 0; i < D; ++i) X[a][i] = coords[(int64_t)gid[a] * D + i];
                Xp[a] = X[a];
            }
            const Geom<D, double> gm = geom<D, double>(Xp);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double c0 = 0.0;
#pragma unroll
                for (int a = 1; a < NV; ++a) {
                    out[a * D + i] = (float)gm.c[a - 1][i];
                    c0 -= gm.c[a - 1][i];
                }
                out[i] = (float)c0;
            }
            out[12] = (float)((chi[e] ? 1.0 : ersatz) * inv_measure_det2<D, double>(gm.det));
        }
        f32x4 *g4 = reinterpret_cast<f32x4 *>(geo + sl * 16);
#pragma unroll
        for (int k = 0; k < 4; ++k) g4[k] = f32x4{out[4 * k], out[4 * k + 1], out[4 * k + 2], out[4 * k + 3]};
    }
}

// Q = K(phi) P for S = 16 NC columns, p.q partials per tile and column.
// Every block first decides whether the solve is over (all columns done or
// the iteration cap reached) from state that no kernel of this launch
// writes, so all blocks agree; block 0 records the decision.
//
// Per batch of kBatchKB slots: (A) element data to LDS (prefetched into
// registers during the previous batch), (B) K_e[:, b>=1] in MFMA fragment
// order, (C) groups of G node-disjoint elements: a wave loads the operands
// of the next group while it contracts the current one, and since no two
// elements of a group share a node, the group's read-add-writes of the node
// rows are all in flight together.  A wave owns its columns, so the rows sum
// in slot order without atomics.
template <int D, int NC, int G>
__global__ __launch_bounds__(64 * NC) void k_batch_apply(
    BatchTileArgs ta, const float *__restrict__ geo, float lam, float mu, const float *__restrict__ P,
    float *__restrict__ Q, float *__restrict__ halo, const uint8_t *__restrict__ fixed,
    double *__restrict__ pq_part, BatchCtl *ctl, const BatchCol *__restrict__ cols)
{
    constexpr int S = 16 * NC, NV = D + 1, NR = D * NV, NK = D * D, KS = (NK + 3) / 4, NT = 64 * NC;
    constexpr int KB = kBatchKB;
    static_assert(KB % G == 0, "groups tile a batch");
    __shared__ int s_stop;
    const int tid = threadIdx.x;
    const int t = xcd_tile(blockIdx.x, ta.n_tiles);
    if (t < 0) return;
    if (tid == 0) s_stop = batch_stop(ctl, cols, S);
    __syncthreads();
    if (s_stop) return;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *sY = reinterpret_cast<float *>(smem_raw);       // [MN][D][S]
    float *sDummy = sY + (size_t)ta.MN * D * S;            // [S * 4]: sink of rows without a node
    float *sK = sDummy + S * 4;                            // [KB][KS][64] K_e fragments
    const int sink = (int)(sDummy - sY);
    float *sC = sK + KB * KS * 64;                         // [KB][NV][D] cofactor vectors
    float *sW = sC + KB * NV * D;                          // [KB] w
    int4 *sEN = reinterpret_cast<int4 *>(sW + KB);         // [KB] global vertex ids
    uint2 *sEL = reinterpret_cast<uint2 *>(sEN + KB);      // [KB] local vertex ids (4 x uint16)
    int32_t *sNode = reinterpret_cast<int32_t *>(sEL + KB);  // [MN]
    int32_t *sHp = sNode + ta.MN;                          // [MN] halo slot, -1 interior
    uint8_t *sFix = reinterpret_cast<uint8_t *>(sHp + ta.MN);  // [MN*D]

    const int32_t *inf = ta.info + (int64_t)t * kTileInfo;
    const int ns = inf[kTileNE], nn = inf[kTileNN], nint = inf[kTileNInt];
    for (int l = tid; l < nn; l += NT) {
        const int32_t gn = ta.nodes[(int64_t)t * ta.MN + l];
        sNode[l] = gn;
        sHp[l] = l < nint ? -1 : ta.hpos[(int64_t)t * ta.MN + l];
#pragma unroll
        for (int i = 0; i < D; ++i) sFix[l * D + i] = fixed[(int64_t)gn * D + i];
    }
    {
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
        f32x4 *y4 = reinterpret_cast<f32x4 *>(sY);
        for (int i = tid; i < nn * D * S / 4; i += NT) y4[i] = z;
        f32x4 *k4 = reinterpret_cast<f32x4 *>(sK);
        for (int i = tid; i < KB * KS * 16; i += NT) k4[i] = z;  // padding stays zero
    }
    f32x4 pg[4];
    int4 pn = make_int4(0, 0, 0, 0);
    uint64_t plc = 0;
    const int64_t slot0 = (int64_t)t * ta.MS;
    auto fetch = [&](int base) {
        if (tid < KB && base + tid < ns) {
            const int64_t sl = slot0 + base + tid;
            const f32x4 *g4 = reinterpret_cast<const f32x4 *>(geo + sl * 16);
#pragma unroll
            for (int k = 0; k < 4; ++k) pg[k] = g4[k];
            pn = ta.sgconn[sl];
            plc = ta.slconn[sl];
        }
    };
    fetch(0);
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63, g = lane >> 4;
    const int colg = wave * 16 + (lane & 15);
    const int a0 = (4 * g) / D, a1 = (4 * g + 3) / D;  // vertices of this lane's output rows
    for (int base = 0; base < ns; base += KB) {
        const int nb = min(KB, ns - base);
        // (A) element data of this batch to LDS
        if (tid < nb) {
            float gv[16];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                gv[4 * k] = pg[k].x;
                gv[4 * k + 1] = pg[k].y;
                gv[4 * k + 2] = pg[k].z;
                gv[4 * k + 3] = pg[k].w;
            }
#pragma unroll
            for (int k = 0; k < NV * D; ++k) sC[tid * NV * D + k] = gv[k];
            sW[tid] = gv[12];
            sEN[tid] = pn;
            sEL[tid] = make_uint2((uint32_t)plc, (uint32_t)(plc >> 32));
        }
        __syncthreads();
        // (B) K_e[:, b>=1] in fragment order: row r = (a, i), column
        // k = (b-1, j); lane (row r, k-group) of k-step s reads its A entry
        // at [s][16 (k mod 4) + r]
        for (int task = tid; task < nb * NV * D; task += NT) {
            const int e = task / (NV * D), ab = task - e * (NV * D), a = ab / D, b = ab - a * D + 1;
            const float *ca = sC + (e * NV + a) * D, *cb = sC + (e * NV + b) * D;
            float d = 0.f;
#pragma unroll
            for (int i = 0; i < D; ++i) d += ca[i] * cb[i];
            const float w = sW[e];
            float *ke = sK + e * KS * 64;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const float v = w * (lam * ca[i] * cb[j] + mu * ca[j] * cb[i] + (i == j ? mu * d : 0.f));
                    const int r = a * D + i, k = (b - 1) * D + j;
                    ke[(k >> 2) * 64 + ((k & 3) << 4) + r] = v;
                }
        }
        __syncthreads();
        // (C) node-disjoint groups, operands double-buffered
        const int ngr = nb / G;
        float avA[G][KS], bvA[G][KS], avB[G][KS], bvB[G][KS];
        uint32_t lvA[G], lvB[G];
        auto load = [&](int gi, float (&av)[G][KS], float (&bv)[G][KS], uint32_t (&lv)[G]) {
#pragma unroll
            for (int e = 0; e < G; ++e) {
                const int el = gi * G + e;
                const int4 en = sEN[el];
                const uint2 lc = sEL[el];
                float v0[D];
#pragma unroll
                for (int j = 0; j < D; ++j) v0[j] = P[((int64_t)en.x * D + j) * S + colg];
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    // lanes past the contraction length (k >= NK) load a valid
                    // row and use 0: no divergent branch, so no wait here
                    const int k = 4 * s + g, kc = k < NK ? k : NK - 1, j = kc % D;
                    const float x0 = D == 2 ? (j == 0 ? v0[0] : v0[D - 1])
                                            : (j == 0 ? v0[0] : j == 1 ? v0[1] : v0[D - 1]);
                    const float xb = P[((int64_t)pick4(en, 1 + kc / D) * D + j) * S + colg];
                    bv[e][s] = k < NK ? xb - x0 : 0.f;
                    av[e][s] = sK[(el * KS + s) * 64 + lane];
                }
                const uint32_t l0 = (a0 < 2 ? lc.x >> (16 * a0) : lc.y >> (16 * (a0 - 2))) & 0xFFFF;
                const uint32_t l1 = (a1 < 2 ? lc.x >> (16 * a1) : lc.y >> (16 * (a1 - 2))) & 0xFFFF;
                lv[e] = l0 | (l1 << 16);
            }
        };
        auto contract = [&](const float (&av)[G][KS], const float (&bv)[G][KS], const uint32_t (&lv)[G]) {
            f32x4 acc[G];
#pragma unroll
            for (int e = 0; e < G; ++e) {
                acc[e] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < KS; ++s)
                    acc[e] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[e][s], bv[e][s], acc[e], 0, 0, 0);
            }
            // the group's elements share no node: all reads, then all writes.
            // Rows past d(d+1) and padding slots go to a per-lane sink in LDS
            // (no divergent branch); the sink is never read back.
            int ad[G][4];
#pragma unroll
            for (int e = 0; e < G; ++e)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = 4 * g + q;
                    const bool ok = r < NR && (lv[e] & 0xFFFF) != 0xFFFF;
                    const int ln = (int)(r / D == a0 ? (lv[e] & 0xFFFF) : (lv[e] >> 16));
                    ad[e][q] = ok ? (ln * D + (r % D)) * S + colg : sink + q * S + colg;
                }
            float old[G][4];
#pragma unroll
            for (int e = 0; e < G; ++e)
#pragma unroll
                for (int q = 0; q < 4; ++q) old[e][q] = sY[ad[e][q]];
#pragma unroll
            for (int e = 0; e < G; ++e)
#pragma unroll
                for (int q = 0; q < 4; ++q) sY[ad[e][q]] = old[e][q] + acc[e][q];
        };
        load(0, avA, bvA, lvA);
        fetch(base + KB);
        for (int gi = 0; gi < ngr; gi += 2) {
            if (gi + 1 < ngr) load(gi + 1, avB, bvB, lvB);
            contract(avA, bvA, lvA);
            if (gi + 1 < ngr) {
                if (gi + 2 < ngr) load(gi + 2, avA, bvA, lvA);
                contract(avB, bvB, lvB);
            }
        }
        __syncthreads();
    }

    // outputs: 4 columns per thread, 16 rows per pass; interior rows to Q,
    // shared rows to the halo; p.q partials per column (the K_e area is free)
    constexpr int C4 = S / 4, RP = NT / C4;  // RP = 16
    double *s_red = reinterpret_cast<double *>(sK);   // [RP][S]
    const int c4 = tid % C4, rp = tid / C4;
    double pq[4] = {0.0, 0.0, 0.0, 0.0};
    const f32x4 *P4 = reinterpret_cast<const f32x4 *>(P);
    f32x4 *Q4 = reinterpret_cast<f32x4 *>(Q);
    f32x4 *H4 = reinterpret_cast<f32x4 *>(halo);
    const f32x4 *Y4 = reinterpret_cast<const f32x4 *>(sY);
#pragma unroll 2
    for (int row = rp; row < nn * D; row += RP) {
        const int ln = row / D, i = row - ln * D;
        const int64_t gr = (int64_t)sNode[ln] * D + i;
        const int hp = sHp[ln];
        const bool fx = sFix[row] != 0;
        const f32x4 y = Y4[row * C4 + c4];
        if (hp < 0)
            Q4[gr * C4 + c4] = fx ? f32x4{0.f, 0.f, 0.f, 0.f} : y;
        else
            H4[((int64_t)hp * D + i) * C4 + c4] = y;
        if (!fx) {
            const f32x4 p = P4[gr * C4 + c4];
#pragma unroll
            for (int k = 0; k < 4; ++k) pq[k] += (double)p[k] * (double)y[k];
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) s_red[rp * S + 4 * c4 + k] = pq[k];
    __syncthreads();
    if (tid < S) {
        double sum = 0.0;
        for (int k = 0; k < RP; ++k) sum += s_red[k * S + tid];
        pq_part[(int64_t)t * S + tid] = sum;
    }
}

// This thread's share of sum_i v[i * stride], i < n (i = threadIdx.x,
// + blockDim.x, ...), added in that order with eight loads in flight.
__device__ __forceinline__ double strided_sum(const double *__restrict__ v, int stride, int n)
{
    constexpr int U = 8;
    const int nt = (int)blockDim.x;
    double s = 0.0;
    for (int base = (int)threadIdx.x; base < n; base += U * nt) {
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = v[(int64_t)min(base + u * nt, n - 1) * stride];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * nt < n) s += t[u];
    }
    return s;
}

// alpha_k = rho_k / (p_k . q_k), one block per column.
__global__ __launch_bounds__(256) void k_batch_alpha(const BatchCtl *ctl, BatchCol *cols,
                                                     const double *__restrict__ pq_part,
                                                     int n_tiles, int S)
{
    __shared__ double lds[4];
    const int k = blockIdx.x;
    // the partials' loads go out together with the control loads: the grid is
    // one round of blocks, so a chain of dependent loads is not hidden
    const int stop = ctl->done, col_done = cols[k].done;
    const double part = strided_sum(pq_part + k, S, n_tiles);
    if (stop) return;
    if (col_done) {
        if (threadIdx.x == 0) cols[k].alpha = 0.0;
        return;
    }
    const double s = block_sum(part, lds);
    if (threadIdx.x == 0) {
        BatchCol &c = cols[k];
        c.pq = s;
        if (s > 0.0 && isfinite(s)) {
            c.alpha = c.rho / s;
        } else {  // not SPD or non-finite: this column stops and restarts next phase
            c.alpha = 0.0;
            c.status = FO_ERR_BREAKDOWN;
            c.done = 1;
            c.fresh = 1;
        }
    }
}

// r -= alpha q (q of shared nodes: their halo slots in tile order; hrange
// null: every row of q is in Q; clamped rows q = 0); partials of r.D^-1 r
// and r.r per column.  (x += alpha p is done by the direction kernel, which
// reads p anyway.)
template <int D, int S>
__global__ __launch_bounds__(256) void k_batch_update(
    const BatchCtl *ctl, const BatchCol *__restrict__ cols, float *__restrict__ R,
    const float *__restrict__ Q, const float *__restrict__ dinv, const int2 *__restrict__ hrange,
    const float *__restrict__ halo, int64_t ndof, double *__restrict__ rz_part)
{
    constexpr int RG = 256 / S;
    constexpr int U = 4;
    __shared__ double red[2][256];
    const int tid = threadIdx.x, col = tid % S, rg = tid / S;
    const int64_t step = (int64_t)gridDim.x * RG;
    int64_t row = rg < RG ? (int64_t)blockIdx.x * RG + rg : ndof;
    // every row of q in Q (hrange null): four rows per thread and step, the
    // next step's loads issued before this step's stores (they are the
    // thread's own later rows); the first step's go out together with the
    // control loads, since the grid is one round of blocks and a chain of
    // dependent loads ahead of the data would not be hidden
    float qv[U], rv[U], dv[U];
    auto load = [&](int64_t r0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t rw = min(r0 + u * step, ndof - 1);
            qv[u] = Q[rw * S + col];
            rv[u] = R[rw * S + col];
            dv[u] = dinv[rw];
        }
    };
    if (!hrange && row < ndof) load(row);
    const int stop = ctl->done;
    const float alpha = (float)cols[col].alpha;
    if (stop) return;
    double rz = 0.0, rr = 0.0;
    if (!hrange) {
        for (; row < ndof; row += U * step) {
            float qc[U], rc[U], dc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                qc[u] = qv[u];
                rc[u] = rv[u];
                dc[u] = dv[u];
            }
            if (row + U * step < ndof) load(row + U * step);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (row + u * step >= ndof) break;
                const float q = dc[u] == 0.f ? 0.f : qc[u];
                const float r = rc[u] - alpha * q;
                R[(row + u * step) * S + col] = r;
                rz += (double)r * (double)(dc[u] * r);
                rr += (double)r * (double)r;
            }
        }
    }
    for (; row < ndof; row += step) {
        const int64_t node = row / D;
        const int i = (int)(row - node * D);
        const int2 hr = hrange[node];
        float q;
        if (hr.x < 0) {
            q = Q[row * S + col];
        } else {
            q = halo_row_sum(halo, hr, (int64_t)i * S + col, (int64_t)D * S);
        }
        const float di = dinv[row];
        if (di == 0.f) q = 0.f;
        const int64_t ix = row * S + col;
        const float r = R[ix] - alpha * q;
        R[ix] = r;
        rz += (double)r * (double)(di * r);
        rr += (double)r * (double)r;
    }
    red[0][tid] = rz;
    red[1][tid] = rr;
    __syncthreads();
    if (tid < S) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < RG; ++k) {
            a += red[0][k * S + tid];
            b += red[1][k * S + tid];
        }
        rz_part[(int64_t)blockIdx.x * S + tid] = a;
        rz_part[((int64_t)gridDim.x + blockIdx.x) * S + tid] = b;
    }
}

// Per column: the phase target on r.r, beta = rho_new / rho.  A column at
// its target is marked reached and keeps iterating: the operator costs the
// same for every column of the block, and the host ends phases only at the
// end of a chunk of iterations, so the iterations up to there lower its
// residual further instead of idling.  A column stopped at its cap keeps the
// rho of the residual that built its direction (the direction is not
// updated), so the next phase continues it with the CG coefficient of the
// replaced residual; a reached column's direction already belongs to its
// latest residual and the next phase keeps it as it is (rescaled).
__global__ __launch_bounds__(256) void k_batch_beta(BatchCtl *ctl, BatchCol *cols,
                                                    const double *__restrict__ rz_part, int nb,
                                                    int S)
{
    __shared__ double lds[4];
    const int k = blockIdx.x;
    const int stop = ctl->done, col_done = cols[k].done;  // loaded together with the partials
    double a = strided_sum(rz_part + k, S, nb), b = strided_sum(rz_part + (int64_t)nb * S + k, S, nb);
    if (stop) return;
    if (k == 0 && threadIdx.x == 0) ctl->it += 1;
    if (col_done) return;
    a = block_sum(a, lds);
    b = block_sum(b, lds);
    if (threadIdx.x == 0) {
        BatchCol &c = cols[k];
        c.rho_new = a;
        c.rr = b;
        if (!(a >= 0.0) || !isfinite(a) || !isfinite(b)) {
            c.status = FO_ERR_BREAKDOWN;
            c.done = 1;
            c.fresh = 1;
        } else {
            if (b <= c.tol2) c.reached = 1;
            if (++c.it >= c.cap) {  // at the cap: stop; short of the target it stagnated (restart)
                c.done = 1;
                if (!c.reached) {
                    c.capped = 1;
                    c.fresh = 1;
                }
            } else {
                c.beta = c.rho > 0.0 ? a / c.rho : 0.0;
                c.rho = a;
            }
        }
    }
}

// Per iteration (mask null): x += alpha p for every column that took a step
// in this iteration (alpha != 0), then p = D^-1 r + beta p for the columns
// still running.  Phase start (mask != null): p = D^-1 r + beta p for the
// columns whose residual was just replaced (beta = the phase coefficient),
// or p = beta p for those that keep their direction (keep), x untouched.
// Two rows per thread and step, loads first.
template <int S>
__global__ __launch_bounds__(256) void k_batch_direction(const BatchCtl *ctl,
                                                         const BatchCol *__restrict__ cols,
                                                         const uint8_t *__restrict__ mask,
                                                         float *__restrict__ P, float *__restrict__ X,
                                                         const float *__restrict__ R,
                                                         const float *__restrict__ dinv, int64_t ndof)
{
    constexpr int RG = 256 / S;
    const int tid = threadIdx.x, col = tid % S, rg = tid / S;
    const int64_t step = (int64_t)gridDim.x * RG;
    int64_t row = rg < RG ? (int64_t)blockIdx.x * RG + rg : ndof;
    // the next step's loads are issued before this step's stores (the
    // thread's own later rows); the first step's, all four streams, go out
    // together with the control loads.  x is read and written only here, so
    // it streams past the caches (non-temporal): the iteration's other
    // streams and the operator (about 200 MB on 64x32x32 with 64 columns)
    // then stay in the 256 MB Infinity Cache between iterations.
    float pv[2] = {0.f, 0.f}, xv[2] = {0.f, 0.f}, rv[2] = {0.f, 0.f}, dv[2] = {0.f, 0.f};
    auto load = [&](int64_t r0, bool lx, bool lr) {
        const bool two = r0 + step < ndof;
        const int64_t ix0 = r0 * S + col, ix1 = two ? ix0 + step * S : ix0;
        pv[0] = P[ix0];
        pv[1] = P[ix1];
        if (lx) {
            xv[0] = __builtin_nontemporal_load(X + ix0);
            xv[1] = __builtin_nontemporal_load(X + ix1);
        }
        if (lr) {
            rv[0] = R[ix0];
            rv[1] = R[ix1];
            dv[0] = dinv[r0];
            dv[1] = dinv[two ? r0 + step : r0];
        }
    };
    if (row < ndof) load(row, true, true);
    if (!mask && ctl->done) return;
    const bool dir = mask ? mask[col] != 0 : !cols[col].done;
    const float alpha = mask ? 0.f : (float)cols[col].alpha;
    if (!dir && alpha == 0.f) return;
    const float beta = (float)cols[col].beta;
    const bool keep = mask && cols[col].keep;
    for (; row < ndof; row += 2 * step) {
        const bool two = row + step < ndof;
        const int64_t ix0 = row * S + col, ix1 = two ? ix0 + step * S : ix0;
        const float p0 = pv[0], p1 = pv[1];
        const float x0 = xv[0], x1 = xv[1];
        const float z0 = dv[0] * rv[0], z1 = dv[1] * rv[1];
        if (row + 2 * step < ndof) load(row + 2 * step, alpha != 0.f, dir);
        if (alpha != 0.f) {
            __builtin_nontemporal_store(x0 + alpha * p0, X + ix0);
            if (two) __builtin_nontemporal_store(x1 + alpha * p1, X + ix1);
        }
        if (dir) {
            P[ix0] = keep ? beta * p0 : (beta == 0.f ? z0 : z0 + beta * p0);
            if (two) P[ix1] = keep ? beta * p1 : (beta == 0.f ? z1 : z1 + beta * p1);
        }
    }
}

// Phase start of the masked columns: r32 = r64 / s_k (s_k^2 in s2new),
// x32 = 0; partials r.z, r.r (columns outside the mask are left alone).
template <int S>
__global__ __launch_bounds__(256) void k_batch_rescale(const double *__restrict__ R64,
                                                       const double *__restrict__ s2new,
                                                       const uint8_t *__restrict__ mask,
                                                       float *__restrict__ R32,
                                                       float *__restrict__ X32,
                                                       const float *__restrict__ dinv, int64_t ndof,
                                                       double *__restrict__ rz_part)
{
    constexpr int RG = 256 / S;
    __shared__ double red[2][256];
    const int tid = threadIdx.x, col = tid % S, rg = tid / S;
    const double sn = s2new[col];
    const double inv = sn > 0.0 ? 1.0 / sqrt(sn) : 0.0;
    double rz = 0.0, rr = 0.0;
    if (mask[col]) {
        for (int64_t row = rg < RG ? (int64_t)blockIdx.x * RG + rg : ndof; row < ndof;
             row += (int64_t)gridDim.x * RG) {
            const int64_t ix = row * S + col;
            const float r = (float)(R64[ix] * inv);
            R32[ix] = r;
            X32[ix] = 0.f;
            rz += (double)r * (double)(dinv[row] * r);
            rr += (double)r * (double)r;
        }
    }
    red[0][tid] = rz;
    red[1][tid] = rr;
    __syncthreads();
    if (tid < S) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < RG; ++k) {
            a += red[0][k * S + tid];
            b += red[1][k * S + tid];
        }
        rz_part[(int64_t)blockIdx.x * S + tid] = a;
        rz_part[((int64_t)gridDim.x + blockIdx.x) * S + tid] = b;
    }
}

// New phase state of the masked columns after a residual replacement (the
// single-load rule per column): with old scale s_o and new scale s_n, the
// first direction is D^-1 r32 + beta (s_o / s_n) p_old, beta = rho_n s_n^2 /
// (rho_o s_o^2); a fresh column restarts (coefficient 0); its phase target
// is ptol[k] (phase_target).  Other columns keep running; the solve is
// marked live again.
__global__ __launch_bounds__(256) void k_batch_phase(BatchCtl *ctl, BatchCol *cols,
                                                     const double *__restrict__ rz_part, int nb,
                                                     int S, double *s2, const uint8_t *mask,
                                                     const int32_t *caps, const double *__restrict__ ptol)
{
    __shared__ double lds[4];
    const int k = blockIdx.x;
    if (k == 0 && threadIdx.x == 0) ctl->done = 0;
    if (!mask[k]) return;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        a += rz_part[(int64_t)i * S + k];
        b += rz_part[((int64_t)nb + i) * S + k];
    }
    a = block_sum(a, lds);
    b = block_sum(b, lds);
    if (threadIdx.x == 0) {
        const BatchCol c = cols[k];
        const double so2 = s2[k], sn2 = s2[S + k];
        double coef = 0.0;
        int keep = 0;
        if (!c.fresh && so2 > 0.0 && sn2 > 0.0) {
            if (c.reached && !c.done) {
                // iterated on past its target: the direction was built from
                // the residual just replaced; it is kept (residual
                // replacement leaves the direction alone), in the new
                // phase's scale
                coef = sqrt(so2 / sn2);
                keep = 1;
            } else if (c.rho > 0.0 && isfinite(c.rho)) {
                coef = (a * sn2) / (c.rho * so2) * sqrt(so2 / sn2);
            }
        }
        BatchCol n{};
        n.keep = keep;
        n.rho = a;
        n.rho_new = a;
        n.rr = b;
        n.tol2 = ptol[k] * ptol[k];
        n.beta = coef;
        n.fresh = 0;
        n.it = 0;
        n.cap = caps[k];
        n.done = b <= n.tol2 ? 1 : 0;
        if (!(a >= 0.0) || !isfinite(a)) {
            n.status = FO_ERR_BREAKDOWN;
            n.done = 1;
            n.fresh = 1;
        }
        cols[k] = n;
        s2[k] = sn2;
    }
}

// Column sums of squares of a [n_dofs][S] FP64 block: partials per block.
template <int S>
__global__ __launch_bounds__(256) void k_batch_colsq(const double *__restrict__ V, int64_t ndof,
                                                     double *__restrict__ part)
{
    constexpr int RG = 256 / S;
    __shared__ double red[256];
    const int tid = threadIdx.x, col = tid % S, rg = tid / S;
    double s = 0.0;
    for (int64_t row = rg < RG ? (int64_t)blockIdx.x * RG + rg : ndof; row < ndof; row += (int64_t)gridDim.x * RG) {
        const double v = V[row * S + col];
        s += v * v;
    }
    red[tid] = s;
    __syncthreads();
    if (tid < S) {
        double a = 0.0;
        for (int k = 0; k < RG; ++k) a += red[k * S + tid];
        part[(int64_t)blockIdx.x * S + tid] = a;
    }
}

__global__ __launch_bounds__(256) void k_batch_colsum(const double *__restrict__ part, int nb, int S,
                                                      double *__restrict__ out)
{
    __shared__ double lds[4];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[(int64_t)i * S + k];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[k] = s;
}

// x64 += s_k x32 (s_k^2 in s2) for the masked columns.
__global__ __launch_bounds__(256) void k_batch_accumulate(double *__restrict__ X64,
                                                          const float *__restrict__ X32,
                                                          const double *__restrict__ s2,
                                                          const uint8_t *__restrict__ mask, int S,
                                                          int64_t n)
{
    for (int64_t ix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ix < n;
         ix += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(ix % S);
        if (mask[k]) X64[ix] += sqrt(s2[k]) * (double)X32[ix];
    }
}

// r64[:, k] = b[:, k] - q (clamped rows 0).
__global__ __launch_bounds__(256) void k_batch_residual_col(const double *__restrict__ B,
                                                            const double *__restrict__ q,
                                                            const uint8_t *__restrict__ fixed,
                                                            double *__restrict__ R, int S, int k,
                                                            int64_t ndof)
{
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < ndof;
         row += (int64_t)gridDim.x * blockDim.x)
        R[row * S + k] = fixed[row] ? 0.0 : B[row * S + k] - q[row];
}

// X[:, k] += d (one column of a [n_dofs][S] block).
__global__ __launch_bounds__(256) void k_batch_add_col(double *__restrict__ X, const double *__restrict__ d,
                                                       int S, int k, int64_t ndof)
{
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < ndof;
         row += (int64_t)gridDim.x * blockDim.x)
        X[row * S + k] += d[row];
}

// Caller's b [n_dofs][ld] (columns c0..c0+n-1) -> [n_dofs][S], clamped rows
// and padding columns zero.
__global__ __launch_bounds__(256) void k_batch_pack(const double *__restrict__ b, int64_t ld,
                                                    int n, const uint8_t *__restrict__ fixed,
                                                    double *__restrict__ B, int S, int64_t ndof)
{
    const int64_t total = ndof * S;
    for (int64_t ix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ix < total;
         ix += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = ix / S;
        const int k = (int)(ix - row * S);
        B[ix] = (k < n && !fixed[row]) ? b[row * ld + k] : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_batch_unpack(const double *__restrict__ X, int S, int n,
                                                      double *__restrict__ u, int64_t ld,
                                                      int64_t ndof)
{
    const int64_t total = ndof * n;
    for (int64_t ix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ix < total;
         ix += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = ix / n;
        const int k = (int)(ix - row * n);
        u[row * ld + k] = X[row * S + k];
    }
}

// Y = K(phi) X assembled from the apply's outputs: interior rows from Q,
// shared rows summed over their halo slots in tile order (hrange null: all
// rows from Q), clamped rows 0.
template <int D, int S>
__global__ __launch_bounds__(256) void k_batch_collect(const float *__restrict__ Q,
                                                       const float *__restrict__ halo,
                                                       const int2 *__restrict__ hrange,
                                                       const uint8_t *__restrict__ fixed,
                                                       float *__restrict__ Y, int64_t ndof)
{
    constexpr int RG = 256 / S;
    const int tid = threadIdx.x, col = tid % S, rg = tid / S;
    for (int64_t row = rg < RG ? (int64_t)blockIdx.x * RG + rg : ndof; row < ndof; row += (int64_t)gridDim.x * RG) {
        const int64_t node = row / D;
        const int i = (int)(row - node * D);
        const int2 hr = hrange ? hrange[node] : make_int2(-1, -1);
        float q;
        if (hr.x < 0) {
            q = Q[row * S + col];
        } else {
            q = halo_row_sum(halo, hr, (int64_t)i * S + col, (int64_t)D * S);
        }
        Y[row * S + col] = fixed[row] ? 0.f : q;
    }
}

// ---------------------------------------------------------------------------
// launchers

static int grid_of(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

template <int D, int NC, int G>
static int set_apply_lds1(int bytes)
{
    return hipFuncSetAttribute((const void *)k_batch_apply<D, NC, G>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess;
}

template <int D, int NC>
static int set_apply_lds(int bytes)
{
    return set_apply_lds1<D, NC, 4>(bytes) | set_apply_lds1<D, NC, 8>(bytes);
}

// Allows the largest dynamic LDS for every instance (outside graph capture).
static int batch_prepare_lds(int D)
{
    const int cap = kBatchLds - kBatchStaticLds;
    if (D == 2)
        return set_apply_lds<2, 1>(cap) | set_apply_lds<2, 2>(cap) | set_apply_lds<2, 3>(cap) |
               set_apply_lds<2, 4>(cap);
    return set_apply_lds<3, 1>(cap) | set_apply_lds<3, 2>(cap) | set_apply_lds<3, 3>(cap) |
           set_apply_lds<3, 4>(cap);
}

template <int D, int NC, int G>
static void apply_t(const fo_ctx *c, const float *P, float *Q, BatchCtl *ctl, const BatchCol *cols,
                    hipStream_t s)
{
    const BatchState &b = c->batch;
    const size_t lds = batch_lds_bytes(D, 16 * NC, b.tiles.max_nodes);
    hipLaunchKernelGGL((k_batch_apply<D, NC, G>), dim3(xcd_grid(b.tiles.n_tiles)), dim3(64 * NC), lds, s,
                       batch_tile_args(c), b.geo, (float)c->lam, (float)c->mu, P, Q, b.halo, c->fixed,
                       b.pq_part, ctl, cols);
}

template <int D, int NC>
static void apply_g(const fo_ctx *c, const float *P, float *Q, BatchCtl *ctl, const BatchCol *cols,
                    hipStream_t s)
{
    if (c->batch.group == 4)
        apply_t<D, NC, 4>(c, P, Q, ctl, cols, s);
    else
        apply_t<D, NC, 8>(c, P, Q, ctl, cols, s);
}

static void launch_element_apply(const fo_ctx *c, int NC, const float *P, float *Q, BatchCtl *ctl,
                                 const BatchCol *cols, hipStream_t s)
{
    if (c->dim == 2) {
        switch (NC) {
        case 1: apply_g<2, 1>(c, P, Q, ctl, cols, s); break;
        case 2: apply_g<2, 2>(c, P, Q, ctl, cols, s); break;
        case 3: apply_g<2, 3>(c, P, Q, ctl, cols, s); break;
        default: apply_g<2, 4>(c, P, Q, ctl, cols, s); break;
        }
    } else {
        switch (NC) {
        case 1: apply_g<3, 1>(c, P, Q, ctl, cols, s); break;
        case 2: apply_g<3, 2>(c, P, Q, ctl, cols, s); break;
        case 3: apply_g<3, 3>(c, P, Q, ctl, cols, s); break;
        default: apply_g<3, 4>(c, P, Q, ctl, cols, s); break;
        }
    }
}

// The operator of the context's batched solves (fo_set_batch_operator).
static void launch_batch_apply(const fo_ctx *c, int NC, const float *P, float *Q, BatchCtl *ctl,
                               const BatchCol *cols, hipStream_t s)
{
    if (c->batch.op == FO_BATCH_OP_NODAL)
        nodal_apply_launch(c, NC, P, Q, ctl, cols, s);
    else
        launch_element_apply(c, NC, P, Q, ctl, cols, s);
}

void batch_apply_launch(const fo_ctx *c, int NC, const float *P, float *Q, BatchCtl *ctl, const BatchCol *cols,
                        hipStream_t s)
{
    launch_batch_apply(c, NC, P, Q, ctl, cols, s);
}

// Shared rows of Q live in the halo (element operator) or Q holds every row
// (nodal operator: null).
static const int2 *q_hrange(const fo_ctx *c)
{
    return c->batch.op == FO_BATCH_OP_NODAL ? nullptr : reinterpret_cast<const int2 *>(c->batch.tiles.node_hrange);
}

// The p.q partials of the apply at S columns: per tile or per nodal block.
static const double *pq_parts(const fo_ctx *c) { return c->batch.op == FO_BATCH_OP_NODAL ? c->batch.pq_nodal : c->batch.pq_part; }
static int pq_count(const fo_ctx *c, int S)
{
    return c->batch.op == FO_BATCH_OP_NODAL ? nodal_blocks(c, S) : c->batch.tiles.n_tiles;
}

// Dispatch on S = 16 NC for the node-parallel kernels.
template <template <int> class K, class... A>
static void by_s(int S, A... a)
{
    switch (S) {
    case 16: K<16>::run(a...); break;
    case 32: K<32>::run(a...); break;
    case 48: K<48>::run(a...); break;
    default: K<64>::run(a...); break;
    }
}

template <int S>
struct UpdateL {
    static void run(const fo_ctx *c, hipStream_t s)
    {
        const BatchState &b = c->batch;
        const int2 *hr = q_hrange(c);
        if (c->dim == 2)
            hipLaunchKernelGGL((k_batch_update<2, S>), dim3(b.n_upd), dim3(256), 0, s, b.ctl, b.cols, b.r32,
                               b.q32, c->dinv32, hr, b.halo, c->ndof, b.rz_part);
        else
            hipLaunchKernelGGL((k_batch_update<3, S>), dim3(b.n_upd), dim3(256), 0, s, b.ctl, b.cols, b.r32,
                               b.q32, c->dinv32, hr, b.halo, c->ndof, b.rz_part);
    }
};

template <int S>
struct DirectionL {
    static void run(const fo_ctx *c, const uint8_t *mask, hipStream_t s)
    {
        const BatchState &b = c->batch;
        hipLaunchKernelGGL(k_batch_direction<S>, dim3(b.n_upd), dim3(256), 0, s, b.ctl, b.cols, mask,
                           b.p32, b.x32, b.r32, c->dinv32, c->ndof);
    }
};

template <int S>
struct RescaleL {
    static void run(const fo_ctx *c, hipStream_t s)
    {
        const BatchState &b = c->batch;
        hipLaunchKernelGGL(k_batch_rescale<S>, dim3(b.n_upd), dim3(256), 0, s, b.r64, b.s2 + S, b.mask,
                           b.r32, b.x32, c->dinv32, c->ndof, b.rz_part);
    }
};

template <int S>
struct ColsqL {
    static void run(const fo_ctx *c, const double *V, double *out, hipStream_t s)
    {
        const BatchState &b = c->batch;
        hipLaunchKernelGGL(k_batch_colsq<S>, dim3(b.n_upd), dim3(256), 0, s, V, c->ndof, b.rz_part);
        hipLaunchKernelGGL(k_batch_colsum, dim3(S), dim3(256), 0, s, b.rz_part, b.n_upd, S, out);
    }
};

// One CG iteration for all columns: apply, alpha, update, beta, direction.
static void batch_iteration(const fo_ctx *c, int NC, hipStream_t s)
{
    const BatchState &b = c->batch;
    const int S = 16 * NC;
    launch_batch_apply(c, NC, b.p32, b.q32, b.ctl, b.cols, s);
    hipLaunchKernelGGL(k_batch_alpha, dim3(S), dim3(256), 0, s, b.ctl, b.cols, pq_parts(c), pq_count(c, S), S);
    by_s<UpdateL>(S, c, s);
    hipLaunchKernelGGL(k_batch_beta, dim3(S), dim3(256), 0, s, b.ctl, b.cols, b.rz_part, b.n_upd, S);
    by_s<DirectionL>(S, c, (const uint8_t *)nullptr, s);
}

// ---------------------------------------------------------------------------
// host side: tiles, buffers, solve

// Batch buffers: the block vectors are the context's; the tile arrays of a
// context with its own memory are separate allocations, released when
// fo_batch_tune rebuilds the tiles (a context on a caller's workspace keeps
// the tiles of its creation).
static int balloc(fo_ctx *c, void **p, size_t bytes, bool tile)
{
    if (!tile || c->ws || c->measure) return ctx_alloc(c, p, bytes);
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;  // counted as ctx_alloc counts
    void *v = nullptr;
    if (device_malloc(&v, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return FO_ERR_NOMEM;
    }
    c->batch.tile_allocs.push_back(v);
    c->bytes += bytes;
    c->batch.tile_bytes += bytes;
    *p = v;
    return FO_OK;
}

template <typename T>
static int bup(fo_ctx *c, T **dst, const std::vector<T> &v)
{
    FO_TRY(balloc(c, (void **)dst, v.size() * sizeof(T), true));
    if (!c->measure && !v.empty() && (hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream) !=
                           hipSuccess ||
                       fo::wait_stream(c->stream) != hipSuccess))
        return FO_ERR_HIP;
    return FO_OK;
}

static void free_batch_tiles(fo_ctx *c)
{
    BatchState &b = c->batch;
    for (void *p : b.tile_allocs) (void)hipFree(p);
    b.tile_allocs.clear();
    c->bytes -= b.tile_bytes;
    b.tile_bytes = 0;
    b.tiles = TileSet{};
}

void batch_release(fo_ctx *c)
{
    free_batch_tiles(c);
    BatchState &b = c->batch;
    if (b.ctl_host) (void)hipHostFree(b.ctl_host);
    if (b.cols_host) (void)hipHostFree(b.cols_host);
    if (b.s2_host) (void)hipHostFree(b.s2_host);
    if (b.mask_host) (void)hipHostFree(b.mask_host);
    if (b.caps_host) (void)hipHostFree(b.caps_host);
    if (b.ptol_host) (void)hipHostFree(b.ptol_host);
    b.ptol_host = nullptr;
    if (b.bcg_host) (void)hipHostFree(b.bcg_host);
    b.caps_host = nullptr;
    b.bcg_host = nullptr;
    b.ctl_host = nullptr;
    b.cols_host = nullptr;
    b.s2_host = nullptr;
    b.mask_host = nullptr;
}

int batch_max_nodes(int D, int S)
{
    const int fixed = (int)batch_lds_bytes(D, S, 0) + 16;
    const int per = D * S * 4 + 8 + D;
    return std::max(0, (kBatchLds - kBatchStaticLds - fixed) / per);
}

// Batch tiles with at most `mn` nodes over the context's element order; the
// elements of each tile are packed into groups of G with pairwise disjoint
// node sets (greedy first fit in Morton order), each group padded to G
// slots.  Slot arrays get a fixed per-tile stride.
static int build_batch_tiles(fo_ctx *c, int mn, int G, const std::vector<double> &X,
                             const std::vector<int32_t> &conn)
{
    BatchState &b = c->batch;
    const int D = c->dim, NV = D + 1;
    HostTiles h;
    build_tiles(D, c->N, c->E, X.data(), conn.data(), 16383, &h, mn, true);
    const int T = h.n_tiles;
    const int words = (h.max_nodes + 63) / 64;
    std::vector<std::vector<int32_t>> tslots(T);  // per tile: slot -> tile element index, -1 padding
    int MS = 0;
    for (int t = 0; t < T; ++t) {
        const int ne = h.info[(size_t)t * kTileInfo + kTileNE];
        std::vector<std::vector<int32_t>> groups;
        std::vector<std::vector<uint64_t>> masks;
        size_t first_open = 0;
        for (int i = 0; i < ne; ++i) {
            const uint16_t *lc = &h.lconn[((size_t)t * h.max_elems + i) * 4];
            size_t gsel = groups.size();
            for (size_t k = first_open; k < groups.size(); ++k) {
                if ((int)groups[k].size() >= G) continue;
                bool clash = false;
                for (int a = 0; a < NV && !clash; ++a) clash = (masks[k][lc[a] >> 6] >> (lc[a] & 63)) & 1;
                if (!clash) {
                    gsel = k;
                    break;
                }
            }
            if (gsel == groups.size()) {
                groups.emplace_back();
                masks.emplace_back(words, 0);
            }
            groups[gsel].push_back(i);
            for (int a = 0; a < NV; ++a) masks[gsel][lc[a] >> 6] |= 1ULL << (lc[a] & 63);
            while (first_open < groups.size() && (int)groups[first_open].size() >= G) ++first_open;
        }
        std::vector<int32_t> &sl = tslots[t];
        for (auto &gr : groups) {
            for (int32_t i : gr) sl.push_back(i);
            for (size_t k = gr.size(); k < (size_t)G; ++k) sl.push_back(-1);
        }
        MS = std::max(MS, (int)sl.size());
    }
    std::vector<int32_t> selem((size_t)T * MS, -1);
    std::vector<uint64_t> slconn((size_t)T * MS, ~0ULL);
    std::vector<int32_t> sgconn((size_t)T * MS * 4, 0);
    std::vector<int32_t> info(h.info);
    for (int t = 0; t < T; ++t) {
        const int e0 = h.info[(size_t)t * kTileInfo + kTileE0];
        const std::vector<int32_t> &sl = tslots[t];
        info[(size_t)t * kTileInfo + kTileNE] = (int32_t)sl.size();
        for (size_t k = 0; k < sl.size(); ++k) {
            const size_t o = (size_t)t * MS + k;
            if (sl[k] < 0) continue;
            const int64_t e = e0 + sl[k];
            selem[o] = (int32_t)e;
            const uint16_t *lc = &h.lconn[((size_t)t * h.max_elems + sl[k]) * 4];
            uint64_t v = 0;
            for (int a = 0; a < 4; ++a) v |= (uint64_t)(a < NV ? lc[a] : 0) << (16 * a);
            slconn[o] = v;
            for (int a = 0; a < NV; ++a) sgconn[o * 4 + a] = conn[(size_t)a * c->E + e];
        }
    }
    free_batch_tiles(c);
    TileSet &ts = b.tiles;
    ts.n_tiles = T;
    ts.max_nodes = h.max_nodes;
    ts.max_elems = MS;
    ts.n_slots = h.n_slots;
    ts.n_shared_nodes = (int64_t)h.halo_node.size();
    ts.n_shared_slots = h.halo_ptr.empty() ? 0 : (int64_t)h.halo_ptr.back();
    FO_TRY(bup(c, &ts.info, info));
    FO_TRY(bup(c, &ts.nodes, h.nodes));
    FO_TRY(bup(c, &ts.hpos, h.hpos));
    FO_TRY(bup(c, &ts.node_hrange, h.node_hrange));
    FO_TRY(bup(c, &ts.halo_node, h.halo_node));
    FO_TRY(bup(c, &ts.halo_ptr, h.halo_ptr));
    FO_TRY(bup(c, &b.selem, selem));
    FO_TRY(bup(c, &b.slconn, slconn));
    int32_t *sg = nullptr;
    FO_TRY(bup(c, &sg, sgconn));
    b.sgconn = reinterpret_cast<int4 *>(sg);
    b.slot_stride = MS;
    b.n_slot_total = (int64_t)T * MS;
    b.group = G;
    FO_TRY(balloc(c, (void **)&b.geo, (size_t)std::max<int64_t>(b.n_slot_total, 1) * 16 * sizeof(float), true));
    b.halo_cap = (size_t)std::max<int64_t>(ts.n_shared_slots, 1) * c->dim * b.S;
    FO_TRY(balloc(c, (void **)&b.halo, b.halo_cap * sizeof(float), true));
    const size_t need_pq = (size_t)std::max(T, 1) * b.S;
    FO_TRY(balloc(c, (void **)&b.pq_part, need_pq * sizeof(double), true));
    b.pq_cap = need_pq;
    b.mn_cap = mn;
    ++b.version;
    if (c->have_phi) FO_TRY(batch_levelset(c));
    return FO_OK;
}

// Host copies of the mesh in the context's element order (for tile builds).
static int mesh_host(fo_ctx *c, std::vector<double> &X, std::vector<int32_t> &conn)
{
    X.resize((size_t)c->N * c->dim);
    conn.resize((size_t)(c->dim + 1) * c->E);
    if (hipMemcpyAsync(X.data(), c->coords, X.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(conn.data(), c->conn, conn.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        fo::wait_stream(c->stream) != hipSuccess)
        return FO_ERR_HIP;
    return FO_OK;
}

int batch_default_nodes(int D) { return D == 2 ? 256 : 160; }

int batch_setup(fo_ctx *c, int max_rhs, const double *coords, const std::vector<int32_t> &conn_t)
{
    BatchState &b = c->batch;
    const int D = c->dim;
    b.S = 16 * std::min(4, (max_rhs + 15) / 16);
    const int64_t n = c->ndof * b.S;
    const int RG = 256 / b.S;
    b.n_upd = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (c->ndof + RG - 1) / RG));
    FO_TRY(balloc(c, (void **)&b.x32, n * sizeof(float), false));
    FO_TRY(balloc(c, (void **)&b.r32, n * sizeof(float), false));
    FO_TRY(balloc(c, (void **)&b.p32, n * sizeof(float), false));
    FO_TRY(balloc(c, (void **)&b.q32, n * sizeof(float), false));
    FO_TRY(balloc(c, (void **)&b.x64, n * sizeof(double), false));
    FO_TRY(balloc(c, (void **)&b.r64, n * sizeof(double), false));
    FO_TRY(balloc(c, (void **)&b.b64, n * sizeof(double), false));
    FO_TRY(balloc(c, (void **)&b.rz_part, (size_t)2 * b.n_upd * b.S * sizeof(double), false));
    FO_TRY(balloc(c, (void **)&b.s2, (size_t)3 * b.S * sizeof(double), false));
    FO_TRY(balloc(c, (void **)&b.mask, (size_t)b.S, false));
    FO_TRY(balloc(c, (void **)&b.caps, (size_t)b.S * sizeof(int32_t), false));
    FO_TRY(balloc(c, (void **)&b.ptol, (size_t)b.S * sizeof(double), false));
    FO_TRY(balloc(c, (void **)&b.cols, (size_t)b.S * sizeof(BatchCol), false));
    FO_TRY(balloc(c, (void **)&b.ctl, sizeof(BatchCtl), false));
    FO_TRY(balloc(c, (void **)&b.bcg.st, sizeof(BcgState), false));
    FO_TRY(balloc(c, (void **)&b.bcg.sums, (size_t)2 * b.S * b.S * sizeof(double), false));
    FO_TRY(balloc(c, (void **)&b.bcg.part, bcg_part_floats(b.S) * sizeof(float), false));
    if (!c->measure) {
        if (hipHostMalloc((void **)&b.ctl_host, sizeof(BatchCtl)) != hipSuccess ||
            hipHostMalloc((void **)&b.cols_host, b.S * sizeof(BatchCol)) != hipSuccess ||
            hipHostMalloc((void **)&b.s2_host, b.S * sizeof(double)) != hipSuccess ||
            hipHostMalloc((void **)&b.mask_host, b.S) != hipSuccess ||
            hipHostMalloc((void **)&b.caps_host, b.S * sizeof(int32_t)) != hipSuccess ||
            hipHostMalloc((void **)&b.ptol_host, b.S * sizeof(double)) != hipSuccess ||
            hipHostMalloc((void **)&b.bcg_host, sizeof(BcgState)) != hipSuccess)
            return FO_ERR_NOMEM;
        if (bcg_prepare()) return FO_ERR_HIP;
        // directions start at zero (the first direction of a column ignores them,
        // but stale non-finite bits must not survive a zero coefficient)
        launch_fill<float>(b.p32, n, 0.0f, c->stream);
        launch_fill<float>(b.q32, n, 0.0f, c->stream);
        if (batch_prepare_lds(D)) return FO_ERR_HIP;
    }
    // host copies of the mesh in the context's element order (for the tiles)
    const std::vector<double> X(coords, coords + (size_t)c->N * D);
    const int mn = std::min(batch_default_nodes(D), batch_max_nodes(D, b.S));
    FO_TRY(nodal_setup(c, conn_t));
    FO_TRY(build_batch_tiles(c, mn, 8, X, conn_t));
    if (!c->measure) FO_HIP(fo::wait_stream(c->stream));
    return FO_OK;
}

static void destroy_batch_graphs(fo_ctx *c)
{
    for (auto it = c->graphs.begin(); it != c->graphs.end();) {
        if (std::get<0>(it->first) >= 100 && std::get<0>(it->first) < 300) {  // batched solver families
            (void)hipGraphExecDestroy(it->second);
            it = c->graphs.erase(it);
        } else {
            ++it;
        }
    }
}

// Times `reps` back-to-back launches of the batched apply (NC column
// chunks; op: FO_BATCH_OP_*, or -1 for the context's operator); columns are
// all active.
int batch_time_apply(fo_ctx *c, int NC, int reps, double *avg_us, int op)
{
    if (op < 0) op = c->batch.op;
    BatchState &b = c->batch;
    hipStream_t s = c->stream;
    const int S = 16 * NC;
    std::vector<BatchCol> cols(S);
    for (auto &col : cols) col = BatchCol{};
    BatchCtl ctl{0, 0, INT32_MAX, 0};
    FO_HIP(hipMemcpyAsync(b.cols, cols.data(), S * sizeof(BatchCol), hipMemcpyHostToDevice, s));
    FO_HIP(hipMemcpyAsync(b.ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, s));
    launch_fill<float>(b.p32, c->ndof * S, 1.0f, s);
    auto apply = [&]() {
        if (op == FO_BATCH_OP_NODAL)
            nodal_apply_launch(c, NC, b.p32, b.q32, b.ctl, b.cols, s);
        else
            launch_element_apply(c, NC, b.p32, b.q32, b.ctl, b.cols, s);
    };
    apply();
    hipEvent_t e0, e1;
    FO_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FO_ERR_HIP;
    }
    (void)hipEventRecord(e0, s);
    for (int k = 0; k < reps; ++k) apply();
    (void)hipEventRecord(e1, s);
    float ms = 0.0f;
    int rc = FO_OK;
    if (fo::wait_event(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        hipGetLastError() != hipSuccess)
        rc = FO_ERR_HIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    launch_fill<float>(b.p32, c->ndof * S, 0.0f, s);
    if (rc == FO_OK) *avg_us = 1e3 * (double)ms / reps;
    return rc;
}

template <int S>
struct CollectL {
    static void run(const fo_ctx *c, float *Y, hipStream_t s)
    {
        const BatchState &b = c->batch;
        const int2 *hr = q_hrange(c);
        if (c->dim == 2)
            hipLaunchKernelGGL((k_batch_collect<2, S>), dim3(b.n_upd), dim3(256), 0, s, b.q32, b.halo, hr,
                               c->fixed, Y, c->ndof);
        else
            hipLaunchKernelGGL((k_batch_collect<3, S>), dim3(b.n_upd), dim3(256), 0, s, b.q32, b.halo, hr,
                               c->fixed, Y, c->ndof);
    }
};

// Y = K(phi) X for one FP32 block of S = 16 NC columns (device [n_dofs][S]).
int batch_apply_block(fo_ctx *c, int NC, const float *X, float *Y)
{
    BatchState &b = c->batch;
    hipStream_t s = c->stream;
    const int S = 16 * NC;
    std::vector<BatchCol> cols(S);
    for (auto &col : cols) col = BatchCol{};
    BatchCtl ctl{0, 0, INT32_MAX, 0};
    FO_HIP(hipMemcpyAsync(b.cols, cols.data(), S * sizeof(BatchCol), hipMemcpyHostToDevice, s));
    FO_HIP(hipMemcpyAsync(b.ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, s));
    FO_HIP(hipMemcpyAsync(b.p32, X, c->ndof * S * sizeof(float), hipMemcpyDeviceToDevice, s));
    launch_batch_apply(c, NC, b.p32, b.q32, b.ctl, b.cols, s);
    by_s<CollectL>(S, (const fo_ctx *)c, Y, s);
    FO_HIP(hipGetLastError());
    FO_HIP(fo::wait_stream(s));
    return FO_OK;
}

// Tries the node caps that fit the LDS and both group sizes, and keeps the
// fastest apply.
int batch_tune(fo_ctx *c, int n_rhs, int *best_nodes, int *best_group, double *best_us)
{
    if (c->ws) return FO_ERR_STATE;  // the tiles of a workspace context are the ones of its creation
    BatchState &b = c->batch;
    const int NC = std::min(4, std::max(1, (n_rhs + 15) / 16));
    const int S = 16 * NC;
    const int D = c->dim;
    const int cap = batch_max_nodes(D, S);
    std::vector<int> cand = D == 2 ? std::vector<int>{96, 128, 192, 256, 288}
                                   : std::vector<int>{64, 96, 128, 160, 176};
    std::vector<double> X;
    std::vector<int32_t> conn;
    FO_TRY(mesh_host(c, X, conn));
    destroy_batch_graphs(c);
    int best = 0, bg = 8;
    double best_t = 1e300;
    for (int mn : cand) {
        if (mn > cap) continue;
        for (int G : {4, 8}) {
            FO_TRY(build_batch_tiles(c, mn, G, X, conn));
            double us = 0.0;
            FO_TRY(batch_time_apply(c, NC, 20, &us, FO_BATCH_OP_ELEMENT));
            if (us < best_t) {
                best_t = us;
                best = mn;
                bg = G;
            }
        }
    }
    if (best == 0) return FO_ERR_ARG;
    if (best != b.mn_cap || bg != b.group) FO_TRY(build_batch_tiles(c, best, bg, X, conn));
    FO_HIP(fo::wait_stream(c->stream));
    if (best_nodes) *best_nodes = best;
    if (best_group) *best_group = bg;
    if (best_us) *best_us = best_t;
    return FO_OK;
}

static int poll_batch(fo_ctx *c)
{
    FO_HIP(hipMemcpyAsync(c->batch.ctl_host, c->batch.ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost,
                          c->stream));
    FO_HIP(fo::wait_stream(c->stream));
    return FO_OK;
}

// Column norms^2 of the FP64 residual block into s2[S..2S) and the host.
static int residual_norms(fo_ctx *c, int S)
{
    BatchState &b = c->batch;
    by_s<ColsqL>(S, (const fo_ctx *)c, (const double *)b.r64, b.s2 + S, c->stream);
    FO_HIP(hipMemcpyAsync(b.s2_host, b.s2 + S, S * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    FO_HIP(fo::wait_stream(c->stream));
    return FO_OK;
}

// Element data of the batched operator for the current level set.
int batch_levelset(fo_ctx *c)
{
    const BatchState &b = c->batch;
    if (b.S == 0) return FO_OK;
    FO_TRY(nodal_levelset(c));
    if (b.n_slot_total == 0) return FO_OK;
    const int grid = grid_of(b.n_slot_total);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_batch_geom<2>, dim3(grid), dim3(256), 0, c->stream, b.selem, b.sgconn,
                           b.n_slot_total, c->coords, c->chi, c->ersatz, b.geo);
    else
        hipLaunchKernelGGL(k_batch_geom<3>, dim3(grid), dim3(256), 0, c->stream, b.selem, b.sgconn,
                           b.n_slot_total, c->coords, c->chi, c->ersatz, b.geo);
    FO_HIP(hipGetLastError());
    return FO_OK;
}

// FP32 CG on all columns of one block with FP64 residual replacement per
// column: a column whose FP32 residual fell by its phase target iterates on
// to the end of the chunk of iterations, then its x64 += s x32 and r64 =
// b - K x64 (FP64) are formed, and it continues from the replaced residual
// with its direction (rescaled), while the other columns keep iterating.  With the nodal operator, K x64 of all the columns
// that finished together is one launch over the FP64 node blocks; the
// element operator takes them one at a time through the FP64 element apply.
// Columns c0..c0+n-1 of b (ld) -> u.
static int batch_group(fo_ctx *c, const double *b_in, double *u, int n, int64_t ld,
                       const fo_solve_opts *o, fo_solve_stats *st)
{
    BatchState &b = c->batch;
    hipStream_t s = c->stream;
    const int NC = std::min(4, (n + 15) / 16);
    const int S = 16 * NC;
    const int64_t nd = c->ndof;
    // iterations per graph chunk (host poll); on 64x32x32 with 64 load cases
    // 24 beat 8, 12 and 16 (fewer polls) and 32 tied; 48 lost to the later phase ends
    const int chunk = o->check_every > 0 ? o->check_every : 24;
    const int max_outer = o->max_outer > 0 ? o->max_outer : 60;
    const double phase_rtol = o->inner_rtol > 0 ? o->inner_rtol : 0.1;
    hipLaunchKernelGGL(k_batch_pack, dim3(grid_of(nd * S)), dim3(256), 0, s, b_in, ld, n, c->fixed, b.b64,
                       S, nd);
    launch_fill<double>(b.x64, nd * S, 0.0, s);
    FO_HIP(hipMemcpyAsync(b.r64, b.b64, nd * S * sizeof(double), hipMemcpyDeviceToDevice, s));
    {
        std::vector<BatchCol> cols(S);
        for (auto &col : cols) {
            col = BatchCol{};
            col.fresh = 1;
            col.done = 1;
        }
        BatchCtl ctl{0, 0, o->max_iter, 0};
        FO_HIP(hipMemcpyAsync(b.cols, cols.data(), S * sizeof(BatchCol), hipMemcpyHostToDevice, s));
        FO_HIP(hipMemcpyAsync(b.ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, s));
        FO_HIP(fo::wait_stream(s));
    }
    FO_TRY(residual_norms(c, S));
    std::vector<double> bnorm(S), rn(S);
    std::vector<int> conv(S, 0), status(S, FO_OK), restart(S, 1), outer(S, 0), fail(S, 0);
    std::vector<int64_t> longest(S, 0);  // longest phase of a column that reached its target
    std::vector<int> capped_run(S, 0), finish64(S, 0);
    for (int k = 0; k < S; ++k) {
        bnorm[k] = rn[k] = std::sqrt(b.s2_host[k]);
        conv[k] = k >= n || bnorm[k] == 0.0;
    }
    // columns to (re)start from r64: mask_host
    // a phase four times as long as the column's longest completed one (at
    // least 256 iterations) has stagnated: it is stopped and restarted after
    // the replacement (the single-load rule)
    auto select = [&](const std::vector<int> &fin) {
        bool any = false;
        for (int k = 0; k < S; ++k) {
            b.mask_host[k] = (fin[k] && !conv[k]) ? 1 : 0;
            b.caps_host[k] = (int32_t)std::min<int64_t>(
                INT32_MAX / 2, longest[k] > 0 ? std::max<int64_t>(4 * longest[k], 256) : first_phase_cap(nd));
            b.ptol_host[k] = phase_target(phase_rtol, o->rtol, bnorm[k], rn[k]);
            any = any || b.mask_host[k];
        }
        return any;
    };
    auto restart_columns = [&]() -> int {
        FO_HIP(hipMemcpyAsync(b.mask, b.mask_host, S, hipMemcpyHostToDevice, s));
        by_s<RescaleL>(S, (const fo_ctx *)c, s);
        FO_HIP(hipMemcpyAsync(b.caps, b.caps_host, S * sizeof(int32_t), hipMemcpyHostToDevice, s));
        FO_HIP(hipMemcpyAsync(b.ptol, b.ptol_host, S * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_batch_phase, dim3(S), dim3(256), 0, s, b.ctl, b.cols, b.rz_part, b.n_upd, S, b.s2,
                           b.mask, b.caps, (const double *)b.ptol);
        by_s<DirectionL>(S, (const fo_ctx *)c, (const uint8_t *)b.mask, s);
        FO_HIP(hipGetLastError());
        return FO_OK;
    };
    std::vector<int> fin(S, 1);
    if (select(fin)) FO_TRY(restart_columns());
    int result = FO_NOT_CONVERGED;
    int32_t it_total = 0;
    // the host copy of the control state is current after each chunk's
    // readback; a restart (which clears done) makes it stale
    bool ctl_stale = true;
    while (true) {
        bool all = true;
        for (int k = 0; k < S; ++k) all = all && conv[k];
        if (all) {
            result = FO_OK;
            break;
        }
        if (ctl_stale) FO_TRY(poll_batch(c));
        ctl_stale = false;
        it_total = b.ctl_host->it;
        if (it_total >= o->max_iter) break;
        const bool ran = !b.ctl_host->done;
        const int32_t before = b.ctl_host->it;
        if (ran) {
            auto key = std::make_tuple(100 + NC, chunk, b.version, b.op);  // the operator is captured
            FO_TRY(graph_chunk(c, key, [&](hipStream_t ws) {
                for (int j = 0; j < chunk; ++j) batch_iteration(c, NC, ws);
                return (int)FO_OK;
            }));
        }
        // the control state and the columns that finished their phase (or
        // broke down): one readback, one wait
        FO_HIP(hipMemcpyAsync(b.ctl_host, b.ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, s));
        FO_HIP(hipMemcpyAsync(b.cols_host, b.cols, S * sizeof(BatchCol), hipMemcpyDeviceToHost, s));
        FO_HIP(fo::wait_stream(s));
        if (ran && !b.ctl_host->done && b.ctl_host->it == before) {
            hipError_t e = hipGetLastError();
            std::fprintf(stderr, "libfo: batched CG chunk made no progress (%s)\n", hipGetErrorString(e));
            return FO_ERR_HIP;
        }
        bool any = false;
        for (int k = 0; k < S; ++k) {
            fin[k] = !conv[k] && (b.cols_host[k].done || b.cols_host[k].reached);
            b.mask_host[k] = fin[k] ? 1 : 0;
            any = any || fin[k];
        }
        if (!any) continue;
        FO_HIP(hipMemcpyAsync(b.mask, b.mask_host, S, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_batch_accumulate, dim3(grid_of(nd * S)), dim3(256), 0, s, b.x64, b.x32, b.s2,
                           b.mask, S, nd * S);
        if (b.op == FO_BATCH_OP_NODAL && b.kb64) {
            // every finished column at once, from the FP64 node blocks, with
            // the norms of the finished columns (the only ones read below)
            int nbk = 0;
            FO_TRY(nodal_residual64(c, S, b.x64, b.b64, b.mask, b.r64, b.rz_part, (int64_t)2 * b.n_upd * b.S, &nbk,
                                    s));
            hipLaunchKernelGGL(k_batch_colsum, dim3(S), dim3(256), 0, s, b.rz_part, nbk, S, b.s2 + S);
            FO_HIP(hipMemcpyAsync(b.s2_host, b.s2 + S, S * sizeof(double), hipMemcpyDeviceToHost, s));
            FO_HIP(fo::wait_stream(s));
        } else {
            for (int k = 0; k < S; ++k) {
                if (!fin[k]) continue;
                launch_gather_col<double, double>(b.x64 + k, S, nd, c->t64, nullptr, s);
                FO_TRY(elas_apply64(c, c->t64, c->q64, s));
                hipLaunchKernelGGL(k_batch_residual_col, dim3(grid_of(nd)), dim3(256), 0, s, b.b64, c->q64,
                                   c->fixed, b.r64, S, k, nd);
            }
            FO_TRY(residual_norms(c, S));
        }
        for (int k = 0; k < S; ++k) {
            if (!fin[k]) continue;
            ++outer[k];
            const double r = std::sqrt(b.s2_host[k]);
            if (!(r == r)) {  // non-finite FP64 residual: the column fails
                status[k] = FO_ERR_BREAKDOWN;
                conv[k] = 1;
                fail[k] = 1;
                continue;
            }
            // a column restarted in the last phase that made no progress
            // cannot improve in FP32 any more
            const bool stalled = restart[k] && r >= rn[k];
            restart[k] = b.cols_host[k].fresh;
            if (!b.cols_host[k].capped && b.cols_host[k].status == 0)
                longest[k] = std::max<int64_t>(longest[k], b.cols_host[k].it);
            capped_run[k] = b.cols_host[k].capped ? capped_run[k] + 1 : 0;
            rn[k] = r;
            if (r <= o->rtol * bnorm[k]) {
                conv[k] = 1;
            } else if (capped_run[k] >= 2) {  // FP32 stagnates on this column: finish it in FP64
                conv[k] = 1;
                finish64[k] = 1;
            } else if (stalled || outer[k] >= max_outer) {
                conv[k] = 1;
                fail[k] = 1;
            }
        }
        if (select(fin)) {
            FO_TRY(restart_columns());
            ctl_stale = true;
        }
    }
    // columns that FP32 cannot resolve: FP64 CG on their residual equation
    int64_t extra = 0;
    for (int k = 0; k < n; ++k) {
        if (!finish64[k]) continue;
        launch_gather_col<double, double>(b.r64 + k, S, nd, c->t64, nullptr, s);
        fo_solve_opts o2 = *o;
        o2.rtol = o->rtol * bnorm[k] / rn[k];
        fo_solve_stats s2st{};
        const int rc = fp64_solve(c, c->t64, &o2, &s2st);
        if (rc < 0 && rc != FO_ERR_BREAKDOWN) return rc;
        extra += s2st.iters_inner;
        hipLaunchKernelGGL(k_batch_add_col, dim3(grid_of(nd)), dim3(256), 0, s, b.x64, c->x64, S, k, nd);
        launch_gather_col<double, double>(b.x64 + k, S, nd, c->t64, nullptr, s);
        FO_TRY(elas_apply64(c, c->t64, c->q64, s));
        hipLaunchKernelGGL(k_batch_residual_col, dim3(grid_of(nd)), dim3(256), 0, s, b.b64, c->q64, c->fixed,
                           b.r64, S, k, nd);
        FO_TRY(residual_norms(c, S));
        rn[k] = std::sqrt(b.s2_host[k]);
        ++outer[k];
        if (rc == FO_ERR_BREAKDOWN) status[k] = FO_ERR_BREAKDOWN;
        else if (!(rn[k] <= o->rtol * bnorm[k])) fail[k] = 1;
    }
    hipLaunchKernelGGL(k_batch_unpack, dim3(grid_of(nd * n)), dim3(256), 0, s, b.x64, S, n, u, ld, nd);
    FO_HIP(fo::wait_stream(s));
    double worst = 0.0;
    int max_outer_seen = 0;
    for (int k = 0; k < n; ++k) {
        if (bnorm[k] > 0) worst = std::max(worst, rn[k] / bnorm[k]);
        max_outer_seen = std::max(max_outer_seen, outer[k]);
        if (fail[k] && result == FO_OK) result = FO_NOT_CONVERGED;
    }
    for (int k = 0; k < n; ++k)
        if (status[k] == FO_ERR_BREAKDOWN) result = FO_ERR_BREAKDOWN;
    if (st) {
        st->status = result;
        st->iters_inner += it_total + (int32_t)extra;
        st->iters_outer = std::max(st->iters_outer, max_outer_seen);
        st->rel_res = std::max(st->rel_res, worst);
    }
    return result;
}

// Block CG (O'Leary) on the columns of one block inside the FP64 residual
// replacement: every phase restarts the block from the FP64 residuals of the
// columns not yet converged, each scaled to unit norm, and runs block CG in
// FP32 (fo_bcg.hip) until every column's residual fell by the phase target,
// a column leaving the block when it gets there, or the phase reaches its
// cap; then x64 += s x32 and r64 = b - K x64 in FP64 for the phase's
// columns.  The block narrows (16 columns at a time) between chunks of
// iterations as columns converge.  A column whose FP64 residual did not
// fall in a phase is finished by FP64 CG on its residual equation.
static int bcg_group(fo_ctx *c, const double *b_in, double *u, int n, int64_t ld, const fo_solve_opts *o,
                     fo_solve_stats *st)
{
    BatchState &b = c->batch;
    hipStream_t s = c->stream;
    const int NS = std::min(4, (n + 15) / 16);
    const int S = 16 * NS;
    const int64_t nd = c->ndof;
    const int chunk = o->check_every > 0 ? o->check_every : 8;
    const int max_outer = o->max_outer > 0 ? o->max_outer : 60;
    const double phase_rtol = o->inner_rtol > 0 ? o->inner_rtol : 0.1;
    hipLaunchKernelGGL(k_batch_pack, dim3(grid_of(nd * S)), dim3(256), 0, s, b_in, ld, n, c->fixed, b.b64,
                       S, nd);
    launch_fill<double>(b.x64, nd * S, 0.0, s);
    launch_fill<float>(b.x32, nd * S, 0.0f, s);
    FO_HIP(hipMemcpyAsync(b.r64, b.b64, nd * S * sizeof(double), hipMemcpyDeviceToDevice, s));
    {
        std::vector<BatchCol> cols(S);
        for (auto &col : cols) col = BatchCol{};  // not done: the apply runs while the block does
        BatchCtl ctl{0, 0, o->max_iter, 0};
        FO_HIP(hipMemcpyAsync(b.cols, cols.data(), S * sizeof(BatchCol), hipMemcpyHostToDevice, s));
        FO_HIP(hipMemcpyAsync(b.ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, s));
        FO_HIP(fo::wait_stream(s));
    }
    FO_TRY(residual_norms(c, S));
    std::vector<double> bnorm(S), rn(S);
    std::vector<int> conv(S, 0), status(S, FO_OK), outer(S, 0), fail(S, 0), finish64(S, 0);
    for (int k = 0; k < S; ++k) {
        bnorm[k] = rn[k] = std::sqrt(b.s2_host[k]);
        conv[k] = k >= n || bnorm[k] == 0.0;
    }
    int64_t longest = 0;   // longest phase that reached its target
    int result = FO_NOT_CONVERGED;
    int32_t it_total = 0;
    BcgState &h = *b.bcg_host;
    while (true) {
        int na = 0;
        for (int k = 0; k < S; ++k) {
            b.mask_host[k] = conv[k] ? 0 : 1;
            na += b.mask_host[k];
        }
        if (na == 0) {
            result = FO_OK;
            break;
        }
        FO_TRY(poll_batch(c));
        it_total = b.ctl_host->it;
        if (it_total >= o->max_iter) break;
        // phase start: R32 = R64 / ||R64||, X32 = 0 on the phase's columns
        FO_HIP(hipMemcpyAsync(b.mask, b.mask_host, S, hipMemcpyHostToDevice, s));
        by_s<RescaleL>(S, (const fo_ctx *)c, s);
        // the phase's scales (k_batch_accumulate reads s2[0..S))
        FO_HIP(hipMemcpyAsync(b.s2, b.s2 + S, S * sizeof(double), hipMemcpyDeviceToDevice, s));
        std::memset(&h, 0, offsetof(BcgState, rr));
        h.np = na;
        h.first = 1;
        h.cap = (int32_t)std::min<int64_t>(INT32_MAX / 2, longest > 0 ? std::max<int64_t>(2 * longest, 64)
                                                                      : first_phase_cap(nd));
        h.tol2 = phase_rtol * phase_rtol;
        h.drop = kBcgDrop;
        for (int q = 0, k = 0; q < 64; ++q) {
            while (k < S && !b.mask_host[k]) ++k;
            h.act[q] = (q < na) ? k++ : -1;
        }
        for (int k = 0; k < 64; ++k) h.run[k] = k < S ? b.mask_host[k] : 0;
        FO_HIP(hipMemcpyAsync(b.bcg.st, &h, offsetof(BcgState, rr), hipMemcpyHostToDevice, s));
        b.ctl_host->done = 0;
        b.ctl_host->max_it = o->max_iter;
        b.ctl_host->pad = na;
        FO_HIP(hipMemcpyAsync(b.ctl, b.ctl_host, sizeof(BatchCtl), hipMemcpyHostToDevice, s));
        int NP = (na + 15) / 16;
        bcg_direction(c, b.bcg, NP, NS, s);
        FO_HIP(hipGetLastError());
        while (true) {
            const int32_t before = b.ctl_host->it;
            auto key = std::make_tuple(200 + 8 * NP + NS, chunk, b.version, b.op);
            FO_TRY(graph_chunk(c, key, [&](hipStream_t ws) {
                for (int j = 0; j < chunk; ++j) bcg_iteration(c, b.bcg, NP, NS, ws);
                return (int)FO_OK;
            }));
            FO_TRY(poll_batch(c));
            if (b.ctl_host->done) break;
            if (b.ctl_host->it == before) {
                hipError_t e = hipGetLastError();
                std::fprintf(stderr, "libfo: block CG chunk made no progress (%s)\n", hipGetErrorString(e));
                return FO_ERR_HIP;
            }
            const int np2 = (b.ctl_host->pad + 15) / 16;
            if (np2 >= 1 && np2 < NP) {  // narrower block: re-stride P for the next chunk
                bcg_restride(c, 16 * NP, 16 * np2, s);
                NP = np2;
            }
        }
        FO_HIP(hipMemcpyAsync(&h, b.bcg.st, offsetof(BcgState, rr), hipMemcpyDeviceToHost, s));
        FO_HIP(fo::wait_stream(s));
        if (!h.capped && h.status == 0) longest = std::max<int64_t>(longest, h.it_phase);
        // FP64 refinement of the phase's columns
        hipLaunchKernelGGL(k_batch_accumulate, dim3(grid_of(nd * S)), dim3(256), 0, s, b.x64, b.x32, b.s2,
                           b.mask, S, nd * S);
        for (int k = 0; k < S; ++k) {
            if (!b.mask_host[k]) continue;
            launch_gather_col<double, double>(b.x64 + k, S, nd, c->t64, nullptr, s);
            FO_TRY(elas_apply64(c, c->t64, c->q64, s));
            hipLaunchKernelGGL(k_batch_residual_col, dim3(grid_of(nd)), dim3(256), 0, s, b.b64, c->q64,
                               c->fixed, b.r64, S, k, nd);
        }
        FO_TRY(residual_norms(c, S));
        for (int k = 0; k < S; ++k) {
            if (!b.mask_host[k]) continue;
            ++outer[k];
            const double r = std::sqrt(b.s2_host[k]);
            if (!(r == r)) {  // non-finite FP64 residual: the column fails
                status[k] = FO_ERR_BREAKDOWN;
                conv[k] = 1;
                fail[k] = 1;
                continue;
            }
            const bool stalled = !(r < 0.5 * rn[k]);
            rn[k] = r;
            if (r <= o->rtol * bnorm[k]) {
                conv[k] = 1;
            } else if (stalled) {  // FP32 makes no progress on this column: finish it in FP64
                conv[k] = 1;
                finish64[k] = 1;
            } else if (outer[k] >= max_outer) {
                conv[k] = 1;
                fail[k] = 1;
            }
        }
    }
    // columns that FP32 cannot resolve: FP64 CG on their residual equation
    int64_t extra = 0;
    for (int k = 0; k < n; ++k) {
        if (!finish64[k]) continue;
        launch_gather_col<double, double>(b.r64 + k, S, nd, c->t64, nullptr, s);
        fo_solve_opts o2 = *o;
        o2.rtol = o->rtol * bnorm[k] / rn[k];
        fo_solve_stats s2st{};
        const int rc = fp64_solve(c, c->t64, &o2, &s2st);
        if (rc < 0 && rc != FO_ERR_BREAKDOWN) return rc;
        extra += s2st.iters_inner;
        hipLaunchKernelGGL(k_batch_add_col, dim3(grid_of(nd)), dim3(256), 0, s, b.x64, c->x64, S, k, nd);
        launch_gather_col<double, double>(b.x64 + k, S, nd, c->t64, nullptr, s);
        FO_TRY(elas_apply64(c, c->t64, c->q64, s));
        hipLaunchKernelGGL(k_batch_residual_col, dim3(grid_of(nd)), dim3(256), 0, s, b.b64, c->q64, c->fixed,
                           b.r64, S, k, nd);
        FO_TRY(residual_norms(c, S));
        rn[k] = std::sqrt(b.s2_host[k]);
        ++outer[k];
        if (rc == FO_ERR_BREAKDOWN) status[k] = FO_ERR_BREAKDOWN;
        else if (!(rn[k] <= o->rtol * bnorm[k])) fail[k] = 1;
    }
    hipLaunchKernelGGL(k_batch_unpack, dim3(grid_of(nd * n)), dim3(256), 0, s, b.x64, S, n, u, ld, nd);
    FO_HIP(fo::wait_stream(s));
    double worst = 0.0;
    int max_outer_seen = 0;
    for (int k = 0; k < n; ++k) {
        if (bnorm[k] > 0) worst = std::max(worst, rn[k] / bnorm[k]);
        max_outer_seen = std::max(max_outer_seen, outer[k]);
        if (fail[k] && result == FO_OK) result = FO_NOT_CONVERGED;
    }
    for (int k = 0; k < n; ++k)
        if (status[k] == FO_ERR_BREAKDOWN) result = FO_ERR_BREAKDOWN;
    if (st) {
        st->status = result;
        st->iters_inner += it_total + (int32_t)extra;
        st->iters_outer = std::max(st->iters_outer, max_outer_seen);
        st->rel_res = std::max(st->rel_res, worst);
    }
    return result;
}

int batch_solve(fo_ctx *c, const double *b, double *u, int n_rhs, int64_t ld, const fo_solve_opts *o,
                fo_solve_stats *st)
{
    const int G = c->batch.S;
    int worst = FO_OK;
    for (int c0 = 0; c0 < n_rhs; c0 += G) {
        const int n = std::min(G, n_rhs - c0);
        int rc = c->batch.method == FO_BATCH_COLUMN_CG ? batch_group(c, b + c0, u + c0, n, ld, o, st)
                                                       : bcg_group(c, b + c0, u + c0, n, ld, o, st);
        if (rc < 0 && rc != FO_ERR_BREAKDOWN) return rc;
        if (rc != FO_OK && (worst == FO_OK || rc < worst)) worst = rc;
    }
    return worst;
}

}  // namespace fo

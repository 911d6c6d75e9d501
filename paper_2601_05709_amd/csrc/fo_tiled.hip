// Deterministic element-to-node scatter through LDS tiles (see fo_tiles.h),
// the fused CG operator kernel, and the node-parallel boundary-facet term of
// the descent operator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#include "fo_element.h"
#include "fo_internal.h"
#include "fo_launch.h"
#include "fo_ops.h"
#include "fo_reduce.h"
#include "fo_tiles.h"
#include "fo_xcd.h"

namespace fo {

struct TileArgs {
    const int32_t *info;            // [n_tiles][8]
    const uint64_t *lconn, *lslot;  // [n_tiles][ME], 4 x uint16 each
    const int32_t *nodes;           // [n_tiles][MN]
    const uint16_t *seg;            // [n_tiles][MN+1]
    const int32_t *hpos;            // [n_tiles][MN]
    const float *tx32;              // [n_tiles][MN][D] node offsets from the tile's first node
    int ME, MN, n_tiles;
};

static TileArgs tile_args(const fo_ctx *c)
{
    const TileSet &t = c->tiles;
    return TileArgs{t.info, reinterpret_cast<const uint64_t *>(t.lconn),
                    reinterpret_cast<const uint64_t *>(t.lslot), t.nodes, t.seg, t.hpos, t.tx32,
                    t.max_elems, t.max_nodes, t.n_tiles};
}


// Nodal values an operator stages per tile besides the coordinates and its
// input (Op::NA values per node from op.aux; none unless the Op says so).
template <class Op, class = void>
struct OpAux {
    static constexpr int NA = 0;
};
template <class Op>
struct OpAux<Op, std::void_t<decltype(Op::NA)>> {
    static constexpr int NA = Op::NA;
};

// Element phase shared by the tile kernels: thread = element of the tile;
// writes its (d+1) x NV vertex values into the node-sorted LDS slots.
template <int D, typename T, class Op>
__device__ __forceinline__ void tile_elements(const Op &op, typename Op::Elem ed, uint64_t lc,
                                              uint64_t ls, const T *sX, const T *sU, const T *sA, T *sS)
{
    constexpr int NX = Op::NX, NV = Op::NV, NA = OpAux<Op>::NA;
    const T *Xp[D + 1];
    const T *Up[D + 1];
    const T *Ap[D + 1];
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        int l = (int)((lc >> (16 * a)) & 0xFFFF);
        Xp[a] = sX + l * D;
        Up[a] = sU + l * NX;
        Ap[a] = sA + l * NA;
    }
    T res[D + 1][NV];
    if constexpr (NA > 0)
        op(ed, Xp, Up, Ap, res);
    else
        op(ed, Xp, Up, res);
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        int sl = (int)((ls >> (16 * a)) & 0xFFFF);
#pragma unroll
        for (int v = 0; v < NV; ++v) sS[sl * NV + v] = res[a][v];
    }
}

// Generic scatter: out = sum over elements of op(element) at its vertices.
// One block per tile, one thread per element (blockDim >= elements and nodes
// of every tile).  LDS: node coordinates [nn][D], staged inputs [nn][NX],
// slots [ne*(d+1)][NV].  Interior nodes are written to `out` (zero on clamped
// unknowns when `fixed` is given); shared nodes to their halo slot.
// Optional dot_part[tile] = sum over the tile's nodes of xin . (the tile's
// share of the output), so the partials add up to xin . out (NX == NV).
// `done` (nullable) turns the launch into a no-op.
template <int D, typename T, class Op>
__global__ __launch_bounds__(1024) void k_tile_apply(Op op, TileArgs ta,
                                                     const T *__restrict__ coords,
                                                     const T *__restrict__ xin,
                                                     T *__restrict__ out, T *__restrict__ halo,
                                                     const uint8_t *__restrict__ fixed,
                                                     double *__restrict__ dot_part,
                                                     const int32_t *__restrict__ done)
{
    constexpr int NX = Op::NX, NV = Op::NV, NA = OpAux<Op>::NA;
    using Elem = typename Op::Elem;
    if (done && *done) return;
    const int t = xcd_tile(blockIdx.x, ta.n_tiles);
    if (t < 0) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *smem = reinterpret_cast<T *>(smem_raw);
    const int tid = threadIdx.x;
    const int32_t *inf = ta.info + (int64_t)t * kTileInfo;
    const int e0 = inf[kTileE0], ne = inf[kTileNE], nn = inf[kTileNN], nint = inf[kTileNInt];
    T *sX = smem;
    T *sU = sX + nn * D;
    T *sA = sU + nn * NX;
    T *sS = sA + nn * NA;

    uint64_t lc = 0, ls = 0;
    Elem ed{};
    if (tid < ne) {
        lc = ta.lconn[(int64_t)t * ta.ME + tid];
        ls = ta.lslot[(int64_t)t * ta.ME + tid];
        ed = op.load(e0 + tid);
    }
    int64_t g = 0;
    int sa = 0, sb = 0, hp = -1;
    if (tid < nn) {
        const int64_t tn = (int64_t)t * ta.MN + tid;
        g = ta.nodes[tn];
        hp = ta.hpos[tn];
        sa = ta.seg[(int64_t)t * (ta.MN + 1) + tid];
        sb = ta.seg[(int64_t)t * (ta.MN + 1) + tid + 1];
        T xv[D], uv[NX > 0 ? NX : 1];
        // FP32 geometry from tile-local offsets (formed in FP64 on the host):
        // edge vectors then keep FP32 accuracy relative to the element size
#pragma unroll
        for (int q = 0; q < D; ++q)
            if constexpr (sizeof(T) == 4) xv[q] = ta.tx32[tn * D + q];
            else xv[q] = coords[g * D + q];
#pragma unroll
        for (int k = 0; k < NX; ++k) uv[k] = xin[g * NX + k];
#pragma unroll
        for (int q = 0; q < D; ++q) sX[tid * D + q] = xv[q];
#pragma unroll
        for (int k = 0; k < NX; ++k) sU[tid * NX + k] = uv[k];
        if constexpr (NA > 0) {
            T av[NA];
#pragma unroll
            for (int k = 0; k < NA; ++k) av[k] = op.aux[g * NA + k];
#pragma unroll
            for (int k = 0; k < NA; ++k) sA[tid * NA + k] = av[k];
        }
    }
    __syncthreads();
    if (tid < ne) tile_elements<D, T, Op>(op, ed, lc, ls, sX, sU, sA, sS);
    __syncthreads();
    double dsum = 0.0;
    if (tid < nn) {
        T acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = T(0);
        for (int k = sa; k < sb; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += sS[k * NV + v];
        if (tid < nint) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T val = acc[v];
                if (fixed && fixed[g * NV + v]) val = T(0);
                out[g * NV + v] = val;
                if constexpr (NX == NV) dsum += (double)sU[tid * NX + v] * (double)val;
            }
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                halo[(int64_t)hp * NV + v] = acc[v];
                if constexpr (NX == NV) {
                    bool fx = fixed && fixed[g * NV + v];
                    dsum += fx ? 0.0 : (double)sU[tid * NX + v] * (double)acc[v];
                }
            }
        }
    }
    if (dot_part) {
        __shared__ double lds[16];
        double s = block_sum_any(dsum, lds);
        if (tid == 0) dot_part[t] = s;
    }
}

// Boundary-facet term of the descent operator in tile form (fptr null: none).
template <typename T>
struct FacetArgs {
    const int32_t *fptr;    // [n_tiles][MN+1] incidence ranges per tile node
    const uint64_t *fconn;  // [n_fent] local ids of the facet's vertices
    const T *fa;            // [n_fent][4] a = sqrt(|F| / (d (d+1))) n
    T gamma_n;
};

// LDS layout of the fused CG operator kernel (k_tile_cg):
//   node records [nn][8]: position (D values) in the first 16-byte half,
//     the direction p in the second; the global node id and the packed
//     halo slot / clamp bits sit in the two halves' last entries;
//   element-vertex slots [ne * (D+1)][SS]: one padded D-vector each.
// Whole-record vector reads and writes replace one LDS access per value.
template <int D, typename T>
struct CgLds {
    static constexpr int RS = 8;             // T per node record
    static constexpr int PO = 4;             // offset of p in the record
    static constexpr int SS = D == 3 ? 4 : 2;  // T per slot
    static size_t bytes(int nn, int ne) { return ((size_t)nn * RS + (size_t)ne * (D + 1) * SS) * sizeof(T); }
};

template <typename T>
__device__ __forceinline__ T int_bits(int32_t v)
{
    if constexpr (sizeof(T) == 4) return __int_as_float(v);
    else return __longlong_as_double((long long)v);
}

template <typename T>
__device__ __forceinline__ int32_t bits_int(T v)
{
    if constexpr (sizeof(T) == 4) return __float_as_int(v);
    else return (int32_t)__double_as_longlong(v);
}

// N contiguous values of T at a 16-byte (N * sizeof(T) >= 16) or 8-byte
// aligned LDS address, moved as 16- or 8-byte vectors.
template <typename T, int N>
__device__ __forceinline__ void lds_get(const T *p, T (&out)[N])
{
    constexpr int B = N * (int)sizeof(T);
    static_assert(B % 8 == 0, "vector size");
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int i = 0; i < B / 16; ++i) {
            const float4 v = reinterpret_cast<const float4 *>(p)[i];
            __builtin_memcpy(reinterpret_cast<char *>(out) + 16 * i, &v, 16);
        }
    } else {
#pragma unroll
        for (int i = 0; i < B / 8; ++i) {
            const float2 v = reinterpret_cast<const float2 *>(p)[i];
            __builtin_memcpy(reinterpret_cast<char *>(out) + 8 * i, &v, 8);
        }
    }
}

template <typename T, int N>
__device__ __forceinline__ void lds_put(T *p, const T (&in)[N])
{
    constexpr int B = N * (int)sizeof(T);
    static_assert(B % 8 == 0, "vector size");
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int i = 0; i < B / 16; ++i) {
            float4 v;
            __builtin_memcpy(&v, reinterpret_cast<const char *>(in) + 16 * i, 16);
            reinterpret_cast<float4 *>(p)[i] = v;
        }
    } else {
#pragma unroll
        for (int i = 0; i < B / 8; ++i) {
            float2 v;
            __builtin_memcpy(&v, reinterpret_cast<const char *>(in) + 8 * i, 8);
            reinterpret_cast<float2 *>(p)[i] = v;
        }
    }
}

// Operator kernel of one fused CG iteration (tiled; elasticity, or the
// descent operator with its boundary-facet term added at the nodes):
//   rho_k = r.D^-1 r and rr_k = r.r from the partials of the previous update
//   (summed by wave 0 while the other waves load their nodes); convergence
//   test; beta = rho_k / rho_{k-1} (or the slot's first-iteration
//   coefficient); p_k = D^-1 r + beta p_{k-1} at node staging (the owner tile
//   writes p_k); q = K p_k with interior nodes in q (zero on unknowns with
//   dinv = 0: clamped, or in no element) and shared nodes in the halo;
//   pq_part[tile] = p_k . (the tile's share of q) over the unknowns with
//   dinv != 0.
// Node phase: L = 4, 2 or 1 lanes per node (as many as the block holds)
// each add every L-th slot of the node's segment, then the L partial sums
// are combined by a butterfly (every lane of the group gets the same value).
// Reads scalar slot A, writes slot A ^ 1 (block 0).
template <int D, typename T, class Op>
__global__ __launch_bounds__(1024) void k_tile_cg(Op op, TileArgs ta, FacetArgs<T> fa,
                                                  const T *__restrict__ coords,
                                                  const T *__restrict__ r,
                                                  const T *__restrict__ dinv,
                                                  const T *__restrict__ pin, T *__restrict__ pout,
                                                  T *__restrict__ q, T *__restrict__ halo,
                                                  SolveScalars *sc, int A,
                                                  const double *__restrict__ rz_part, int rz_nb,
                                                  double *__restrict__ pq_part)
{
    using L_ = CgLds<D, T>;
    constexpr int RS = L_::RS, PO = L_::PO, SS = L_::SS;
    __shared__ double lds[16];
    __shared__ double s_beta;
    __shared__ int s_go;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int t = xcd_tile(blockIdx.x, ta.n_tiles);
    const int tid = threadIdx.x;
    if (t < 0) return;
    // wave 0 issues the loads of the r.z / r.r partials first: they depend on
    // nothing, and their latency then overlaps the index and node loads
    PartLoad<4> prz, prr;
    SolveScalars cur;
    if (tid < 64) {
        part_issue(prz, rz_part, rz_nb, tid, 64);
        part_issue(prr, rz_part + rz_nb, rz_nb, tid, 64);
        cur = sc[A];
    }
    // Index loads at fixed strides: they do not wait for the tile's counts
    // (every thread below ME / MN reads inside the tile's arrays; padding
    // entries are never used).  Lanes per node from the node stride MN.
    const int32_t *inf = ta.info + (int64_t)t * kTileInfo;
    const int nt = blockDim.x;
    const int lg = ta.MN * 4 <= nt ? 2 : (ta.MN * 2 <= nt ? 1 : 0);  // log2 of lanes per node
    const int m = tid >> lg, sub = tid & ((1 << lg) - 1);
    uint64_t lc = 0, ls = 0;
    if (tid < ta.ME) {
        lc = ta.lconn[(int64_t)t * ta.ME + tid];
        ls = ta.lslot[(int64_t)t * ta.ME + tid];
    }
    int sa = 0, sb = 0, fk0 = 0, fk1 = 0;
    if (m < ta.MN) {
        sa = ta.seg[(int64_t)t * (ta.MN + 1) + m];
        sb = ta.seg[(int64_t)t * (ta.MN + 1) + m + 1];
        if (fa.fptr) {
            fk0 = fa.fptr[(int64_t)t * (ta.MN + 1) + m];
            fk1 = fa.fptr[(int64_t)t * (ta.MN + 1) + m + 1];
        }
    }
    int32_t g = 0, hp = -1;
    T xv[D];
    if (tid < ta.MN) {
        const int64_t tn = (int64_t)t * ta.MN + tid;
        g = ta.nodes[tn];
        hp = ta.hpos[tn];
#pragma unroll
        for (int v = 0; v < D; ++v) {
            // FP32 geometry from tile-local offsets (formed in FP64 on the host)
            if constexpr (sizeof(T) == 4) xv[v] = ta.tx32[tn * D + v];
        }
    }
    const int e0 = inf[kTileE0], ne = inf[kTileNE], nn = inf[kTileNN], nint = inf[kTileNInt],
              nown = inf[kTileNOwn];
    if (m >= nn) sa = sb = fk0 = fk1 = 0;
    typename Op::Elem ed{};
    if (tid < ne) ed = op.load(e0 + tid);
    unsigned clamp = 0;  // bit v: dinv = 0 (clamped unknown, or no element): q = 0 there
    T zv[D], po[D];
    if (tid < nn) {
#pragma unroll
        for (int v = 0; v < D; ++v) {
            if constexpr (sizeof(T) == 8) xv[v] = coords[(int64_t)g * D + v];
            const T di = dinv[(int64_t)g * D + v];
            zv[v] = di * r[(int64_t)g * D + v];
            po[v] = pin[(int64_t)g * D + v];
            clamp |= (di == T(0) ? 1u : 0u) << v;
        }
    }
    if (tid < 64) {
        const double rho_k = wave_sum(part_finish(prz, rz_part, rz_nb, tid, 64));
        const double rr_k = wave_sum(part_finish(prr, rz_part + rz_nb, rz_nb, tid, 64));
        if (tid == 0) {
            if (cur.done) {  // converged or failed earlier: the launch is a no-op
                s_go = 0;
                if (t == 0) sc[A ^ 1] = cur;
            } else {
                const bool bad = !(rho_k >= 0.0) || rho_k != rho_k || rr_k != rr_k ||
                                 rho_k == INFINITY || rr_k == INFINITY;
                const bool stop = bad || rr_k <= cur.tol2 || cur.it >= cur.max_it;
                s_go = !stop;
                s_beta = cur.first ? cur.beta : (cur.rho > 0.0 ? rho_k / cur.rho : 0.0);
                if (t == 0) {
                    SolveScalars nx = cur;
                    nx.rr = rr_k;
                    nx.rho_new = rho_k;
                    if (stop) {
                        nx.done = 1;
                        nx.status = bad ? FO_ERR_BREAKDOWN : 0;
                    } else {
                        nx.rho = rho_k;
                        nx.beta = s_beta;
                        nx.first = 0;
                        nx.it = cur.it + 1;
                    }
                    sc[A ^ 1] = nx;
                }
            }
        }
    }
    __syncthreads();
    if (!s_go) return;
    const T beta = (T)s_beta;
    const bool fresh = beta == T(0);
    T *sN = reinterpret_cast<T *>(smem_raw);
    T *sS = sN + (size_t)nn * RS;
    if (tid < nn) {
        T rec[RS];
#pragma unroll
        for (int k = 0; k < RS; ++k) rec[k] = T(0);
#pragma unroll
        for (int v = 0; v < D; ++v) {
            rec[v] = xv[v];
            rec[PO + v] = fresh ? zv[v] : zv[v] + beta * po[v];
        }
        rec[PO - 1] = int_bits<T>(g);
        rec[RS - 1] = int_bits<T>((int32_t)(((uint32_t)(hp + 1) << 3) | clamp));
        lds_put(sN + (size_t)tid * RS, rec);
        if (tid < nown)
#pragma unroll
            for (int v = 0; v < D; ++v) pout[(int64_t)g * D + v] = rec[PO + v];
    }
    __syncthreads();
    if (tid < ne) {
        T X[D + 1][PO], U[D + 1][PO];
        const T *Xp[D + 1];
        const T *Up[D + 1];
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            const int l = (int)((lc >> (16 * a)) & 0xFFFF);
            T rec[RS];
            lds_get(sN + (size_t)l * RS, rec);
#pragma unroll
            for (int k = 0; k < PO; ++k) {
                X[a][k] = rec[k];
                U[a][k] = rec[PO + k];
            }
            Xp[a] = X[a];
            Up[a] = U[a];
        }
        T res[D + 1][D];
        op(ed, Xp, Up, res);
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            const int sl = (int)((ls >> (16 * a)) & 0xFFFF);
            T o[SS];
#pragma unroll
            for (int k = 0; k < SS; ++k) o[k] = k < D ? res[a][k] : T(0);
            lds_put(sS + (size_t)sl * SS, o);
        }
    }
    __syncthreads();
    T acc[D];
#pragma unroll
    for (int v = 0; v < D; ++v) acc[v] = T(0);
    for (int k = sa + sub; k < sb; k += 1 << lg) {
        T sv[SS];
        lds_get(sS + (size_t)k * SS, sv);
#pragma unroll
        for (int v = 0; v < D; ++v) acc[v] += sv[v];
    }
    if (lg >= 1)
#pragma unroll
        for (int v = 0; v < D; ++v) acc[v] += quad_xor<1>(acc[v]);
    if (lg >= 2)
#pragma unroll
        for (int v = 0; v < D; ++v) acc[v] += quad_xor<2>(acc[v]);
    double dsum = 0.0;
    if (m < nn && sub == 0) {
        T rec[RS];
        lds_get(sN + (size_t)m * RS, rec);
        const int64_t gm = bits_int<T>(rec[PO - 1]);
        const uint32_t hc = (uint32_t)bits_int<T>(rec[RS - 1]);
        const unsigned cm = hc & 7u;
        // boundary facets of this tile at node m (descent operator):
        // gamma_n a (a . (p_m + sum over the facet's vertices p_b))
        for (int k = fk0; k < fk1; ++k) {
            const uint64_t fc = fa.fconn[k];
            T av[D], sn = T(0), self = T(0);
#pragma unroll
            for (int v = 0; v < D; ++v) av[v] = fa.fa[(int64_t)k * 4 + v];
#pragma unroll
            for (int b = 0; b < D; ++b) {
                const T *pb = sN + (size_t)((fc >> (16 * b)) & 0xFFFF) * RS + PO;
#pragma unroll
                for (int v = 0; v < D; ++v) sn += av[v] * pb[v];
            }
#pragma unroll
            for (int v = 0; v < D; ++v) self += av[v] * rec[PO + v];
            const T c = fa.gamma_n * (self + sn);
#pragma unroll
            for (int v = 0; v < D; ++v) acc[v] += c * av[v];
        }
        if (m < nint) {
#pragma unroll
            for (int v = 0; v < D; ++v) {
                const T val = (cm >> v) & 1u ? T(0) : acc[v];
                q[gm * D + v] = val;
                dsum += (double)rec[PO + v] * (double)val;
            }
        } else {
            const int64_t hm = (int64_t)(hc >> 3) - 1;
#pragma unroll
            for (int v = 0; v < D; ++v) {
                halo[hm * D + v] = acc[v];
                dsum += (cm >> v) & 1u ? 0.0 : (double)rec[PO + v] * (double)acc[v];
            }
        }
    }
    const double s = block_sum_last(dsum, lds);
    if (tid == 0) pq_part[t] = s;
}

// Shared nodes: sum the node's halo slots (contiguous, in tile order).
template <typename T, int NV>
__global__ void k_halo(const int32_t *__restrict__ hnode, const int32_t *__restrict__ hptr,
                       int64_t S, const T *__restrict__ halo, T *__restrict__ out,
                       const uint8_t *__restrict__ fixed, const int32_t *__restrict__ done)
{
    if (done && *done) return;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < S;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t g = hnode[k];
        int j0 = hptr[k], j1 = hptr[k + 1];
        T acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = T(0);
        for (int j = j0; j < j1; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += halo[(int64_t)j * NV + v];
#pragma unroll
        for (int v = 0; v < NV; ++v) out[g * NV + v] = (fixed && fixed[g * NV + v]) ? T(0) : acc[v];
    }
}

// ---------------------------------------------------------------------------
// launch configuration

template <int D, typename T, int NX, int NV>
static size_t tile_lds_bytes(int max_nodes, int max_elems)
{
    return ((size_t)max_nodes * (D + NX) + (size_t)max_elems * (D + 1) * NV) * sizeof(T);
}

static int tile_threads(const fo_ctx *c)
{
    int m = std::max(c->tiles.max_elems, c->tiles.max_nodes);
    return std::min(1024, (m + 63) / 64 * 64);
}

static int set_lds(const void *fn, size_t cap)
{
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap) !=
           hipSuccess;
}

// Allows the dynamic LDS of the largest possible tile, once per kernel
// instance (must happen outside graph capture: see tiled_prepare).
template <int D, typename T, class Op>
static int ensure_lds_attr()
{
    static std::atomic<bool> done{false};
    if (done.load(std::memory_order_acquire)) return 0;
    size_t cap = tile_lds_bytes<D, T, Op::NX + OpAux<Op>::NA, Op::NV>(tile_max_nodes(D), tile_max_elems(D));
    if (set_lds((const void *)k_tile_apply<D, T, Op>, cap)) return 1;
    done.store(true, std::memory_order_release);
    return 0;
}

template <int D, typename T, class Op>
static int ensure_lds_attr_cg()
{
    static std::atomic<bool> done{false};
    if (done.load(std::memory_order_acquire)) return 0;
    size_t cap = CgLds<D, T>::bytes(tile_max_nodes(D), tile_max_elems(D));
    if (set_lds((const void *)k_tile_cg<D, T, Op>, cap)) return 1;
    done.store(true, std::memory_order_release);
    return 0;
}

template <int D>
static int prepare_dim()
{
    return ensure_lds_attr<D, double, ElasOp<D, double>>() | ensure_lds_attr<D, float, ElasOp<D, float>>() |
           ensure_lds_attr<D, double, ElasDiagOp<D, double>>() | ensure_lds_attr<D, double, DescentOp<D>>() |
           ensure_lds_attr<D, double, DescentDiagOp<D>>() | ensure_lds_attr<D, double, SdRhsOp<D>>() |
           ensure_lds_attr<D, double, PhiGradOp<D>>() | ensure_lds_attr_cg<D, double, ElasOp<D, double>>() |
           ensure_lds_attr_cg<D, float, ElasOp<D, float>>() |
           ensure_lds_attr_cg<D, double, DescentOp<D, double>>() |
           ensure_lds_attr_cg<D, float, DescentOp<D, float>>() | ensure_lds_attr<D, double, TransportOp<D>>() |
           ensure_lds_attr<D, double, TransportDiagOp<D>>() | ensure_lds_attr<D, double, ReinitOp<D>>() |
           ensure_lds_attr<D, double, ReinitDiagOp<D>>() | ensure_lds_attr<D, double, ReinitRhsOp<D>>() |
           ensure_lds_attr<D, double, HeatOp<D>>() | ensure_lds_attr<D, double, HeatDiagOp<D>>() |
           ensure_lds_attr<D, double, MassOp<D>>() | ensure_lds_attr<D, double, HeatSdOp<D>>() |
           ensure_lds_attr<D, double, VecMassOp<D>>() | ensure_lds_attr<D, double, InvSdOp<D>>();
}

int tiled_prepare(const fo_ctx *c)
{
    if (c->tiles.max_nodes > tile_max_nodes(c->dim) || c->tiles.max_elems > tile_max_elems(c->dim))
        return FO_ERR_MESH;
    return (c->dim == 2 ? prepare_dim<2>() : prepare_dim<3>()) ? FO_ERR_HIP : FO_OK;
}

// Event pair for one timed launch (fo_profile_enable), or null when off.
static std::pair<hipEvent_t, hipEvent_t> *prof_slot(const fo_ctx *cc, int which)
{
    fo_ctx *c = const_cast<fo_ctx *>(cc);
    if (!c->prof || which < 0) return nullptr;
    auto &v = c->prof_events[which];
    size_t &used = c->prof_used[which];
    if (used == v.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return nullptr;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return nullptr;
        }
        v.emplace_back(a, b);
    }
    return &v[used++];
}

template <int D, typename T, class Op>
static int run_tiled(const fo_ctx *c, const Op &op, const T *coords, const T *xin, T *out,
                     const uint8_t *fixed, hipStream_t s, int prof_tile = -1, int prof_halo = -1,
                     double *dot_part = nullptr, const int32_t *done = nullptr,
                     bool skip_halo = false)
{
    size_t lds = tile_lds_bytes<D, T, Op::NX + OpAux<Op>::NA, Op::NV>(c->tiles.max_nodes, c->tiles.max_elems);
    if (ensure_lds_attr<D, T, Op>()) return FO_ERR_HIP;
    auto *pt = prof_slot(c, prof_tile);
    if (pt) (void)hipEventRecord(pt->first, s);
    hipLaunchKernelGGL((k_tile_apply<D, T, Op>), dim3(xcd_grid(c->tiles.n_tiles)), dim3(tile_threads(c)), lds,
                       s, op, tile_args(c), coords, xin, out, reinterpret_cast<T *>(c->halo), fixed,
                       dot_part, done);
    if (pt) (void)hipEventRecord(pt->second, s);
    if (c->tiles.n_shared_nodes > 0 && !skip_halo) {
        int64_t S = c->tiles.n_shared_nodes;
        int nb = (int)std::min<int64_t>((S + 255) / 256, 65535);
        auto *ph = prof_slot(c, prof_halo);
        if (ph) (void)hipEventRecord(ph->first, s);
        hipLaunchKernelGGL((k_halo<T, Op::NV>), dim3(nb), dim3(256), 0, s, c->tiles.halo_node,
                           c->tiles.halo_ptr, S, reinterpret_cast<const T *>(c->halo), out, fixed,
                           done);
        if (ph) (void)hipEventRecord(ph->second, s);
    }
    return FO_OK;
}

template <int D, typename T, class Op>
static int launch_tile_cg_op(const fo_ctx *c, Op op, FacetArgs<T> fa, const T *r, const T *dinv,
                             const T *pin, T *pout, T *q, SolveScalars *sc, int A, hipStream_t s)
{
    if (ensure_lds_attr_cg<D, T, Op>()) return FO_ERR_HIP;
    const T *coords;
    if constexpr (sizeof(T) == 8) coords = c->coords;
    else coords = c->coords32;
    size_t lds = CgLds<D, T>::bytes(c->tiles.max_nodes, c->tiles.max_elems);
    // with folded partials every tile reads two values (see launch_tile_cg)
    const double *rz = c->fold_rz ? c->fold : c->rz_part;
    const int nrz = c->fold_rz ? 1 : upd_blocks(c->N);
    hipLaunchKernelGGL((k_tile_cg<D, T, Op>), dim3(xcd_grid(c->tiles.n_tiles)), dim3(tile_threads(c)), lds,
                       s, op, tile_args(c), fa, coords, r, dinv, pin, pout, q,
                       reinterpret_cast<T *>(c->halo), sc, A, rz, nrz, c->pq_part);
    return FO_OK;
}

template <int D, typename T>
static int launch_tile_cg_dim(const fo_ctx *c, int kind, const T *r, const T *dinv, const T *pin,
                              T *pout, T *q, SolveScalars *sc, int A, hipStream_t s)
{
    if (kind == FUSED_ELAS)
        return launch_tile_cg_op<D, T>(c, ElasOp<D, T>{c->chi, (T)c->ersatz, (T)c->lam, (T)c->mu},
                                       FacetArgs<T>{nullptr, nullptr, nullptr, T(0)}, r, dinv, pin, pout,
                                       q, sc, A, s);
    const DescentSetup &d = c->descent;
    const TileSet &ts = c->tiles;
    FacetArgs<T> fa{nullptr, nullptr, nullptr, T(0)};
    if (ts.n_fent > 0 && d.gamma_n != 0.0) {
        const T *a;
        if constexpr (sizeof(T) == 8) a = ts.fa64;
        else a = ts.fa32;
        fa = FacetArgs<T>{ts.fptr, ts.fconn, a, (T)d.gamma_n};
    }
    return launch_tile_cg_op<D, T>(c, DescentOp<D, T>{d.in0, (T)d.alpha, (T)d.gamma_s}, fa, r, dinv,
                                   pin, pout, q, sc, A, s);
}

template <typename T>
int launch_tile_cg(const fo_ctx *c, int kind, const T *r, const T *dinv, const T *pin, T *pout, T *q,
                   SolveScalars *sc, int A, hipStream_t s, bool fold)
{
    // large meshes: one block folds the update's r.z / r.r partials first
    if (c->fold_rz && fold) launch_fold(c->rz_part, upd_blocks(c->N), 2, c->fold, s);
    int which = -1;
    if (kind == FUSED_ELAS) which = sizeof(T) == 8 ? FO_PROF_ELAS_TILE_FP64 : FO_PROF_ELAS_TILE_FP32;
    auto *pt = which >= 0 ? prof_slot(c, which) : nullptr;
    if (pt) (void)hipEventRecord(pt->first, s);
    const int rc = c->dim == 2 ? launch_tile_cg_dim<2, T>(c, kind, r, dinv, pin, pout, q, sc, A, s)
                               : launch_tile_cg_dim<3, T>(c, kind, r, dinv, pin, pout, q, sc, A, s);
    if (pt) (void)hipEventRecord(pt->second, s);
    return rc;
}
template int launch_tile_cg<double>(const fo_ctx *, int, const double *, const double *, const double *,
                                    double *, double *, SolveScalars *, int, hipStream_t, bool);
template int launch_tile_cg<float>(const fo_ctx *, int, const float *, const float *, const float *,
                                   float *, float *, SolveScalars *, int, hipStream_t, bool);

// ---------------------------------------------------------------------------
// boundary facets of the descent operator, node-parallel (deterministic)

template <int D>
__device__ __forceinline__ double facet_measure(const double *const *P)
{
    if constexpr (D == 2) {
        double dx = P[1][0] - P[0][0], dy = P[1][1] - P[0][1];
        return sqrt(dx * dx + dy * dy);
    } else {
        double u[3], v[3];
        for (int i = 0; i < 3; ++i) {
            u[i] = P[1][i] - P[0][i];
            v[i] = P[2][i] - P[0][i];
        }
        double c0 = u[1] * v[2] - u[2] * v[1], c1 = u[2] * v[0] - u[0] * v[2],
               c2 = u[0] * v[1] - u[1] * v[0];
        return 0.5 * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    }
}

// For each boundary node g and each facet f containing it (fixed order):
//   y_g += gamma_n |F| / (d(d+1)) n (n . (x_g + sum_b x_b))     (apply), or
//   y_g += 2 gamma_n |F| / (d(d+1)) n_i^2                       (diagonal).
template <int D>
__global__ void k_facet_nodes(const int32_t *__restrict__ bnode, const int32_t *__restrict__ bptr,
                              const int32_t *__restrict__ bfac, int64_t NB,
                              const int32_t *__restrict__ bf, const double *__restrict__ bn,
                              int64_t F, const double *__restrict__ coords, double gamma_n,
                              const double *__restrict__ x, double *__restrict__ y,
                              const int32_t *__restrict__ done)
{
    if (done && *done) return;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < NB;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t g = bnode[k];
        double acc[D];
        for (int i = 0; i < D; ++i) acc[i] = 0.0;
        for (int j = bptr[k]; j < bptr[k + 1]; ++j) {
            int64_t f = bfac[j];
            const double *P[D];
            int32_t nd[D];
            for (int a = 0; a < D; ++a) {
                nd[a] = bf[(int64_t)a * F + f];
                P[a] = coords + (int64_t)nd[a] * D;
            }
            double c = gamma_n * facet_measure<D>(P) / (double)(D * (D + 1));
            const double *n = bn + f * D;
            if (x) {
                double sn = 0.0, self = 0.0;
                for (int a = 0; a < D; ++a) {
                    double t = 0.0;
                    for (int i = 0; i < D; ++i) t += n[i] * x[(int64_t)nd[a] * D + i];
                    sn += t;
                    if (nd[a] == g) self = t;
                }
                for (int i = 0; i < D; ++i) acc[i] += c * n[i] * (self + sn);
            } else {
                for (int i = 0; i < D; ++i) acc[i] += 2.0 * c * n[i] * n[i];
            }
        }
        for (int i = 0; i < D; ++i) y[g * D + i] += acc[i];
    }
}

static void facet_terms(const fo_ctx *c, const double *x, double *y, hipStream_t s,
                        const int32_t *done = nullptr)
{
    if (c->n_bnodes == 0 || c->descent.gamma_n == 0.0) return;
    int nb = (int)std::min<int64_t>((c->n_bnodes + 255) / 256, 65535);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_facet_nodes<2>, dim3(nb), dim3(256), 0, s, c->bnodes, c->bnode_ptr,
                           c->bnode_fac, c->n_bnodes, c->bfacets, c->bnormal, c->nbf, c->coords,
                           c->descent.gamma_n, x, y, done);
    else
        hipLaunchKernelGGL(k_facet_nodes<3>, dim3(nb), dim3(256), 0, s, c->bnodes, c->bnode_ptr,
                           c->bnode_fac, c->n_bnodes, c->bfacets, c->bnormal, c->nbf, c->coords,
                           c->descent.gamma_n, x, y, done);
}

void launch_facet_terms(const fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    facet_terms(c, x, y, s);
}

// P1 mass on the boundary facets, node-parallel over the boundary nodes in
// the same fixed facet order: y_g = sum_f |F| / (d(d+1)) (x_g + sum_b x_b)
// (y is written on the boundary nodes only).
template <int D>
__global__ void k_facet_mass(const int32_t *__restrict__ bnode, const int32_t *__restrict__ bptr,
                             const int32_t *__restrict__ bfac, int64_t NB, const int32_t *__restrict__ bf, int64_t F,
                             const double *__restrict__ coords, const double *__restrict__ x,
                             double *__restrict__ y)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < NB;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = bnode[k];
        double acc[D];
        for (int i = 0; i < D; ++i) acc[i] = 0.0;
        for (int j = bptr[k]; j < bptr[k + 1]; ++j) {
            const int64_t f = bfac[j];
            const double *P[D];
            int64_t nd[D];
            for (int a = 0; a < D; ++a) {
                nd[a] = bf[(int64_t)a * F + f];
                P[a] = coords + nd[a] * D;
            }
            const double cf = facet_measure<D>(P) / (double)(D * (D + 1));
            for (int i = 0; i < D; ++i) {
                double t = x[g * D + i];
                for (int a = 0; a < D; ++a) t += x[nd[a] * D + i];
                acc[i] += cf * t;
            }
        }
        for (int i = 0; i < D; ++i) y[g * D + i] = acc[i];
    }
}

void launch_facet_mass(const fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    launch_fill<double>(y, c->ndof, 0.0, s);
    if (c->n_bnodes == 0) return;
    const int nb = (int)std::min<int64_t>((c->n_bnodes + 255) / 256, 65535);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_facet_mass<2>, dim3(nb), dim3(256), 0, s, c->bnodes, c->bnode_ptr, c->bnode_fac,
                           c->n_bnodes, c->bfacets, c->nbf, c->coords, x, y);
    else
        hipLaunchKernelGGL(k_facet_mass<3>, dim3(nb), dim3(256), 0, s, c->bnodes, c->bnode_ptr, c->bnode_fac,
                           c->n_bnodes, c->bfacets, c->nbf, c->coords, x, y);
}

// ---------------------------------------------------------------------------
// tiled launchers

template <typename T>
int launch_elas_apply_tiled(const fo_ctx *c, const T *coords, const T *x, T *y, hipStream_t s,
                            double *dot_part, const int32_t *done, bool skip_halo)
{
    const bool f64 = sizeof(T) == 8;
    const int pt = f64 ? FO_PROF_ELAS_TILE_FP64 : FO_PROF_ELAS_TILE_FP32;
    const int ph = f64 ? FO_PROF_HALO_FP64 : FO_PROF_HALO_FP32;
    if (c->dim == 2)
        return run_tiled<2, T>(c, ElasOp<2, T>{c->chi, (T)c->ersatz, (T)c->lam, (T)c->mu}, coords,
                               x, y, c->fixed, s, pt, ph, dot_part, done, skip_halo);
    return run_tiled<3, T>(c, ElasOp<3, T>{c->chi, (T)c->ersatz, (T)c->lam, (T)c->mu}, coords, x,
                           y, c->fixed, s, pt, ph, dot_part, done, skip_halo);
}
template int launch_elas_apply_tiled<double>(const fo_ctx *, const double *, const double *,
                                             double *, hipStream_t, double *, const int32_t *, bool);
template int launch_elas_apply_tiled<float>(const fo_ctx *, const float *, const float *, float *,
                                            hipStream_t, double *, const int32_t *, bool);

int launch_elas_diag_tiled(const fo_ctx *c, double *diag, hipStream_t s)
{
    if (c->dim == 2)
        return run_tiled<2, double>(c, ElasDiagOp<2, double>{c->chi, c->ersatz, c->lam, c->mu},
                                    c->coords, (const double *)nullptr, diag, nullptr, s);
    return run_tiled<3, double>(c, ElasDiagOp<3, double>{c->chi, c->ersatz, c->lam, c->mu},
                                c->coords, (const double *)nullptr, diag, nullptr, s);
}

int launch_descent_apply_tiled(const fo_ctx *c, const double *x, double *y, hipStream_t s,
                               const int32_t *done)
{
    const DescentSetup &d = c->descent;
    int rc;
    if (c->dim == 2)
        rc = run_tiled<2, double>(c, DescentOp<2>{d.in0, d.alpha, d.gamma_s}, c->coords, x, y,
                                  nullptr, s, -1, -1, nullptr, done);
    else
        rc = run_tiled<3, double>(c, DescentOp<3>{d.in0, d.alpha, d.gamma_s}, c->coords, x, y,
                                  nullptr, s, -1, -1, nullptr, done);
    if (rc) return rc;
    facet_terms(c, x, y, s, done);
    return FO_OK;
}

int launch_descent_diag_tiled(const fo_ctx *c, double *diag, hipStream_t s)
{
    const DescentSetup &d = c->descent;
    int rc;
    if (c->dim == 2)
        rc = run_tiled<2, double>(c, DescentDiagOp<2>{d.in0, d.alpha, d.gamma_s}, c->coords,
                                  (const double *)nullptr, diag, nullptr, s);
    else
        rc = run_tiled<3, double>(c, DescentDiagOp<3>{d.in0, d.alpha, d.gamma_s}, c->coords,
                                  (const double *)nullptr, diag, nullptr, s);
    if (rc) return rc;
    facet_terms(c, nullptr, diag, s);
    return FO_OK;
}

int launch_transport_apply(const fo_ctx *c, const double *theta, const double *par, int which, const double *x,
                           double *y, hipStream_t s, const int32_t *done)
{
    if (c->has_isolated) launch_fill<double>(y, c->N, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, TransportOp<2>{theta, par, which}, c->coords, x, y, nullptr, s, -1, -1,
                                    nullptr, done);
    return run_tiled<3, double>(c, TransportOp<3>{theta, par, which}, c->coords, x, y, nullptr, s, -1, -1,
                                nullptr, done);
}

int launch_transport_diag(const fo_ctx *c, const double *theta, const double *par, double *diag, hipStream_t s)
{
    launch_fill<double>(diag, c->N, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, TransportDiagOp<2>{theta, par}, c->coords, (const double *)nullptr, diag,
                                    nullptr, s);
    return run_tiled<3, double>(c, TransportDiagOp<3>{theta, par}, c->coords, (const double *)nullptr, diag,
                                nullptr, s);
}

int launch_reinit_apply(const fo_ctx *c, const double *w, const double *par, const double *x, double *y,
                        hipStream_t s, const int32_t *done)
{
    if (c->has_isolated) launch_fill<double>(y, c->N, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, ReinitOp<2>{w, par}, c->coords, x, y, nullptr, s, -1, -1, nullptr, done);
    return run_tiled<3, double>(c, ReinitOp<3>{w, par}, c->coords, x, y, nullptr, s, -1, -1, nullptr, done);
}

int launch_reinit_diag(const fo_ctx *c, const double *w, const double *par, double *diag, hipStream_t s)
{
    launch_fill<double>(diag, c->N, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, ReinitDiagOp<2>{w, par}, c->coords, (const double *)nullptr, diag,
                                    nullptr, s);
    return run_tiled<3, double>(c, ReinitDiagOp<3>{w, par}, c->coords, (const double *)nullptr, diag, nullptr,
                                s);
}

int launch_reinit_rhs(const fo_ctx *c, const double *w, const double *par, double *rhs, hipStream_t s)
{
    launch_fill<double>(rhs, c->N, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, ReinitRhsOp<2>{w, par}, c->coords, (const double *)nullptr, rhs, nullptr,
                                    s);
    return run_tiled<3, double>(c, ReinitRhsOp<3>{w, par}, c->coords, (const double *)nullptr, rhs, nullptr, s);
}

int launch_heat_apply(const fo_ctx *c, const uint8_t *fixed, const double *x, double *y, hipStream_t s,
                      const int32_t *done)
{
    if (c->has_isolated) launch_fill<double>(y, c->N, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, HeatOp<2>{c->chi, c->ersatz}, c->coords, x, y, fixed, s, -1, -1, nullptr,
                                    done);
    return run_tiled<3, double>(c, HeatOp<3>{c->chi, c->ersatz}, c->coords, x, y, fixed, s, -1, -1, nullptr, done);
}

int launch_heat_diag(const fo_ctx *c, const uint8_t *fixed, double *diag, hipStream_t s)
{
    launch_fill<double>(diag, c->N, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, HeatDiagOp<2>{c->chi, c->ersatz}, c->coords, (const double *)nullptr, diag,
                                    fixed, s);
    return run_tiled<3, double>(c, HeatDiagOp<3>{c->chi, c->ersatz}, c->coords, (const double *)nullptr, diag,
                                fixed, s);
}

int launch_mass_apply(const fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    launch_fill<double>(y, c->N, 0.0, s);
    if (c->dim == 2) return run_tiled<2, double>(c, MassOp<2>{}, c->coords, x, y, nullptr, s);
    return run_tiled<3, double>(c, MassOp<3>{}, c->coords, x, y, nullptr, s);
}

int launch_heat_rhs(const fo_ctx *c, const double *u, const double *f, double lambda_vol, double V, double *rhs,
                    hipStream_t s)
{
    launch_fill<double>(rhs, c->ndof, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, HeatSdOp<2>{c->chi, f, c->ersatz, lambda_vol, V}, c->coords, u, rhs,
                                    nullptr, s);
    return run_tiled<3, double>(c, HeatSdOp<3>{c->chi, f, c->ersatz, lambda_vol, V}, c->coords, u, rhs, nullptr,
                                s);
}

int launch_elas_apply_free(const fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    if (c->has_isolated) launch_fill<double>(y, c->ndof, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, ElasOp<2, double>{c->chi, c->ersatz, c->lam, c->mu}, c->coords, x, y,
                                    nullptr, s);
    return run_tiled<3, double>(c, ElasOp<3, double>{c->chi, c->ersatz, c->lam, c->mu}, c->coords, x, y, nullptr,
                                s);
}

int launch_vec_mass(const fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    launch_fill<double>(y, c->ndof, 0.0, s);
    if (c->dim == 2) return run_tiled<2, double>(c, VecMassOp<2>{}, c->coords, x, y, nullptr, s);
    return run_tiled<3, double>(c, VecMassOp<3>{}, c->coords, x, y, nullptr, s);
}

int launch_inverse_rhs(const fo_ctx *c, const double *u, const double *aux, double kappa, double alpha,
                       double *rhs, hipStream_t s)
{
    launch_fill<double>(rhs, c->ndof, 0.0, s);
    if (c->dim == 2)
        return run_tiled<2, double>(c, InvSdOp<2>{c->chi, aux, kappa, alpha, c->lam, c->mu}, c->coords, u, rhs,
                                    nullptr, s);
    return run_tiled<3, double>(c, InvSdOp<3>{c->chi, aux, kappa, alpha, c->lam, c->mu}, c->coords, u, rhs,
                                nullptr, s);
}

int launch_sd_rhs_tiled(const fo_ctx *c, double *rhs, hipStream_t s)
{
    if (c->dim == 2)
        return run_tiled<2, double>(c, SdRhsOp<2>{c->s1buf}, c->coords, (const double *)nullptr,
                                    rhs, nullptr, s);
    return run_tiled<3, double>(c, SdRhsOp<3>{c->s1buf}, c->coords, (const double *)nullptr, rhs,
                                nullptr, s);
}

int launch_phigrad_tiled(const fo_ctx *c, const double *phi, double *gbuf, hipStream_t s)
{
    if (c->dim == 2)
        return run_tiled<2, double>(c, PhiGradOp<2>{}, c->coords, phi, gbuf, nullptr, s);
    return run_tiled<3, double>(c, PhiGradOp<3>{}, c->coords, phi, gbuf, nullptr, s);
}

// ---------------------------------------------------------------------------

template <typename T>
static int up_vec(fo_ctx *c, T **dst, const std::vector<T> &src)
{
    FO_TRY(ctx_alloc_n(c, dst, std::max<size_t>(src.size(), 1)));
    void *p = *dst;
    if (!c->measure && !src.empty() &&
        hipMemcpyAsync(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess)
        return FO_ERR_HIP;
    return FO_OK;
}

int upload_tiles(fo_ctx *c, const HostTiles &h)
{
    TileSet &t = c->tiles;
    t.n_tiles = h.n_tiles;
    t.max_nodes = h.max_nodes;
    t.max_elems = h.max_elems;
    t.n_slots = h.n_slots;
    t.n_shared_nodes = (int64_t)h.halo_node.size();
    t.n_shared_slots = h.halo_ptr.empty() ? 0 : (int64_t)h.halo_ptr.back();
    int rc;
    if ((rc = up_vec(c, &t.info, h.info)) || (rc = up_vec(c, &t.lconn, h.lconn)) ||
        (rc = up_vec(c, &t.lslot, h.lslot)) || (rc = up_vec(c, &t.nodes, h.nodes)) ||
        (rc = up_vec(c, &t.seg, h.seg)) || (rc = up_vec(c, &t.hpos, h.hpos)) ||
        (rc = up_vec(c, &t.halo_node, h.halo_node)) || (rc = up_vec(c, &t.halo_ptr, h.halo_ptr)) ||
        (rc = up_vec(c, &t.node_hrange, h.node_hrange)))
        return rc;
    // halo partials: widest op has d+1 values per node
    return ctx_alloc_n(c, &c->halo, std::max<size_t>((size_t)t.n_shared_slots * (c->dim + 1), 1));
}

}  // namespace fo

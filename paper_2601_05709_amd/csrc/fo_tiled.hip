// Deterministic element-to-node scatter through LDS tiles (see fo_tiles.h),
// and the node-parallel boundary-facet term of the descent operator.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fo_element.h"
#include "fo_internal.h"
#include "fo_launch.h"
#include "fo_ops.h"
#include "fo_reduce.h"
#include "fo_tiles.h"

namespace fo {

struct TileArgs {
    const int32_t *elem_off, *node_off, *node_int, *halo_off, *nodes, *sub_off, *seg_off;
    const uint64_t *lconn, *lslot;  // 4 x uint16 per element
    const uint16_t *seg_node, *seg_start;
};

static TileArgs tile_args(const fo_ctx *c)
{
    const TileSet &t = c->tiles;
    return TileArgs{t.tile_elem_off, t.tile_node_off, t.tile_node_interior, t.tile_halo_off,
                    t.tile_nodes,    t.sub_off,       t.seg_off,
                    reinterpret_cast<const uint64_t *>(t.lconn),
                    reinterpret_cast<const uint64_t *>(t.lslot), t.seg_node, t.seg_start};
}

// One block per tile.  LDS: node coordinates [nn][D], staged inputs [nn][NX],
// node accumulators [nn][NV], sub-batch slots [kSub*(D+1)][NV].
template <int D, typename T, class Op>
__global__ __launch_bounds__(kSub) void k_tile_scatter(Op op, TileArgs ta,
                                                       const T *__restrict__ coords,
                                                       const T *__restrict__ xin,
                                                       T *__restrict__ out, T *__restrict__ halo,
                                                       const uint8_t *__restrict__ fixed)
{
    constexpr int NX = Op::NX, NV = Op::NV;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *smem = reinterpret_cast<T *>(smem_raw);
    const int t = blockIdx.x;
    const int n0 = ta.node_off[t];
    const int nn = ta.node_off[t + 1] - n0;
    const int nint = ta.node_int[t];
    T *sX = smem;
    T *sU = sX + nn * D;
    T *sA = sU + nn * NX;
    T *sS = sA + nn * NV;
    for (int l = threadIdx.x; l < nn; l += kSub) {
        int64_t g = ta.nodes[n0 + l];
#pragma unroll
        for (int i = 0; i < D; ++i) sX[l * D + i] = coords[g * D + i];
#pragma unroll
        for (int k = 0; k < NX; ++k) sU[l * NX + k] = xin[g * NX + k];
#pragma unroll
        for (int v = 0; v < NV; ++v) sA[l * NV + v] = T(0);
    }
    __syncthreads();
    const int e0 = ta.elem_off[t], e1 = ta.elem_off[t + 1];
    const int s0 = ta.sub_off[t], s1 = ta.sub_off[t + 1];
    for (int sb = s0; sb < s1; ++sb) {
        int i = e0 + (sb - s0) * kSub + threadIdx.x;
        if (i < e1) {
            uint64_t lc = ta.lconn[i], ls = ta.lslot[i];
            const T *Xp[D + 1];
            const T *Up[D + 1];
            int32_t unused[D + 1];
#pragma unroll
            for (int a = 0; a <= D; ++a) {
                int l = (int)((lc >> (16 * a)) & 0xFFFF);
                Xp[a] = sX + l * D;
                Up[a] = sU + l * NX;
                unused[a] = l;
            }
            T res[D + 1][NV];
            op(i, unused, Xp, Up, res);
#pragma unroll
            for (int a = 0; a <= D; ++a) {
                int sl = (int)((ls >> (16 * a)) & 0xFFFF);
#pragma unroll
                for (int v = 0; v < NV; ++v) sS[sl * NV + v] = res[a][v];
            }
        }
        __syncthreads();
        const int g0 = ta.seg_off[sb], g1 = ta.seg_off[sb + 1] - 1;  // last entry = sentinel
        for (int s = g0 + threadIdx.x; s < g1; s += kSub) {
            int node = ta.seg_node[s];
            int a = ta.seg_start[s], b = ta.seg_start[s + 1];
            T acc[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = T(0);
            for (int k = a; k < b; ++k)
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] += sS[k * NV + v];
#pragma unroll
            for (int v = 0; v < NV; ++v) sA[node * NV + v] += acc[v];
        }
        __syncthreads();
    }
    const int hoff = ta.halo_off[t];
    for (int l = threadIdx.x; l < nn; l += kSub) {
        int64_t g = ta.nodes[n0 + l];
        if (l < nint) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T val = sA[l * NV + v];
                if (fixed && fixed[g * NV + v]) val = T(0);
                out[g * NV + v] = val;
            }
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) halo[(int64_t)(hoff + l - nint) * NV + v] = sA[l * NV + v];
        }
    }
}

// Shared nodes: sum the halo slots of each node in tile order.
template <typename T, int NV>
__global__ void k_halo(const int32_t *__restrict__ hnode, const int32_t *__restrict__ hptr,
                       const int32_t *__restrict__ hsrc, int64_t S, const T *__restrict__ halo,
                       T *__restrict__ out, const uint8_t *__restrict__ fixed)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < S;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t g = hnode[k];
        T acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = T(0);
        for (int j = hptr[k]; j < hptr[k + 1]; ++j) {
            int64_t src = hsrc[j];
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += halo[src * NV + v];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) out[g * NV + v] = (fixed && fixed[g * NV + v]) ? T(0) : acc[v];
    }
}

template <int D, typename T, class Op>
static size_t tile_lds_bytes(int max_nodes)
{
    return ((size_t)max_nodes * (D + Op::NX + Op::NV) + (size_t)kSub * (D + 1) * Op::NV) * sizeof(T);
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
                     const uint8_t *fixed, hipStream_t s, int prof_tile = -1, int prof_halo = -1)
{
    size_t lds = tile_lds_bytes<D, T, Op>(c->tiles.max_nodes);
    static bool attr_done = false;  // one per template instance: allow the largest tile
    if (!attr_done) {
        size_t cap = tile_lds_bytes<D, T, Op>(tile_max_nodes(D));
        if (hipFuncSetAttribute((const void *)k_tile_scatter<D, T, Op>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap) != hipSuccess)
            return FO_ERR_HIP;
        attr_done = true;
    }
    if (c->tiles.max_nodes > tile_max_nodes(D)) return FO_ERR_MESH;
    auto *pt = prof_slot(c, prof_tile);
    if (pt) (void)hipEventRecord(pt->first, s);
    hipLaunchKernelGGL((k_tile_scatter<D, T, Op>), dim3(c->tiles.n_tiles), dim3(kSub), lds, s, op,
                       tile_args(c), coords, xin, out, reinterpret_cast<T *>(c->halo), fixed);
    if (pt) (void)hipEventRecord(pt->second, s);
    if (c->tiles.n_shared_nodes > 0) {
        int64_t S = c->tiles.n_shared_nodes;
        int nb = (int)std::min<int64_t>((S + 255) / 256, 65535);
        auto *ph = prof_slot(c, prof_halo);
        if (ph) (void)hipEventRecord(ph->first, s);
        hipLaunchKernelGGL((k_halo<T, Op::NV>), dim3(nb), dim3(256), 0, s, c->tiles.halo_node,
                           c->tiles.halo_ptr, c->tiles.halo_src, S,
                           reinterpret_cast<const T *>(c->halo), out, fixed);
        if (ph) (void)hipEventRecord(ph->second, s);
    }
    return FO_OK;
}

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
                              const double *__restrict__ x, double *__restrict__ y)
{
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

static void facet_terms(const fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    if (c->n_bnodes == 0 || c->descent.gamma_n == 0.0) return;
    int nb = (int)std::min<int64_t>((c->n_bnodes + 255) / 256, 65535);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_facet_nodes<2>, dim3(nb), dim3(256), 0, s, c->bnodes, c->bnode_ptr,
                           c->bnode_fac, c->n_bnodes, c->bfacets, c->bnormal, c->nbf, c->coords,
                           c->descent.gamma_n, x, y);
    else
        hipLaunchKernelGGL(k_facet_nodes<3>, dim3(nb), dim3(256), 0, s, c->bnodes, c->bnode_ptr,
                           c->bnode_fac, c->n_bnodes, c->bfacets, c->bnormal, c->nbf, c->coords,
                           c->descent.gamma_n, x, y);
}

void launch_facet_terms(const fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    facet_terms(c, x, y, s);
}

// ---------------------------------------------------------------------------
// tiled launchers

template <typename T>
int launch_elas_apply_tiled(const fo_ctx *c, const T *coords, const T *x, T *y, hipStream_t s)
{
    const bool f64 = sizeof(T) == 8;
    const int pt = f64 ? FO_PROF_ELAS_TILE_FP64 : FO_PROF_ELAS_TILE_FP32;
    const int ph = f64 ? FO_PROF_HALO_FP64 : FO_PROF_HALO_FP32;
    if (c->dim == 2)
        return run_tiled<2, T>(c, ElasOp<2, T>{c->chi, (T)c->ersatz, (T)c->lam, (T)c->mu}, coords,
                               x, y, c->fixed, s, pt, ph);
    return run_tiled<3, T>(c, ElasOp<3, T>{c->chi, (T)c->ersatz, (T)c->lam, (T)c->mu}, coords, x,
                           y, c->fixed, s, pt, ph);
}
template int launch_elas_apply_tiled<double>(const fo_ctx *, const double *, const double *,
                                             double *, hipStream_t);
template int launch_elas_apply_tiled<float>(const fo_ctx *, const float *, const float *, float *,
                                            hipStream_t);

int launch_elas_diag_tiled(const fo_ctx *c, double *diag, hipStream_t s)
{
    if (c->dim == 2)
        return run_tiled<2, double>(c, ElasDiagOp<2, double>{c->chi, c->ersatz, c->lam, c->mu},
                                    c->coords, (const double *)nullptr, diag, nullptr, s);
    return run_tiled<3, double>(c, ElasDiagOp<3, double>{c->chi, c->ersatz, c->lam, c->mu},
                                c->coords, (const double *)nullptr, diag, nullptr, s);
}

int launch_descent_apply_tiled(const fo_ctx *c, const double *x, double *y, hipStream_t s)
{
    const DescentSetup &d = c->descent;
    int rc;
    if (c->dim == 2)
        rc = run_tiled<2, double>(c, DescentOp<2>{d.in0, d.alpha, d.gamma_s}, c->coords, x, y,
                                  nullptr, s);
    else
        rc = run_tiled<3, double>(c, DescentOp<3>{d.in0, d.alpha, d.gamma_s}, c->coords, x, y,
                                  nullptr, s);
    if (rc) return rc;
    facet_terms(c, x, y, s);
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
    size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return FO_ERR_NOMEM;
    c->allocations.push_back(p);
    c->bytes += bytes;
    *dst = static_cast<T *>(p);
    if (!src.empty() &&
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
    t.max_sub = h.max_sub;
    t.n_slots = (int64_t)h.tile_nodes.size();
    t.n_shared_nodes = (int64_t)h.halo_node.size();
    t.n_shared_slots = (int64_t)h.halo_src.size();
    int rc;
    if ((rc = up_vec(c, &t.tile_elem_off, h.tile_elem_off)) ||
        (rc = up_vec(c, &t.tile_node_off, h.tile_node_off)) ||
        (rc = up_vec(c, &t.tile_node_interior, h.tile_node_interior)) ||
        (rc = up_vec(c, &t.tile_halo_off, h.tile_halo_off)) ||
        (rc = up_vec(c, &t.tile_nodes, h.tile_nodes)) || (rc = up_vec(c, &t.lconn, h.lconn)) ||
        (rc = up_vec(c, &t.lslot, h.lslot)) || (rc = up_vec(c, &t.sub_off, h.sub_off)) ||
        (rc = up_vec(c, &t.seg_off, h.seg_off)) || (rc = up_vec(c, &t.seg_node, h.seg_node)) ||
        (rc = up_vec(c, &t.seg_start, h.seg_start)) || (rc = up_vec(c, &t.halo_node, h.halo_node)) ||
        (rc = up_vec(c, &t.halo_ptr, h.halo_ptr)) || (rc = up_vec(c, &t.halo_src, h.halo_src)))
        return rc;
    // halo partials: widest op has d+1 values per node
    std::vector<double> zero;
    size_t n = std::max<size_t>((size_t)t.n_shared_slots * (c->dim + 1), 1);
    void *p = nullptr;
    if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) return FO_ERR_NOMEM;
    c->allocations.push_back(p);
    c->bytes += n * sizeof(double);
    c->halo = static_cast<double *>(p);
    return FO_OK;
}

}  // namespace fo

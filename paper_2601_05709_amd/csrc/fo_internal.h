// Internal declarations shared by the host runtime and the kernels of libfo.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <map>
#include <tuple>
#include <vector>

#include "../../include/fo.h"
#include "fo_wait.h"

// Status plumbing of the host runtime: a failing HIP call is reported on
// stderr and turns into FO_ERR_HIP; FO_TRY forwards any non-OK status.
#define FO_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t _e = (call);                                                         \
        if (_e != hipSuccess) {                                                         \
            std::fprintf(stderr, "libfo: %s failed: %s\n", #call, hipGetErrorString(_e)); \
            return FO_ERR_HIP;                                                          \
        }                                                                               \
    } while (0)

#define FO_TRY(x)              \
    do {                       \
        int _rc = (x);         \
        if (_rc != FO_OK) {    \
            return _rc;        \
        }                      \
    } while (0)

namespace fo {

// Every device allocation of the library goes through device_malloc, which
// counts them (fo_device_allocations).
hipError_t device_malloc(void **p, size_t bytes);

// Device memory owned by a context: allocated (and recorded for fo_destroy)
// or, for a context on a caller's workspace, carved from it (256-byte
// aligned).  FO_ERR_NOMEM when it does not fit.
int ctx_alloc(fo_ctx *c, void **p, size_t bytes);

template <typename T>
int ctx_alloc_n(fo_ctx *c, T **p, size_t count)
{
    void *v = nullptr;
    const int rc = ctx_alloc(c, &v, count * sizeof(T));
    *p = static_cast<T *>(v);
    return rc;
}

// fo_optimize's loop on caller-provided work vectors of
// optimize_work_doubles(c) doubles (u, rhs, theta, three scalars).
size_t optimize_work_doubles(const fo_ctx *c);
int optimize_on(fo_ctx *c, const fo_loop_opts *o, const double *b, double *phi, fo_loop_record *records,
                int32_t *n_done, int32_t *stopped, double *work);

constexpr int kMaxBoxes = 64;      // boxes of Omega0 in the velocity options

// Relative residual reduction asked of an FP32 phase of the refinement: the
// inner tolerance, but no more than the solve still needs (with a margin for
// the drift of the FP32 residual from the true one), so that the last phase
// does not overshoot the target by up to the inner factor.
constexpr double kPhaseMargin = 0.5;
inline double phase_target(double inner_rtol, double rtol, double bnorm, double rn)
{
    const double need = rn > 0.0 ? kPhaseMargin * rtol * bnorm / rn : 1.0;
    return need > inner_rtol ? (need < 1.0 ? need : 1.0) : inner_rtol;
}

constexpr int kBlock = 256;        // threads per block of the vector kernels
constexpr int kRedBlocks = 1024;   // partial sums per reduction (fixed: deterministic)
constexpr int kUpdBlock = 1024;    // threads per block of the fused CG update (one node each)
constexpr int kFoldGroups = 256;   // most p.q partial groups of 1024 folded in parallel (fused CG)

// Device-resident scalars of one Krylov solve.  The host polls a copy of
// `done`/`status`/`it` every few iterations; everything else stays on the GPU.
struct SolveScalars {
    double rho;      // r . z of the current iterate
    double pq;       // p . A p
    double rr;       // r . r
    double alpha, beta;
    double tol2;     // (rtol ||b||)^2 on the working-precision recursive residual
    double bnorm2;   // ||b||^2 of the current (inner) system
    double rho_new;  // r . z after the last update (also when done)
    int32_t it;      // operator applications performed
    int32_t done;    // 1: converged or failed, kernels become no-ops
    int32_t status;  // 0 ok, FO_ERR_BREAKDOWN
    int32_t max_it;  // cap for this (inner) solve
    int32_t first;   // fused CG: next direction uses `beta` as given (restart)
    int32_t pad;
};

// Element-to-node scatter tiles (deterministic mode), see fo_tiles.h.
// Per-tile arrays use fixed strides MN (nodes) and ME (elements).
struct TileSet {
    int32_t n_tiles = 0;
    int32_t max_nodes = 0;              // MN: node stride, LDS sizing
    int32_t max_elems = 0;              // ME: element stride, block size
    int64_t n_slots = 0;                // tile-node pairs
    int64_t n_shared_slots = 0;         // halo slots (tile-node pairs of shared nodes)
    int64_t n_shared_nodes = 0;
    // device arrays
    int32_t *info = nullptr;            // [n_tiles][8] first element, counts (kTile*)
    uint16_t *lconn = nullptr;          // [n_tiles][ME][4] local vertex ids
    uint16_t *lslot = nullptr;          // [n_tiles][ME][4] LDS slot of each (element, vertex)
    int32_t *nodes = nullptr;           // [n_tiles][MN] global node of each tile node
    uint16_t *seg = nullptr;            // [n_tiles][MN+1] first slot of each node's segment
    int32_t *hpos = nullptr;            // [n_tiles][MN] halo slot of a shared tile node
    int32_t *halo_node = nullptr;       // [n_shared_nodes] global node of each shared node
    int32_t *halo_ptr = nullptr;        // [n_shared_nodes+1] node-major halo slot ranges
    int32_t *node_hrange = nullptr;     // [N][2] halo range of a node, (-1,-1) if interior
    float *tx32 = nullptr;              // [n_tiles][MN][dim] node coordinates minus the tile's
                                        // first node, formed in FP64 (FP32 operator geometry)
    // boundary facets of the descent operator, per tile node (see fo_create)
    bool facets_ok = false;             // every facet lies in a tile (else: node-parallel facets)
    int64_t n_fent = 0;                 // tile-node / facet incidences
    int32_t *fptr = nullptr;            // [n_tiles][MN+1] first incidence of each tile node
    uint64_t *fconn = nullptr;          // [n_fent] local ids of the facet's vertices (4 x uint16)
    double *fa64 = nullptr;             // [n_fent][4] a = sqrt(|F| / (d (d+1))) n
    float *fa32 = nullptr;              // [n_fent][4] FP32 copy
};

// Per-column state of the batched (multi-load) CG, one entry per column of
// the block of right-hand sides.
struct BatchCol {
    double rho;      // r . z of the residual that built the current direction
    double rho_new;  // r . z of the latest residual
    double rr;       // r . r of the latest residual
    double alpha, beta;
    double tol2;     // phase target for r . r (rescaled residual)
    double pq;       // p . A p
    int32_t done;    // converged in this phase, breakdown, capped, or inactive
    int32_t status;  // 0 ok, FO_ERR_BREAKDOWN
    int32_t fresh;   // next phase restarts this column's direction
    int32_t it;      // iterations of the current phase
    int32_t cap;     // iteration cap of the current phase
    int32_t capped;  // the phase ended at its cap
    int32_t reached; // reached the phase target; iterates on until the host ends the phase
    int32_t keep;    // phase start: the direction is kept, only rescaled (beta = the scale)
    int32_t pad;
};

// Iteration control of the batched CG (device; the host polls a copy).
struct BatchCtl {
    int32_t it;      // completed iterations of the current phase
    int32_t done;    // every column done, or it >= max_it
    int32_t max_it;
    int32_t pad;
};

// Device state of the block CG (one block of up to 64 load cases).
constexpr int kBcgBlocks = 512;     // row blocks of its Gram products (fixed: deterministic sums)
constexpr double kBcgDrop = 1e-5;   // relative pivot below which a block direction is dropped
struct BcgState {
    int32_t np;          // directions in the block P (columns >= np are zero)
    int32_t first;       // the next direction kernel builds P = Z[:, act] (phase start)
    int32_t status;      // 0 ok, FO_ERR_BREAKDOWN
    int32_t it_phase;    // iterations of the current phase
    int32_t cap;         // iteration cap of the phase
    int32_t capped;      // the phase ended at its cap
    int32_t pad[2];
    double tol2;         // phase target of r.r per column (rescaled residuals)
    double drop;         // relative pivot below which a direction is dropped
    int32_t act[64];     // direction q was built from residual column act[q] (-1: none)
    int32_t run[64];     // residual column still running in this phase
    double rr[64];       // r.r of every column after the last update
    double Gi[64 * 64];  // (P^T K P)^-1 on the kept directions (dropped ones zero)
    float gam[64 * 64];  // Gamma [sp][S]
    float del[64 * 64];  // Delta [sp][sp]
};

struct BcgBufs {
    BcgState *st = nullptr;
    double *sums = nullptr;   // Gram sums [sp*sp + sp*S] or [sp*S + S]
    float *part = nullptr;    // per-block partials
};

// Buffers of the batched path: block vectors are [n_dofs][S] (column
// fastest), S = 16 NC right-hand sides per block, NC = 1..4.
struct BatchState {
    int S = 0;                          // column stride of the allocated block vectors
    int mn_cap = 0;                     // node cap of the current batch tiles
    int group = 8;                      // G: node-disjoint elements per contraction group
    int slot_stride = 0;                // MS: element slots per tile (fixed stride)
    int64_t n_slot_total = 0;           // n_tiles * MS
    int version = 0;                    // bumps when the tiles change (graph keys)
    int n_upd = 0;                      // blocks of the node-parallel batch kernels
    TileSet tiles;                      // batch tiles over the context's element order
    int32_t *selem = nullptr;           // [n_tiles][MS] element of each slot, -1 padding
    uint64_t *slconn = nullptr;         // [n_tiles][MS] local vertex ids (4 x uint16)
    int4 *sgconn = nullptr;             // [n_tiles][MS] global vertex ids
    std::vector<void *> tile_allocs;    // released when the tiles are rebuilt
    size_t tile_bytes = 0;
    float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr;
    float *halo = nullptr;              // [halo_cap]
    size_t halo_cap = 0;
    double *x64 = nullptr, *r64 = nullptr, *b64 = nullptr;
    double *pq_part = nullptr;          // [pq_cap] per tile and column
    size_t pq_cap = 0;
    double *rz_part = nullptr;          // [2][n_upd][S]
    double *s2 = nullptr;               // [3][S]: scale^2 of the phase, new residual^2, b^2
    uint8_t *mask = nullptr;            // [S] columns selected for a residual replacement
    int32_t *caps = nullptr;            // [S] phase iteration caps of the selected columns
    int32_t *caps_host = nullptr;       // pinned [S]
    double *ptol = nullptr;             // [S] phase targets of the selected columns (phase_target)
    double *ptol_host = nullptr;        // pinned [S]
    float *geo = nullptr;               // [n_tiles][MS][16] slot cofactors and weight (per level set)
    BatchCol *cols = nullptr;           // [S]
    BatchCtl *ctl = nullptr;
    BatchCtl *ctl_host = nullptr;       // pinned
    BatchCol *cols_host = nullptr;      // pinned [S]
    double *s2_host = nullptr;          // pinned [S]
    uint8_t *mask_host = nullptr;       // pinned [S]
    BcgBufs bcg;                        // block CG
    BcgState *bcg_host = nullptr;       // pinned copy (status, counts)
    int method = FO_BATCH_COLUMN_CG;    // FO_BATCH_COLUMN_CG (default) or FO_BATCH_BLOCK_CG
    // the operator: FO_BATCH_OP_NODAL (default: assembled node blocks) or
    // FO_BATCH_OP_ELEMENT (element tiles above)
    int op = FO_BATCH_OP_NODAL;
    int nb = 0;                         // NB: neighbour slots per node (a multiple of nb_chunk)
    int nb_chunk = 8;                   // neighbours per round of loads of the apply: 7 or 8
    int kw = 0;                         // floats of blocks per node: NB d^2 rounded up to a multiple of 4
    int n_apply = 0;                    // blocks of the nodal apply at S columns (p.q partials)
    int32_t *nbr = nullptr;             // [N][NB] neighbour nodes, ascending, padded with the node
    int32_t *inc_ptr = nullptr;         // [N+1] node -> element incidence
    int32_t *inc_elem = nullptr;        // [(d+1) E] incident elements, ascending per node
    float *kb = nullptr;                // [N][kw] blocks K_ij, [NB][d][d] then zeros (per level set; 0 for padding)
    double *kb64 = nullptr;             // [N][NB][d][d] the same blocks unrounded (FP64 residuals)
    double *pq_nodal = nullptr;         // [n_apply][S] p.q partials of the nodal apply
    int nodal_occ[4] = {0, 0, 0, 0};    // resident blocks of the apply at S = 16, 32, 48, 64
    int64_t n_offdiag = 0;              // off-diagonal blocks (ordered node pairs sharing an element)
    int64_t nodal_bytes = 0;            // device bytes of the nodal arrays
};

struct DescentSetup {
    bool valid = false;
    double alpha = 0, gamma_n = 0, gamma_s = 0;
    std::vector<double> boxes;
    uint8_t *in0 = nullptr;   // [E] element centroid in Omega0 (tile element order)
    double *diag = nullptr;   // [n_dofs]
    double *dinv = nullptr;   // [n_dofs]
    float *dinv32 = nullptr;  // [n_dofs]
    const uint8_t *fixed = nullptr;  // the mask in use (theta = 0 there): mask_copy, or null
    const uint8_t *fixed_src = nullptr;  // the caller's mask of the current options (identity only)
    uint8_t *mask_copy = nullptr;    // [n_dofs] copy of the caller's mask, taken at set-up
    double *rhs = nullptr;    // [n_dofs] right-hand side with the masked entries zeroed
    double *boxes_dev = nullptr;  // [kMaxBoxes][2 dim] device copy of the boxes
};

}  // namespace fo

struct fo_ctx {
    int dim = 0;
    int64_t N = 0, E = 0, ndof = 0;
    int32_t max_rhs = 1;
    double lam = 0, mu = 0, ersatz = 1e-3;
    hipStream_t stream = nullptr;
    int device = 0;
    int scatter = FO_SCATTER_TILED;
    bool have_phi = false;
    bool has_isolated = false;         // some node belongs to no element
    size_t bytes = 0;                  // device footprint
    std::vector<void *> allocations;   // everything hipMalloc'ed by this ctx
    char *ws = nullptr;                // caller's workspace (device), or null
    size_t ws_cap = 0;                 // its size
    bool measure = false;              // dry run of fo_create: count the bytes, touch no device

    // mesh, tile element order (elem_perm[tile order] = input element id)
    double *coords = nullptr;          // [N][dim]
    float *coords32 = nullptr;         // [N][dim]
    int32_t *conn = nullptr;           // [dim+1][E] SoA, tile element order
    int32_t *elem_perm = nullptr;      // [E] tile order -> input order
    uint8_t *fixed = nullptr;          // [ndof]
    int64_t nbf = 0;
    int32_t *bfacets = nullptr;        // [dim][nbf]
    double *bnormal = nullptr;         // [nbf][dim]
    fo::TileSet tiles;

    // level-set dependent
    uint8_t *chi = nullptr;            // [E] element in Omega (tile order)
    double *diag64 = nullptr;          // [ndof] diagonal of K(phi)
    double *dinv64 = nullptr;          // [ndof] Jacobi (0 on clamped)
    float *dinv32 = nullptr;

    // descent operator
    fo::DescentSetup descent;

    // Krylov workspace (single RHS); FP64 and FP32 copies
    double *x64 = nullptr, *r64 = nullptr, *p64 = nullptr, *q64 = nullptr, *b64 = nullptr,
           *t64 = nullptr, *p64b = nullptr, *x64b = nullptr;  // x64b: saved iterate (FP64 finish)
    float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *b32 = nullptr,
          *p32b = nullptr;  // p*b: second direction buffer of the fused CG
    double *halo = nullptr;            // [n_shared_slots * dim] halo partials
    double *partials = nullptr;        // [kRedBlocks * 4] general partial sums
    double *pq_part = nullptr;         // [max(n_tiles, kRedBlocks)] p.Ap partials
    double *rz_part = nullptr;         // [2 * kRedBlocks] r.z, r.r partials
    // Folded partials of the fused CG on large meshes: r.z, r.r (0, 1) and
    // p.q (2), each summed by one block in a fixed order before the kernel that
    // needs it, so that the tile kernel's blocks (and the update's) read one
    // value instead of every partial.  Used when there are more partials than
    // those kernels sum in one pass of loads.
    double *fold = nullptr;            // [4 + kFoldGroups]: folded r.z, r.r, p.q; the p.q group sums from 4
    bool fold_rz = false, fold_pq = false;
    double *bb_part = nullptr;         // [kRedBlocks] b.b partials
    fo::SolveScalars *scal = nullptr;  // device, two parity slots
    fo::SolveScalars *scal_host = nullptr;  // pinned [2]: copies of slot 0 (final state in [0])
    hipStream_t work = nullptr;        // private non-blocking stream on which graphs are captured
    hipEvent_t ev_poll[2] = {nullptr, nullptr};  // status copies of chunks in flight
    // captured CG iteration chunks: key (operator, chunk, scatter, descent version)
    std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;
    int descent_version = 0;
    double *red_host = nullptr;        // pinned scratch for scalar results
    double *dscratch = nullptr;        // [8] device scratch scalars

    // node-recovery buffers for the level-set update
    double *gbuf = nullptr;            // [N][dim+1]

    // shape derivative: element tensors (tile order) and partial sums
    double *s1buf = nullptr;           // [E][dim*dim]
    double *sd_part = nullptr;         // [(max_rhs+1)][blocks]
    int sd_part_cap = 0;

    // kernel timing (fo_profile_*): event pairs per counter
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events[FO_PROF_COUNT];
    size_t prof_used[FO_PROF_COUNT] = {0, 0, 0, 0};

    // transport step: h^2 of the diffusion term (the paper's mesh-size
    // expression) and the work buffers of transport and reinitialisation
    double transport_h2 = 0.0;
    void *tr_buf = nullptr;

    // graph_chunk enqueues chunks that have no captured graph yet directly
    // instead of capturing them (no graph instantiation during the call)
    bool no_capture = false;

    // inverse elasticity work buffers, allocated on the first call
    void *inv_buf = nullptr;
    size_t inv_cap = 0;                // doubles in inv_buf

    // fixed nodes of the heat state solve in progress (device [N])
    const uint8_t *heat_mask = nullptr;

    // batched multi-load solves (allocated when max_rhs > 1)
    fo::BatchState batch;

    // boundary nodes -> incident facets (descent normal penalty)
    int64_t n_bnodes = 0;
    int32_t *bnodes = nullptr, *bnode_ptr = nullptr, *bnode_fac = nullptr;
};

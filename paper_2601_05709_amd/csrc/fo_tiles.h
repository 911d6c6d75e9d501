// Element tiles for the deterministic LDS scatter.
//
// A tile is a run of at most tile_max_elems elements along a Morton curve of
// element centroids; one thread block processes it with one thread per
// element.  Within a tile:
//   - nodes are numbered locally: interior nodes (all of whose elements lie in
//     the tile) first, then the shared nodes this tile owns, then the other
//     shared nodes.  A shared node is owned by the first tile that touches it;
//     the owner writes node vectors that every touching tile computes alike;
//   - every (element, vertex) pair owns one LDS slot, and slots are ordered by
//     local node, so the contributions to one node form a contiguous segment
//     that one thread sums in a fixed order.
// Interior nodes are written straight to the output; shared nodes go to a
// node-major halo buffer whose slots a second, node-parallel pass (or the CG
// update) sums in tile order.  Results are bitwise reproducible for a mesh.
#pragma once

#include <cstdint>
#include <vector>

struct fo_ctx;

namespace fo {

// Per-tile arrays have a fixed stride (the largest tile), so every index a
// thread needs is addressable from the tile id alone.
enum { kTileE0 = 0, kTileNE, kTileNN, kTileNInt, kTileNOwn, kTileInfo = 8 };

struct HostTiles {
    std::vector<int32_t> perm;             // tile order -> input element id
    int32_t n_tiles = 0, max_nodes = 0, max_elems = 0;  // strides MN, ME
    int64_t n_slots = 0;                   // tile-node pairs (unpadded)
    std::vector<int32_t> info;             // [n_tiles][8]: first element, elements, nodes,
                                           //   interior nodes, owned nodes (see kTile*)
    std::vector<uint16_t> lconn;           // [n_tiles][ME][4] local vertex ids
    std::vector<uint16_t> lslot;           // [n_tiles][ME][4] LDS slot of (element, vertex)
    std::vector<int32_t> nodes;            // [n_tiles][MN] global node of each tile node
    std::vector<uint16_t> seg;             // [n_tiles][MN+1] first slot of each node's segment
    std::vector<int32_t> hpos;             // [n_tiles][MN] halo slot of a shared tile node, -1
    std::vector<int32_t> halo_node;        // [n_shared_nodes] global node id
    std::vector<int32_t> halo_ptr;         // [n_shared_nodes+1] node-major halo slot ranges
    std::vector<int32_t> node_hrange;      // [N][2] halo slot range of a node, (-1,-1) interior
    std::vector<int32_t> tile_elem_off_tmp;  // build scratch
};

// Limits on a tile.  Elements per tile bound the block size (one thread per
// element) and the LDS slot array; nodes per tile bound the node staging.
int tile_max_nodes(int dim);
int tile_max_elems(int dim);

// Element count per tile for a mesh of E elements on a GPU with `cus`
// compute units: about eight tiles per CU, within [128, tile_max_elems].
int tile_target_elems(int dim, int64_t E, int cus);

// Builds tiles of at most max_elems elements.  Never fails for a valid mesh.
// With max_nodes > 0 the tiles hold at most max_nodes nodes and max_elems is
// not clamped to tile_max_elems (tiles of the batched operator); presorted
// keeps the given element order instead of sorting along a Morton curve
// (perm is then the identity).
void build_tiles(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                 int max_elems, HostTiles *out, int max_nodes = 0, bool presorted = false);

// Copies the tiles to the device arrays of c->tiles (allocated in c).
int upload_tiles(fo_ctx *c, const HostTiles &h);

}  // namespace fo

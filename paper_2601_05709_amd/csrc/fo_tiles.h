// Element tiles for the deterministic LDS scatter.
//
// A tile is a run of elements along a Morton curve of element centroids, cut
// so that its nodes fit in LDS.  Within a tile:
//   - nodes are numbered locally, interior nodes (all of whose elements lie in
//     the tile) first, shared nodes after them;
//   - elements are processed in sub-batches of kSub (one element per thread);
//     every (element, vertex) pair of a sub-batch owns one LDS slot, and the
//     slots are ordered by local node, so each node's contributions form a
//     contiguous segment that one thread sums in a fixed order.
// Interior nodes are written straight to the output; shared nodes go to a halo
// buffer that a second, node-parallel pass sums in a fixed (tile) order.  The
// result is bitwise reproducible for a given mesh.
#pragma once

#include <cstdint>
#include <vector>

struct fo_ctx;

namespace fo {

constexpr int kSub = 256;  // elements per sub-batch = threads per tile block

struct HostTiles {
    std::vector<int32_t> perm;             // tile order -> input element id
    int32_t n_tiles = 0, max_nodes = 0, max_sub = 0;
    std::vector<int32_t> tile_elem_off;    // [n_tiles+1]
    std::vector<int32_t> tile_node_off;    // [n_tiles+1]
    std::vector<int32_t> tile_node_interior;  // [n_tiles]
    std::vector<int32_t> tile_halo_off;    // [n_tiles]
    std::vector<int32_t> tile_nodes;       // [n_slots]
    std::vector<uint16_t> lconn;           // [E][4]
    std::vector<uint16_t> lslot;           // [E][4]
    std::vector<int32_t> sub_off;          // [n_tiles+1] sub-batch index of each tile
    std::vector<int32_t> seg_off;          // [n_sub+1] into seg_node/seg_start
    std::vector<uint16_t> seg_node;        // segment local node (0xFFFF = end sentinel)
    std::vector<uint16_t> seg_start;       // segment first slot (sentinel: slot count)
    std::vector<int32_t> halo_node;        // [n_shared_nodes]
    std::vector<int32_t> halo_ptr;         // [n_shared_nodes+1]
    std::vector<int32_t> halo_src;         // [n_halo_slots]
    std::vector<int32_t> owner_tile;       // [N] tile that writes node-owned vectors
};

// Limits on a tile (chosen so the FP64 3D staging fits twice per CU's LDS).
int tile_max_nodes(int dim);
int tile_max_elems(int dim);

// Builds tiles for the mesh.  Never fails for a valid mesh.
void build_tiles(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                 HostTiles *out);

// Copies the tiles to the device arrays of c->tiles (allocated in c).
int upload_tiles(fo_ctx *c, const HostTiles &h);

}  // namespace fo

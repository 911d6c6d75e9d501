// Block-to-tile mapping for launches over element tiles.
#pragma once

#include <hip/hip_runtime.h>

namespace fo {

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous run
// of tiles (spatial neighbours) so shared nodes are fetched into one L2.
// Launch with xcd_grid(n_tiles) blocks; returns -1 for the few spare blocks.
__device__ __forceinline__ int xcd_tile(int b, int n_tiles)
{
    const int per = (n_tiles + 7) >> 3;
    const int t = (b & 7) * per + (b >> 3);
    return t < n_tiles ? t : -1;
}

static inline int xcd_grid(int n_tiles) { return 8 * ((n_tiles + 7) / 8); }

}  // namespace fo

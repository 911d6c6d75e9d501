// Device helpers shared by the batched operator kernels (element tiles in
// fo_batch.hip, assembled node blocks in fo_nodal.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "fo_internal.h"

namespace fo {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Whether the batched solve is over: marked done, the iteration cap reached,
// or every one of the S columns done or at its phase target.  Read by thread 0 of every block of an
// operator launch from state that no kernel of that launch writes (block 0
// may set done, which only confirms the same decision), so all blocks agree;
// block 0 records the decision.  Every field is loaded at once: one round
// trip, not one per test.
__device__ __forceinline__ int batch_stop(BatchCtl *ctl, const BatchCol *cols, int S)
{
    const int done = ctl->done, it = ctl->it, max_it = ctl->max_it;
    int all = 1;
    for (int k = 0; k < S; ++k) all &= cols[k].done | cols[k].reached;
    const int stop = done || it >= max_it || all;
    if (stop && !done && blockIdx.x == 0) ctl->done = 1;
    return stop;
}

}  // namespace fo

// fo_optimize without device allocation: the loop's work vectors live in a
// fixed device array of the library instead of a per-call allocation, for
// callers that cannot allocate device memory (code under graph capture,
// serving loops that keep the allocator out of the request path).
//
// `scratch` is one array per GPU, allocated with the code object when the
// library is loaded on that device and held until the process ends.  Host
// code never uses the array's name as an address: its device address is
// looked up once per device (hipGetSymbolAddress, with the device current)
// and kept here.  Every call on a GPU shares that GPU's array, so calls
// that overlap on one GPU race on it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <vector>

#include "fo_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
static_assert((3 * (size_t)FO_NOALLOC_MAX_DOFS + 4) * sizeof(double) <= kScratchBytes &&
                  (3 * ((size_t)FO_NOALLOC_MAX_DOFS + 1) + 4) * sizeof(double) > kScratchBytes,
              "FO_NOALLOC_MAX_DOFS is the largest n_dofs whose work vectors fit");

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
std::vector<double *> g_ptr;  // device address of scratch per device, null until looked up

// scratch's device address on `device` (null on failure).
double *scratch_on(int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_ptr.size() <= device) g_ptr.resize((size_t)device + 1, nullptr);
    if (g_ptr[(size_t)device]) return g_ptr[(size_t)device];
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != device && hipSetDevice(device) != hipSuccess) return nullptr;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
        std::fprintf(stderr, "libfo: hipGetSymbolAddress(scratch) failed: %s\n", hipGetErrorString(e));
        return nullptr;
    }
    g_ptr[(size_t)device] = static_cast<double *>(p);
    return g_ptr[(size_t)device];
}

}  // namespace

extern "C" {

int fo_optimize_noalloc(fo_ctx *c, const fo_loop_opts *o, const double *b, double *phi, fo_loop_record *records,
                        int32_t *n_done, int32_t *stopped)
{
    if (!c) return FO_ERR_ARG;
    if (fo::optimize_work_doubles(c) * sizeof(double) > kScratchBytes) {
        std::fprintf(stderr, "libfo: fo_optimize_noalloc: %lld unknowns exceed the static work array (%d)\n",
                     (long long)c->ndof, (int)FO_NOALLOC_MAX_DOFS);
        return FO_ERR_ARG;
    }
    double *work = scratch_on(c->device);
    if (!work) return FO_ERR_HIP;
    const bool before = c->no_capture;
    c->no_capture = true;
    const int rc = fo::optimize_on(c, o, b, phi, records, n_done, stopped, work);
    c->no_capture = before;
    return rc;
}

}  // extern "C"

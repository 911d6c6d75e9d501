// Recording stand-in for the few HIP runtime calls that the serving pool and
// the fiber waits make (host-only CPU build of tests/pool_host).
#pragma once
#include <cstddef>

typedef enum { hipSuccess = 0, hipErrorNotReady = 600, hipErrorInvalidValue = 1 } hipError_t;
typedef struct StubStream *hipStream_t;
typedef struct StubEvent *hipEvent_t;
typedef enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 } hipMemcpyKind;
#define hipStreamNonBlocking 1u

hipError_t hipGetDevice(int *d);
hipError_t hipSetDevice(int d);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamQuery(hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipMalloc(void **p, size_t bytes);
hipError_t hipFree(void *p);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind k, hipStream_t s);
template <class T>
inline hipError_t hipMalloc(T **p, size_t bytes)
{
    return hipMalloc(reinterpret_cast<void **>(p), bytes);
}

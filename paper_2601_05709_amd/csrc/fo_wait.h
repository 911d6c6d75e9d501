// Device waits of the host runtime, and the cooperative fibers of the
// serving pool.
//
// Every place where the library waits for the device (a stream drained, a
// status event reached) goes through wait_stream / wait_event.  On an
// ordinary thread they block like hipStreamSynchronize / hipEventSynchronize.
// Inside a pool fiber they poll the stream or event and, while it is not
// ready, hand control back to the pool's scheduler, which resumes the other
// requests' fibers; so all requests of a pool run on the caller's one host
// thread while their work overlaps on the device (each on its own stream).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace fo {

hipError_t wait_stream(hipStream_t s);
hipError_t wait_event(hipEvent_t e);

// A fiber runs fn(arg) on its own stack, on the thread that resumes it.
struct Fiber;
Fiber *fiber_create(void (*fn)(void *), void *arg, size_t stack_bytes);
// Runs the fiber until it yields or finishes; true once it has finished.
bool fiber_resume(Fiber *f);
// Frees a fiber that has finished or was never started.
void fiber_destroy(Fiber *f);
// The fiber running on this thread, or null.
Fiber *fiber_current();
// Returns control to the fiber's resumer (only inside a fiber).
void fiber_yield();

}  // namespace fo

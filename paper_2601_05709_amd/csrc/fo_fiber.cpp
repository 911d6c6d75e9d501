// Fibers (ucontext) and fiber-aware device waits; see fo_wait.h.
#include "fo_wait.h"

#include <sys/mman.h>
#include <ucontext.h>
#include <unistd.h>

#include <cstdint>

#if defined(__SANITIZE_ADDRESS__)
#define FO_ASAN_FIBERS 1
#elif defined(__has_feature)
#if __has_feature(address_sanitizer)
#define FO_ASAN_FIBERS 1
#endif
#endif
#ifdef FO_ASAN_FIBERS
#include <sanitizer/common_interface_defs.h>
#endif

namespace fo {

struct Fiber {
    ucontext_t ctx;
    ucontext_t *back = nullptr;  // context of the resumer while the fiber runs
    void *map = nullptr;         // stack mapping (lowest page is a guard)
    size_t map_bytes = 0;
    void (*fn)(void *) = nullptr;
    void *arg = nullptr;
    bool started = false;
    bool finished = false;
#ifdef FO_ASAN_FIBERS
    const void *back_stack = nullptr;  // resumer's stack, for the sanitizer's bookkeeping
    size_t back_size = 0;
    void *fake = nullptr;
#endif
};

namespace {

thread_local Fiber *t_cur = nullptr;

// Switches from `from` to `to`; the sanitizer is told which stack runs next.
void switch_to(ucontext_t *from, ucontext_t *to, Fiber *f, bool into_fiber, bool leaving_for_good)
{
#ifdef FO_ASAN_FIBERS
    void *fake = nullptr;
    if (into_fiber)
        __sanitizer_start_switch_fiber(&fake, (char *)f->map + getpagesize(), f->map_bytes - getpagesize());
    else
        __sanitizer_start_switch_fiber(leaving_for_good ? nullptr : &f->fake, f->back_stack, f->back_size);
    swapcontext(from, to);
    if (into_fiber)
        __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
    else
        __sanitizer_finish_switch_fiber(f->fake, &f->back_stack, &f->back_size);
#else
    (void)f;
    (void)into_fiber;
    (void)leaving_for_good;
    swapcontext(from, to);
#endif
}

void trampoline(unsigned hi, unsigned lo)
{
    Fiber *f = reinterpret_cast<Fiber *>(((uintptr_t)hi << 32) | (uintptr_t)lo);
#ifdef FO_ASAN_FIBERS
    __sanitizer_finish_switch_fiber(nullptr, &f->back_stack, &f->back_size);
#endif
    f->fn(f->arg);
    f->finished = true;
    switch_to(&f->ctx, f->back, f, false, true);  // never resumed again
}

}  // namespace

Fiber *fiber_create(void (*fn)(void *), void *arg, size_t stack_bytes)
{
    const size_t page = (size_t)getpagesize();
    const size_t bytes = ((stack_bytes + page - 1) / page + 1) * page;
    void *m = mmap(nullptr, bytes, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (m == MAP_FAILED) return nullptr;
    if (mprotect(m, page, PROT_NONE) != 0) {
        munmap(m, bytes);
        return nullptr;
    }
    Fiber *f = new Fiber();
    f->map = m;
    f->map_bytes = bytes;
    f->fn = fn;
    f->arg = arg;
    if (getcontext(&f->ctx) != 0) {
        munmap(m, bytes);
        delete f;
        return nullptr;
    }
    f->ctx.uc_stack.ss_sp = (char *)m + page;
    f->ctx.uc_stack.ss_size = bytes - page;
    f->ctx.uc_link = nullptr;
    const uintptr_t v = reinterpret_cast<uintptr_t>(f);
    makecontext(&f->ctx, (void (*)())trampoline, 2, (unsigned)(v >> 32), (unsigned)(v & 0xFFFFFFFFu));
    return f;
}

bool fiber_resume(Fiber *f)
{
    if (!f || f->finished) return true;
    ucontext_t here;
    Fiber *prev = t_cur;
    f->back = &here;
    f->started = true;
    t_cur = f;
    switch_to(&here, &f->ctx, f, true, false);
    t_cur = prev;
    return f->finished;
}

void fiber_destroy(Fiber *f)
{
    if (!f) return;
    if (f->map) munmap(f->map, f->map_bytes);
    delete f;
}

Fiber *fiber_current() { return t_cur; }

void fiber_yield()
{
    Fiber *f = t_cur;
    if (!f) return;
    switch_to(&f->ctx, f->back, f, false, false);
}

hipError_t wait_stream(hipStream_t s)
{
    if (!t_cur) return hipStreamSynchronize(s);
    for (;;) {
        const hipError_t q = hipStreamQuery(s);
        if (q != hipErrorNotReady) return q;
        fiber_yield();
    }
}

hipError_t wait_event(hipEvent_t e)
{
    if (!t_cur) return hipEventSynchronize(e);
    for (;;) {
        const hipError_t q = hipEventQuery(e);
        if (q != hipErrorNotReady) return q;
        fiber_yield();
    }
}

}  // namespace fo

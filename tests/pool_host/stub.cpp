// Recording stand-ins for the HIP runtime and for the context calls that a
// pool request makes.  Every stream, device allocation and context records
// the thread that made and released it; "device work" is a countdown per
// stream that hipStreamQuery runs down, so the fiber waits really yield.
// At exit the records must show each object released exactly once, on the
// thread that made it, and no call on an object that was already released.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>

#include "../../include/fo.h"
#include "stub.h"

namespace {

struct Rec {
    std::thread::id made, gone;
    bool live = true;
    int kind = 0;  // 1 stream, 2 device buffer, 3 context
    size_t bytes = 0;
};

std::mutex g_mu;
std::map<const void *, Rec> g_objs;
int g_errors = 0;
long g_live_bytes = 0;

void fail(const char *what, const void *p)
{
    std::fprintf(stderr, "stub: %s (%p)\n", what, p);
    ++g_errors;
}

void make(const void *p, int kind, size_t bytes = 0)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_objs.find(p);
    if (it != g_objs.end() && it->second.live) fail("object made twice", p);
    Rec r;
    r.made = std::this_thread::get_id();
    r.kind = kind;
    r.bytes = bytes;
    g_objs[p] = r;
    g_live_bytes += (long)bytes;
}

void release(const void *p, int kind)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_objs.find(p);
    if (it == g_objs.end()) return fail("release of an unknown object", p);
    if (!it->second.live) return fail("object released twice", p);
    if (it->second.kind != kind) return fail("release with the wrong call", p);
    it->second.live = false;
    it->second.gone = std::this_thread::get_id();
    if (it->second.gone != it->second.made) fail("object released on another thread than the one that made it", p);
    g_live_bytes -= (long)it->second.bytes;
}

void use(const void *p, int kind)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_objs.find(p);
    if (it == g_objs.end()) return fail("use of an unknown object", p);
    if (!it->second.live) return fail("use of a released object", p);
    if (it->second.kind != kind) return fail("object used as the wrong kind", p);
    if (it->second.made != std::this_thread::get_id()) fail("object used on another thread", p);
}

}  // namespace

struct StubStream {
    int pending = 0;  // queries until the enqueued work counts as done
};

struct fo_ctx {
    hipStream_t stream = nullptr;
    int64_t n = 0;
    double phi_sum = 0.0;
    bool have_phi = false;
};

// ------------------------------------------------------------------ HIP

hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    *s = new StubStream();
    make(*s, 1);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    release(s, 1);
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s)
{
    use(s, 1);
    s->pending = 0;
    return hipSuccess;
}
hipError_t hipStreamQuery(hipStream_t s)
{
    use(s, 1);
    if (s->pending > 0) {
        --s->pending;
        return hipErrorNotReady;
    }
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipMalloc(void **p, size_t bytes)
{
    *p = std::calloc(1, bytes ? bytes : 1);
    make(*p, 2, bytes);
    return hipSuccess;
}
hipError_t hipFree(void *p)
{
    if (!p) return hipSuccess;
    release(p, 2);
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s)
{
    use(s, 1);
    std::memcpy(dst, src, bytes);
    s->pending += 1;
    return hipSuccess;
}

// ------------------------------------------------------------------ libfo

namespace fo {
hipError_t wait_stream(hipStream_t s);
hipError_t device_malloc(void **p, size_t bytes) { return hipMalloc(p, bytes); }
}

extern "C" {

const char *fo_status_string(int) { return "stub status"; }

size_t fo_footprint_estimate(const fo_mesh *m)
{
    if (!m || m->n_nodes <= 0) return 0;
    return (size_t)m->n_nodes * 1000;
}

size_t fo_footprint_bytes(const fo_ctx *c) { return c ? (size_t)(c->n / 2) * 1000 : 0; }

int fo_create(fo_ctx **out, const fo_mesh *m, const fo_material *, int32_t, void *stream)
{
    use(stream, 1);
    fo_ctx *c = new fo_ctx();
    c->stream = (hipStream_t)stream;
    c->n = m->n_nodes * m->dim;
    make(c, 3);
    stub_count_create();
    *out = c;
    return FO_OK;
}

int fo_destroy(fo_ctx *c)
{
    if (!c) return FO_ERR_ARG;
    use(c->stream, 1);
    release(c, 3);
    delete c;
    return FO_OK;
}

int fo_set_levelset(fo_ctx *c, const double *phi)
{
    use(c, 3);
    c->have_phi = true;
    c->phi_sum = phi[0];
    c->stream->pending += 2;
    return FO_OK;
}

// "solve": a few chunks, each waited for as the CG loop does
int fo_state_solve(fo_ctx *c, const double *b, double *u, int32_t, int64_t, const fo_solve_opts *,
                   fo_solve_stats *st)
{
    use(c, 3);
    if (!c->have_phi) return FO_ERR_STATE;
    const int chunks = 2 + (int)(c->n % 5);
    for (int k = 0; k < chunks; ++k) {
        c->stream->pending += 3;
        if (fo::wait_stream(c->stream) != hipSuccess) return FO_ERR_HIP;
    }
    for (int64_t i = 0; i < c->n; ++i) u[i] = 2.0 * b[i] + c->phi_sum;
    if (st) {
        st->status = FO_OK;
        st->iters_inner = 16 * chunks;
    }
    return FO_OK;
}

int fo_shape_derivative(fo_ctx *c, const double *u, int32_t, int64_t, double, double, double *rhs, double *,
                        double *J, double *vol)
{
    use(c, 3);
    double s = 0.0;
    for (int64_t i = 0; i < c->n; ++i) {
        rhs[i] = -u[i];
        s += u[i];
    }
    *J = s;
    *vol = (double)c->n;
    c->stream->pending += 1;
    return FO_OK;
}

int fo_descent_solve(fo_ctx *c, const fo_descent_opts *, const double *rhs, double *theta, const fo_solve_opts *,
                     fo_solve_stats *st, double *B_tt)
{
    use(c, 3);
    for (int k = 0; k < 2; ++k) {
        c->stream->pending += 2;
        if (fo::wait_stream(c->stream) != hipSuccess) return FO_ERR_HIP;
    }
    double s = 0.0;
    for (int64_t i = 0; i < c->n; ++i) {
        theta[i] = 0.5 * rhs[i];
        s += theta[i] * rhs[i];
    }
    *B_tt = s;
    if (st) st->status = FO_OK;
    return FO_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ report

static int g_creates = 0;
void stub_count_create() { ++g_creates; }
int stub_creates() { return g_creates; }

int stub_report()
{
    std::lock_guard<std::mutex> lk(g_mu);
    int leaks = 0;
    for (auto &kv : g_objs)
        if (kv.second.live) {
            std::fprintf(stderr, "stub: object %p (kind %d) never released\n", kv.first, kv.second.kind);
            ++leaks;
        }
    std::printf("stub: %zu objects, %d errors, %d leaks, %ld live bytes\n", g_objs.size(), g_errors, leaks,
                g_live_bytes);
    return g_errors + leaks;
}

// Serving pool: continuous batching of hot-path requests on one GPU.
//
// Every admitted request runs as a fiber on the thread that drives the pool
// (fo_pool_step, fo_pool_wait): the fiber makes the request's library calls
// on its own context and HIP stream, and wherever a call waits for the
// device (a CG chunk's status, a stream drain) it yields to the scheduler,
// which resumes the next request.  So requests admitted while others run
// overlap on the device, and every HIP object of the pool -- contexts,
// their streams, events, graphs and host buffers, the request buffers -- is
// created, used and destroyed on that one host thread.
//
// Contexts stay resident after their request finishes and are reused by
// requests with the same mesh key; idle ones are evicted least recently used
// first when a new context needs the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "../../include/fo.h"
#include "fo_wait.h"

namespace fo {
hipError_t device_malloc(void **p, size_t bytes);  // the library's counted allocation
}

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kFiberStack = 8u << 20;  // host stack of a request (virtual, touched on use)

// A context with its stream and request buffers, resident on the device.
struct Resident {
    uint64_t key = 0;
    fo_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    double *buf = nullptr;   // phi [N] | b, u, rhs, theta [n] | J, vol, B_tt
    size_t bytes = 0;        // reserved: the estimate until created, then the actual footprint
    bool busy = false;
    bool created = false;
    int64_t N = 0, n = 0;
    uint64_t last_use = 0;
};

size_t buffer_bytes(const fo_mesh &m) { return (size_t)(m.n_nodes + 4 * m.n_nodes * m.dim + 3) * 8; }

void free_resident(Resident *r)
{
    if (r->ctx) (void)fo_destroy(r->ctx);
    if (r->buf) (void)hipFree(r->buf);
    if (r->stream) (void)hipStreamDestroy(r->stream);
    r->ctx = nullptr;
    r->buf = nullptr;
    r->stream = nullptr;
}

int worst(int a, int b)
{
    if (a < 0 || b < 0) return std::min(a, b);
    return std::max(a, b);
}

}  // namespace

struct fo_pool {
    struct Slot {
        enum State { FREE, RUNNING, DONE } state = FREE;
        Resident *res = nullptr;
        fo_request req{};
        std::vector<double> boxes;
        fo::Fiber *fiber = nullptr;
        fo_pool_result result{};
        fo_pool *pool = nullptr;
        int index = 0;
    };
    int device = 0;
    std::thread::id owner;
    size_t budget = 0, used = 0;
    std::vector<std::unique_ptr<Resident>> residents;
    std::vector<Slot> slots;
    Clock::time_point t0;
    uint64_t tick = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    bool mine() const { return std::this_thread::get_id() == owner; }

    // Drops an idle resident.
    void evict(size_t i)
    {
        Resident *r = residents[i].get();
        used -= std::min(used, r->bytes);
        free_resident(r);
        residents.erase(residents.begin() + (long)i);
    }

    void run(Slot &sl);      // a request's work (inside its fiber)
    void finish(Slot &sl);   // bookkeeping once its fiber has ended
    int step(int *progressed);
};

void fo_pool::run(Slot &sl)
{
    Resident *r = sl.res;
    const fo_request &q = sl.req;
    fo_pool_result &res = sl.result;
    res.t_start = now();
    int st = FO_OK;
    if (!r->created) {
        int rc = FO_OK;
        if (hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking) != hipSuccess) rc = FO_ERR_HIP;
        if (rc == FO_OK) rc = fo_create(&r->ctx, &q.mesh, &q.mat, 1, r->stream);
        if (rc == FO_OK && fo::device_malloc((void **)&r->buf, buffer_bytes(q.mesh)) != hipSuccess) rc = FO_ERR_NOMEM;
        if (rc == FO_OK) {
            const size_t actual = fo_footprint_bytes(r->ctx) + buffer_bytes(q.mesh);
            used = used + actual - std::min(used, r->bytes);
            r->bytes = actual;
            r->created = true;
            r->N = q.mesh.n_nodes;
            r->n = q.mesh.n_nodes * q.mesh.dim;
        } else {
            st = rc;
        }
    } else {
        res.reused_context = 1;
    }
    if (st == FO_OK) {
        const int64_t N = r->N, n = r->n;
        double *phi = r->buf, *b = phi + N, *u = b + n, *rhs = u + n, *theta = rhs + n, *J = theta + n,
               *vol = J + 1, *btt = vol + 1;
        hipStream_t hs = r->stream;
        if (hipMemcpyAsync(phi, q.phi, N * 8, hipMemcpyHostToDevice, hs) != hipSuccess ||
            hipMemcpyAsync(b, q.b, n * 8, hipMemcpyHostToDevice, hs) != hipSuccess)
            st = FO_ERR_HIP;
        if (st == FO_OK) st = fo_set_levelset(r->ctx, phi);
        if (st >= 0) st = worst(st, fo_state_solve(r->ctx, b, u, 1, 1, &q.state_opts, &res.state));
        if (st >= 0) st = worst(st, fo_shape_derivative(r->ctx, u, 1, 1, q.lambda_vol, q.V, rhs, nullptr, J, vol));
        if (st >= 0) {
            fo_descent_opts d = q.descent;
            d.boxes = sl.boxes.empty() ? nullptr : sl.boxes.data();
            st = worst(st, fo_descent_solve(r->ctx, &d, rhs, theta, &q.descent_solve_opts, &res.descent, btt));
        }
        // drain the stream (yielding) before the copies into pageable host
        // memory, which would otherwise block the scheduler's thread
        if (fo::wait_stream(hs) != hipSuccess) st = worst(st, FO_ERR_HIP);
        if (st >= 0) {
            double scal[3] = {0, 0, 0};
            bool ok = hipMemcpyAsync(scal, J, 3 * 8, hipMemcpyDeviceToHost, hs) == hipSuccess;
            if (q.u_out) ok = ok && hipMemcpyAsync(q.u_out, u, n * 8, hipMemcpyDeviceToHost, hs) == hipSuccess;
            if (q.rhs_out) ok = ok && hipMemcpyAsync(q.rhs_out, rhs, n * 8, hipMemcpyDeviceToHost, hs) == hipSuccess;
            if (q.theta_out)
                ok = ok && hipMemcpyAsync(q.theta_out, theta, n * 8, hipMemcpyDeviceToHost, hs) == hipSuccess;
            // the copies must have landed before the request is reported done
            if (fo::wait_stream(hs) != hipSuccess) ok = false;
            if (!ok) st = FO_ERR_HIP;
            res.J = scal[0];
            res.vol = scal[1];
            res.B_tt = scal[2];
        }
    }
    if (st < 0)
        std::fprintf(stderr, "libfo pool: request in slot %d failed: %s (%d)\n", sl.index, fo_status_string(st), st);
    res.status = st;
    res.t_end = now();
}

void fo_pool::finish(Slot &sl)
{
    fo::fiber_destroy(sl.fiber);
    sl.fiber = nullptr;
    Resident *r = sl.res;
    r->busy = false;
    r->last_use = ++tick;
    if (r->key == 0 || !r->created) {  // not shareable, or failed: give the memory back now
        for (size_t i = 0; i < residents.size(); ++i)
            if (residents[i].get() == r) {
                evict(i);
                break;
            }
    }
    sl.res = nullptr;
    sl.state = Slot::DONE;
}

// Resumes every running request once; *progressed counts those that ran
// past a wait (finished or not) rather than finding their device work still
// pending.  Returns the number still running.
int fo_pool::step(int *progressed)
{
    int running = 0, moved = 0;
    for (Slot &sl : slots) {
        if (sl.state != Slot::RUNNING) continue;
        const bool fin = fo::fiber_resume(sl.fiber);
        ++moved;
        if (fin)
            finish(sl);
        else
            ++running;
    }
    if (progressed) *progressed = moved;
    return running;
}

namespace {

void fiber_main(void *arg)
{
    auto *sl = static_cast<fo_pool::Slot *>(arg);
    sl->pool->run(*sl);
}

}  // namespace

extern "C" {

int fo_pool_create(fo_pool **out, size_t budget_bytes, int32_t max_slots)
{
    if (!out || budget_bytes == 0 || max_slots < 1 || max_slots > 64) return FO_ERR_ARG;
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FO_ERR_HIP;
    fo_pool *p = new fo_pool();
    p->device = dev;
    p->owner = std::this_thread::get_id();
    p->budget = budget_bytes;
    p->slots = std::vector<fo_pool::Slot>((size_t)max_slots);
    for (int i = 0; i < max_slots; ++i) {
        p->slots[(size_t)i].pool = p;
        p->slots[(size_t)i].index = i;
    }
    p->t0 = Clock::now();
    *out = p;
    return FO_OK;
}

int fo_pool_admit(fo_pool *p, const fo_request *q, int32_t *slot)
{
    if (!p || !q || !slot || !q->phi || !q->b || !(q->V > 0)) return FO_ERR_ARG;
    if (!p->mine()) return FO_ERR_STATE;
    if (q->descent.n_boxes < 0 || (q->descent.n_boxes > 0 && !q->descent.boxes)) return FO_ERR_ARG;
    if (q->descent.fixed) return FO_ERR_ARG;  // a device mask cannot follow a request to its context
    const size_t est = fo_footprint_estimate(&q->mesh);
    if (est == 0) return FO_ERR_ARG;
    int s = -1;
    for (size_t i = 0; i < p->slots.size(); ++i)
        if (p->slots[i].state == fo_pool::Slot::FREE) {
            s = (int)i;
            break;
        }
    if (s < 0) return FO_ERR_BUSY;
    Resident *r = nullptr;
    if (q->mesh_key != 0)
        for (auto &rp : p->residents)
            if (rp->key == q->mesh_key && rp->created && !rp->busy) {
                r = rp.get();
                break;
            }
    const bool fresh = r == nullptr;
    if (fresh) {
        const size_t need = est + buffer_bytes(q->mesh);
        while (p->used + need > p->budget) {  // evict idle residents, least recently used first
            long lru = -1;
            for (size_t i = 0; i < p->residents.size(); ++i) {
                const Resident *c = p->residents[i].get();
                if (!c->busy && c->created && (lru < 0 || c->last_use < p->residents[(size_t)lru]->last_use))
                    lru = (long)i;
            }
            if (lru < 0) return FO_ERR_BUSY;
            p->evict((size_t)lru);
        }
    }
    fo_pool::Slot &sl = p->slots[(size_t)s];
    fo::Fiber *f = fo::fiber_create(fiber_main, &sl, kFiberStack);
    if (!f) return FO_ERR_NOMEM;
    if (fresh) {
        p->residents.emplace_back(new Resident());
        r = p->residents.back().get();
        r->key = q->mesh_key;
        r->bytes = est + buffer_bytes(q->mesh);
        p->used += r->bytes;
    }
    r->busy = true;
    sl.req = *q;
    sl.boxes.assign(q->descent.boxes, q->descent.boxes + (size_t)std::max(0, q->descent.n_boxes) * 2 * q->mesh.dim);
    sl.res = r;
    sl.fiber = f;
    sl.result = fo_pool_result{};
    sl.result.t_admit = p->now();
    sl.state = fo_pool::Slot::RUNNING;
    *slot = s;
    return FO_OK;
}

int fo_pool_step(fo_pool *p, int32_t *running)
{
    if (!p) return FO_ERR_ARG;
    if (!p->mine()) return FO_ERR_STATE;
    const int r = p->step(nullptr);
    if (running) *running = r;
    return FO_OK;
}

int fo_pool_wait(fo_pool *p, int64_t timeout_us, int32_t *slot)
{
    if (!p || !slot) return FO_ERR_ARG;
    if (!p->mine()) return FO_ERR_STATE;
    *slot = -1;
    const auto start = Clock::now();
    for (;;) {
        for (size_t i = 0; i < p->slots.size(); ++i)
            if (p->slots[i].state == fo_pool::Slot::DONE) {
                *slot = (int32_t)i;
                return FO_OK;
            }
        int moved = 0;
        const int running = p->step(&moved);
        bool done = false;
        for (const auto &sl : p->slots) done = done || sl.state == fo_pool::Slot::DONE;
        if (done) continue;
        if (running == 0) return FO_OK;
        if (timeout_us >= 0 &&
            std::chrono::duration_cast<std::chrono::microseconds>(Clock::now() - start).count() >= timeout_us)
            return FO_OK;
        // every request is waiting for its device work: a short pause keeps
        // the host from spinning on the queries
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

int fo_pool_poll(fo_pool *p, int32_t slot, int32_t *done, fo_pool_result *res)
{
    if (!p || !done || slot < 0 || slot >= (int32_t)p->slots.size()) return FO_ERR_ARG;
    if (!p->mine()) return FO_ERR_STATE;
    const fo_pool::Slot &sl = p->slots[(size_t)slot];
    *done = sl.state == fo_pool::Slot::DONE ? 1 : 0;
    if (*done && res) *res = sl.result;
    return FO_OK;
}

int fo_pool_release(fo_pool *p, int32_t slot)
{
    if (!p || slot < 0 || slot >= (int32_t)p->slots.size()) return FO_ERR_ARG;
    if (!p->mine()) return FO_ERR_STATE;
    fo_pool::Slot &sl = p->slots[(size_t)slot];
    if (sl.state != fo_pool::Slot::DONE) return FO_ERR_STATE;
    sl.state = fo_pool::Slot::FREE;
    return FO_OK;
}

int fo_pool_stats(const fo_pool *p, size_t *used_bytes, int32_t *running, int32_t *resident)
{
    if (!p) return FO_ERR_ARG;
    int32_t run = 0;
    for (const auto &sl : p->slots) run += sl.state == fo_pool::Slot::RUNNING ? 1 : 0;
    if (used_bytes) *used_bytes = p->used;
    if (running) *running = run;
    if (resident) *resident = (int32_t)p->residents.size();
    return FO_OK;
}

int fo_pool_destroy(fo_pool *p)
{
    if (!p) return FO_ERR_ARG;
    if (!p->mine()) return FO_ERR_STATE;
    while (p->step(nullptr) > 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    (void)hipSetDevice(p->device);
    for (auto &r : p->residents) free_resident(r.get());
    delete p;
    return FO_OK;
}

}  // extern "C"

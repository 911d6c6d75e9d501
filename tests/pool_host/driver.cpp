// Drives the serving pool (fo_pool.cpp, fo_fiber.cpp) on the recording stub:
// results alone and in the mix, budget admission and release, context reuse,
// least-recently-used eviction, teardown with requests still running, and
// calls from a thread that does not own the pool.  Exit status 0 = clean.
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/fo.h"
#include "stub.h"

namespace {

int g_fail = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "driver: check failed at %d: %s\n", __LINE__, #c); \
            ++g_fail;                                                      \
        }                                                                  \
    } while (0)

struct Req {
    int64_t nodes;
    uint64_t key;
    std::vector<double> phi, b, u, rhs, theta;
    fo_request q{};
    explicit Req(int id, int64_t nn, uint64_t k) : nodes(nn), key(k)
    {
        const int64_t n = nn * 2;
        phi.assign((size_t)nn, 0.25 * id - 1.0);
        b.resize((size_t)n);
        for (int64_t i = 0; i < n; ++i) b[(size_t)i] = 0.001 * (double)((i * 7 + id * 13) % 101);
        u.assign((size_t)n, 0.0);
        rhs.assign((size_t)n, 0.0);
        theta.assign((size_t)n, 0.0);
        q.mesh.dim = 2;
        q.mesh.n_nodes = nn;
        q.mesh.n_elems = 2 * nn;
        q.mat.E = 1.0;
        q.mat.nu = 0.3;
        q.mesh_key = k;
        q.phi = phi.data();
        q.b = b.data();
        q.V = 1.0;
        q.u_out = u.data();
        q.rhs_out = rhs.data();
        q.theta_out = theta.data();
    }
};

fo_pool_result run_all(fo_pool *p, std::vector<Req *> rs)
{
    std::vector<int> slot_of(64, -1);
    fo_pool_result last{};
    for (size_t i = 0; i < rs.size(); ++i) {
        int32_t s = -1;
        CHECK(fo_pool_admit(p, &rs[i]->q, &s) == FO_OK);
        if (s >= 0) slot_of[(size_t)s] = (int)i;
    }
    size_t done = 0;
    while (done < rs.size()) {
        int32_t s = -1;
        CHECK(fo_pool_wait(p, -1, &s) == FO_OK);
        if (s < 0) break;
        int32_t d = 0;
        CHECK(fo_pool_poll(p, s, &d, &last) == FO_OK && d == 1);
        CHECK(last.status == FO_OK);
        CHECK(fo_pool_release(p, s) == FO_OK);
        ++done;
    }
    CHECK(done == rs.size());
    return last;
}

}  // namespace

int main()
{
    // results alone and in the mix
    std::vector<Req> alone, mix;
    for (int i = 0; i < 6; ++i) alone.emplace_back(i, 40 + 7 * i, 0);
    for (int i = 0; i < 6; ++i) mix.emplace_back(i, 40 + 7 * i, 0);
    for (auto &r : alone) {
        fo_pool *p = nullptr;
        CHECK(fo_pool_create(&p, 1 << 30, 1) == FO_OK);
        run_all(p, {&r});
        CHECK(fo_pool_destroy(p) == FO_OK);
    }
    {
        fo_pool *p = nullptr;
        CHECK(fo_pool_create(&p, 1 << 30, 6) == FO_OK);
        std::vector<Req *> rp;
        for (auto &r : mix) rp.push_back(&r);
        std::vector<int32_t> slots;
        for (auto *r : rp) {
            int32_t s = -1;
            CHECK(fo_pool_admit(p, &r->q, &s) == FO_OK);
            slots.push_back(s);
        }
        int32_t running = 0;
        CHECK(fo_pool_step(p, &running) == FO_OK && running == 6);  // all started, all waiting
        double first_end = 1e30, last_start = -1;
        for (int k = 0; k < 6; ++k) {
            int32_t s = -1;
            CHECK(fo_pool_wait(p, -1, &s) == FO_OK && s >= 0);
            fo_pool_result res{};
            int32_t d = 0;
            CHECK(fo_pool_poll(p, s, &d, &res) == FO_OK && d == 1);
            first_end = std::min(first_end, res.t_end);
            last_start = std::max(last_start, res.t_start);
            CHECK(fo_pool_release(p, s) == FO_OK);
        }
        CHECK(last_start < first_end);  // they overlapped
        CHECK(fo_pool_destroy(p) == FO_OK);
        for (int i = 0; i < 6; ++i) {
            CHECK(std::memcmp(alone[i].u.data(), mix[i].u.data(), alone[i].u.size() * 8) == 0);
            CHECK(std::memcmp(alone[i].theta.data(), mix[i].theta.data(), alone[i].theta.size() * 8) == 0);
        }
    }
    // budget admission: one unkeyed context fits
    {
        Req a(1, 100, 0), b(2, 100, 0);
        const size_t one = (size_t)100 * 1000 + (size_t)(100 + 4 * 200 + 3) * 8;
        fo_pool *p = nullptr;
        CHECK(fo_pool_create(&p, one + one / 2, 4) == FO_OK);
        int32_t s = -1, s2 = -1;
        CHECK(fo_pool_admit(p, &a.q, &s) == FO_OK);
        CHECK(fo_pool_admit(p, &b.q, &s2) == FO_ERR_BUSY);
        CHECK(fo_pool_wait(p, -1, &s) == FO_OK && s >= 0);
        CHECK(fo_pool_release(p, s) == FO_OK);
        size_t used = 1;
        int32_t run = -1, res = -1;
        CHECK(fo_pool_stats(p, &used, &run, &res) == FO_OK && used == 0 && res == 0);
        CHECK(fo_pool_admit(p, &b.q, &s2) == FO_OK);
        CHECK(fo_pool_release(p, s2) == FO_ERR_STATE);  // still running
        CHECK(fo_pool_wait(p, -1, &s2) == FO_OK && s2 >= 0);
        CHECK(fo_pool_release(p, s2) == FO_OK);
        CHECK(fo_pool_destroy(p) == FO_OK);
    }
    // reuse by key, and LRU eviction when a third mesh needs the memory
    {
        Req a(1, 100, 11), a2(2, 100, 11), b(3, 120, 12), c(4, 110, 13);
        const size_t per = (size_t)120 * 1000 + (size_t)(120 + 4 * 240 + 3) * 8;
        fo_pool *p = nullptr;
        CHECK(fo_pool_create(&p, 2 * per + per / 2, 2) == FO_OK);
        const int c0 = stub_creates();
        run_all(p, {&a});
        fo_pool_result r = run_all(p, {&a2});
        CHECK(r.reused_context == 1 && stub_creates() == c0 + 1);
        run_all(p, {&b});
        int32_t resident = 0;
        CHECK(fo_pool_stats(p, nullptr, nullptr, &resident) == FO_OK && resident == 2);
        run_all(p, {&c});  // evicts the least recently used (key 11)
        CHECK(fo_pool_stats(p, nullptr, nullptr, &resident) == FO_OK && resident <= 2);
        Req a3(5, 100, 11);
        r = run_all(p, {&a3});
        CHECK(r.reused_context == 0);
        CHECK(fo_pool_destroy(p) == FO_OK);
    }
    // teardown while requests run; calls from a thread that is not the owner
    {
        Req a(1, 60, 21), b(2, 70, 0), c(3, 80, 22);
        fo_pool *p = nullptr;
        CHECK(fo_pool_create(&p, 1 << 30, 4) == FO_OK);
        int32_t s = -1;
        CHECK(fo_pool_admit(p, &a.q, &s) == FO_OK);
        CHECK(fo_pool_admit(p, &b.q, &s) == FO_OK);
        CHECK(fo_pool_admit(p, &c.q, &s) == FO_OK);
        int32_t running = 0;
        CHECK(fo_pool_step(p, &running) == FO_OK && running == 3);
        int other[4] = {0, 0, 0, 0};
        std::thread t([&]() {
            int32_t x = -1;
            other[0] = fo_pool_step(p, &x);
            other[1] = fo_pool_wait(p, 0, &x);
            other[2] = fo_pool_release(p, 0);
            other[3] = fo_pool_destroy(p);
        });
        t.join();
        for (int k = 0; k < 4; ++k) CHECK(other[k] == FO_ERR_STATE);
        CHECK(fo_pool_destroy(p) == FO_OK);
        CHECK(a.u[0] != 0.0 && c.u[0] != 0.0);  // ran to completion
    }
    const int bad = stub_report();
    std::printf("driver: %d failed checks\n", g_fail);
    return (g_fail || bad) ? 1 : 0;
}

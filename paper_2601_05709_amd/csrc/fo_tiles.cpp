// Host construction of element tiles (see fo_tiles.h).
#include "fo_tiles.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace fo {

int tile_max_nodes(int dim) { return dim == 2 ? 1024 : 768; }
int tile_max_elems(int dim) { return dim == 2 ? 2048 : 3072; }

namespace {

// Spreads the low 21 bits of v so that bit k moves to bit 3k.
uint64_t spread3(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

uint64_t spread2(uint64_t v)
{
    v &= 0xffffffff;
    v = (v | v << 16) & 0x0000ffff0000ffffULL;
    v = (v | v << 8) & 0x00ff00ff00ff00ffULL;
    v = (v | v << 4) & 0x0f0f0f0f0f0f0f0fULL;
    v = (v | v << 2) & 0x3333333333333333ULL;
    v = (v | v << 1) & 0x5555555555555555ULL;
    return v;
}

}  // namespace

void build_tiles(int D, int64_t N, int64_t E, const double *X, const int32_t *conn, HostTiles *h)
{
    const int NV = D + 1;
    // 1. Morton order of element centroids in the bounding cube
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t n = 0; n < N; ++n)
        for (int i = 0; i < D; ++i) {
            lo[i] = std::min(lo[i], X[n * D + i]);
            hi[i] = std::max(hi[i], X[n * D + i]);
        }
    double ext = 0.0;
    for (int i = 0; i < D; ++i) ext = std::max(ext, hi[i] - lo[i]);
    if (!(ext > 0)) ext = 1.0;
    const double levels = D == 3 ? 2097151.0 : 4294967295.0;
    std::vector<uint64_t> key(E);
    for (int64_t e = 0; e < E; ++e) {
        double c[3] = {0, 0, 0};
        for (int a = 0; a < NV; ++a)
            for (int i = 0; i < D; ++i) c[i] += X[(int64_t)conn[a * E + e] * D + i];
        uint64_t q[3];
        for (int i = 0; i < D; ++i) {
            double t = (c[i] / NV - lo[i]) / ext;
            t = std::min(std::max(t, 0.0), 1.0);
            q[i] = (uint64_t)std::llround(t * levels);
        }
        key[e] = D == 3 ? (spread3(q[0]) | spread3(q[1]) << 1 | spread3(q[2]) << 2)
                        : (spread2(q[0]) | spread2(q[1]) << 1);
    }
    h->perm.resize(E);
    std::iota(h->perm.begin(), h->perm.end(), 0);
    std::stable_sort(h->perm.begin(), h->perm.end(),
                     [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    key.clear();
    key.shrink_to_fit();

    // 2. greedy tiles bounded by element and node counts
    const int max_n = tile_max_nodes(D), max_e = tile_max_elems(D);
    std::vector<int32_t> mark(N, -1);  // tile currently holding the node
    h->tile_elem_off.assign(1, 0);
    {
        int32_t tile = 0;
        int nn = 0, ne = 0;
        for (int64_t i = 0; i < E; ++i) {
            int32_t e = h->perm[i];
            int fresh = 0;
            for (int a = 0; a < NV; ++a)
                if (mark[conn[a * E + e]] != tile) ++fresh;
            if (ne > 0 && (ne + 1 > max_e || nn + fresh > max_n)) {
                h->tile_elem_off.push_back((int32_t)i);
                ++tile;
                nn = ne = 0;
            }
            for (int a = 0; a < NV; ++a) {
                int32_t n = conn[a * E + e];
                if (mark[n] != tile) {
                    mark[n] = tile;
                    ++nn;
                }
            }
            ++ne;
        }
        h->tile_elem_off.push_back((int32_t)E);
    }
    const int32_t T = (int32_t)h->tile_elem_off.size() - 1;
    h->n_tiles = T;

    // 3. how many tiles touch each node; owner = first tile touching it
    std::vector<int32_t> ntouch(N, 0);
    h->owner_tile.assign(N, -1);
    std::fill(mark.begin(), mark.end(), -1);
    for (int32_t t = 0; t < T; ++t)
        for (int32_t i = h->tile_elem_off[t]; i < h->tile_elem_off[t + 1]; ++i) {
            int32_t e = h->perm[i];
            for (int a = 0; a < NV; ++a) {
                int32_t n = conn[a * E + e];
                if (mark[n] != t) {
                    mark[n] = t;
                    ++ntouch[n];
                    if (h->owner_tile[n] < 0) h->owner_tile[n] = t;
                }
            }
        }

    // 4. per tile: local numbering (interior first), local conn, sub-batch slots
    h->tile_node_off.assign(1, 0);
    h->tile_node_interior.resize(T);
    h->tile_halo_off.resize(T);
    h->lconn.assign((size_t)E * 4, 0);
    h->lslot.assign((size_t)E * 4, 0);
    h->sub_off.assign(1, 0);
    h->seg_off.assign(1, 0);
    h->tile_nodes.clear();
    std::vector<int32_t> local(N, -1);
    std::vector<int32_t> inter, shared;
    int32_t halo_total = 0;
    h->max_nodes = 0;
    h->max_sub = 0;
    struct SlotKey {
        uint16_t node;
        uint16_t elem;
        uint8_t vert;
    };
    std::vector<SlotKey> keys;
    for (int32_t t = 0; t < T; ++t) {
        inter.clear();
        shared.clear();
        int32_t e0 = h->tile_elem_off[t], e1 = h->tile_elem_off[t + 1];
        for (int32_t i = e0; i < e1; ++i) {
            int32_t e = h->perm[i];
            for (int a = 0; a < NV; ++a) {
                int32_t n = conn[a * E + e];
                if (local[n] == -1) {
                    local[n] = -2;
                    (ntouch[n] == 1 ? inter : shared).push_back(n);
                }
            }
        }
        std::sort(inter.begin(), inter.end());
        std::sort(shared.begin(), shared.end());
        int32_t li = 0;
        for (int32_t n : inter) {
            local[n] = li++;
            h->tile_nodes.push_back(n);
        }
        for (int32_t n : shared) {
            local[n] = li++;
            h->tile_nodes.push_back(n);
        }
        h->tile_node_off.push_back((int32_t)h->tile_nodes.size());
        h->tile_node_interior[t] = (int32_t)inter.size();
        h->tile_halo_off[t] = halo_total;
        halo_total += (int32_t)shared.size();
        h->max_nodes = std::max(h->max_nodes, li);
        for (int32_t i = e0; i < e1; ++i) {
            int32_t e = h->perm[i];
            for (int a = 0; a < NV; ++a) h->lconn[(size_t)i * 4 + a] = (uint16_t)local[conn[a * E + e]];
        }
        int nsub = 0;
        for (int32_t s0 = e0; s0 < e1; s0 += kSub) {
            int32_t s1 = std::min(e1, s0 + kSub);
            keys.clear();
            for (int32_t i = s0; i < s1; ++i)
                for (int a = 0; a < NV; ++a)
                    keys.push_back({h->lconn[(size_t)i * 4 + a], (uint16_t)(i - s0), (uint8_t)a});
            std::sort(keys.begin(), keys.end(), [](const SlotKey &x, const SlotKey &y) {
                if (x.node != y.node) return x.node < y.node;
                if (x.elem != y.elem) return x.elem < y.elem;
                return x.vert < y.vert;
            });
            for (size_t k = 0; k < keys.size(); ++k) {
                h->lslot[(size_t)(s0 + keys[k].elem) * 4 + keys[k].vert] = (uint16_t)k;
                if (k == 0 || keys[k].node != keys[k - 1].node) {
                    h->seg_node.push_back(keys[k].node);
                    h->seg_start.push_back((uint16_t)k);
                }
            }
            h->seg_node.push_back(0xFFFF);  // sentinel: end of the last segment
            h->seg_start.push_back((uint16_t)keys.size());
            h->seg_off.push_back((int32_t)h->seg_node.size());
            ++nsub;
        }
        h->sub_off.push_back(h->sub_off.back() + nsub);
        h->max_sub = std::max(h->max_sub, nsub);
        for (int32_t n : inter) local[n] = -1;
        for (int32_t n : shared) local[n] = -1;
    }

    // 5. halo: each shared node sums its halo slots in tile order
    std::vector<int32_t> cnt(N, 0);
    for (int32_t t = 0; t < T; ++t)
        for (int32_t l = h->tile_node_interior[t]; l < h->tile_node_off[t + 1] - h->tile_node_off[t]; ++l)
            ++cnt[h->tile_nodes[h->tile_node_off[t] + l]];
    std::vector<int32_t> hidx(N, -1);
    h->halo_node.clear();
    for (int64_t n = 0; n < N; ++n)
        if (cnt[n] > 0) {
            hidx[n] = (int32_t)h->halo_node.size();
            h->halo_node.push_back((int32_t)n);
        }
    const int32_t S = (int32_t)h->halo_node.size();
    h->halo_ptr.assign(S + 1, 0);
    for (int32_t k = 0; k < S; ++k) h->halo_ptr[k + 1] = h->halo_ptr[k] + cnt[h->halo_node[k]];
    h->halo_src.assign(h->halo_ptr[S], 0);
    std::vector<int32_t> fill(h->halo_ptr.begin(), h->halo_ptr.end() - 1);
    for (int32_t t = 0; t < T; ++t) {
        int32_t base = h->tile_node_off[t];
        int32_t nint = h->tile_node_interior[t];
        int32_t nn = h->tile_node_off[t + 1] - base;
        for (int32_t l = nint; l < nn; ++l) {
            int32_t n = h->tile_nodes[base + l];
            h->halo_src[fill[hidx[n]]++] = h->tile_halo_off[t] + (l - nint);
        }
    }
}

}  // namespace fo

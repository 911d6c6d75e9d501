// Host construction of element tiles (see fo_tiles.h).
#include "fo_tiles.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace fo {

int tile_max_nodes(int dim) { return dim == 2 ? 512 : 320; }
int tile_max_elems(int dim) { return dim == 2 ? 512 : 512; }

int tile_target_elems(int dim, int64_t E, int cus)
{
    int64_t per = E / std::max<int64_t>(8 * (int64_t)std::max(cus, 1), 1);
    per = (per + 63) / 64 * 64;
    return (int)std::min<int64_t>(std::max<int64_t>(per, 128), tile_max_elems(dim));
}

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

// Stable order of the elements along a Morton curve of their centroids.
void morton_order(int D, int64_t N, int64_t E, const double *X, const int32_t *conn,
                  std::vector<int32_t> &perm)
{
    const int NV = D + 1;
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
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int32_t a, int32_t b) { return key[a] < key[b]; });
}

}  // namespace

void build_tiles(int D, int64_t N, int64_t E, const double *X, const int32_t *conn, int max_elems,
                 HostTiles *h, int max_nodes, bool presorted)
{
    const int NV = D + 1;
    h->perm.resize(E);
    std::iota(h->perm.begin(), h->perm.end(), 0);
    if (!presorted) morton_order(D, N, E, X, conn, h->perm);

    // greedy tiles bounded by element and node counts
    const int max_n = max_nodes > 0 ? std::min(max_nodes, 65535) : tile_max_nodes(D);
    const int max_e = max_nodes > 0 ? std::min(std::max(max_elems, 1), 16383)
                                    : std::min(std::max(max_elems, 1), tile_max_elems(D));
    std::vector<int32_t> mark(N, -1);  // tile currently holding the node
    h->tile_elem_off_tmp.assign(1, 0);
    {
        int32_t tile = 0;
        int nn = 0, ne = 0;
        for (int64_t i = 0; i < E; ++i) {
            int32_t e = h->perm[i];
            int fresh = 0;
            for (int a = 0; a < NV; ++a)
                if (mark[conn[a * E + e]] != tile) ++fresh;
            if (ne > 0 && (ne + 1 > max_e || nn + fresh > max_n)) {
                h->tile_elem_off_tmp.push_back((int32_t)i);
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
        h->tile_elem_off_tmp.push_back((int32_t)E);
    }
    const int32_t T = (int32_t)h->tile_elem_off_tmp.size() - 1;
    h->n_tiles = T;

    // how many tiles touch each node; owner = first tile touching it
    std::vector<int32_t> ntouch(N, 0), owner(N, -1);
    std::fill(mark.begin(), mark.end(), -1);
    for (int32_t t = 0; t < T; ++t)
        for (int32_t i = h->tile_elem_off_tmp[t]; i < h->tile_elem_off_tmp[t + 1]; ++i) {
            int32_t e = h->perm[i];
            for (int a = 0; a < NV; ++a) {
                int32_t n = conn[a * E + e];
                if (mark[n] != t) {
                    mark[n] = t;
                    ++ntouch[n];
                    if (owner[n] < 0) owner[n] = t;
                }
            }
        }

    // per tile: local numbering (interior, owned shared, other shared),
    //    local connectivity and node-sorted LDS slots (unpadded first)
    struct Tile {
        int32_t e0, ne, nint, nown;
        std::vector<int32_t> nodes;
        std::vector<uint16_t> seg;
    };
    std::vector<Tile> tiles(T);
    std::vector<uint16_t> lconn((size_t)E * 4, 0), lslot((size_t)E * 4, 0);
    std::vector<int32_t> local(N, -1);
    std::vector<int32_t> inter, own, other;
    h->max_nodes = 0;
    h->max_elems = 0;
    h->n_slots = 0;
    struct SlotKey {
        uint16_t node;
        uint16_t elem;
        uint8_t vert;
    };
    std::vector<SlotKey> keys;
    for (int32_t t = 0; t < T; ++t) {
        inter.clear();
        own.clear();
        other.clear();
        const int32_t e0 = h->tile_elem_off_tmp[t], e1 = h->tile_elem_off_tmp[t + 1];
        for (int32_t i = e0; i < e1; ++i) {
            int32_t e = h->perm[i];
            for (int a = 0; a < NV; ++a) {
                int32_t n = conn[a * E + e];
                if (local[n] == -1) {
                    local[n] = -2;
                    (ntouch[n] == 1 ? inter : owner[n] == t ? own : other).push_back(n);
                }
            }
        }
        std::sort(inter.begin(), inter.end());
        std::sort(own.begin(), own.end());
        std::sort(other.begin(), other.end());
        Tile &tl = tiles[t];
        tl.e0 = e0;
        tl.ne = e1 - e0;
        tl.nint = (int32_t)inter.size();
        tl.nown = (int32_t)(inter.size() + own.size());
        int32_t li = 0;
        for (const std::vector<int32_t> *grp : {&inter, &own, &other})
            for (int32_t n : *grp) {
                local[n] = li++;
                tl.nodes.push_back(n);
            }
        h->n_slots += li;
        h->max_nodes = std::max(h->max_nodes, li);
        h->max_elems = std::max(h->max_elems, tl.ne);
        keys.clear();
        for (int32_t i = e0; i < e1; ++i) {
            int32_t e = h->perm[i];
            for (int a = 0; a < NV; ++a) {
                uint16_t l = (uint16_t)local[conn[a * E + e]];
                lconn[(size_t)i * 4 + a] = l;
                keys.push_back({l, (uint16_t)(i - e0), (uint8_t)a});
            }
        }
        std::sort(keys.begin(), keys.end(), [](const SlotKey &x, const SlotKey &y) {
            if (x.node != y.node) return x.node < y.node;
            if (x.elem != y.elem) return x.elem < y.elem;
            return x.vert < y.vert;
        });
        // every tile node has at least one slot, so segments follow node order
        size_t k = 0;
        for (int32_t l = 0; l < li; ++l) {
            tl.seg.push_back((uint16_t)k);
            while (k < keys.size() && keys[k].node == l) {
                lslot[(size_t)(e0 + keys[k].elem) * 4 + keys[k].vert] = (uint16_t)k;
                ++k;
            }
        }
        tl.seg.push_back((uint16_t)k);  // sentinel
        for (int32_t n : tl.nodes) local[n] = -1;
    }

    // halo: node-major slots; each shared node owns a contiguous range that
    //    its tiles fill in tile order
    std::vector<int32_t> cnt(N, 0);
    for (int32_t t = 0; t < T; ++t)
        for (int32_t l = tiles[t].nint; l < (int32_t)tiles[t].nodes.size(); ++l) ++cnt[tiles[t].nodes[l]];
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
    h->node_hrange.assign((size_t)N * 2, -1);
    for (int32_t k = 0; k < S; ++k) {
        h->node_hrange[(size_t)h->halo_node[k] * 2] = h->halo_ptr[k];
        h->node_hrange[(size_t)h->halo_node[k] * 2 + 1] = h->halo_ptr[k + 1];
    }
    std::vector<int32_t> fill(h->halo_ptr.begin(), h->halo_ptr.end() - 1);

    // padded per-tile arrays
    const int64_t MN = h->max_nodes, ME = h->max_elems;
    h->info.assign((size_t)T * kTileInfo, 0);
    h->lconn.assign((size_t)T * ME * 4, 0);
    h->lslot.assign((size_t)T * ME * 4, 0);
    h->nodes.assign((size_t)T * MN, 0);
    h->seg.assign((size_t)T * (MN + 1), 0);
    h->hpos.assign((size_t)T * MN, -1);
    for (int32_t t = 0; t < T; ++t) {
        const Tile &tl = tiles[t];
        int32_t *inf = &h->info[(size_t)t * kTileInfo];
        inf[kTileE0] = tl.e0;
        inf[kTileNE] = tl.ne;
        inf[kTileNN] = (int32_t)tl.nodes.size();
        inf[kTileNInt] = tl.nint;
        inf[kTileNOwn] = tl.nown;
        for (int32_t i = 0; i < tl.ne; ++i)
            for (int a = 0; a < 4; ++a) {
                h->lconn[((size_t)t * ME + i) * 4 + a] = lconn[((size_t)tl.e0 + i) * 4 + a];
                h->lslot[((size_t)t * ME + i) * 4 + a] = lslot[((size_t)tl.e0 + i) * 4 + a];
            }
        for (size_t l = 0; l < tl.nodes.size(); ++l) {
            h->nodes[(size_t)t * MN + l] = tl.nodes[l];
            if ((int32_t)l >= tl.nint) h->hpos[(size_t)t * MN + l] = fill[hidx[tl.nodes[l]]]++;
        }
        for (size_t l = 0; l < tl.seg.size(); ++l) h->seg[(size_t)t * (MN + 1) + l] = tl.seg[l];
    }
    h->tile_elem_off_tmp.clear();
    h->tile_elem_off_tmp.shrink_to_fit();
}

}  // namespace fo

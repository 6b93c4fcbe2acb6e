// Tile and halo tables for the LDS-staged step kernel.
//
// Cells are processed in tiles of T consecutive cells (in the reordered
// index).  A workgroup stages its tile, the tile's first halo ring (face
// neighbours outside the tile) and second ring (face neighbours of the first
// ring outside tile and ring 1) in LDS, computes the gradients of the tile and
// ring-1 cells once, and reads neighbour values and gradients from LDS.  These
// tables map every slot of a tile cell and of a ring-1 cell to a local index.
#include <algorithm>
#include <cstring>

#include "fvlbm_internal.h"

namespace fvlbm {
namespace {
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

void build_tile_tables_host(const std::vector<int> &nb, int n, int nf, int np, int T, HostTiles &h) {
    h.T = T;
    h.n_tiles = (n + T - 1) / T;
    h.hmax = 0;
    h.h1max = 0;
    h.lnbr.assign((size_t)np * 4, (uint16_t)(int16_t)LN_PAD);
    h.hdr.assign((size_t)h.n_tiles * 4, 0);
    h.halo_idx.clear();
    h.halo_code.clear();
    std::vector<int> r1, r2;
    for (int t = 0; t < h.n_tiles; t++) {
        const int t0 = t * T, t1 = std::min(n, t0 + T);
        auto in_tile = [&](int j) { return j >= t0 && j < t1; };
        r1.clear();
        r2.clear();
        for (int i = t0; i < t1; i++)
            for (int k = 0; k < nf; k++) {
                int j = nb[(size_t)i * nf + k];
                if (j >= 0 && !in_tile(j)) r1.push_back(j);
            }
        std::sort(r1.begin(), r1.end());
        r1.erase(std::unique(r1.begin(), r1.end()), r1.end());
        auto in_r1 = [&](int j) { return std::binary_search(r1.begin(), r1.end(), j); };
        for (int c : r1)
            for (int k = 0; k < nf; k++) {
                int j = nb[(size_t)c * nf + k];
                if (j >= 0 && !in_tile(j) && !in_r1(j)) r2.push_back(j);
            }
        std::sort(r2.begin(), r2.end());
        r2.erase(std::unique(r2.begin(), r2.end()), r2.end());
        const int n1 = (int)r1.size(), n2 = (int)r2.size();
        auto local = [&](int j) -> int {
            if (in_tile(j)) return j - t0;
            auto p = std::lower_bound(r1.begin(), r1.end(), j);
            if (p != r1.end() && *p == j) return T + (int)(p - r1.begin());
            auto q = std::lower_bound(r2.begin(), r2.end(), j);
            return T + n1 + (int)(q - r2.begin());          // every 2-ring cell is staged
        };
        for (int i = t0; i < t1; i++)
            for (int k = 0; k < nf; k++) {
                int j = nb[(size_t)i * nf + k];
                int code = j >= 0 ? local(j) : (j == NB_PAD ? LN_PAD : j);
                h.lnbr[(size_t)i * 4 + k] = (uint16_t)(int16_t)code;
            }
        h.hdr[(size_t)t * 4 + 0] = (int)h.halo_idx.size();
        h.hdr[(size_t)t * 4 + 1] = n1;
        h.hdr[(size_t)t * 4 + 2] = n2;
        h.hdr[(size_t)t * 4 + 3] = (int)h.halo_code.size();
        for (int c : r1) h.halo_idx.push_back(c);
        for (int c : r2) h.halo_idx.push_back(c);
        for (int c : r1)
            for (int k = 0; k < nf; k++) {
                int j = nb[(size_t)c * nf + k];
                h.halo_code.push_back(j >= 0 ? local(j) : j);   // boundary group code or NB_PAD
            }
        h.hmax = std::max(h.hmax, n1 + n2);
        h.h1max = std::max(h.h1max, n1);
    }
}

fvlbm_status get_tiles(MeshDev &mesh, int T, const TileTables **out, std::string &err) {
    auto it = mesh.tiles.find(T);
    if (it != mesh.tiles.end()) {
        *out = &it->second;
        return FVLBM_OK;
    }
    HostTiles h;
    build_tile_tables_host(mesh.nbr_host, mesh.n_cells, mesh.nf, mesh.np, T, h);
    if (T + h.hmax >= 32767) { err = "tile halo too large for 16-bit local indices"; return FVLBM_E_MESH; }
    const std::vector<uint16_t> &lnbr = h.lnbr;
    const std::vector<int> &halo_ptr = h.hdr, &halo_idx = h.halo_idx, &halo_code = h.halo_code;
    TileTables tt;
    tt.T = T;
    tt.n_tiles = h.n_tiles;
    tt.hmax = h.hmax;
    tt.h1max = h.h1max;
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off = align256(off + b); return o; };
    size_t o_l = take(lnbr.size() * sizeof(uint16_t));
    size_t o_p = take(halo_ptr.size() * sizeof(int));
    size_t o_i = take(std::max<size_t>(1, halo_idx.size()) * sizeof(int));
    size_t o_c = take(std::max<size_t>(1, halo_code.size()) * sizeof(int));
    char *blk = nullptr;
    if (hipMalloc(&blk, off) != hipSuccess) { err = "device allocation of tile tables failed"; return FVLBM_E_NOMEM; }
    hipError_t e = hipMemcpy(blk + o_l, lnbr.data(), lnbr.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(blk + o_p, halo_ptr.data(), halo_ptr.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && !halo_idx.empty()) e = hipMemcpy(blk + o_i, halo_idx.data(), halo_idx.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && !halo_code.empty()) e = hipMemcpy(blk + o_c, halo_code.data(), halo_code.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) { hipFree(blk); err = "tile table upload failed"; return FVLBM_E_DEVICE; }
    tt.block = blk;
    tt.bytes = off;
    tt.lnbr = reinterpret_cast<uint2 *>(blk + o_l);
    tt.hdr = reinterpret_cast<int4 *>(blk + o_p);
    tt.halo_idx = reinterpret_cast<int *>(blk + o_i);
    tt.halo_code = reinterpret_cast<int *>(blk + o_c);
    auto res = mesh.tiles.emplace(T, tt);
    *out = &res.first->second;
    return FVLBM_OK;
}

void free_tiles(MeshDev &mesh) {
    for (auto &kv : mesh.tiles)
        if (kv.second.block) hipFree(kv.second.block);
    mesh.tiles.clear();
}

}  // namespace fvlbm

// Tile and halo tables for the LDS-staged step kernel.
//
// Cells are processed in tiles of T consecutive cells (in the reordered
// index).  A workgroup stages its tile, the tile's first halo ring (face
// neighbours outside the tile) and second ring (face neighbours of the first
// ring outside tile and ring 1) in LDS, computes the gradients of the tile and
// ring-1 cells once, and reads neighbour values and gradients from LDS.  These
// tables map every slot of a tile cell and of a ring-1 cell to a local index.
// Every tile gets the same number of ring slots (the largest over tiles), so a
// thread's halo cell sits at a fixed position: the kernel's first round of
// loads needs no per-tile header.
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
    h.h1max = 0;
    h.h2max = 0;
    std::vector<std::vector<int>> R1(h.n_tiles), R2(h.n_tiles);
    for (int t = 0; t < h.n_tiles; t++) {
        const int t0 = t * T, t1 = std::min(n, t0 + T);
        auto in_tile = [&](int j) { return j >= t0 && j < t1; };
        std::vector<int> &r1 = R1[t], &r2 = R2[t];
        for (int i = t0; i < t1; i++)
            for (int k = 0; k < nf; k++) {
                int j = nb[(size_t)i * nf + k];
                if (j >= 0 && !in_tile(j)) r1.push_back(j);
            }
        std::sort(r1.begin(), r1.end());
        r1.erase(std::unique(r1.begin(), r1.end()), r1.end());
        for (int c : r1)
            for (int k = 0; k < nf; k++) {
                int j = nb[(size_t)c * nf + k];
                if (j >= 0 && !in_tile(j) && !std::binary_search(r1.begin(), r1.end(), j)) r2.push_back(j);
            }
        std::sort(r2.begin(), r2.end());
        r2.erase(std::unique(r2.begin(), r2.end()), r2.end());
        h.h1max = std::max(h.h1max, (int)r1.size());
        h.h2max = std::max(h.h2max, (int)r2.size());
    }
    const int hs = h.h1max + h.h2max;
    h.lnbr.assign((size_t)np * 4, (uint16_t)(int16_t)LN_PAD);
    h.halo_idx.assign((size_t)h.n_tiles * hs, -1);
    h.halo_code.assign((size_t)h.n_tiles * h.h1max * 4, (uint16_t)(int16_t)LN_PAD);
    for (int t = 0; t < h.n_tiles; t++) {
        const int t0 = t * T, t1 = std::min(n, t0 + T);
        const std::vector<int> &r1 = R1[t], &r2 = R2[t];
        auto code = [&](int j) -> int {
            if (j == NB_PAD) return LN_PAD;
            if (j < 0) return j;                                   // boundary group -1-g
            if (j >= t0 && j < t1) return j - t0;
            auto p = std::lower_bound(r1.begin(), r1.end(), j);
            if (p != r1.end() && *p == j) return T + (int)(p - r1.begin());
            auto q = std::lower_bound(r2.begin(), r2.end(), j);   // every ring-2 cell is staged
            return T + h.h1max + (int)(q - r2.begin());
        };
        for (int i = t0; i < t1; i++)
            for (int k = 0; k < nf; k++) h.lnbr[(size_t)i * 4 + k] = (uint16_t)(int16_t)code(nb[(size_t)i * nf + k]);
        for (size_t k = 0; k < r1.size(); k++) {
            h.halo_idx[(size_t)t * hs + k] = r1[k];
            for (int s = 0; s < nf; s++)
                h.halo_code[((size_t)t * h.h1max + k) * 4 + s] = (uint16_t)(int16_t)code(nb[(size_t)r1[k] * nf + s]);
        }
        for (size_t k = 0; k < r2.size(); k++) h.halo_idx[(size_t)t * hs + h.h1max + k] = r2[k];
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
    if (T + h.h1max + h.h2max >= 32767) { err = "tile halo too large for 16-bit local indices"; return FVLBM_E_MESH; }
    TileTables tt;
    tt.T = T;
    tt.n_tiles = h.n_tiles;
    tt.h1max = h.h1max;
    tt.h2max = h.h2max;
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off = align256(off + std::max<size_t>(b, 16)); return o; };
    const size_t b_l = h.lnbr.size() * sizeof(uint16_t), b_i = h.halo_idx.size() * sizeof(int),
                 b_c = h.halo_code.size() * sizeof(uint16_t);
    const size_t o_l = take(b_l), o_i = take(b_i), o_c = take(b_c);
    char *blk = nullptr;
    if (hipMalloc(&blk, off) != hipSuccess) { err = "device allocation of tile tables failed"; return FVLBM_E_NOMEM; }
    hipError_t e = hipMemcpy(blk + o_l, h.lnbr.data(), b_l, hipMemcpyHostToDevice);
    if (e == hipSuccess && b_i) e = hipMemcpy(blk + o_i, h.halo_idx.data(), b_i, hipMemcpyHostToDevice);
    if (e == hipSuccess && b_c) e = hipMemcpy(blk + o_c, h.halo_code.data(), b_c, hipMemcpyHostToDevice);
    if (e != hipSuccess) { hipFree(blk); err = "tile table upload failed"; return FVLBM_E_DEVICE; }
    tt.block = blk;
    tt.bytes = off;
    tt.lnbr = reinterpret_cast<uint2 *>(blk + o_l);
    tt.halo_idx = reinterpret_cast<int *>(blk + o_i);
    tt.halo_code = reinterpret_cast<uint2 *>(blk + o_c);
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

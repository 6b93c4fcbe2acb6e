// Tile and halo tables for the LDS-staged step kernel.
//
// Cells are processed in tiles of T consecutive cells (in the reordered
// index).  A workgroup stages its tile and the tile's halo (face neighbours
// outside the tile) in LDS, computes every gradient once, and reads the
// neighbours' values and gradients from LDS.  These tables map each slot to a
// local LDS index; halo cells' own stencils (needed for their gradients) point
// to a local index when the neighbour is staged, else to the global cell.
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
    std::vector<uint16_t> &lnbr = h.lnbr;
    std::vector<int> &halo_ptr = h.halo_ptr, &halo_idx = h.halo_idx, &halo_code = h.halo_code;
    lnbr.assign((size_t)np * 4, (uint16_t)(int16_t)LN_PAD);
    halo_ptr.assign(h.n_tiles + 1, 0);
    halo_idx.clear();
    halo_code.clear();
    std::vector<int> halo;
    for (int t = 0; t < h.n_tiles; t++) {
        const int t0 = t * T, t1 = std::min(n, t0 + T);
        halo.clear();
        for (int i = t0; i < t1; i++)
            for (int k = 0; k < nf; k++) {
                int j = nb[(size_t)i * nf + k];
                if (j >= 0 && (j < t0 || j >= t1)) halo.push_back(j);
            }
        std::sort(halo.begin(), halo.end());
        halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
        auto local = [&](int j) -> int {       // local index of j, or -1 if not staged
            if (j >= t0 && j < t1) return j - t0;
            auto p = std::lower_bound(halo.begin(), halo.end(), j);
            if (p != halo.end() && *p == j) return T + (int)(p - halo.begin());
            return -1;
        };
        for (int i = t0; i < t1; i++)
            for (int k = 0; k < nf; k++) {
                int j = nb[(size_t)i * nf + k];
                int code = j >= 0 ? local(j) : (j == NB_PAD ? LN_PAD : j);
                lnbr[(size_t)i * 4 + k] = (uint16_t)(int16_t)code;
            }
        for (int h : halo) {
            halo_idx.push_back(h);
            for (int k = 0; k < nf; k++) {
                int j = nb[(size_t)h * nf + k];
                int code;
                if (j >= 0) {
                    int l = local(j);
                    code = l >= 0 ? l : LOCAL_LIM + j;
                } else {
                    code = j;                      // boundary group code or NB_PAD
                }
                halo_code.push_back(code);
            }
        }
        halo_ptr[t + 1] = (int)halo_idx.size();
        h.hmax = std::max(h.hmax, (int)halo.size());
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
    const std::vector<int> &halo_ptr = h.halo_ptr, &halo_idx = h.halo_idx, &halo_code = h.halo_code;
    TileTables tt;
    tt.T = T;
    tt.n_tiles = h.n_tiles;
    tt.hmax = h.hmax;
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
    tt.halo_ptr = reinterpret_cast<int *>(blk + o_p);
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

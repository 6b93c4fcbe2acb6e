// Sanitizer driver for the library's host mesh code (test infrastructure):
// topology, validation and every cell order, then the tile and halo tables at
// several tile sizes, on a raw mesh written by tests/test_sanitizers_cpu.py.
// Built for the host only with -fsanitize=address,undefined; a memory or
// undefined-behaviour error aborts with a report.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "fvlbm_internal.h"

template <class T>
static std::vector<T> rd(FILE *fp, size_t n) {
    std::vector<T> v(n);
    if (n && fread(v.data(), sizeof(T), n, fp) != n) { fprintf(stderr, "short mesh file\n"); exit(2); }
    return v;
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    int h[6];
    if (fread(h, sizeof(int), 6, fp) != 6) return 2;
    auto xy = rd<double>(fp, 2 * (size_t)h[0]);
    auto cptr = rd<int32_t>(fp, (size_t)h[1] + 1), cn = rd<int32_t>(fp, (size_t)h[2]);
    auto bfn = rd<int32_t>(fp, 2 * (size_t)h[3]), bfg = rd<int32_t>(fp, (size_t)h[3]);
    auto gk = rd<int32_t>(fp, (size_t)h[4]), gi = rd<int32_t>(fp, (size_t)h[4]);
    auto gu = rd<double>(fp, 2 * (size_t)h[4]), gr = rd<double>(fp, (size_t)h[4]);
    auto pp = rd<int32_t>(fp, 2 * (size_t)h[5]);
    auto ps = rd<double>(fp, 2 * (size_t)h[5]);
    fclose(fp);
    std::vector<fvlbm_bc> groups(h[4]);
    for (int g = 0; g < h[4]; g++) groups[g] = fvlbm_bc{gk[g], gi[g], {gu[2 * g], gu[2 * g + 1]}, gr[g]};
    int status = 0;
    for (int reorder = 0; reorder < 4; reorder++) {
        fvlbm::HostTopology topo;
        std::string err;
        const fvlbm_status st = fvlbm::build_topology(h[0], xy.data(), h[1], cptr.data(), cn.data(), h[3], bfn.data(),
                                                      bfg.data(), h[4], groups.data(), h[5], pp.data(), ps.data(),
                                                      reorder, topo, err);
        if (st != FVLBM_OK) {
            printf("reorder %d rejected (%d): %s\n", reorder, (int)st, err.c_str());
            status = 3;
            continue;
        }
        const int n = topo.n_cells, np = (n + 511) / 512 * 512;
        long slots = 0;
        for (int T : {64, 128, 192, 256, 384, 512}) {
            fvlbm::HostTiles tiles;
            fvlbm::build_tile_tables_host(topo.nbr, n, topo.nf, np, T, tiles);
            slots += (long)tiles.h1max + tiles.h2max;
        }
        printf("reorder %d cells %d nf %d halo slots %ld\n", reorder, n, topo.nf, slots);
    }
    return status;
}

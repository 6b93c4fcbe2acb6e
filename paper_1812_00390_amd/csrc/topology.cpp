// Host-side mesh topology: edge matching, boundary groups, periodic pairs,
// validation, and cell reordering (reverse Cuthill-McKee, Hilbert curve or
// recursive graph bisection) so that a wavefront's neighbour gathers stay
// within a few cache lines and a tile of consecutive cells has a short halo.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>
#include <unordered_map>

#include "fvlbm_internal.h"

namespace fvlbm {
namespace {

inline uint64_t edge_key(int a, int b) {
    uint32_t lo = (uint32_t)std::min(a, b), hi = (uint32_t)std::max(a, b);
    return ((uint64_t)lo << 32) | hi;
}

// d2xy inverse: position on a 2^order x 2^order Hilbert curve.
uint64_t hilbert_index(uint32_t x, uint32_t y, int order) {
    uint64_t d = 0;
    for (uint32_t s = 1u << (order - 1); s > 0; s >>= 1) {
        uint32_t rx = (x & s) ? 1 : 0;
        uint32_t ry = (y & s) ? 1 : 0;
        d += (uint64_t)s * s * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = s - 1 - x;
                y = s - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

std::vector<int> order_hilbert(const std::vector<double> &cx, const std::vector<double> &cy) {
    int n = (int)cx.size();
    double x0 = *std::min_element(cx.begin(), cx.end()), x1 = *std::max_element(cx.begin(), cx.end());
    double y0 = *std::min_element(cy.begin(), cy.end()), y1 = *std::max_element(cy.begin(), cy.end());
    double span = std::max(x1 - x0, y1 - y0);
    if (span <= 0) span = 1;
    const int order = 20;
    const double scale = (double)((1u << order) - 1) / span;
    std::vector<std::pair<uint64_t, int>> key(n);
    for (int i = 0; i < n; i++) {
        uint32_t hx = (uint32_t)((cx[i] - x0) * scale), hy = (uint32_t)((cy[i] - y0) * scale);
        key[i] = {hilbert_index(hx, hy, order), i};
    }
    std::sort(key.begin(), key.end());
    std::vector<int> perm(n);
    for (int i = 0; i < n; i++) perm[i] = key[i].second;
    return perm;
}

// Recursive graph bisection over the cell adjacency (CSR).  A part is split
// by the graph distances d1, d2 to the two ends p1, p2 of a pseudo-diameter:
// cells with smaller d1 - d2 (closer to p1) form the first half.  The cut is
// a level set of a graph coordinate, so both halves stay compact in graph
// distance whatever the cell aspect ratios, and every aligned block of 512
// (at the top levels) or 64 cells (below) is one compact part: tiles of
// consecutive cells get short halos.
class Bisector {
  public:
    Bisector(int n, const std::vector<int> &ptr, const std::vector<int> &adj)
        : n_(n), ptr_(ptr), adj_(adj), part_(n, -1), d1_(n, -1), d2_(n, -1) {}

    std::vector<int> order() {
        std::vector<int> cells(n_);
        std::iota(cells.begin(), cells.end(), 0);
        out_.reserve(n_);
        split(cells, 0);
        return out_;
    }

  private:
    // BFS distances from s within the current part; returns a farthest reached cell.
    int bfs(int s, int tag, std::vector<int> &dist, const std::vector<int> &cells) {
        for (int c : cells) dist[c] = -1;
        q_.clear();
        q_.push_back(s);
        dist[s] = 0;
        int last = s;
        for (size_t h = 0; h < q_.size(); h++) {
            const int c = q_[h];
            last = c;
            for (int e = ptr_[c]; e < ptr_[c + 1]; e++) {
                const int j = adj_[e];
                if (part_[j] == tag && dist[j] < 0) { dist[j] = dist[c] + 1; q_.push_back(j); }
            }
        }
        return last;
    }

    static int split_size(size_t m) {
        const size_t blk = m >= 1024 ? 512 : 64;
        size_t left = (m / 2 + blk / 2) / blk * blk;
        if (left < blk) left = blk;
        if (left >= m) left = m - 1;
        return (int)left;
    }

    void split(std::vector<int> &cells, int depth) {
        const int tag = ++tag_;
        for (int c : cells) part_[c] = tag;
        if (cells.size() > 1) {
            const int p1 = bfs(bfs(cells[0], tag, d1_, cells), tag, d1_, cells);
            int p2 = p1, far = -1;
            for (int c : cells)
                if (d1_[c] > far) { far = d1_[c]; p2 = c; }
            bfs(p2, tag, d2_, cells);
            // key: reached cells by d1 - d2, cells of other components last
            const long span = (long)n_ + 1;
            auto key = [&](int c) -> long {
                if (d1_[c] < 0 || d2_[c] < 0) return (2 * span + 1) * span + c;
                return ((long)(d1_[c] - d2_[c]) + span) * span + c;
            };
            if (cells.size() <= 64) {
                std::sort(cells.begin(), cells.end(), [&](int a, int b) { return key(a) < key(b); });
            } else {
                const int left = split_size(cells.size());
                std::nth_element(cells.begin(), cells.begin() + left, cells.end(),
                                 [&](int a, int b) { return key(a) < key(b); });
                std::vector<int> a(cells.begin(), cells.begin() + left), b(cells.begin() + left, cells.end());
                std::vector<int>().swap(cells);
                split(a, depth + 1);
                split(b, depth + 1);
                return;
            }
        }
        out_.insert(out_.end(), cells.begin(), cells.end());
    }

    int n_;
    const std::vector<int> &ptr_, &adj_;
    std::vector<int> part_, d1_, d2_, q_, out_;
    int tag_ = 0;
};

// Reverse Cuthill-McKee over the cell adjacency (CSR).
std::vector<int> order_rcm(int n, const std::vector<int> &adj_ptr, const std::vector<int> &adj) {
    std::vector<int> deg(n);
    for (int i = 0; i < n; i++) deg[i] = adj_ptr[i + 1] - adj_ptr[i];
    std::vector<char> seen(n, 0);
    std::vector<int> order;
    order.reserve(n);
    std::vector<int> level(n, -1);
    auto bfs_last = [&](int s) {    // returns a farthest cell of s's component
        std::vector<int> q{s};
        level[s] = 0;
        int last = s;
        for (size_t h = 0; h < q.size(); h++) {
            int c = q[h];
            last = c;
            for (int e = adj_ptr[c]; e < adj_ptr[c + 1]; e++)
                if (level[adj[e]] < 0) { level[adj[e]] = level[c] + 1; q.push_back(adj[e]); }
        }
        for (int c : q) level[c] = -1;
        return last;
    };
    for (int s0 = 0; s0 < n; s0++) {
        if (seen[s0]) continue;
        // pseudo-peripheral start: two sweeps of breadth-first search
        int s = bfs_last(bfs_last(s0));
        size_t head = order.size();
        order.push_back(s);
        seen[s] = 1;
        std::vector<int> nb;
        for (size_t h = head; h < order.size(); h++) {
            int c = order[h];
            nb.clear();
            for (int e = adj_ptr[c]; e < adj_ptr[c + 1]; e++)
                if (!seen[adj[e]]) { nb.push_back(adj[e]); seen[adj[e]] = 1; }
            std::sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

}  // namespace

fvlbm_status build_topology(int32_t n_nodes, const double *xy, int32_t n_cells,
                            const int32_t *cell_ptr, const int32_t *cell_nodes, int32_t n_bfaces,
                            const int32_t *bface_nodes, const int32_t *bface_group, int32_t n_groups,
                            const fvlbm_bc *groups, int32_t n_periodic,
                            const int32_t *periodic_pairs, const double *periodic_shift,
                            int32_t reorder, HostTopology &topo, std::string &err) {
    if (n_nodes <= 0 || !xy || n_cells <= 0 || !cell_ptr || !cell_nodes || n_bfaces < 0 ||
        (n_bfaces > 0 && (!bface_nodes || !bface_group)) || n_groups < 0 || n_groups > MAX_GROUPS ||
        (n_groups > 0 && !groups) || n_periodic < 0 ||
        (n_periodic > 0 && (!periodic_pairs || !periodic_shift)) || reorder < 0 || reorder > 3) {
        err = "bad arguments to fvlbm_create_mesh";
        return FVLBM_E_ARG;
    }
    if (cell_ptr[0] != 0) { err = "cell_ptr[0] must be 0"; return FVLBM_E_MESH; }
    int nf = 3;
    for (int c = 0; c < n_cells; c++) {
        int m = cell_ptr[c + 1] - cell_ptr[c];
        if (m < 3 || m > 4) { err = "cells must have 3 or 4 nodes"; return FVLBM_E_MESH; }
        if (m == 4) nf = 4;
        for (int k = 0; k < m; k++) {
            int v = cell_nodes[cell_ptr[c] + k];
            if (v < 0 || v >= n_nodes) { err = "cell node index out of range"; return FVLBM_E_MESH; }
        }
    }
    for (int g = 0; g < n_groups; g++) {
        if (groups[g].kind < FVLBM_BC_WALL || groups[g].kind > FVLBM_BC_SYMMETRY) { err = "unknown boundary kind"; return FVLBM_E_ARG; }
    }
    // convexity and orientation: every corner turns left
    for (int c = 0; c < n_cells; c++) {
        int p0 = cell_ptr[c], m = cell_ptr[c + 1] - p0;
        for (int k = 0; k < m; k++) {
            const double *a = &xy[2 * cell_nodes[p0 + (k + m - 1) % m]];
            const double *b = &xy[2 * cell_nodes[p0 + k]];
            const double *d = &xy[2 * cell_nodes[p0 + (k + 1) % m]];
            double cr = (b[0] - a[0]) * (d[1] - b[1]) - (b[1] - a[1]) * (d[0] - b[0]);
            if (!(cr > 0)) { err = "cell is not convex and counter-clockwise"; return FVLBM_E_MESH; }
        }
    }
    // edge matching (input order)
    const int MAXS = 4;
    std::vector<int> nbr_in((size_t)n_cells * MAXS, NB_PAD), back_in((size_t)n_cells * MAXS, -1);
    std::vector<double> shift_in((size_t)n_cells * MAXS * 2, 0.0);
    std::unordered_map<uint64_t, int> open;        // edge -> cell*MAXS + slot, awaiting a partner
    open.reserve((size_t)n_cells * 2);
    for (int c = 0; c < n_cells; c++) {
        int p0 = cell_ptr[c], m = cell_ptr[c + 1] - p0;
        for (int k = 0; k < m; k++) {
            uint64_t key = edge_key(cell_nodes[p0 + k], cell_nodes[p0 + (k + 1) % m]);
            auto it = open.find(key);
            if (it == open.end()) {
                open.emplace(key, c * MAXS + k);
            } else {
                int s = it->second;
                if (s < 0) { err = "edge shared by more than two cells"; return FVLBM_E_MESH; }
                nbr_in[(size_t)c * MAXS + k] = s / MAXS;
                back_in[(size_t)c * MAXS + k] = s % MAXS;
                nbr_in[s] = c;
                back_in[s] = k;
                it->second = -1;                    // closed
            }
        }
    }
    std::vector<int> bslot(n_bfaces, -1);
    for (int b = 0; b < n_bfaces; b++) {
        auto it = open.find(edge_key(bface_nodes[2 * b], bface_nodes[2 * b + 1]));
        if (it == open.end() || it->second < 0) { err = "boundary edge is not an open cell edge"; return FVLBM_E_MESH; }
        int s = it->second;
        bslot[b] = s;
        int g = bface_group[b];
        if (g >= n_groups || g < -1) { err = "boundary group index out of range"; return FVLBM_E_MESH; }
        if (g >= 0) nbr_in[s] = -1 - g;
    }
    for (int p = 0; p < n_periodic; p++) {
        int a = periodic_pairs[2 * p], b = periodic_pairs[2 * p + 1];
        if (a < 0 || b < 0 || a >= n_bfaces || b >= n_bfaces || a == b) { err = "periodic pair out of range"; return FVLBM_E_MESH; }
        int sa = bslot[a], sb = bslot[b];
        // the two edges must be congruent under the shift
        const double *pa0 = &xy[2 * bface_nodes[2 * a]], *pa1 = &xy[2 * bface_nodes[2 * a + 1]];
        const double *pb0 = &xy[2 * bface_nodes[2 * b]], *pb1 = &xy[2 * bface_nodes[2 * b + 1]];
        double sx = periodic_shift[2 * p], sy = periodic_shift[2 * p + 1];
        double mxa = 0.5 * (pa0[0] + pa1[0]), mya = 0.5 * (pa0[1] + pa1[1]);
        double mxb = 0.5 * (pb0[0] + pb1[0]) + sx, myb = 0.5 * (pb0[1] + pb1[1]) + sy;
        double la = std::hypot(pa1[0] - pa0[0], pa1[1] - pa0[1]);
        if (std::hypot(mxa - mxb, mya - myb) > 1e-9 * (la + std::hypot(sx, sy))) { err = "periodic edges do not match under the shift"; return FVLBM_E_MESH; }
        nbr_in[sa] = sb / MAXS; back_in[sa] = sb % MAXS;
        shift_in[2 * (size_t)sa] = sx; shift_in[2 * (size_t)sa + 1] = sy;
        nbr_in[sb] = sa / MAXS; back_in[sb] = sa % MAXS;
        shift_in[2 * (size_t)sb] = -sx; shift_in[2 * (size_t)sb + 1] = -sy;
    }
    for (int c = 0; c < n_cells; c++) {
        int m = cell_ptr[c + 1] - cell_ptr[c];
        for (int k = 0; k < m; k++)
            if (nbr_in[(size_t)c * MAXS + k] == NB_PAD) { err = "open boundary edge without a group or periodic partner"; return FVLBM_E_MESH; }
    }
    // reorder
    std::vector<int> perm(n_cells);
    std::iota(perm.begin(), perm.end(), 0);
    if (reorder == FVLBM_REORDER_RCM || reorder == FVLBM_REORDER_BISECT) {
        std::vector<int> ptr(n_cells + 1, 0), adj;
        adj.reserve((size_t)n_cells * 4);
        for (int c = 0; c < n_cells; c++) {
            for (int k = 0; k < MAXS; k++) {
                int j = nbr_in[(size_t)c * MAXS + k];
                if (j >= 0) adj.push_back(j);
            }
            ptr[c + 1] = (int)adj.size();
        }
        if (reorder == FVLBM_REORDER_RCM) perm = order_rcm(n_cells, ptr, adj);
        else perm = Bisector(n_cells, ptr, adj).order();
    } else if (reorder == FVLBM_REORDER_HILBERT) {
        std::vector<double> cx(n_cells), cy(n_cells);
        for (int c = 0; c < n_cells; c++) {
            int p0 = cell_ptr[c], m = cell_ptr[c + 1] - p0;
            double sx = 0, sy = 0;
            for (int k = 0; k < m; k++) { sx += xy[2 * cell_nodes[p0 + k]]; sy += xy[2 * cell_nodes[p0 + k] + 1]; }
            cx[c] = sx / m; cy[c] = sy / m;
        }
        perm = order_hilbert(cx, cy);
    }
    topo.n_cells = n_cells;
    topo.nf = nf;
    topo.perm = perm;
    topo.iperm.assign(n_cells, 0);
    for (int i = 0; i < n_cells; i++) topo.iperm[perm[i]] = i;
    topo.ncorner.assign(n_cells, 0);
    topo.corner_xy.assign((size_t)n_cells * nf * 2, 0.0);
    topo.nbr.assign((size_t)n_cells * nf, NB_PAD);
    topo.back.assign((size_t)n_cells * nf, -1);
    topo.shift.assign((size_t)n_cells * nf * 2, 0.0);
    topo.n_boundary_cells = 0;
    for (int i = 0; i < n_cells; i++) {
        int c = perm[i];
        int p0 = cell_ptr[c], m = cell_ptr[c + 1] - p0;
        topo.ncorner[i] = m;
        bool bnd = false;
        for (int k = 0; k < m; k++) {
            int v = cell_nodes[p0 + k];
            topo.corner_xy[((size_t)i * nf + k) * 2] = xy[2 * v];
            topo.corner_xy[((size_t)i * nf + k) * 2 + 1] = xy[2 * v + 1];
            int j = nbr_in[(size_t)c * MAXS + k];
            topo.nbr[(size_t)i * nf + k] = j >= 0 ? topo.iperm[j] : j;
            topo.back[(size_t)i * nf + k] = back_in[(size_t)c * MAXS + k];
            topo.shift[((size_t)i * nf + k) * 2] = shift_in[2 * ((size_t)c * MAXS + k)];
            topo.shift[((size_t)i * nf + k) * 2 + 1] = shift_in[2 * ((size_t)c * MAXS + k) + 1];
            if (j < 0) bnd = true;
        }
        topo.n_boundary_cells += bnd;
    }
    topo.bface_cell.assign(n_bfaces, -1);
    topo.bface_slot.assign(n_bfaces, -1);
    topo.bface_group.assign(bface_group, bface_group + n_bfaces);
    for (int b = 0; b < n_bfaces; b++) {
        topo.bface_cell[b] = topo.iperm[bslot[b] / MAXS];
        topo.bface_slot[b] = bslot[b] % MAXS;
    }
    return FVLBM_OK;
}

}  // namespace fvlbm

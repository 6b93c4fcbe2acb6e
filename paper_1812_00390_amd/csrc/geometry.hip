// FP64 geometry and least-squares precompute on the device (once per mesh).
//
// Per cell: area and area centroid (Section 2.2: f lives at the polygon's
// centre), bounding-box extents for the CFL length of Eq. 14.  Per face slot:
// outward unit normal, length, midpoint; the least-squares stencil point
// (neighbour centre or its periodic image, the wall-face centre P, or the
// ghost mirrored across the face line); the 2x2 weighted normal matrix of
// Eq. 12 with w = 1/|d|^2 and its inverse.  The streaming coefficients
// handed to the step kernels are rounded to FP32 only at the end.
#include <cmath>
#include <cstring>

#include "fvlbm_internal.h"

namespace fvlbm {
namespace {

__global__ void k_cell_geometry(int n, int nf, const int *__restrict__ ncorner,
                                const double *__restrict__ xy, double *__restrict__ cen,
                                double *__restrict__ area, double *__restrict__ cfl_len) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int m = ncorner[i];
    const double *p = xy + (size_t)i * nf * 2;
    // corners relative to corner 0: the cross products then carry the cell's
    // size, not its distance from the origin (a cell of 1e-5 at x = 1 would
    // otherwise keep only about seven digits of its area and centroid)
    const double bx = p[0], by = p[1];
    double a2 = 0, sx = 0, sy = 0;
    double x0 = 0, x1 = 0, y0 = 0, y1 = 0;
    for (int k = 0; k < m; k++) {
        int k1 = (k + 1 == m) ? 0 : k + 1;
        double xa = p[2 * k] - bx, ya = p[2 * k + 1] - by, xb = p[2 * k1] - bx, yb = p[2 * k1 + 1] - by;
        double cr = __dmul_rn(xa, yb) - __dmul_rn(xb, ya);
        a2 += cr;
        sx += (xa + xb) * cr;
        sy += (ya + yb) * cr;
        x0 = fmin(x0, xa); x1 = fmax(x1, xa);
        y0 = fmin(y0, ya); y1 = fmax(y1, ya);
    }
    area[i] = 0.5 * a2;
    cen[2 * i] = bx + sx / (3.0 * a2);
    cen[2 * i + 1] = by + sy / (3.0 * a2);
    cfl_len[i] = 0.5 * a2 / ((x1 - x0) + (y1 - y0));
}

// Compact FP32 per-cell description consumed by the step kernels:
//   v[k]   corner k minus the centroid (corners padded with corner 0 up to nf)
//   d[k]   least-squares stencil offset x_n - x_i of slot k (0 on padded slots)
// From these the kernels form 1/A (shoelace over the v[k]), the face midpoint
// offset (v_k + v_k+1)/2, the scaled normal rot(v_k+1 - v_k)/A = n dl / A, the
// least-squares matrix M = sum_k w_k d_k d_k^T with w_k = 1/|d_k|^2 and its
// inverse (Eq. 12; M is dimensionless and well scaled, so this is done in FP32
// in registers, which reads 16 B per cell less than storing M^-1 and 1/A), the
// gradient coefficient M^-1 w_k d_k, and the neighbour's offset to the face
// (midpoint - d_k).  Here M is formed in FP64 only to reject a singular
// stencil.
__global__ void k_face_coefficients(int n, int nf, int np, const int *__restrict__ ncorner,
                                    const double *__restrict__ xy, const int *__restrict__ nbr_in,
                                    const double *__restrict__ shift, const double *__restrict__ cen,
                                    const double *__restrict__ area, const int *__restrict__ gkind,
                                    float2 *__restrict__ vxy, float2 *__restrict__ dxy,
                                    int *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int m = ncorner[i];
    const double *p = xy + (size_t)i * nf * 2;
    const double cx = cen[2 * i], cy = cen[2 * i + 1];
    double m11 = 0, m12 = 0, m22 = 0;
    for (int k = 0; k < nf; k++) {
        size_t s = (size_t)k * np + i;
        int kc = k < m ? k : 0;           // padded corner repeats corner 0
        vxy[s] = make_float2((float)(p[2 * kc] - cx), (float)(p[2 * kc + 1] - cy));
        if (k >= m) {
            dxy[s] = make_float2(0.f, 0.f);
            continue;
        }
        int k1 = (k + 1 == m) ? 0 : k + 1;
        double ex = p[2 * k1] - p[2 * k], ey = p[2 * k1 + 1] - p[2 * k + 1];
        double len = sqrt(ex * ex + ey * ey);
        double nx = ey / len, ny = -ex / len;          // outward for CCW corners
        double fx = 0.5 * (p[2 * k] + p[2 * k1]), fy = 0.5 * (p[2 * k + 1] + p[2 * k1 + 1]);
        int code = nbr_in[(size_t)i * nf + k];
        double stx, sty;
        if (code >= 0) {
            stx = cen[2 * code] + shift[((size_t)i * nf + k) * 2];
            sty = cen[2 * code + 1] + shift[((size_t)i * nf + k) * 2 + 1];
        } else if (gkind[-1 - code] == FVLBM_BC_WALL) {
            stx = fx; sty = fy;                        // wall-face centre P
        } else {
            double dn = (fx - cx) * nx + (fy - cy) * ny;
            stx = cx + 2.0 * dn * nx; sty = cy + 2.0 * dn * ny;   // mirrored ghost
        }
        double dx = stx - cx, dy = sty - cy;
        double w = 1.0 / (dx * dx + dy * dy);
        m11 += w * dx * dx; m12 += w * dx * dy; m22 += w * dy * dy;
        dxy[s] = make_float2((float)dx, (float)dy);
    }
    double det = m11 * m22 - m12 * m12;
    double tr = m11 + m22;
    if (!(det > 1e-12 * tr * tr)) atomicOr(bad, 1);
}

__global__ void k_min_reduce(const double *__restrict__ v, int n, double *__restrict__ out) {
    __shared__ double sh[1024];
    double m = 1e300;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmin(m, v[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

fvlbm_status build_device_mesh(const HostTopology &topo, const fvlbm_bc *groups, int n_groups,
                               hipStream_t stream, MeshDev &mesh, std::string &err) {
    const int n = topo.n_cells, nf = topo.nf;
    const int np = (n + 511) / 512 * 512;
    mesh.n_cells = n; mesh.np = np; mesh.nf = nf; mesh.n_groups = n_groups;
    for (int g = 0; g < n_groups; g++) mesh.groups_host[g] = groups[g];
    mesh.n_boundary_cells = topo.n_boundary_cells;
    mesh.perm = topo.perm;

    // persistent arrays
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    size_t o_vxy = take((size_t)nf * np * sizeof(float2));
    size_t o_dxy = take((size_t)nf * np * sizeof(float2));
    size_t o_area = take((size_t)n * sizeof(double));
    size_t o_perm = take((size_t)n * sizeof(int));
    // boundary faces by group, the caller's order within each group
    std::vector<int2> gfaces;
    for (int g = 0; g < n_groups; g++) {
        mesh.gface_off[g] = (int)gfaces.size();
        for (size_t b = 0; b < topo.bface_group.size(); b++)
            if (topo.bface_group[b] == g) gfaces.push_back(make_int2(topo.bface_cell[b], topo.bface_slot[b]));
    }
    for (int g = n_groups; g <= MAX_GROUPS; g++) mesh.gface_off[g] = (int)gfaces.size();
    size_t o_gf = take(std::max<size_t>(1, gfaces.size()) * sizeof(int2));
    size_t total = off;
    char *blk = nullptr;
    if (hipMalloc(&blk, total) != hipSuccess) { err = "device allocation of mesh arrays failed"; return FVLBM_E_NOMEM; }
    mesh.block = blk; mesh.bytes = total;
    mesh.vxy = (float2 *)(blk + o_vxy);
    mesh.dxy = (float2 *)(blk + o_dxy);
    mesh.nbr_host = topo.nbr;
    mesh.area = (double *)(blk + o_area);
    mesh.perm_dev = (int *)(blk + o_perm);
    mesh.gfaces_dev = (int2 *)(blk + o_gf);

    // scratch for the FP64 pass
    size_t soff = 0;
    auto stake = [&](size_t bytes) { size_t o = soff; soff = align256(soff + bytes); return o; };
    size_t s_nc = stake((size_t)n * sizeof(int));
    size_t s_xy = stake((size_t)n * nf * 2 * sizeof(double));
    size_t s_nb = stake((size_t)n * nf * sizeof(int));
    size_t s_sh = stake((size_t)n * nf * 2 * sizeof(double));
    size_t s_cen = stake((size_t)n * 2 * sizeof(double));
    size_t s_cfl = stake((size_t)n * sizeof(double));
    size_t s_gk = stake(MAX_GROUPS * sizeof(int));
    size_t s_bad = stake(sizeof(int) + sizeof(double));
    char *scr = nullptr;
    if (hipMalloc(&scr, soff) != hipSuccess) { err = "device allocation of geometry scratch failed"; return FVLBM_E_NOMEM; }
    int gk[MAX_GROUPS] = {0};
    for (int g = 0; g < n_groups; g++) gk[g] = groups[g].kind;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    chk(hipMemcpyAsync(scr + s_nc, topo.ncorner.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, stream));
    chk(hipMemcpyAsync(scr + s_xy, topo.corner_xy.data(), (size_t)n * nf * 2 * sizeof(double), hipMemcpyHostToDevice, stream));
    chk(hipMemcpyAsync(scr + s_nb, topo.nbr.data(), (size_t)n * nf * sizeof(int), hipMemcpyHostToDevice, stream));
    chk(hipMemcpyAsync(scr + s_sh, topo.shift.data(), (size_t)n * nf * 2 * sizeof(double), hipMemcpyHostToDevice, stream));
    chk(hipMemcpyAsync(scr + s_gk, gk, sizeof(gk), hipMemcpyHostToDevice, stream));
    chk(hipMemsetAsync(scr + s_bad, 0, sizeof(int), stream));
    chk(hipMemcpyAsync(mesh.perm_dev, topo.perm.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, stream));
    if (!gfaces.empty())
        chk(hipMemcpyAsync(mesh.gfaces_dev, gfaces.data(), gfaces.size() * sizeof(int2), hipMemcpyHostToDevice, stream));
    // zero the padded tails of every plane so stray reads see finite values
    chk(hipMemsetAsync(blk, 0, o_area, stream));
    int nb = (n + 255) / 256;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_cell_geometry, dim3(nb), dim3(256), 0, stream, n, nf, (const int *)(scr + s_nc),
                           (const double *)(scr + s_xy), (double *)(scr + s_cen), mesh.area, (double *)(scr + s_cfl));
        chk(hipGetLastError());
        hipLaunchKernelGGL(k_face_coefficients, dim3(nb), dim3(256), 0, stream, n, nf, np,
                           (const int *)(scr + s_nc), (const double *)(scr + s_xy), (const int *)(scr + s_nb),
                           (const double *)(scr + s_sh), (const double *)(scr + s_cen), mesh.area,
                           (const int *)(scr + s_gk), mesh.vxy, mesh.dxy,
                           (int *)(scr + s_bad));
        chk(hipGetLastError());
        hipLaunchKernelGGL(k_min_reduce, dim3(1), dim3(1024), 0, stream, (const double *)(scr + s_cfl), n,
                           (double *)(scr + s_bad + 8));
        chk(hipGetLastError());
    }
    struct { int bad; int pad; double minlen; } res = {0, 0, 0};
    chk(hipMemcpyAsync(&res, scr + s_bad, sizeof(res), hipMemcpyDeviceToHost, stream));
    chk(hipStreamSynchronize(stream));
    hipFree(scr);
    if (e != hipSuccess) { err = std::string("HIP error in geometry pass: ") + hipGetErrorString(e); return FVLBM_E_DEVICE; }
    if (res.bad) { err = "singular least-squares stencil"; return FVLBM_E_MESH; }
    mesh.cfl_length = res.minlen;
    return FVLBM_OK;
}

}  // namespace fvlbm

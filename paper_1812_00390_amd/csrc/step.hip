// The FVLBM right-hand side and time-integrator update, fused per cell.
//
// One thread owns one cell and all nine directions.  Per RHS evaluation
// (paper Section 2.5, Steps 1-5):
//   Step 1/3  wall value f_P and ghost values f_GC of the cell's boundary
//             slots (Eqs. 18-22), from the cell's own current-stage state;
//   Step 2    least-squares gradient (Eq. 12) as sum_k c_k (phi_k - f_i),
//             with c_k = M^-1 w_k d_k precomputed in FP64;
//   Step 4    upwind face values (Eq. 11; border faces Eqs. 23-26): the
//             outgoing side uses the cell's own gradient, the incoming side
//             the upwind neighbour's gradient, which this thread recomputes
//             from the neighbour's stencil (a cell-centric gather: no atomics
//             and no gradient array in HBM);
//             flux sum over faces of (e.n dl/A) phi and the BGK source;
//   Step 5    dst = base + coef * RHS (Euler, and each stage of the
//             four-stage scheme), or the AB2 combination.
// Everything is computed on deviations h = f - f_eq(rho0, u_dev) in FP32,
// so the constant part of f never enters a flux difference; storage is FP32
// f, FP32 h, or FP16 h/(w S).
#include "fvlbm_internal.h"

namespace fvlbm {
namespace {

// D2Q9 (Eq. 2, c = 1) and weights (Eq. 4)
__device__ constexpr int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr float WT[Q] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                                    1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};

// ---------------------------------------------------------------- rounding
//
// Every state store rounds without bias: the new value's exact residual is
// carried (two-product / two-sum), and the stored neighbour is picked with
// probability proportional to the distance, driven by a hash of the value's
// own bits and the slot index.  Round-to-nearest would drop every increment
// smaller than half an ulp, so a run can freeze short of its steady state
// (FP32) or drift (FP16); unbiased rounding keeps the expected increment.
// The hash makes the rounding a pure function of (value, cell, direction):
// results do not depend on launch order, schedule, batching or graphs.

__device__ inline uint32_t mix32(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352dU;
    x ^= x >> 15; x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

struct Exact {
    float s, e;   // value = s + e, |e| <= ulp(s)/2 (approximately)
};

// b + c * r with its residual
__device__ inline Exact fma_exact(float c, float r, float b) {
#pragma clang fp contract(off)
    const float p = c * r;
    const float pe = fmaf(c, r, -p);
    const float s = b + p;
    const float bb = s - b;
    const float e = (b - (s - bb)) + (p - bb);
    return {s, e + pe};
}

// a + x with its residual (x carries its own residual xe)
__device__ inline Exact add_exact(float a, Exact x) {
#pragma clang fp contract(off)
    const float s = a + x.s;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (x.s - bb);
    return {s, e + x.e};
}

__device__ inline float unit_random(uint32_t h) { return (float)(h >> 8) * (1.0f / 16777216.0f); }

// unbiased rounding of s + e to FP32
__device__ inline float round_fp32(Exact v, uint32_t salt) {
    if (v.e == 0.f) return v.s;
    const float nb = nextafterf(v.s, v.e > 0.f ? INFINITY : -INFINITY);
    const float gap = fabsf(nb - v.s);
    const uint32_t h = mix32(__float_as_uint(v.e) ^ mix32(__float_as_uint(v.s) ^ salt));
    return unit_random(h) * gap < fabsf(v.e) ? nb : v.s;
}

// unbiased rounding of a float to FP16: add 13 random bits below the FP16
// mantissa, then truncate (exact for FP16 normals)
__device__ inline __half round_fp16(float v, uint32_t salt) {
    const uint32_t b = __float_as_uint(v);
    const uint32_t h = mix32(b ^ mix32(salt));
    const uint32_t mag = (b & 0x7fffffffu) + (h & 0x1fffu);
    return __float2half_rz(__uint_as_float((b & 0x80000000u) | mag));
}

template <int STORE>
struct Storage;

template <>
struct Storage<FVLBM_STORE_FP32> {
    __device__ static float load(const void *p, size_t idx, int a, const RefDev &r) {
        return static_cast<const float *>(p)[idx] - r.fref[a];
    }
    __device__ static void store(void *p, size_t idx, int a, Exact h, const RefDev &r, uint32_t salt) {
        static_cast<float *>(p)[idx] = round_fp32(add_exact(r.fref[a], h), salt);
    }
};
template <>
struct Storage<FVLBM_STORE_FP32_DEV> {
    __device__ static float load(const void *p, size_t idx, int, const RefDev &) {
        return static_cast<const float *>(p)[idx];
    }
    __device__ static void store(void *p, size_t idx, int, Exact h, const RefDev &, uint32_t salt) {
        static_cast<float *>(p)[idx] = round_fp32(h, salt);
    }
};
template <>
struct Storage<FVLBM_STORE_FP16_DEV> {
    __device__ static float load(const void *p, size_t idx, int a, const RefDev &r) {
        return __half2float(static_cast<const __half *>(p)[idx]) * (WT[a] * r.scale);
    }
    __device__ static void store(void *p, size_t idx, int a, Exact h, const RefDev &r, uint32_t salt) {
        static_cast<__half *>(p)[idx] = round_fp16((h.s + h.e) / (WT[a] * r.scale), salt);
    }
};

constexpr int NO_CELL = 0x7fffffff;   // matches no neighbour-slot code

struct Macro {
    float drho, rho;   // rho - rho0, rho
    float jx, jy;      // momentum rho u
    float ux, uy;
};

// Eq. 5 on deviations h = f - f_eq(rho0, u_dev): rho = rho0 + sum h, rho u = rho0 u_dev + sum e h.
__device__ inline Macro moments(const float h[Q], const RefDev &r) {
    Macro m;
    float s = 0.f, mx = 0.f, my = 0.f;
#pragma unroll
    for (int a = 0; a < Q; a++) {
        s += h[a];
        if (EX[a]) mx += EX[a] * h[a];
        if (EY[a]) my += EY[a] * h[a];
    }
    m.drho = s;
    m.rho = r.rho0 + s;
    m.jx = r.jx0 + mx;
    m.jy = r.jy0 + my;
    const float ir = 1.f / m.rho;
    m.ux = m.jx * ir;
    m.uy = m.jy * ir;
    return m;
}

// Eq. 3 as a deviation from the reference equilibrium, written with the momentum j = rho u:
// f_eq(rho, u) - f_eq(rho0, u_dev) = w [ (rho - rho0) + 3 e.(j - j0) + (4.5 (e.j)^2 - 1.5 |j|^2)/rho - c0 ]
__device__ inline void heq(float drho, float rho, float jx, float jy, const RefDev &r, float out[Q]) {
    const float ir = 1.f / rho;
    const float jj = 1.5f * (jx * jx + jy * jy);
    const float dx = jx - r.jx0, dy = jy - r.jy0;
#pragma unroll
    for (int a = 0; a < Q; a++) {
        const float ej = EX[a] * jx + EY[a] * jy;
        const float ed = EX[a] * dx + EY[a] * dy;
        out[a] = WT[a] * (drho + 3.f * ed + (4.5f * ej * ej - jj) * ir - r.c0[a]);
    }
}

// Boundary stencil value of a cell's boundary slot (Eqs. 18-22), deviation form.
__device__ inline void boundary_value(const GroupDev &g, const float h[Q], const Macro &m,
                                      const float heq_c[Q], float2 gn, const RefDev &r, float out[Q]) {
    float e[Q];
    switch (g.kind) {
    case FVLBM_BC_WALL:                 // Eq. 18: f_eq(rho_k, u_w) + f_k - f_eq,k
        heq(m.drho, m.rho, m.rho * g.ux, m.rho * g.uy, r, e);
#pragma unroll
        for (int a = 0; a < Q; a++) out[a] = e[a] + (h[a] - heq_c[a]);
        break;
    case FVLBM_BC_INLET: {              // Eq. 19: rho* = rho_inf (external) or rho_k (internal)
        const float dr = g.internal ? m.drho : g.drho;
        const float rs = g.internal ? m.rho : g.rho;
        heq(dr, rs, rs * g.ux, rs * g.uy, r, e);
#pragma unroll
        for (int a = 0; a < Q; a++) out[a] = e[a] + (h[a] - heq_c[a]);
        break;
    }
    case FVLBM_BC_OUTLET:
        if (!g.internal) {              // Eq. 20: f_GC = f_i
#pragma unroll
            for (int a = 0; a < Q; a++) out[a] = h[a];
        } else {                        // Eq. 21: f_eq(rho_inf, u_i) + f_k - f_eq,k
            heq(g.drho, g.rho, g.rho * m.ux, g.rho * m.uy, r, e);
#pragma unroll
            for (int a = 0; a < Q; a++) out[a] = e[a] + (h[a] - heq_c[a]);
        }
        break;
    default: {                          // Eq. 22: mirrored normal velocity
        const float il = rsqrtf(gn.x * gn.x + gn.y * gn.y);
        const float nx = gn.x * il, ny = gn.y * il;
        const float jn = m.jx * nx + m.jy * ny;
        heq(m.drho, m.rho, m.jx - 2.f * jn * nx, m.jy - 2.f * jn * ny, r, out);
        break;
    }
    }
}

template <int NF, int STORE>
struct Cell {
    // Gradient of cell c (Eq. 12) given its own deviations hc.  If one
    // neighbour's deviations are already in registers (known, hk) they are reused.
    __device__ static void gradient(const InstDesc &d, int c, const float hc[Q], int known,
                                    const float hk[Q], float gx[Q], float gy[Q]) {
#pragma unroll
        for (int a = 0; a < Q; a++) { gx[a] = 0.f; gy[a] = 0.f; }
        bool have_m = false;
        Macro m;
        float he[Q];
#pragma unroll
        for (int k = 0; k < NF; k++) {
            const size_t s = (size_t)k * d.np + c;
            const int j = d.nbr[s];
            if (NF == 4 && j == NB_PAD) continue;
            const float2 w = d.cg[s];
            float phi[Q];
            if (j == known) {
#pragma unroll
                for (int a = 0; a < Q; a++) phi[a] = hk[a];
            } else if (j >= 0) {
#pragma unroll
                for (int a = 0; a < Q; a++)
                    phi[a] = Storage<STORE>::load(d.src, (size_t)a * d.np + j, a, d.ref);
            } else {
                if (!have_m) {
                    m = moments(hc, d.ref);
                    heq(m.drho, m.rho, m.jx, m.jy, d.ref, he);
                    have_m = true;
                }
                boundary_value(d.groups[-1 - j], hc, m, he, d.gn[s], d.ref, phi);
            }
#pragma unroll
            for (int a = 0; a < Q; a++) {
                float df = phi[a] - hc[a];
                gx[a] = fmaf(w.x, df, gx[a]);
                gy[a] = fmaf(w.y, df, gy[a]);
            }
        }
    }
};

__device__ inline int remap_block(int b, int nb, int xcd_remap) {
    // Blocks are dispatched round-robin over the 8 XCDs; renumber them so that
    // each XCD walks one contiguous range of tiles (neighbour gathers then hit
    // that XCD's L2).
    if (!xcd_remap) return b;
    const int x = b & 7, r = b >> 3;
    const int per = nb >> 3, extra = nb & 7;
    // XCD x owns per (+1 for x < extra) consecutive logical blocks
    return x * per + (x < extra ? x : extra) + r;
}

template <int NF, int STORE>
__global__ void __launch_bounds__(512) k_stage(const InstDesc *__restrict__ descs,
                                               const int2 *__restrict__ units, int n_units,
                                               int xcd_remap) {
    const int lb = remap_block(blockIdx.x, n_units, xcd_remap);
    const int2 u = units[lb];
    const InstDesc &d = descs[u.x];
    const int i = u.y + threadIdx.x;
    if (i >= d.n_cells) return;
    float hi[Q];
#pragma unroll
    for (int a = 0; a < Q; a++) hi[a] = Storage<STORE>::load(d.src, (size_t)a * d.np + i, a, d.ref);
    const Macro mi = moments(hi, d.ref);
    float hei[Q];
    heq(mi.drho, mi.rho, mi.jx, mi.jy, d.ref, hei);

    float gxi[Q], gyi[Q];
    Cell<NF, STORE>::gradient(d, i, hi, NO_CELL, hi, gxi, gyi);

    float acc[Q];
#pragma unroll
    for (int a = 0; a < Q; a++) acc[a] = 0.f;

#pragma unroll
    for (int k = 0; k < NF; k++) {
        const size_t s = (size_t)k * d.np + i;
        const int j = d.nbr[s];
        if (NF == 4 && j == NB_PAD) continue;
        const float2 g = d.gn[s];
        const float2 r = d.rf[s];
        if (j >= 0) {
            float hj[Q], gxj[Q], gyj[Q];
#pragma unroll
            for (int a = 0; a < Q; a++)
                hj[a] = Storage<STORE>::load(d.src, (size_t)a * d.np + j, a, d.ref);
            Cell<NF, STORE>::gradient(d, j, hj, i, hi, gxj, gyj);
            const float2 q = d.rj[s];
#pragma unroll
            for (int a = 1; a < Q; a++) {
                const float en = EX[a] * g.x + EY[a] * g.y;
                const float own = fmaf(gyi[a], r.y, fmaf(gxi[a], r.x, hi[a]));
                const float nb = fmaf(gyj[a], q.y, fmaf(gxj[a], q.x, hj[a]));
                acc[a] = fmaf(en, en > 0.f ? own : nb, acc[a]);
            }
        } else {
            const GroupDev &gr = d.groups[-1 - j];
            float bv[Q];
            boundary_value(gr, hi, mi, hei, g, d.ref, bv);
            const bool upwind = gr.kind == FVLBM_BC_INLET || (gr.kind == FVLBM_BC_OUTLET && gr.internal);
#pragma unroll
            for (int a = 1; a < Q; a++) {
                const float en = EX[a] * g.x + EY[a] * g.y;
                float phi;
                if (gr.kind == FVLBM_BC_WALL) {
                    phi = bv[a];
                } else if (upwind) {
                    phi = en > 0.f ? fmaf(gyi[a], r.y, fmaf(gxi[a], r.x, hi[a])) : bv[a];
                } else if (gr.kind == FVLBM_BC_OUTLET) {
                    phi = hi[a];
                } else {
                    phi = 0.5f * (hi[a] + bv[a]);
                }
                acc[a] = fmaf(en, phi, acc[a]);
            }
        }
    }

    // RHS = -sum (e.n dl/A) phi - (f - f_eq)/tau  (Eq. 10), then the update.
#pragma unroll
    for (int a = 0; a < Q; a++) {
        const float rhs = -acc[a] - (hi[a] - hei[a]) * d.inv_tau;
        const size_t idx = (size_t)a * d.np + i;
        const uint32_t salt = (uint32_t)i * 9u + (uint32_t)a;
        Exact out;
        if (d.mode == 0) {
            const float b = (d.base == d.src) ? hi[a] : Storage<STORE>::load(d.base, idx, a, d.ref);
            out = fma_exact(d.coef, rhs, b);
        } else if (d.mode == 3) {
            static_cast<float *>(d.dst)[idx] = rhs;
            continue;
        } else {
            const float prev = (d.mode == 1) ? rhs : d.rhs_prev[idx];
            out = fma_exact(0.5f * d.coef, 3.f * rhs - prev, hi[a]);
            d.rhs_prev[idx] = rhs;
        }
        Storage<STORE>::store(d.dst, idx, a, out, d.ref, salt);
    }
}

template <int NF, int STORE>
const void *stage_fn() { return reinterpret_cast<const void *>(&k_stage<NF, STORE>); }

const void *pick(int nf, int storage) {
    if (nf == 3) {
        if (storage == FVLBM_STORE_FP32) return stage_fn<3, FVLBM_STORE_FP32>();
        if (storage == FVLBM_STORE_FP32_DEV) return stage_fn<3, FVLBM_STORE_FP32_DEV>();
        return stage_fn<3, FVLBM_STORE_FP16_DEV>();
    }
    if (storage == FVLBM_STORE_FP32) return stage_fn<4, FVLBM_STORE_FP32>();
    if (storage == FVLBM_STORE_FP32_DEV) return stage_fn<4, FVLBM_STORE_FP32_DEV>();
    return stage_fn<4, FVLBM_STORE_FP16_DEV>();
}

}  // namespace

hipError_t launch_stage(const InstDesc *descs_dev, const UnitTable &ut, int nf, int storage,
                        int xcd_remap, hipStream_t stream) {
    if (ut.n_units == 0) return hipSuccess;
    const int2 *units = ut.units;
    int n_units = ut.n_units;
    void *args[] = {(void *)&descs_dev, (void *)&units, (void *)&n_units, (void *)&xcd_remap};
    return hipLaunchKernel(pick(nf, storage), dim3(ut.n_units), dim3(ut.block), args, 0, stream);
}

hipError_t add_stage_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, int ndeps,
                          const InstDesc *descs_dev, const UnitTable &ut, int nf, int storage,
                          int xcd_remap, void **argbuf) {
    // argbuf: caller-owned storage for the 4 argument values, alive until the graph is instantiated
    struct Args { const InstDesc *d; const int2 *u; int n; int x; };
    Args *a = reinterpret_cast<Args *>(argbuf[0]);
    a->d = descs_dev; a->u = ut.units; a->n = ut.n_units; a->x = xcd_remap;
    void **kp = argbuf + 1;
    kp[0] = &a->d; kp[1] = &a->u; kp[2] = &a->n; kp[3] = &a->x;
    hipKernelNodeParams p{};
    p.func = const_cast<void *>(pick(nf, storage));
    p.gridDim = dim3(ut.n_units);
    p.blockDim = dim3(ut.block);
    p.sharedMemBytes = 0;
    p.kernelParams = kp;
    p.extra = nullptr;
    return hipGraphAddKernelNode(node, g, deps, ndeps, &p);
}

}  // namespace fvlbm

// The FVLBM right-hand side and time-integrator update, fused per tile.
//
// A workgroup owns a tile of consecutive cells (one thread per cell, all nine
// directions per thread) and stages the tile and two rings of face-neighbour
// halo in LDS.  Per RHS evaluation (paper Section 2.5, Steps 1-5):
//   Step 1/3  wall value f_P and ghost values f_GC of a cell's boundary
//             slots (Eqs. 18-22), from that cell's own current-stage state;
//   Step 2    least-squares gradient (Eq. 12) as sum_k M^-1 w_k d_k (phi_k - f_i)
//             for every tile and ring-1 cell, once, into LDS;
//   Step 4    upwind face values (Eq. 11; border faces Eqs. 23-26): the
//             outgoing side from the cell's own gradient, the incoming side
//             from the neighbour's staged value and gradient (a cell-centric
//             gather: no atomics and no gradient array in HBM); flux sum over
//             faces of (e.n dl/A) phi and the BGK source;
//   Step 5    dst = base + coef * RHS (Euler, and each stage of the
//             four-stage scheme), or the AB2 combination.
// Everything is computed on deviations h = f - f_eq(rho0, u_dev) in FP32,
// so the constant part of f never enters a flux difference; storage is FP32
// f, FP32 h, or FP16 h/(w S).
#include "fvlbm_internal.h"

// No implicit contraction: every fused multiply-add below is written as fmaf,
// so every kernel variant (tile size, persistent or not, batched or not)
// performs the same roundings and results are bitwise independent of the
// launch schedule.
#pragma clang fp contract(off)

namespace fvlbm {
namespace {

// D2Q9 (Eq. 2, c = 1) and weights (Eq. 4)
__device__ constexpr int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr float WT[Q] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                                    1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};

// ---------------------------------------------------------------- memory
//
// The descriptor's pointers are read from memory, so the compiler cannot
// infer their address space and would emit FLAT instructions (which also
// count against the LDS wait counter).  Every device-memory access goes
// through these global-address-space accessors instead.
#if defined(__HIP_DEVICE_COMPILE__)
#define FVLBM_GLOBAL_AS __attribute__((address_space(1)))   // the device pass only; the host pass never runs these
#else
#define FVLBM_GLOBAL_AS
#endif
template <class T>
__device__ inline T ldg(const T *p, size_t i) {
    return ((const FVLBM_GLOBAL_AS T *)p)[i];
}
template <class T>
__device__ inline void stg(T *p, size_t i, T v) {
    ((FVLBM_GLOBAL_AS T *)p)[i] = v;
}

__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------- rounding
//
// Every state store rounds without bias: the new value's residual is carried
// (Fast2Sum), and the stored neighbour is picked with probability
// proportional to the distance, driven by a multiplicative hash of the
// value's own bits and the slot index.  Round-to-nearest would drop every increment
// smaller than half an ulp, so a run can freeze short of its steady state
// (FP32) or drift (FP16); unbiased rounding keeps the expected increment.
// The hash makes the rounding a pure function of (value, cell, direction):
// results do not depend on launch order, schedule, batching or graphs.

struct Exact {
    float s, e;   // value = s + e, |e| <= ulp(s)/2 (approximately)
};

// b + c * r with its residual: the increment p = c r is rounded once (its
// error is far below an ulp of the sum), then Fast2Sum; when |p| > |b| the
// residual is only approximate, which leaves the rounding nearly unbiased.
__device__ inline Exact fma_exact(float c, float r, float b) {
#pragma clang fp contract(off)
    const float p = c * r;
    const float s = b + p;
    return {s, p - (s - b)};
}

// a + x with its residual (x carries its own residual)
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
    // neighbour of s in the direction of e (s is finite and, as |e| <= ulp(s)/2, nonzero)
    const uint32_t bs = __float_as_uint(v.s);
    const bool up_mag = (v.e > 0.f) == (v.s > 0.f);
    const float nb = __uint_as_float(up_mag ? bs + 1u : bs - 1u);
    const float gap = fabsf(nb - v.s);
    uint32_t h = (__float_as_uint(v.e) ^ (__float_as_uint(v.s) * 0x9e3779b1u) ^ salt) * 0x85ebca6bu;
    h ^= h >> 15;
    return unit_random(h) * gap < fabsf(v.e) ? nb : v.s;
}

// unbiased rounding of a float to FP16: add 13 random bits below the FP16
// mantissa, then truncate (exact for FP16 normals)
__device__ inline __half round_fp16(float v, uint32_t salt) {
    const uint32_t b = __float_as_uint(v);
    uint32_t h = (b ^ (salt * 0x9e3779b1u)) * 0x85ebca6bu;
    h ^= h >> 15;
    const uint32_t mag = (b & 0x7fffffffu) + (h & 0x1fffu);
    return __float2half_rz(__uint_as_float((b & 0x80000000u) | mag));
}

template <int STORE>
struct Storage;

template <>
struct Storage<FVLBM_STORE_FP32> {
    __device__ static float load(const void *p, size_t idx, int a, const RefDev &r) {
        return ldg(static_cast<const float *>(p), idx) - r.fref[a];
    }
    __device__ static void store(void *p, size_t idx, int a, Exact h, const RefDev &r, uint32_t salt) {
        stg(static_cast<float *>(p), idx, round_fp32(add_exact(r.fref[a], h), salt));
    }
};
template <>
struct Storage<FVLBM_STORE_FP32_DEV> {
    __device__ static float load(const void *p, size_t idx, int, const RefDev &) {
        return ldg(static_cast<const float *>(p), idx);
    }
    __device__ static void store(void *p, size_t idx, int, Exact h, const RefDev &, uint32_t salt) {
        stg(static_cast<float *>(p), idx, round_fp32(h, salt));
    }
};
template <>
struct Storage<FVLBM_STORE_FP16_DEV> {
    __device__ static float load(const void *p, size_t idx, int a, const RefDev &r) {
        const __half v = ldg(static_cast<const __half *>(p), idx);
        return __half2float(v) * (WT[a] * r.scale);
    }
    __device__ static void store(void *p, size_t idx, int a, Exact h, const RefDev &r, uint32_t salt) {
        stg(static_cast<__half *>(p), idx, round_fp16((h.s + h.e) * r.inv_unit[a], salt));
    }
};

// e_a . (x, y) for the D2Q9 velocities, folded per direction (no products by 0)
__device__ __forceinline__ float edot(int a, float x, float y) {
    switch (a) {
    case 0: return 0.f;
    case 1: return x;
    case 2: return y;
    case 3: return -x;
    case 4: return -y;
    case 5: return x + y;
    case 6: return y - x;
    case 7: return -x - y;
    default: return x - y;
    }
}

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
    const float ir = frcp(m.rho);
    m.ux = m.jx * ir;
    m.uy = m.jy * ir;
    return m;
}

// Eq. 3 as a deviation from the reference equilibrium, written with the momentum j = rho u:
// f_eq(rho, u) - f_eq(rho0, u_dev) = w [ (rho - rho0) + 3 e.(j - j0) + (4.5 (e.j)^2 - 1.5 |j|^2)/rho - c0 ]
__device__ inline void heq(float drho, float rho, float jx, float jy, const RefDev &r, float out[Q]) {
    const float ir = frcp(rho);
    const float jj = 1.5f * (jx * jx + jy * jy);
    const float dx = jx - r.jx0, dy = jy - r.jy0;
#pragma unroll
    for (int a = 0; a < Q; a++) {
        const float ej = edot(a, jx, jy);
        const float ed = edot(a, dx, dy);
        const float quad = fmaf(fmaf(4.5f * ej, ej, -jj), ir, -r.c0[a]);
        out[a] = WT[a] * (drho + fmaf(3.f, ed, quad));
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

constexpr int PAD_BELOW = -MAX_GROUPS;   // slot codes below this are padded slots

// Least-squares coefficient of slot k of cell c: M^-1 w_k d_k (Eq. 12).
__device__ inline float2 lsq_coef(float2 dk, float m11, float m12, float m22) {
    const float w = frcp(fmaf(dk.x, dk.x, dk.y * dk.y));
    return make_float2(w * fmaf(m11, dk.x, m12 * dk.y), w * fmaf(m12, dk.x, m22 * dk.y));
}

// n dl / A of slot k from the corner offsets v_k, v_k+1 (CCW corners: outward normal).
__device__ inline float2 scaled_normal(float2 v0, float2 v1, float inva) {
    return make_float2((v1.y - v0.y) * inva, -(v1.x - v0.x) * inva);
}

template <int NF>
__device__ inline float2 corner(const InstDesc &d, int k, int c) {
    return ldg(d.vxy, (size_t)(k % NF) * d.np + c);
}

__device__ inline int remap_block(int b, int nb, int xcd_remap) {
    // Blocks are dispatched round-robin over the 8 XCDs; renumber them so that
    // each XCD walks one contiguous range of tiles (halo reads then hit that
    // XCD's L2).
    if (!xcd_remap) return b;
    const int x = b & 7, r = b >> 3;
    const int per = nb >> 3, extra = nb & 7;
    return x * per + (x < extra ? x : extra) + r;
}

__device__ inline int unpack16(uint32_t w, int hi) { return (int)(int16_t)(hi ? (w >> 16) : (w & 0xffffu)); }

// Geometry of one cell held in registers: stencil offsets, least-squares
// inverse, corner offsets and 1/A.
template <int NF>
struct CellGeo {
    float2 dk[NF];
    float m11, m12, m22;
    __device__ void load(const InstDesc &d, int c) {
#pragma unroll
        for (int k = 0; k < NF; k++) dk[k] = ldg(d.dxy, (size_t)k * d.np + c);
        m11 = ldg(d.minv, c);
        m12 = ldg(d.minv, (size_t)d.np + c);
        m22 = ldg(d.minv, 2 * (size_t)d.np + c);
    }
};

// LDS records.  Region A holds tile and ring-1 cells, 28 floats each:
// f0..f8, pad, (gx0,gy0)..(gx8,gy8); region B holds ring-2 cells, 12 floats
// each: f0..f8, pad.  Records are 16-byte aligned, so a cell's values are
// read with 128-bit LDS loads.
constexpr int RA = 7;   // float4 per region-A record
constexpr int RB = 3;   // float4 per region-B record

__device__ inline void rd_f(const float4 *rec, float f[Q]) {
    const float4 x = rec[0], y = rec[1];
    f[0] = x.x; f[1] = x.y; f[2] = x.z; f[3] = x.w;
    f[4] = y.x; f[5] = y.y; f[6] = y.z; f[7] = y.w;
    f[8] = reinterpret_cast<const float *>(rec)[8];
}
__device__ inline void wr_f(float4 *rec, const float f[Q]) {
    rec[0] = make_float4(f[0], f[1], f[2], f[3]);
    rec[1] = make_float4(f[4], f[5], f[6], f[7]);
    reinterpret_cast<float *>(rec)[8] = f[8];
}
__device__ inline void rd_g(const float4 *rec, float gx[Q], float gy[Q]) {
    const float2 p = reinterpret_cast<const float2 *>(rec)[5];
    const float4 a = rec[3], b = rec[4], c = rec[5], d = rec[6];
    gx[0] = p.x; gy[0] = p.y;
    gx[1] = a.x; gy[1] = a.y; gx[2] = a.z; gy[2] = a.w;
    gx[3] = b.x; gy[3] = b.y; gx[4] = b.z; gy[4] = b.w;
    gx[5] = c.x; gy[5] = c.y; gx[6] = c.z; gy[6] = c.w;
    gx[7] = d.x; gy[7] = d.y; gx[8] = d.z; gy[8] = d.w;
}
__device__ inline void wr_g(float4 *rec, const float gx[Q], const float gy[Q]) {
    reinterpret_cast<float2 *>(rec)[5] = make_float2(gx[0], gy[0]);
    rec[3] = make_float4(gx[1], gy[1], gx[2], gy[2]);
    rec[4] = make_float4(gx[3], gy[3], gx[4], gy[4]);
    rec[5] = make_float4(gx[5], gy[5], gx[6], gy[6]);
    rec[6] = make_float4(gx[7], gy[7], gx[8], gy[8]);
}

// Gradient of cell c (Eq. 12) from staged values: sum_k M^-1 w_k d_k (phi_k - f_c),
// phi_k = the staged value of local cell code[k], or the wall / ghost value of
// a boundary slot (Eqs. 18-22) formed from the cell's own state.  Local
// indices below `a_end` are region-A records, the rest region B.
template <int NF>
__device__ inline void gradient_staged(const InstDesc &d, int c, const CellGeo<NF> &geo, const float hc[Q],
                                       const int code[NF], const float4 *A, const float4 *B, int a_end,
                                       float gx[Q], float gy[Q]) {
#pragma unroll
    for (int a = 0; a < Q; a++) { gx[a] = 0.f; gy[a] = 0.f; }
    bool have_m = false;
    Macro m;
    float he[Q];
#pragma unroll
    for (int k = 0; k < NF; k++) {
        if (code[k] < PAD_BELOW) continue;
        const float2 w = lsq_coef(geo.dk[k], geo.m11, geo.m12, geo.m22);
        float phi[Q];
        if (code[k] >= 0) {
            const int l = code[k];
            rd_f(l < a_end ? A + l * RA : B + (l - a_end) * RB, phi);
        } else {
            if (!have_m) {
                m = moments(hc, d.ref);
                heq(m.drho, m.rho, m.jx, m.jy, d.ref, he);
                have_m = true;
            }
            const float2 gn = scaled_normal(corner<NF>(d, k, c), corner<NF>(d, k + 1, c), ldg(d.inva, c));
            boundary_value(d.groups[-1 - code[k]], hc, m, he, gn, d.ref, phi);
        }
#pragma unroll
        for (int a = 0; a < Q; a++) {
            const float df = phi[a] - hc[a];
            gx[a] = fmaf(w.x, df, gx[a]);
            gy[a] = fmaf(w.y, df, gy[a]);
        }
    }
}

// Phase 3 for one tile cell: face values, flux sum, BGK source, update, store.
template <int NF, int STORE>
__device__ __forceinline__ void tile_update(const InstDesc &d, int i, const int code[NF], const CellGeo<NF> &geo,
                                            const float4 *own, const float4 *A) {
    float hi[Q], gxi[Q], gyi[Q];
    rd_f(own, hi);
    rd_g(own, gxi, gyi);
    const Macro mi = moments(hi, d.ref);
    float hei[Q];
    heq(mi.drho, mi.rho, mi.jx, mi.jy, d.ref, hei);
    const float inva = ldg(d.inva, i);
    float acc[Q];
#pragma unroll
    for (int a = 0; a < Q; a++) acc[a] = 0.f;
#pragma unroll
    for (int k = 0; k < NF; k++) {
        if (code[k] < PAD_BELOW) continue;
        const float2 v0 = corner<NF>(d, k, i), v1 = corner<NF>(d, k + 1, i);
        const float2 g = scaled_normal(v0, v1, inva);
        const float2 r = make_float2(0.5f * (v0.x + v1.x), 0.5f * (v0.y + v1.y));   // x_f - x_i
        if (code[k] >= 0) {
            const float4 *rec = A + code[k] * RA;                                     // neighbours are in region A
            const float2 q = make_float2(r.x - geo.dk[k].x, r.y - geo.dk[k].y);       // x_f - x_j
            float hj[Q], gxj[Q], gyj[Q];
            rd_f(rec, hj);
            rd_g(rec, gxj, gyj);
#pragma unroll
            for (int a = 1; a < Q; a++) {
                const float en = edot(a, g.x, g.y);
                const float own = fmaf(gyi[a], r.y, fmaf(gxi[a], r.x, hi[a]));
                const float nb = fmaf(gyj[a], q.y, fmaf(gxj[a], q.x, hj[a]));
                acc[a] = fmaf(en, en > 0.f ? own : nb, acc[a]);
            }
        } else {
            const GroupDev &gr = d.groups[-1 - code[k]];
            float bv[Q];
            boundary_value(gr, hi, mi, hei, g, d.ref, bv);
            const bool upwind = gr.kind == FVLBM_BC_INLET || (gr.kind == FVLBM_BC_OUTLET && gr.internal);
#pragma unroll
            for (int a = 1; a < Q; a++) {
                const float en = edot(a, g.x, g.y);
                float phi;
                if (gr.kind == FVLBM_BC_WALL) {
                    phi = bv[a];                                                    // Eq. 18 face value
                } else if (upwind) {
                    phi = en > 0.f ? fmaf(gyi[a], r.y, fmaf(gxi[a], r.x, hi[a])) : bv[a];   // Eqs. 23, 24
                } else if (gr.kind == FVLBM_BC_OUTLET) {
                    phi = hi[a];                                                    // Eq. 25
                } else {
                    phi = 0.5f * (hi[a] + bv[a]);                                   // Eq. 26
                }
                acc[a] = fmaf(en, phi, acc[a]);
            }
        }
    }

    // RHS = -sum (e.n dl/A) phi - (f - f_eq)/tau  (Eq. 10), then the update.
#pragma unroll
    for (int a = 0; a < Q; a++) {
        const float rhs = fmaf(hei[a] - hi[a], d.inv_tau, -acc[a]);
        const size_t idx = (size_t)a * d.np + i;
        const uint32_t salt = (uint32_t)i * 9u + (uint32_t)a;
        Exact out;
        if (d.mode == 0) {
            const float b = (d.base == d.src) ? hi[a] : Storage<STORE>::load(d.base, idx, a, d.ref);
            out = fma_exact(d.coef, rhs, b);
        } else if (d.mode == 3) {
            stg(static_cast<float *>(d.dst), idx, rhs);
            continue;
        } else {
            const float prev = (d.mode == 1) ? rhs : ldg(d.rhs_prev, idx);
            out = fma_exact(0.5f * d.coef, 3.f * rhs - prev, hi[a]);
            stg(d.rhs_prev, idx, rhs);
        }
        Storage<STORE>::store(d.dst, idx, a, out, d.ref, salt);
    }
}

// One RHS evaluation and update for one tile of T cells.
//   Phase 1  one round of independent device loads: the tile's values, both
//            halo rings' values (to LDS), this thread's cell geometry and its
//            ring-1 cell's geometry (to registers);
//   Phase 2  gradients of tile and ring-1 cells into LDS (each computed once);
//   Phase 3  per tile cell: face values (own gradient outgoing, staged
//            neighbour value and gradient incoming), flux sum, BGK source,
//            update, store.
// Dynamic LDS: nA = T + h1max region-A records, then region-B records for
// up to hmax ring-2 cells (sized by the launcher).
template <int NF, int STORE, int T>
__device__ __forceinline__ void tile_body(const InstDesc *__restrict__ descs, int2 u, float4 *A, float4 *B) {
    const InstDesc &d = descs[u.x];
    const int tile = u.y;
    const int tid = threadIdx.x;
    const int i = tile * T + tid;
    const bool valid = i < d.n_cells;
    const int4 hd = ldg(d.hdr, tile);              // {first entry, n1, n2, first ring-1 code}
    const int n1 = hd.y, nh = hd.y + hd.z;
    const int a_end = T + n1;                      // local indices below this are region A

    // ---- phase 1
    int code[NF];
    CellGeo<NF> geo;
    if (valid) {
        float f[Q];
#pragma unroll
        for (int a = 0; a < Q; a++) f[a] = Storage<STORE>::load(d.src, (size_t)a * d.np + i, a, d.ref);
        wr_f(A + tid * RA, f);
        const uint2 ln = ldg(d.lnbr, i);
#pragma unroll
        for (int k = 0; k < NF; k++) code[k] = unpack16(k < 2 ? ln.x : ln.y, k & 1);
        geo.load(d, i);
    }
    int hcell = -1, hcode[NF];
    CellGeo<NF> hgeo;
    if (tid < n1) {
        hcell = ldg(d.halo_idx, hd.x + tid);
#pragma unroll
        for (int s = 0; s < NF; s++) hcode[s] = ldg(d.halo_code, (size_t)hd.w + (size_t)tid * NF + s);
        hgeo.load(d, hcell);
    }
    for (int k = tid; k < nh; k += T) {
        const int c = ldg(d.halo_idx, hd.x + k);
        float f[Q];
#pragma unroll
        for (int a = 0; a < Q; a++) f[a] = Storage<STORE>::load(d.src, (size_t)a * d.np + c, a, d.ref);
        wr_f(k < n1 ? A + (T + k) * RA : B + (k - n1) * RB, f);
    }
    __syncthreads();

    // ---- phase 2
    {
        float hc[Q], gx[Q], gy[Q];
        if (valid) {
            rd_f(A + tid * RA, hc);
            gradient_staged<NF>(d, i, geo, hc, code, A, B, a_end, gx, gy);
            wr_g(A + tid * RA, gx, gy);
        }
        if (hcell >= 0) {
            rd_f(A + (T + tid) * RA, hc);
            gradient_staged<NF>(d, hcell, hgeo, hc, hcode, A, B, a_end, gx, gy);
            wr_g(A + (T + tid) * RA, gx, gy);
        }
        for (int k = tid + T; k < n1; k += T) {       // ring 1 larger than the tile: geometry loaded here
            const int c = ldg(d.halo_idx, hd.x + k);
            int cc[NF];
#pragma unroll
            for (int s = 0; s < NF; s++) cc[s] = ldg(d.halo_code, (size_t)hd.w + (size_t)k * NF + s);
            CellGeo<NF> g2;
            g2.load(d, c);
            rd_f(A + (T + k) * RA, hc);
            gradient_staged<NF>(d, c, g2, hc, cc, A, B, a_end, gx, gy);
            wr_g(A + (T + k) * RA, gx, gy);
        }
    }
    __syncthreads();
    if (valid) tile_update<NF, STORE>(d, i, code, geo, A + tid * RA, A);
}

template <int NF, int STORE, int T>
__global__ void __launch_bounds__(T) k_tile(const InstDesc *__restrict__ descs,
                                            const int2 *__restrict__ units, int n_units,
                                            int xcd_remap, int nA) {
    extern __shared__ float4 lds4[];
    tile_body<NF, STORE, T>(descs, units[remap_block(blockIdx.x, n_units, xcd_remap)], lds4, lds4 + nA * RA);
}

// Persistent form: a grid sized to the resident capacity walks the unit list
// (a multiple of 8 blocks, so each block stays on one XCD's range of tiles).
template <int NF, int STORE, int T>
__global__ void __launch_bounds__(T) k_tile_persistent(const InstDesc *__restrict__ descs,
                                                       const int2 *__restrict__ units, int n_units,
                                                       int xcd_remap, int nA) {
    extern __shared__ float4 lds4[];
    for (int ub = blockIdx.x; ub < n_units; ub += gridDim.x) {
        tile_body<NF, STORE, T>(descs, units[remap_block(ub, n_units, xcd_remap)], lds4, lds4 + nA * RA);
        __syncthreads();             // the next unit reuses the LDS records
    }
}

template <int NF, int STORE, int T>
const void *fn(bool persistent) {
    return persistent ? reinterpret_cast<const void *>(&k_tile_persistent<NF, STORE, T>)
                      : reinterpret_cast<const void *>(&k_tile<NF, STORE, T>);
}

template <int NF, int STORE>
const void *pick_t(int T, bool persistent) {
    switch (T) {
    case 64: return fn<NF, STORE, 64>(persistent);
    case 128: return fn<NF, STORE, 128>(persistent);
    case 256: return fn<NF, STORE, 256>(persistent);
    default: return fn<NF, STORE, 512>(persistent);
    }
}

const void *pick(int nf, int storage, int T, bool persistent) {
    if (nf == 3) {
        if (storage == FVLBM_STORE_FP32) return pick_t<3, FVLBM_STORE_FP32>(T, persistent);
        if (storage == FVLBM_STORE_FP32_DEV) return pick_t<3, FVLBM_STORE_FP32_DEV>(T, persistent);
        return pick_t<3, FVLBM_STORE_FP16_DEV>(T, persistent);
    }
    if (storage == FVLBM_STORE_FP32) return pick_t<4, FVLBM_STORE_FP32>(T, persistent);
    if (storage == FVLBM_STORE_FP32_DEV) return pick_t<4, FVLBM_STORE_FP32_DEV>(T, persistent);
    return pick_t<4, FVLBM_STORE_FP16_DEV>(T, persistent);
}

// Grid of a launch: one block per unit, or (persistent) the number of blocks
// the device holds at once, rounded down to a multiple of 8 (one per XCD).
int grid_blocks(const UnitTable &ut, int persistent, int nf, int storage, size_t lds) {
    if (!persistent) return ut.n_units;
    int per_cu = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pick(nf, storage, ut.block, true), ut.block, lds);
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int g = std::max(8, (per_cu > 0 ? per_cu : 1) * cus / 8 * 8);
    return std::min(g, (ut.n_units + 7) / 8 * 8);
}

}  // namespace

size_t stage_lds_bytes(int T, int hmax, int h1max) {
    return ((size_t)(T + h1max) * RA + (size_t)(hmax > h1max ? hmax : h1max) * RB) * sizeof(float4);
}

hipError_t launch_stage(const InstDesc *descs_dev, const UnitTable &ut, int nf, int storage,
                        int xcd_remap, int persistent, int hmax, int h1max, hipStream_t stream) {
    if (ut.n_units == 0) return hipSuccess;
    const int2 *units = ut.units;
    int n_units = ut.n_units;
    int nA = ut.block + h1max;
    const size_t lds = stage_lds_bytes(ut.block, hmax, h1max);
    void *args[] = {(void *)&descs_dev, (void *)&units, (void *)&n_units, (void *)&xcd_remap, (void *)&nA};
    return hipLaunchKernel(pick(nf, storage, ut.block, persistent), dim3(grid_blocks(ut, persistent, nf, storage, lds)),
                           dim3(ut.block), args, lds, stream);
}

hipError_t add_stage_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, int ndeps,
                          const InstDesc *descs_dev, const UnitTable &ut, int nf, int storage,
                          int xcd_remap, int persistent, int hmax, int h1max, void **argbuf) {
    // argbuf: caller-owned storage for the argument values, alive until the graph is instantiated
    struct Args { const InstDesc *d; const int2 *u; int n; int x; int nA; };
    Args *a = reinterpret_cast<Args *>(argbuf[0]);
    a->d = descs_dev; a->u = ut.units; a->n = ut.n_units; a->x = xcd_remap; a->nA = ut.block + h1max;
    void **kp = argbuf + 1;
    kp[0] = &a->d; kp[1] = &a->u; kp[2] = &a->n; kp[3] = &a->x; kp[4] = &a->nA;
    hipKernelNodeParams p{};
    const size_t lds = stage_lds_bytes(ut.block, hmax, h1max);
    p.func = const_cast<void *>(pick(nf, storage, ut.block, persistent));
    p.gridDim = dim3(grid_blocks(ut, persistent, nf, storage, lds));
    p.blockDim = dim3(ut.block);
    p.sharedMemBytes = (unsigned)lds;
    p.kernelParams = kp;
    p.extra = nullptr;
    return hipGraphAddKernelNode(node, g, deps, ndeps, &p);
}

}  // namespace fvlbm

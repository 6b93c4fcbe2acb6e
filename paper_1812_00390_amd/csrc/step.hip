// The FVLBM right-hand side and time-integrator update, fused per tile.
//
// A workgroup owns a tile of consecutive cells (one thread per cell, all nine
// directions per thread) and stages the tile and two rings of face-neighbour
// halo in LDS.  Per RHS evaluation (paper Section 2.4.2, Steps 1-5):
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
// f, FP32 h, FP16 h/(w S), or 16-bit block-scaled h (int16 mantissas with a
// per-cell power-of-two scale).
//
// Only directions 1..8 move (e_0 = 0), so a staged record holds h_1..h_8 and
// their gradients; a cell's h_0 stays in its own thread's registers.
// Interior faces are handled in fully unrolled loops; the rare boundary slots
// go through one rolled loop per phase, which keeps the kernel small.
#include "fvlbm_internal.h"

#include <type_traits>

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
// through these global-address-space accessors instead.  Plane accesses take
// a uniform plane base (scalar registers) plus a 32-bit byte offset, which
// maps onto the scalar-base form of the global load and store instructions.
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
__device__ inline T ldo(const void *base, uint32_t off) {
    return *(const FVLBM_GLOBAL_AS T *)((const FVLBM_GLOBAL_AS char *)base + off);
}
// Stores of the new state (and of the other per-cell outputs) are non-temporal:
// nothing reads them again in the same launch, so their lines should not
// displace from L2 the halo values that neighbouring tiles read again.
template <class T>
__device__ inline void sto(void *base, uint32_t off, T v) {
    FVLBM_GLOBAL_AS char *p = (FVLBM_GLOBAL_AS char *)base + off;
    if constexpr (std::is_same<T, __half>::value)
        __builtin_nontemporal_store(__half_as_ushort(v), (FVLBM_GLOBAL_AS unsigned short *)p);
    else
        __builtin_nontemporal_store(v, (FVLBM_GLOBAL_AS T *)p);
}
// Non-temporal loads, for the data a launch reads once: a cell's corner offsets
// and neighbour codes, a tile's halo tables, the update base (the stencil offsets
// and the state are read again as halo values of the neighbouring tiles and stay
// ordinary loads).
typedef float float2v __attribute__((ext_vector_type(2)));
typedef unsigned uint2v __attribute__((ext_vector_type(2)));
template <class V>
__device__ inline V ldn(const void *base, uint32_t off) {
    return __builtin_nontemporal_load((const FVLBM_GLOBAL_AS V *)((const FVLBM_GLOBAL_AS char *)base + off));
}
__device__ inline int ldn1(const int *p, int i) { return __builtin_nontemporal_load((const FVLBM_GLOBAL_AS int *)p + i); }
__device__ inline const void *plane(const void *p, size_t plane_bytes, int a) {
    return static_cast<const char *>(p) + plane_bytes * (size_t)a;
}
__device__ inline void *plane(void *p, size_t plane_bytes, int a) {
    return static_cast<char *>(p) + plane_bytes * (size_t)a;
}

__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------- rounding
//
// Every state store rounds without bias.  Round-to-nearest drops every
// increment smaller than half an ulp, so a run can freeze short of its steady
// state (FP32) or drift (FP16).  Instead a dither uniform over one unit in the
// last place (centred) is added before rounding, so the expected stored value
// is the exact one.  The dither is a hash of the increment's bits and of
// (cell, direction): results do not depend on launch order, schedule,
// batching or graphs.

// Dither bits: the top of a 24-bit product (full-rate multiply) of the input's
// low 24 bits, with one odd multiplier per direction.  The input is the
// increment's bits (its mantissa fills the low 23) xor the cell, so it changes
// from step to step and from cell to cell.
__device__ constexpr uint32_t MIXK[Q] = {0x9e3779u, 0x85ebcbu, 0xc2b2afu, 0x27d4ebu, 0x165667u,
                                         0xd3a265u, 0xfd7047u, 0x6c8e95u, 0x4cf5adu};
__device__ inline uint32_t mix(uint32_t x, int a) { return __umul24(x, MIXK[a]); }

// b + p rounded to FP32 with a centred dither of one ulp of b.  The dither is
// drawn from the increment's bits, never from the bits being rounded away.
__device__ inline float add_sr(float b, float p, uint32_t key, int a) {
    const float g = __uint_as_float(__float_as_uint(b) & 0x7f800000u) * 0x1p-55f;   // ulp(b) / 2^32; 0 for b = 0
    const int32_t r = (int32_t)mix(__float_as_uint(p) ^ key, a);                    // uniform in [-2^31, 2^31)
    return b + fmaf((float)r, g, p);
}

// unbiased rounding of v = (b + p) / unit to FP16: 13 random bits (from the
// increment p) are added below the FP16 mantissa, then truncated (exact for
// FP16 normals)
__device__ inline __half round_fp16(float v, float p, uint32_t key, int a) {
    const uint32_t b = __float_as_uint(v);
    const uint32_t mag = (b & 0x7fffffffu) + (mix(__float_as_uint(p) ^ key, a) >> 19);
    return __float2half_rz(__uint_as_float((b & 0x80000000u) | mag));
}

// FP16 deviations x_a = h_a / (w_a S), rounded so that the stored cell keeps
// its mass and momentum.  Each value is rounded without bias (round_fp16), but
// nine independent roundings leave an error in the cell's conserved moments,
// which the collision does not relax, so it adds up from step to step as a
// random walk.  The values are therefore rounded one after another, each
// target corrected for the moment error of the values rounded before it
// (errors e_a = (q_a - x_a) w_a, in units of S):
//   cardinals by opposite pairs: 1, then 3 carrying 1's error (the pair's
//   momentum e_1 (E_1 - E_3) then keeps only 3's rounding); 2, then 4;
//   the pairs' remaining momentum error R goes to the diagonals as the
//   least-norm change that carries no mass, x_d - (e_d . R) / (4 w_d);
//   diagonals by opposite pairs the same way: 5, then 7; 6, then 8;
//   the mass error of all eight moving values goes to the rest value,
//   x_0 - sum_a e_a / w_0.
// The momentum error left is the rounding of one diagonal per diagonal axis
// (a quarter of a cardinal's weight), and the mass error that of the rest
// value (its deviation is small, second order in the velocity).  Every target
// is the exact value plus zero-mean corrections and every rounding is
// unbiased, so the expected stored value is still the exact one.
// res receives what is left: the stored cell's mass and momentum less the
// exact ones, in units of S.  The last stage of a step stores it beside the
// state and the next step's last stage adds it back to its base (see
// carry_correction), so the conserved moments carry no rounding from step to
// step; only the non-conserved moments keep a rounding error, which the
// collision relaxes.
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

struct ConsF16 {
    __device__ static void store(void *buf, size_t np, int c, const float b[Q], const float inc[Q], const RefDev &r,
                                 uint32_t key0, float res[3]) {
        const uint32_t off = (uint32_t)c * 2u;
        float x[Q], e[Q];
        __half q[Q];
#pragma unroll
        for (int a = 0; a < Q; a++) x[a] = (b[a] + inc[a]) * r.inv_unit[a];
        // rounds value a to target t; returns its rounding error (q - t) w_a and sets e_a = (q - x_a) w_a
        auto rnd = [&](int a, float t) {
            q[a] = round_fp16(t, inc[a], key0, a);
            const float qf = __half2float(q[a]);
            e[a] = (qf - x[a]) * WT[a];
            return (qf - t) * WT[a];
        };
        // cardinal pairs (1, 3) and (2, 4): the second carries the first's rounding (weights equal)
        rnd(3, x[3] + rnd(1, x[1]) * 9.f);                  // 1 / w = 9
        rnd(4, x[4] + rnd(2, x[2]) * 9.f);
        const float rx = e[1] - e[3], ry = e[2] - e[4];
        // diagonal pairs (5, 7) and (6, 8): least-norm share of R, then the pair carry
        const float s57 = rx + ry, s68 = ry - rx;           // e_5 . R, e_6 . R (e_7 = -e_5, e_8 = -e_6)
        const float r5 = rnd(5, fmaf(-9.f, s57, x[5]));      // 1 / (4 w_d) = 9
        rnd(7, fmaf(36.f, r5, fmaf(9.f, s57, x[7])));       // 1 / w_d = 36
        const float r6 = rnd(6, fmaf(-9.f, s68, x[6]));
        rnd(8, fmaf(36.f, r6, fmaf(9.f, s68, x[8])));
        const float rm = ((e[1] + e[2]) + (e[3] + e[4])) + ((e[5] + e[6]) + (e[7] + e[8]));
        rnd(0, fmaf(-2.25f, rm, x[0]));                       // 1 / w_0 = 9/4
#pragma unroll
        for (int a = 0; a < Q; a++) sto<__half>(plane(buf, np * 2, a), off, q[a]);
        res[0] = e[0] + rm;
        res[1] = ((e[1] - e[3]) + (e[5] - e[7])) + (e[8] - e[6]);
        res[2] = ((e[2] - e[4]) + (e[5] - e[7])) + (e[6] - e[8]);
    }
};

// The moment carry of FP16 storage: 3 planes of np FP16 values, 2^20 x the
// residual (mass, x- and y-momentum, units of S) of a cell's last store.  The
// scale keeps residuals from 6e-14 to 6e-2 S representable (a residual is at
// most a few ulps of a value times its weight); larger ones, which only a
// diverged state makes, saturate instead of overflowing.
constexpr float CARRY_SCALE = 1048576.f;
__device__ inline void load_carry(const __half *cp, size_t np, int c, float cr[3]) {
#pragma unroll
    for (int k = 0; k < 3; k++) cr[k] = __half2float(ldo<__half>(plane(cp, np * 2, k), (uint32_t)c * 2u)) * (1.f / CARRY_SCALE);
}
__device__ inline void store_carry(__half *cp, size_t np, int c, const float res[3]) {
#pragma unroll
    for (int k = 0; k < 3; k++)
        sto<__half>(plane(cp, np * 2, k), (uint32_t)c * 2u,
                    __float2half_rn(fminf(fmaxf(res[k] * CARRY_SCALE, -65504.f), 65504.f)));
}
// The exact state is the stored one less the carried residual R: the
// equilibrium-shaped change -S w_a (R_0 + 3 e_a . (R_x, R_y)) carries exactly
// -S R in mass and momentum (sum w = 1, sum w e e = I/3) and nothing else the
// collision does not relax.
__device__ inline float carry_correction(int a, const float cr[3], float S) {
    return -S * WT[a] * fmaf(3.f, edot(a, cr[1], cr[2]), cr[0]);
}

// A storage format: load(plane base, byte offset, direction) returns the
// deviation h; store(.., b, inc, ..) writes b + inc (b a deviation).
template <int STORE>
struct Storage;

template <>
struct Storage<FVLBM_STORE_FP32> {
    static constexpr uint32_t SZ = 4;
    __device__ static float load(const void *p, uint32_t off, int a, const RefDev &r) {
        return ldo<float>(p, off) - r.fref[a];
    }
    __device__ static void store(void *p, uint32_t off, int a, float b, float inc, const RefDev &r, uint32_t key) {
        sto<float>(p, off, add_sr(b + r.fref[a], inc, key, a));   // b + fref is the stored f (b came from it by Sterbenz)
    }
};
template <>
struct Storage<FVLBM_STORE_FP32_DEV> {
    static constexpr uint32_t SZ = 4;
    __device__ static float load(const void *p, uint32_t off, int, const RefDev &) { return ldo<float>(p, off); }
    __device__ static void store(void *p, uint32_t off, int a, float b, float inc, const RefDev &, uint32_t key) {
        sto<float>(p, off, add_sr(b, inc, key, a));
    }
};
template <>
struct Storage<FVLBM_STORE_FP16_DEV> {
    static constexpr uint32_t SZ = 2;
    __device__ static float load(const void *p, uint32_t off, int a, const RefDev &r) {
        return __half2float(ldo<__half>(p, off)) * (WT[a] * r.scale);
    }
    // (stores go through ConsF16: a cell's nine values are rounded together)
};

// 16-bit block-scaled deviations: per cell nine int16 mantissas and one
// exponent byte s, h_a = q_a 2^(s - 142), with 2^(s - 127) just above the
// cell's largest |h_a|.  The largest deviation keeps 15 bits where FP16 keeps
// 11.  Planes: nine int16 planes, then the exponent plane (np bytes).
struct BlockI16 {
    __device__ static float scale(const void *buf, size_t np, int c) {
        const uint32_t sb = ldo<uint8_t>(static_cast<const char *>(buf) + np * 18, (uint32_t)c);
        return __uint_as_float(sb << 23) * 0x1p-15f;                      // 0 when s = 0
    }
    __device__ static float load(const void *buf, size_t np, int c, int a, float sc) {
        return (float)ldo<int16_t>(plane(buf, np * 2, a), (uint32_t)c * 2u) * sc;
    }
    // v[a] = b[a] + inc[a]; unbiased rounding of each mantissa (dither from the increment)
    __device__ static void store(void *buf, size_t np, int c, const float b[Q], const float inc[Q], uint32_t key0) {
        float v[Q], m = 0.f;
#pragma unroll
        for (int a = 0; a < Q; a++) {
            v[a] = b[a] + inc[a];
            m = fmaxf(m, fabsf(v[a]));
        }
        const uint32_t sb = m > 0.f ? min(((__float_as_uint(m) >> 23) & 0xffu) + 1u, 254u) : 0u;
        const int sh = 142 - (int)sb;
#pragma unroll
        for (int a = 0; a < Q; a++) {
            const float x = sb ? ldexpf(v[a], sh) : 0.f;                     // |x| < 2^15, exact scaling
            const float fl = floorf(x);
            const float u = (float)(mix(__float_as_uint(inc[a]) ^ key0, a) >> 8) * 0x1p-24f;
            int q = (int)fl + (u < x - fl ? 1 : 0);
            q = max(-32767, min(32767, q));
            sto<int16_t>(plane(buf, np * 2, a), (uint32_t)c * 2u, (int16_t)q);
        }
        sto<uint8_t>(static_cast<char *>(buf) + np * 18, (uint32_t)c, (uint8_t)sb);
    }
};

// Per-cell access for every storage mode.  load_cell fills f[a0..8] with the
// deviations of cell c; store_cell writes b + inc.  NT: a non-temporal load (the
// update base, which only the cell's own tile reads), for the FP32 storages.
template <int STORE, bool NT = false>
__device__ inline void load_cell(const void *buf, size_t np, int c, float f[Q], const RefDev &r, int a0 = 0,
                                 int a1 = Q) {
    if constexpr (NT && (STORE == FVLBM_STORE_FP32 || STORE == FVLBM_STORE_FP32_DEV)) {
        const uint32_t off = (uint32_t)c * 4u;
#pragma unroll
        for (int a = a0; a < a1; a++) {
            const float x = __builtin_nontemporal_load(
                (const FVLBM_GLOBAL_AS float *)((const FVLBM_GLOBAL_AS char *)plane(buf, np * 4, a) + off));
            f[a] = STORE == FVLBM_STORE_FP32 ? x - r.fref[a] : x;
        }
    } else if constexpr (STORE == FVLBM_STORE_I16_DEV) {
        const float sc = BlockI16::scale(buf, np, c);
#pragma unroll
        for (int a = a0; a < Q; a++) f[a] = BlockI16::load(buf, np, c, a, sc);
    } else {
        using S = Storage<STORE>;
        const uint32_t off = (uint32_t)c * S::SZ;
#pragma unroll
        for (int a = a0; a < a1; a++) f[a] = S::load(plane(buf, np * S::SZ, a), off, a, r);
    }
}
template <int STORE>
__device__ inline void store_cell(void *buf, size_t np, int c, const float b[Q], const float inc[Q], const RefDev &r,
                                  uint32_t key0, __half *carry = nullptr) {
    if constexpr (STORE == FVLBM_STORE_I16_DEV) {
        BlockI16::store(buf, np, c, b, inc, key0);
    } else if constexpr (STORE == FVLBM_STORE_FP16_DEV) {
        float res[3];
        ConsF16::store(buf, np, c, b, inc, r, key0, res);
        if (carry) store_carry(carry, np, c, res);
    } else {
        using S = Storage<STORE>;
        const uint32_t off = (uint32_t)c * S::SZ;
#pragma unroll
        for (int a = 0; a < Q; a++) S::store(plane(buf, np * S::SZ, a), off, a, b[a], inc[a], r, key0);
    }
}

// Direction sets of a split pass: H = -1 all; the halves 0 (directions 0-4)
// and 1 (5-8); the quarters 2 (0, 1, 3), 3 (2, 4), 4 (5, 7) and 5 (6, 8).
// Opposite directions always share a set.
__device__ constexpr bool in_set(int H, int a) {
    return H < 0 ? true
         : H == 0 ? a <= 4
         : H == 1 ? a >= 5
         : H == 2 ? (a == 0 || a == 1 || a == 3)
         : H == 3 ? (a == 2 || a == 4)
         : H == 4 ? (a == 5 || a == 7)
                  : (a == 6 || a == 8);
}
// the set holds directions among 1-4 / among 5-8
__device__ constexpr bool has_lo(int H) { return H < 0 || H == 0 || H == 2 || H == 3; }
__device__ constexpr bool has_hi(int H) { return H < 0 || H == 1 || H == 4 || H == 5; }

// The values of the direction set H of cell c (per-value storage modes).
template <int STORE, int H>
__device__ inline void load_set(const void *buf, size_t np, int c, float f[Q], const RefDev &r) {
    static_assert(STORE != FVLBM_STORE_I16_DEV, "the block-scaled format loads a cell whole");
    using S = Storage<STORE>;
    const uint32_t off = (uint32_t)c * S::SZ;
#pragma unroll
    for (int a = 0; a < Q; a++)
        if (in_set(H, a)) f[a] = S::load(plane(buf, np * S::SZ, a), off, a, r);
}

// store_cell for the directions of set H (per-value storage modes only)
template <int STORE, int H>
__device__ inline void store_half(void *buf, size_t np, int c, const float b[Q], const float inc[Q], const RefDev &r,
                                  uint32_t key0) {
    static_assert(STORE != FVLBM_STORE_I16_DEV && STORE != FVLBM_STORE_FP16_DEV,
                  "the block-scaled and FP16 formats store a cell whole");
    using S = Storage<STORE>;
    const uint32_t off = (uint32_t)c * S::SZ;
#pragma unroll
    for (int a = 0; a < Q; a++)
        if (in_set(H, a)) S::store(plane(buf, np * S::SZ, a), off, a, b[a], inc[a], r, key0);
}

struct Macro {
    float drho, rho;   // rho - rho0, rho
    float jx, jy;      // momentum rho u
    float ux, uy;
    float ir;          // 1 / rho
};

// Eq. 5 on deviations h = f - f_eq(rho0, u_dev): rho = rho0 + sum h, rho u = rho0 u_dev + sum e h.
__device__ inline Macro moments(const float h[Q], const RefDev &r) {
    Macro m;
    float s = h[0];
#pragma unroll
    for (int a = 1; a < Q; a++) s += h[a];
    const float mx = ((((h[1] - h[3]) + h[5]) - h[6]) - h[7]) + h[8];   // sum e_x h
    const float my = ((((h[2] - h[4]) + h[5]) + h[6]) - h[7]) - h[8];   // sum e_y h
    m.drho = s;
    m.rho = r.rho0 + s;
    m.jx = r.jx0 + mx;
    m.jy = r.jy0 + my;
    const float ir = frcp(m.rho);
    m.ux = m.jx * ir;
    m.uy = m.jy * ir;
    m.ir = ir;
    return m;
}

// Eq. 3 as a deviation from the reference equilibrium, written with the momentum j = rho u:
// f_eq(rho, u) - f_eq(rho0, u_dev) = w [ (rho - rho0) + 3 e.(j - j0) + (4.5 (e.j)^2 - 1.5 |j|^2)/rho - c0 ]
// H >= 0: only the directions of set H (in_set), out[0] not formed.
template <int H = -1>
__device__ inline void heq(float drho, float rho, float jx, float jy, const RefDev &r, float out[Q]) {
    const float ir = frcp(rho);
    const float jj = 1.5f * (jx * jx + jy * jy);
    const float dx = jx - r.jx0, dy = jy - r.jy0;
    if (H < 0) out[0] = WT[0] * (drho + fmaf(3.f, 0.f, fmaf(fmaf(0.f, 0.f, -jj), ir, -r.c0[0])));
    // Opposite directions (e_b = -e_a) share (e.j)^2 and c0, and their e.(j - j0)
    // differ in sign only (every negation here is exact): one quadratic term per pair.
    constexpr int PA[4] = {1, 2, 5, 6}, PB[4] = {3, 4, 7, 8};
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const int a = PA[p], b = PB[p];
        if (!in_set(H, a)) continue;
        const float ej = edot(a, jx, jy);
        const float ed = edot(a, dx, dy);
        const float quad = fmaf(fmaf(4.5f * ej, ej, -jj), ir, -r.c0[a]);
        out[a] = WT[a] * (drho + fmaf(3.f, ed, quad));
        out[b] = WT[b] * (drho + fmaf(-3.f, ed, quad));
    }
}

// f_eq(rho, j*) - f_eq(rho, j) (Eq. 3) at one density: the reference terms
// cancel, and with D = j* - j, S = j* + j the quadratic terms factor,
// (e.j*)^2 - (e.j)^2 = (e.D)(e.S) and |j*|^2 - |j|^2 = D.S, so the difference is
// w [3 e.D + (4.5 (e.D)(e.S) - 1.5 D.S) / rho], formed without either equilibrium.
template <int H>
__device__ inline void eq_delta_same_rho(const Macro &m, float jsx, float jsy, float out[Q]) {
    const float Dx = jsx - m.jx, Dy = jsy - m.jy;
    const float Sx = jsx + m.jx, Sy = jsy + m.jy;
    const float C = 1.5f * fmaf(Dx, Sx, Dy * Sy);
    if (H < 0) out[0] = WT[0] * (-C * m.ir);
    constexpr int PA[4] = {1, 2, 5, 6}, PB[4] = {3, 4, 7, 8};   // opposite pairs, e_b = -e_a
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const int a = PA[p], b = PB[p];
        if (!in_set(H, a)) continue;
        const float eD = edot(a, Dx, Dy);
        const float q = fmaf(4.5f * eD, edot(a, Sx, Sy), -C) * m.ir;   // the same for e_b
        out[a] = WT[a] * fmaf(3.f, eD, q);
        out[b] = WT[b] * fmaf(-3.f, eD, q);
    }
}

// f_eq(rho*, j*) - f_eq(rho, j) (Eq. 3) for a density rho* = rho0 + drs: the
// reference terms cancel, leaving
// w [(rho* - rho) + 3 e.(j* - j) + (4.5 (e.j*)^2 - 1.5 |j*|^2) / rho* - (4.5 (e.j)^2 - 1.5 |j|^2) / rho].
template <int H>
__device__ inline void eq_delta(const Macro &m, float drs, float rs, float jsx, float jsy, float out[Q]) {
    const float irs = frcp(rs);
    const float jjs = 1.5f * fmaf(jsx, jsx, jsy * jsy), jj = 1.5f * fmaf(m.jx, m.jx, m.jy * m.jy);
    const float dd = drs - m.drho;
    const float dx = jsx - m.jx, dy = jsy - m.jy;
    if (H < 0) out[0] = WT[0] * (dd + fmaf(-jjs, irs, jj * m.ir));
    constexpr int PA[4] = {1, 2, 5, 6}, PB[4] = {3, 4, 7, 8};
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const int a = PA[p], b = PB[p];
        if (!in_set(H, a)) continue;
        const float es = edot(a, jsx, jsy), ej = edot(a, m.jx, m.jy);
        const float q = fmaf(fmaf(4.5f * es, es, -jjs), irs, -(fmaf(4.5f * ej, ej, -jj) * m.ir));
        const float ed = edot(a, dx, dy);
        out[a] = WT[a] * (dd + fmaf(3.f, ed, q));
        out[b] = WT[b] * (dd + fmaf(-3.f, ed, q));
    }
}

// Boundary stencil value of a cell's boundary slot (Eqs. 18-22) minus the cell's
// own value, phi_k - h.  A wall, an inlet and an internal-density outlet set
// phi_k = f_eq(rho*, j*) + (h - f_eq(rho, j)), so the difference is that of two
// equilibria, formed directly; a symmetry ghost is an equilibrium itself.
// H >= 0: only the directions of set H (opposite directions share a set).
template <int H = -1>
__device__ inline void boundary_delta(const GroupDev &g, const float h[Q], const Macro &m, float2 gn,
                                      const RefDev &r, float out[Q]) {
    switch (g.kind) {
    case FVLBM_BC_WALL:                 // Eq. 18: rho* = rho_k, u* = u_w
        eq_delta_same_rho<H>(m, m.rho * g.ux, m.rho * g.uy, out);
        break;
    case FVLBM_BC_INLET: {              // Eq. 19: rho* = rho_inf (external) or rho_k (internal)
        const float dr = g.internal ? m.drho : g.drho;
        const float rs = g.internal ? m.rho : g.rho;
        eq_delta<H>(m, dr, rs, rs * g.ux, rs * g.uy, out);
        break;
    }
    case FVLBM_BC_OUTLET:
        if (!g.internal) {              // Eq. 20: f_GC = f_i
#pragma unroll
            for (int a = 0; a < Q; a++) out[a] = 0.f;
        } else {                        // Eq. 21: rho* = rho_inf, u* = u_i
            eq_delta<H>(m, g.drho, g.rho, g.rho * m.ux, g.rho * m.uy, out);
        }
        break;
    default: {                          // Eq. 22: mirrored normal velocity
        const float il = rsqrtf(gn.x * gn.x + gn.y * gn.y);
        const float nx = gn.x * il, ny = gn.y * il;
        const float jn = m.jx * nx + m.jy * ny;
        heq<H>(m.drho, m.rho, m.jx - 2.f * jn * nx, m.jy - 2.f * jn * ny, r, out);
#pragma unroll
        for (int a = 0; a < Q; a++)
            if (a > 0 ? in_set(H, a) : H < 0) out[a] -= h[a];
        break;
    }
    }
}

// Least-squares coefficient of slot k of cell c: M^-1 w_k d_k (Eq. 12).
__device__ inline float2 lsq_coef(float2 dk, float m11, float m12, float m22) {
    const float w = frcp(fmaf(dk.x, dk.x, dk.y * dk.y));
    return make_float2(w * fmaf(m11, dk.x, m12 * dk.y), w * fmaf(m12, dk.x, m22 * dk.y));
}

// n dl / A of slot k from the corner offsets v_k, v_k+1 (CCW corners: outward normal).
__device__ inline float2 scaled_normal(float2 v0, float2 v1, float inva) {
    return make_float2((v1.y - v0.y) * inva, -(v1.x - v0.x) * inva);
}

constexpr int PAD_BELOW = -MAX_GROUPS;   // slot codes below this are padded slots

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

// The 64-cell halo-wave form with FP32 storage splits phase 2 and 3 by
// directions over more waves (the 16-bit formats round a cell's nine values
// together, so one thread stores the whole cell).
constexpr bool split_form(int T, int STORE, bool RING) {
    return RING && T == 64 && STORE != FVLBM_STORE_I16_DEV && STORE != FVLBM_STORE_FP16_DEV;
}
// Threads per workgroup of a stage kernel: the tile's cells, one or two waves for
// the halo slots (RING; two when the larger ring holds more than 64 slots, one in
// the split form), two waves for directions 5-8 of the gradients (split form).
constexpr int tile_threads(int T, int STORE, bool RING, int waves = 1) {
    return T + (RING ? 64 * (split_form(T, STORE, RING) ? 1 : waves) : 0) + (split_form(T, STORE, RING) ? 128 : 0);
}
// (A third and fourth wave for rings above 128 slots measured slower: the rare
// tiles with such rings set the block size of the whole launch.)
constexpr int MAX_HALO_WAVES = 2;
// Halo waves of a RING launch whose larger ring holds hmax slots.
inline int halo_waves(int hmax) { return std::min(MAX_HALO_WAVES, std::max(1, (hmax + 63) / 64)); }
// The largest block a stage kernel is launched with.
constexpr int max_tile_threads(int T, int STORE, bool RING) {
    return T ? tile_threads(T, STORE, RING, MAX_HALO_WAVES) : 512;
}

// v[k] from registers by selects (no dynamic register indexing; k may differ
// between lanes)
template <int NF>
__device__ __forceinline__ float2 pick2(const float2 (&v)[NF], int k) {
    float2 r = v[0];
#pragma unroll
    for (int j = 1; j < NF; j++) r = k == j ? v[j] : r;
    return r;
}

// Least-squares data of one cell held in registers: the stencil offsets and
// the inverse of M = sum_k w_k d_k d_k^T, w_k = 1/|d_k|^2 (Eq. 12), formed
// here from the offsets (M is dimensionless and well scaled, so FP32 is
// ample) instead of being read from memory.
template <int NF>
struct CellGeo {
    float2 dk[NF];
    float m11, m12, m22;
    __device__ void load(const float2 *dxy, size_t np, int c) {
        const uint32_t o8 = (uint32_t)c * 8u;
#pragma unroll
        for (int k = 0; k < NF; k++) dk[k] = ldo<float2>(plane(dxy, np * 8, k), o8);
    }
    // padded slots (no face) do not enter M
    __device__ void invert(const int (&code)[NF]) {
        float a = 0.f, b = 0.f, e = 0.f;
#pragma unroll
        for (int k = 0; k < NF; k++) {
            if (code[k] < PAD_BELOW) continue;
            const float w = frcp(fmaf(dk[k].x, dk[k].x, dk[k].y * dk[k].y));
            const float wx = w * dk[k].x, wy = w * dk[k].y;
            a = fmaf(wx, dk[k].x, a);
            b = fmaf(wx, dk[k].y, b);
            e = fmaf(wy, dk[k].y, e);
        }
        const float idet = frcp(fmaf(a, e, -(b * b)));
        m11 = e * idet;
        m12 = -b * idet;
        m22 = a * idet;
    }
};

// Face data of one tile cell: corner offsets from the centroid and 1/A.  A
// triangle's centroid is its vertex mean, so its third offset is minus the sum
// of the other two and is not read.
template <int NF>
struct CellFaces {
    float2 v[NF];
    float inva;
    __device__ void load(const float2 *vxy, size_t np, int c) {
        const uint32_t o8 = (uint32_t)c * 8u;
#pragma unroll
        for (int k = 0; k < (NF == 3 ? 2 : NF); k++) {
            const float2v t = ldn<float2v>(plane(vxy, np * 8, k), o8);
            v[k] = make_float2(t.x, t.y);
        }
    }
    __device__ void finish() {
        if (NF == 3) v[2] = make_float2(-(v[0].x + v[1].x), -(v[0].y + v[1].y));
        float twice_a = 0.f;                    // shoelace over the corner offsets
#pragma unroll
        for (int k = 0; k < NF; k++) {
            const float2 p = v[k], q = v[k + 1 == NF ? 0 : k + 1];
            twice_a = fmaf(p.x, q.y, fmaf(-p.y, q.x, twice_a));
        }
        inva = 2.f * frcp(twice_a);
    }
};

// LDS records.  Region A holds tile and ring-1 cells, 24 floats each:
// h1..h8, (gx1,gy1)..(gx8,gy8), as six float4 planes (float4 c of record l at
// A[c nA + l]), so that the lanes of a wave reading their own records touch
// consecutive addresses (no bank conflicts); region B holds ring-2 cells, 8
// floats each: h1..h8, as consecutive float4 (read at random positions only).
// Every access is a 128-bit LDS load or store; s is the record's float4 stride.
constexpr int RA = 6;   // float4 per region-A record
constexpr int RB = 2;   // float4 per region-B record

__device__ inline void rd_f(const float4 *rec, int s, float f[Q]) {
    const float4 x = rec[0], y = rec[s];
    f[1] = x.x; f[2] = x.y; f[3] = x.z; f[4] = x.w;
    f[5] = y.x; f[6] = y.y; f[7] = y.z; f[8] = y.w;
}
__device__ inline void wr_f(float4 *rec, int s, const float f[Q]) {
    rec[0] = make_float4(f[1], f[2], f[3], f[4]);
    rec[s] = make_float4(f[5], f[6], f[7], f[8]);
}
__device__ inline void rd_g(const float4 *rec, int s, float gx[Q], float gy[Q]) {
    const float4 a = rec[2 * s], b = rec[3 * s], c = rec[4 * s], d = rec[5 * s];
    gx[1] = a.x; gy[1] = a.y; gx[2] = a.z; gy[2] = a.w;
    gx[3] = b.x; gy[3] = b.y; gx[4] = b.z; gy[4] = b.w;
    gx[5] = c.x; gy[5] = c.y; gx[6] = c.z; gy[6] = c.w;
    gx[7] = d.x; gy[7] = d.y; gx[8] = d.z; gy[8] = d.w;
}
// H >= 0: the gradients of half H only (directions 1-4 or 5-8)
template <int H = -1>
__device__ inline void wr_g(float4 *rec, int s, const float gx[Q], const float gy[Q]) {
    if (has_lo(H)) {
        rec[2 * s] = make_float4(gx[1], gy[1], gx[2], gy[2]);
        rec[3 * s] = make_float4(gx[3], gy[3], gx[4], gy[4]);
    }
    if (has_hi(H)) {
        rec[4 * s] = make_float4(gx[5], gy[5], gx[6], gy[6]);
        rec[5 * s] = make_float4(gx[7], gy[7], gx[8], gy[8]);
    }
}

// Boundary-slot terms of the gradient of cell c: phi_k is the wall / ghost
// value (Eqs. 18-22) formed from the cell's own state, taken as phi_k - h_c.
// bm: the cell's boundary slots as bits; each lane walks its own (so a wave
// makes as many passes as its lane with the most boundary faces), in slot order.
// SAVE: phi_k - h_c of the first boundary slot is kept (save, save_k) for the
// cell's boundary flux, which forms the same values from the same state.
// STASH: phi_k - h_c of every boundary slot k also goes to stash[2k ss],
// stash[(2k + 1) ss] (directions 1-4, 5-8), for a flux computed by another wave.
// H >= 0: only the directions of set H.
template <int NF, bool SAVE, bool STASH, int H>
__device__ inline void boundary_gradient_body(const InstDesc &d, const CellGeo<NF> &geo, const float hc[Q],
                                              uint2 packed, uint32_t bm, const GroupDev *lg, float gx[Q], float gy[Q],
                                              float save[Q], int &save_k, float4 *stash, int ss) {
    const Macro m = moments(hc, d.ref);
#pragma unroll 1
    for (uint32_t b = bm; b != 0u; b &= b - 1u) {
        const int k = __builtin_ctz(b);
        const int ck = unpack16(k < 2 ? packed.x : packed.y, k & 1);
        const float2 dk = pick2<NF>(geo.dk, k);
        const float2 w = lsq_coef(dk, geo.m11, geo.m12, geo.m22);
        // the ghost values take only the direction of the face's outward normal (a
        // symmetry face), and a ghost slot's offset is twice the centre-to-face
        // distance along that normal (the mirrored centre): dk has the direction
        const float2 gn = dk;
        const GroupDev g = lg[-1 - ck];
        float df[Q];
        boundary_delta<H>(g, hc, m, gn, d.ref, df);
        if (SAVE && save_k < 0) {
            save_k = k;
#pragma unroll
            for (int a = 1; a < Q; a++)
                if (in_set(H, a)) save[a] = df[a];
        }
        if (STASH) {
            if (has_lo(H)) stash[2 * k * ss] = make_float4(df[1], df[2], df[3], df[4]);
            if (has_hi(H)) stash[(2 * k + 1) * ss] = make_float4(df[5], df[6], df[7], df[8]);
        }
#pragma unroll
        for (int a = 1; a < Q; a++) {
            if (!in_set(H, a)) continue;
            gx[a] = fmaf(w.x, df[a], gx[a]);
            gy[a] = fmaf(w.y, df[a], gy[a]);
        }
    }
}

// Gradient of cell c (Eq. 12) from staged values: sum_k M^-1 w_k d_k (phi_k - h_c),
// phi_k the staged value of local cell code[k] (interior slots first, then
// boundary slots).  Local indices below `a_end` are region-A records (plane
// stride sa), the rest region B.  H >= 0: only the directions of set H.
template <int NF, bool SAVE, bool STASH, int H>
__device__ inline void gradient_staged(const InstDesc &d, const CellGeo<NF> &geo, const float hc[Q],
                                       const int (&code)[NF], uint2 packed, const float4 *A, const float4 *B, int a_end,
                                       const GroupDev *lg, float gx[Q], float gy[Q], float save[Q], int &save_k,
                                       float4 *stash, int ss, int sa) {
#pragma unroll
    for (int a = 1; a < Q; a++) { gx[a] = 0.f; gy[a] = 0.f; }
    uint32_t bm = 0u;                     // boundary slots (padded slots have no face)
#pragma unroll
    for (int k = 0; k < NF; k++) {
        if (code[k] < 0) {
            if (code[k] >= PAD_BELOW) bm |= 1u << k;
            continue;
        }
        const float2 w = lsq_coef(geo.dk[k], geo.m11, geo.m12, geo.m22);
        const int l = code[k];
        float phi[Q];
        rd_f(l < a_end ? A + l : B + (l - a_end) * RB, l < a_end ? sa : 1, phi);
#pragma unroll
        for (int a = 1; a < Q; a++) {
            if (!in_set(H, a)) continue;
            const float df = phi[a] - hc[a];
            gx[a] = fmaf(w.x, df, gx[a]);
            gy[a] = fmaf(w.y, df, gy[a]);
        }
    }
    if (bm) boundary_gradient_body<NF, SAVE, STASH, H>(d, geo, hc, packed, bm, lg, gx, gy, save, save_k, stash, ss);
}

// Boundary-face terms of the flux sum of tile cell i (Eqs. 18, 23-26); bm as in
// boundary_gradient_body; phi_k - h_i of slot save_k was formed in phase 2, and
// with STASH those of every slot (stash as in boundary_gradient_body).
template <int NF, int H, bool STASH>
__device__ inline void boundary_flux(const InstDesc &d, const float hi[Q], const float gxi[Q], const float gyi[Q],
                                     const Macro &mi, uint2 packed, uint32_t bm,
                                     const CellGeo<NF> &geo, const CellFaces<NF> &cf, const GroupDev *lg,
                                     const float save[Q], int save_k, const float4 *stash, int ss, float acc[Q]) {
#pragma unroll 1
    for (uint32_t b = bm; b != 0u; b &= b - 1u) {
        const int k = __builtin_ctz(b);
        const int ck = unpack16(k < 2 ? packed.x : packed.y, k & 1);
        const float2 v0 = pick2<NF>(cf.v, k), v1 = pick2<NF>(cf.v, k + 1 == NF ? 0 : k + 1);   // the interior faces' corners
        const float2 g = scaled_normal(v0, v1, cf.inva);
        const float2 r = make_float2(0.5f * (v0.x + v1.x), 0.5f * (v0.y + v1.y));   // x_f - x_i
        const GroupDev gr = lg[-1 - ck];
        float dv[Q];      // phi_k - h_i
        if (k == save_k) {
#pragma unroll
            for (int a = 1; a < Q; a++) dv[a] = save[a];
        } else if (STASH) {
            if (has_lo(H)) {
                const float4 x = stash[2 * k * ss];
                dv[1] = x.x; dv[2] = x.y; dv[3] = x.z; dv[4] = x.w;
            }
            if (has_hi(H)) {
                const float4 y = stash[(2 * k + 1) * ss];
                dv[5] = y.x; dv[6] = y.y; dv[7] = y.z; dv[8] = y.w;
            }
        } else {          // (the normal direction from the slot offset, as in the gradient)
            boundary_delta(gr, hi, mi, pick2<NF>(geo.dk, k), d.ref, dv);
        }
        const int kind = gr.kind;
        const bool upwind = kind == FVLBM_BC_INLET || (kind == FVLBM_BC_OUTLET && gr.internal);
#pragma unroll
        for (int a = 1; a < Q; a++) {
            if (!in_set(H, a)) continue;
            const float en = edot(a, g.x, g.y);
            const float bv = hi[a] + dv[a];
            float phi;
            if (kind == FVLBM_BC_WALL) {
                phi = bv;                                                       // Eq. 18 face value
            } else if (upwind) {
                phi = en > 0.f ? fmaf(gyi[a], r.y, fmaf(gxi[a], r.x, hi[a])) : bv;   // Eqs. 23, 24
            } else if (kind == FVLBM_BC_OUTLET) {
                phi = hi[a];                                                    // Eq. 25
            } else {
                phi = fmaf(0.5f, dv[a], hi[a]);                                 // Eq. 26: the mean of h_i and phi_k
            }
            acc[a] = fmaf(en, phi, acc[a]);
        }
    }
}

// The BGK collision term f_eq - f of one cell (Eqs. 3-5, deviation form).
// The BGK source moves no mass and no momentum: f_eq carries the density and
// momentum of f.  In FP32 the rounding of f_eq (terms near 0.05, an ulp near
// 4e-9, divided by tau) leaves residual moments that act as a steady momentum
// source and add up over a run.  They are projected out of f_eq - f
// (subtracting w_a (m0 + 3 e_a.m), an identity in exact arithmetic).
__device__ inline void collision_neq(const float h[Q], const RefDev &r, float neq[Q]) {
    const Macro m = moments(h, r);
    float he[Q];
    heq(m.drho, m.rho, m.jx, m.jy, r, he);
#pragma unroll
    for (int a = 0; a < Q; a++) neq[a] = he[a] - h[a];
    const float m0 = ((neq[0] + neq[1]) + (neq[2] + neq[3])) + ((neq[4] + neq[5]) + (neq[6] + neq[7])) + neq[8];
    const float mx = ((neq[1] - neq[3]) + (neq[5] - neq[6])) + (neq[8] - neq[7]);
    const float my = ((neq[2] - neq[4]) + (neq[5] + neq[6])) - (neq[7] + neq[8]);
    neq[0] = fmaf(-WT[0], m0, neq[0]);
#pragma unroll
    for (int a = 1; a < Q; a++) neq[a] = fmaf(-WT[a], fmaf(3.f, edot(a, mx, my), m0), neq[a]);
}

// Phase 3 for one tile cell: face values, flux sum, BGK source, update, store.
// base[] holds f(0) of the update when it is not the evaluated state.  H >= 0:
// only the directions of set H (a base + coef RHS update), the others being
// other waves'; every per-direction value is the one the whole update forms.
// NEQ: the cell's collision term was formed in phase 1 and staged at lneq
// (float4 planes of stride ss: directions 0-3, 4-7, 8).
template <int NF, int STORE, bool M0, int H, bool STASH, bool NEQ>
__device__ __forceinline__ void tile_update(const InstDesc &d, int i, float h0, const float base[Q], bool sep_base,
                                            const int (&code)[NF], uint2 packed, const CellGeo<NF> &geo, const CellFaces<NF> &cf,
                                            const float4 *own, const float4 *A, int sa, const GroupDev *lg,
                                            const float bsave[Q], int bsave_k, const float4 *stash, int ss,
                                            const float4 *lneq, const float (&cr)[3]) {
    float hi[Q], gxi[Q], gyi[Q];
    hi[0] = h0;
    rd_f(own, sa, hi);
    rd_g(own, sa, gxi, gyi);
    const Macro mi = NEQ ? Macro{} : moments(hi, d.ref);   // (boundary values come staged with NEQ)
    float acc[Q];
#pragma unroll
    for (int a = 0; a < Q; a++) acc[a] = 0.f;
    uint32_t bm = 0u;                     // boundary faces (padded slots have no face)
#pragma unroll
    for (int k = 0; k < NF; k++) {
        if (code[k] < 0) {
            if (code[k] >= PAD_BELOW) bm |= 1u << k;
            continue;
        }
        const float2 v0 = cf.v[k], v1 = cf.v[k + 1 == NF ? 0 : k + 1];
        const float2 g = scaled_normal(v0, v1, cf.inva);
        const float2 r = make_float2(0.5f * (v0.x + v1.x), 0.5f * (v0.y + v1.y));   // x_f - x_i
        const float2 q = make_float2(r.x - geo.dk[k].x, r.y - geo.dk[k].y);       // x_f - x_j
        const float4 *rec = A + code[k];                                          // neighbours are in region A
        float hj[Q], gxj[Q], gyj[Q];
        rd_f(rec, sa, hj);
        rd_g(rec, sa, gxj, gyj);
        // upwind side (Eq. 11): one comparison per pair of opposite directions, whose
        // e.n differ in sign only (where e.n = 0 the choice is multiplied by zero)
        bool up[Q];
        up[1] = g.x > 0.f;
        up[2] = g.y > 0.f;
        up[5] = edot(5, g.x, g.y) > 0.f;
        up[6] = edot(6, g.x, g.y) > 0.f;
        up[3] = !up[1];
        up[4] = !up[2];
        up[7] = !up[5];
        up[8] = !up[6];
#pragma unroll
        for (int a = 1; a < Q; a++) {
            if (!in_set(H, a)) continue;
            const float en = edot(a, g.x, g.y);
            const float own_v = fmaf(gyi[a], r.y, fmaf(gxi[a], r.x, hi[a]));
            const float nb_v = fmaf(gyj[a], q.y, fmaf(gxj[a], q.x, hj[a]));
            acc[a] = fmaf(en, up[a] ? own_v : nb_v, acc[a]);
        }
    }
    if (bm) boundary_flux<NF, H, STASH>(d, hi, gxi, gyi, mi, packed, bm, geo, cf, lg, bsave, bsave_k, stash, ss, acc);

    float neq[Q];
    if constexpr (NEQ) {
        const float4 n0 = lneq[0], n1 = lneq[ss], n2 = lneq[2 * ss];
        neq[0] = n0.x; neq[1] = n0.y; neq[2] = n0.z; neq[3] = n0.w;
        neq[4] = n1.x; neq[5] = n1.y; neq[6] = n1.z; neq[7] = n1.w;
        neq[8] = n2.x;
    } else {
        collision_neq(hi, d.ref, neq);
    }

    // RHS = -sum (e.n dl/A) phi - (f - f_eq)/tau  (Eq. 10), then the update.
    // (The uniform mode test stays inside the direction loop.  Written as one
    // switch per cell, hipcc 7.2 emitted the Adams-Bashforth path with its store
    // offset register never set on one branch: the IR was right, the machine code
    // was not.)
    const uint32_t o4 = (uint32_t)i * 4u;
    const size_t pb4 = (size_t)d.np * 4;
    const int mode = M0 ? 0 : d.mode;
    static_assert(H < 0 || M0, "a split update is a base + coef RHS update");
    float bv[Q], inc[Q];
#pragma unroll
    for (int a = 0; a < Q; a++) {
        const float rhs = fmaf(neq[a], d.inv_tau, -acc[a]);
        if (mode == 0) {
            bv[a] = sep_base ? base[a] : hi[a];
            inc[a] = d.coef * rhs;
        } else if (mode == 3) {
            sto<float>(plane(d.dst, pb4, a), o4, rhs);
        } else {
            const float prev = (mode == 1) ? rhs : ldo<float>(plane(d.rhs_prev, pb4, a), o4);
            bv[a] = hi[a];
            inc[a] = (0.5f * d.coef) * (3.f * rhs - prev);
            sto<float>(plane(d.rhs_prev, pb4, a), o4, rhs);
        }
    }
    if constexpr (STORE == FVLBM_STORE_FP16_DEV) {
        // the last stage of a step: the exact base is the stored one less the carried
        // rounding residual of its conserved moments (loaded in phase 1 into cr)
        if (d.mcarry) {
#pragma unroll
            for (int a = 0; a < Q; a++) bv[a] += carry_correction(a, cr, d.ref.scale);
        }
    }
    if constexpr (H >= 0)
        store_half<STORE, H>(d.dst, (size_t)d.np, i, bv, inc, d.ref, (uint32_t)i);
    else if (mode != 3)
        store_cell<STORE>(d.dst, (size_t)d.np, i, bv, inc, d.ref, (uint32_t)i,
                          STORE == FVLBM_STORE_FP16_DEV ? d.mcarry : nullptr);
}

// The values a tile's loads depend on (kernel arguments for a single instance).
struct Hot {
    const void *src, *base;
    const int *halo_idx;
    const uint2 *halo_code, *lnbr;
    const float2 *dxy, *vxy;
    int np, n_cells, h1s, h2s;
};

// One RHS evaluation and update for one tile of T cells.
//   Phase 1  one round of loads: the tile's values, both halo rings' values
//            (to LDS), this thread's cell geometry and faces, its ring-1
//            slot's geometry and the update base (to registers); halo slots
//            sit at fixed positions, so only the halo values wait on an index;
//   Phase 2  gradients of tile and ring-1 cells into LDS (each computed once);
//   Phase 3  per tile cell: face values (own gradient outgoing, staged
//            neighbour value and gradient incoming), flux sum, BGK source,
//            update, store.
// With RING one more wave takes the halo slots: their loads in phase 1 and the
// ring-1 gradients in phase 2, beside the tile's own (and, with 64-cell tiles,
// half of phase 3).
// Dynamic LDS: nA = T + (largest ring-1 slot count) region-A records, then
// region-B records for the largest ring-2 slot count (sized by the launcher).
template <int NF, int STORE, int TC, bool DIRECT, bool M0, bool RING>
__device__ __forceinline__ void tile_body(const InstDesc *__restrict__ descs, int2 u, const Hot &hot, float4 *A,
                                          int sa, float4 *B) {
    // TC: the tile size, or 0 for a tile size chosen at launch (the block size)
    const int T = TC ? TC : (int)blockDim.x;
    const InstDesc &d = descs[u.x];
    // Two descriptor lines (reference state and update coefficients) are first
    // needed at the end of phase 1 (the split form's collision terms) or in
    // phases 2 and 3; one word of each is read here, so that their trip to the
    // scalar cache overlaps the phase-1 loads.
    const float warm0 = d.ref.rho0, warm1 = d.ref.c0[1];
    // the values the first loads depend on: kernel arguments for a single instance
    // (no descriptor load on the path to the first loads), else the descriptor
    const void *src = DIRECT ? hot.src : d.src;
    const int n_cells = DIRECT ? hot.n_cells : d.n_cells;
    const int h1s = DIRECT ? hot.h1s : d.h1s, h2s = DIRECT ? hot.h2s : d.h2s;
    const int *halo_idx = DIRECT ? hot.halo_idx : d.halo_idx;
    const size_t np = (size_t)(DIRECT ? hot.np : d.np);
    const uint2 *halo_code = DIRECT ? hot.halo_code : d.halo_code;
    const uint2 *lnbr = DIRECT ? hot.lnbr : d.lnbr;
    const float2 *dxy = DIRECT ? hot.dxy : d.dxy;
    const float2 *vxy = DIRECT ? hot.vxy : d.vxy;
    const int tile = u.y;
    const int tid = threadIdx.x;
    // RING: threads [0, T) own the tile's cells and one more wave, [T, T + 64),
    // owns the halo slots (outside the split form two waves when the larger ring
    // holds more than 64 slots), so halo loads and ring-1 gradients run
    // beside the tile's own; otherwise thread t owns tile cell t and halo slot t.
    // With 64-cell tiles (SPLIT3) two more waves form directions 5-8 of the
    // phase-2 gradients, one for the tile's cells (thread T + 64 + l: cell l), one
    // for the ring-1 slots (thread T + 128 + s: slot s), the tile and halo waves
    // directions 1-4; phase 3 is split over the four waves by direction sets
    // (0, 1, 3 | 2, 4 | 5, 7 | 6, 8), lane l of each taking tile cell l.
    // Opposite directions share a set, so every value is the one the whole pass
    // forms.
    constexpr bool SPLIT3 = split_form(TC, STORE, RING);
    // halo slots per pass: the halo waves' lanes (RING), else the tile's threads
    const int RS = RING ? (SPLIT3 ? 64 : (int)blockDim.x - T) : T;
    constexpr int GA = SPLIT3 ? 0 : -1;               // gradient half of the tile and halo waves
    // SPLIT3: phi_k - h of the tile cells' boundary slots, formed in phase 2 by
    // the tile's two waves (each its half of the directions), staged for the
    // phase-3 direction sets of every wave (the first slot of each also stays in
    // registers): float4 planes of T cells
    __shared__ float4 lstash[SPLIT3 ? TC * NF * 2 : 1];
    // SPLIT3: the tile cells' phase-3 geometry (neighbour codes, h0, 1/A, stencil
    // offsets, corners), written by the tile's wave in phase 1 for the waves that
    // take the other direction sets: GP float4 planes of T cells
    constexpr int GP = 5;
    __shared__ float4 lgeo[SPLIT3 ? TC * GP : 1];
    // SPLIT3: the tile cells' collision term f_eq - f (a function of the cell's
    // own state), formed once in phase 1 by the wave for directions 5-8 of the
    // tile cells (which waits at the barrier longest): 3 float4 planes
    __shared__ float4 lneq[SPLIT3 ? TC * 3 : 1];
    const int wtid = RING ? __builtin_amdgcn_readfirstlane(tid) : 0;   // (wave-uniform)
    const bool ownw = !RING || wtid < T;                               // the tile's cells
    const bool ownb = SPLIT3 && wtid >= T + 64 && wtid < T + 128;      // their directions 5-8
    const bool halob = SPLIT3 && wtid >= T + 128;                      // ring-1 directions 5-8
    const bool halow = RING && !ownw && !ownb && !halob;               // the halo slots
    const int rj = !RING ? tid : halow ? tid - T : halob ? tid - T - 128 : -1;   // halo slot (< 0: none)
    const int ob = tid - T - 64;                      // ownb: this thread's tile cell
    const int i = tile * T + tid;
    const bool valid = ownw && i < n_cells;
    const bool validb = ownb && tile * T + ob < n_cells;
    const int a_end = T + h1s;                     // local indices below this are region A
    const int *hidx = halo_idx + (size_t)tile * (size_t)(h1s + h2s);

    // ---- phase 1
    // Straight-line loads (indices clamped into range instead of branching, so
    // the compiler can wait on each load precisely): halo slot indices first,
    // then the own cell's data, then the halo values as soon as their indices
    // return; last the loads whose bases may arrive a level later (ring-1 codes,
    // group table, update base).
    const int hs = h1s + h2s;
    const bool rin = rj >= 0;
    float h0 = 0.f, base[Q], f[Q];
    int code[NF];
    CellGeo<NF> geo;
    CellFaces<NF> cf;
    uint2 ln = make_uint2(0u, 0u);
    int hraw1 = -1, hraw2 = -1;
    // (the tile's halo tables are read once here, non-temporally; the later
    // passes that read them again find them in L2 or the Infinity Cache)
    if (!RING)
        hraw1 = ldn1(hidx, tid < hs ? tid : 0), hraw2 = ldn1(hidx, h1s + tid < hs ? h1s + tid : 0);
    const int ic = valid ? i : 0;
    if (ownw) {
        load_cell<STORE>(src, np, ic, f, d.ref);
        const uint2v t = ldn<uint2v>(lnbr, (uint32_t)ic * 8u);
        ln = make_uint2(t.x, t.y);
        geo.load(dxy, np, ic);
        cf.load(vxy, np, ic);
    }
    if (SPLIT3 && ownb) {                             // the cell's state and stencil
        const int icb = validb ? tile * T + ob : 0;
        load_cell<STORE>(src, np, icb, f, d.ref);
        ln = ldo<uint2>(lnbr, (uint32_t)icb * 8u);
        geo.load(dxy, np, icb);
    }
    if (halow)
        hraw1 = ldn1(hidx, rj < hs ? rj : 0), hraw2 = ldn1(hidx, h1s + rj < hs ? h1s + rj : 0);
    if (SPLIT3 && halob) hraw1 = ldg(hidx, rj < hs ? rj : 0);
    const int i3 = tile * T + rj;                     // SPLIT3: this halo lane's tile cell
    const bool valid3 = SPLIT3 && (halow || halob) && i3 < n_cells;
    const bool rin2 = rin && !halob;                  // this thread stages halo values
    const int c1 = rin && rj < h1s ? hraw1 : -1;
    const int c2 = rin2 && rj < h2s ? hraw2 : -1;
    int hcode[NF];
    float hf0 = 0.f, f1[Q], f2[Q];
    CellGeo<NF> hgeo;
    uint2 hl = make_uint2(0u, 0u);
    if (!RING || halow) {
        load_cell<STORE>(src, np, c1 >= 0 ? c1 : 0, f1, d.ref);
        hgeo.load(dxy, np, c1 >= 0 ? c1 : 0);
        load_cell<STORE>(src, np, c2 >= 0 ? c2 : 0, f2, d.ref, 1);
        const uint2v t = ldn<uint2v>(halo_code + (size_t)tile * h1s + (rin && rj < h1s ? rj : 0), 0u);
        hl = make_uint2(t.x, t.y);
    }
    if (SPLIT3 && halob) {                            // the ring-1 cell's h0 and stencil
        load_cell<STORE>(src, np, c1 >= 0 ? c1 : 0, f1, d.ref, 0, 1);
        hgeo.load(dxy, np, c1 >= 0 ? c1 : 0);
        hl = ldg(halo_code, (size_t)tile * h1s + (rin && rj < h1s ? rj : 0));
    }
    // the instance's boundary groups, staged in LDS for the boundary slots (read
    // whole, without waiting for the group count)
    __shared__ GroupDev lg[MAX_GROUPS];
    const int BS = (int)blockDim.x;                   // threads per block
    constexpr int GW = MAX_GROUPS * (int)(sizeof(GroupDev) / sizeof(int));
    const int *gsrc = reinterpret_cast<const int *>(d.groups);
    const int gv0 = ldg(gsrc, tid < GW ? tid : 0);
    const int gv1 = ldg(gsrc, BS < GW && tid + BS < GW ? tid + BS : 0);
    const void *basep = DIRECT ? hot.base : d.base;
    const bool sep_base = (M0 || d.mode == 0) && basep != src;
    // FP16 storage, the last stage of a step: the cell's carried moment residual
    float cr[3] = {0.f, 0.f, 0.f};
    if constexpr (STORE == FVLBM_STORE_FP16_DEV)
        if (ownw && d.mcarry) load_carry(d.mcarry, np, ic, cr);
    // update bases: the planes of this wave's phase-3 set
    if (ownw) {
        if (sep_base) {
            if constexpr (SPLIT3) load_set<STORE, 2>(basep, np, ic, base, d.ref);
            else load_cell<STORE, true>(basep, np, ic, base, d.ref);
        }
        h0 = f[0];
#pragma unroll
        for (int k = 0; k < NF; k++) code[k] = unpack16(k < 2 ? ln.x : ln.y, k & 1);
        geo.invert(code);
        cf.finish();
    } else if constexpr (SPLIT3) {
        if (halow) {
            if (sep_base) load_set<STORE, 3>(basep, np, valid3 ? i3 : 0, base, d.ref);
        } else if (halob) {
            if (sep_base) load_set<STORE, 5>(basep, np, valid3 ? i3 : 0, base, d.ref);
        } else if (ownb) {
            if (sep_base) load_set<STORE, 4>(basep, np, validb ? tile * T + ob : 0, base, d.ref);
            h0 = f[0];
#pragma unroll
            for (int k = 0; k < NF; k++) code[k] = unpack16(k < 2 ? ln.x : ln.y, k & 1);
            geo.invert(code);
        }
    }
    if (valid) wr_f(A + tid, sa, f);
    if constexpr (SPLIT3)
        if (valid) {
            float4 *g = lgeo + tid;
            g[0] = make_float4(__uint_as_float(ln.x), __uint_as_float(ln.y), h0, cf.inva);
            g[T] = make_float4(geo.dk[0].x, geo.dk[0].y, geo.dk[1].x, geo.dk[1].y);
            g[2 * T] = make_float4(geo.dk[2].x, geo.dk[2].y, geo.dk[NF - 1].x, geo.dk[NF - 1].y);
            g[3 * T] = make_float4(cf.v[0].x, cf.v[0].y, cf.v[1].x, cf.v[1].y);
            g[4 * T] = make_float4(cf.v[2].x, cf.v[2].y, cf.v[NF - 1].x, cf.v[NF - 1].y);
        }
    if constexpr (SPLIT3)
        if (validb) {
            float nq[Q];
            collision_neq(f, d.ref, nq);
            float4 *n = lneq + ob;
            n[0] = make_float4(nq[0], nq[1], nq[2], nq[3]);
            n[T] = make_float4(nq[4], nq[5], nq[6], nq[7]);
            n[2 * T] = make_float4(nq[8], 0.f, 0.f, 0.f);
        }
    if (c1 >= 0) {
        hf0 = f1[0];
        if (!halob) wr_f(A + T + rj, sa, f1);
#pragma unroll
        for (int k = 0; k < NF; k++) hcode[k] = unpack16(k < 2 ? hl.x : hl.y, k & 1);
        hgeo.invert(hcode);
    }
    if (c2 >= 0) wr_f(B + rj * RB, 1, f2);
    if (tid < GW) reinterpret_cast<int *>(lg)[tid] = gv0;
    if (BS < GW && tid + BS < GW) reinterpret_cast<int *>(lg)[tid + BS] = gv1;
    for (int k = rin2 ? rj + RS : h1s; k < h1s; k += RS) {   // ring 1 larger than a pass
        const int c = ldg(hidx, k);
        if (c < 0) continue;
        float g[Q];
        load_cell<STORE>(src, np, c, g, d.ref, 1);
        wr_f(A + T + k, sa, g);
    }
    for (int k = rin2 ? rj + RS : h2s; k < h2s; k += RS) {   // ring 2 larger than a pass
        const int c = ldg(hidx, h1s + k);
        if (c < 0) continue;
        float g[Q];
        load_cell<STORE>(src, np, c, g, d.ref, 1);
        wr_f(B + k * RB, 1, g);
    }
    asm volatile("" ::"s"(warm0), "s"(warm1));    // (keeps the two reads above)
    if constexpr (RING && !SPLIT3) {
        // Waves with a boundary face among their cells (own or ring-1) carry the
        // longest phase-2 and phase-3 chains, and their tiles end the launch: they
        // issue first on their SIMD.  (Measured: 1.4 % off the 128-cell ring form's
        // launch on a cylinder O-grid; the same test cost the split form and the
        // one-workgroup-per-tile forms about 1 %, so they do without it.)
        bool bnd = false;
        if (valid) {
#pragma unroll
            for (int k = 0; k < NF; k++) bnd = bnd || (code[k] < 0 && code[k] >= PAD_BELOW);
        }
        if (c1 >= 0) {
#pragma unroll
            for (int k = 0; k < NF; k++) bnd = bnd || (hcode[k] < 0 && hcode[k] >= PAD_BELOW);
        }
        if (__builtin_amdgcn_ballot_w64(bnd) != 0) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    if constexpr (SPLIT3) {
        // the other waves' phase-3 cells: their geometry from the tile's wave,
        // read now so that it has arrived when phase 3 starts (these registers
        // are not used in phase 2 by the waves that read them)
        const int gc = ownb ? ob : rj;
        if (validb || valid3) {
            const float4 *g = lgeo + gc;
            const float4 g0 = g[0], g1 = g[T], g2 = g[2 * T], g3 = g[3 * T], g4 = g[4 * T];
            cf.v[0] = make_float2(g3.x, g3.y);
            cf.v[1] = make_float2(g3.z, g3.w);
            cf.v[2] = make_float2(g4.x, g4.y);
            cf.v[NF - 1] = make_float2(g4.z, g4.w);
            cf.inva = g0.w;
            if (!ownb) {
                ln = make_uint2(__float_as_uint(g0.x), __float_as_uint(g0.y));
                h0 = g0.z;
                geo.dk[0] = make_float2(g1.x, g1.y);
                geo.dk[1] = make_float2(g1.z, g1.w);
                geo.dk[2] = make_float2(g2.x, g2.y);
                geo.dk[NF - 1] = make_float2(g2.z, g2.w);
#pragma unroll
                for (int k = 0; k < NF; k++) code[k] = unpack16(k < 2 ? ln.x : ln.y, k & 1);
            }
        }
    }

    // ---- phase 2
    float bsave[Q];                                // phi_k - h of the cell's first boundary slot, for phase 3
    int bsave_k = -1;
    {
        float hc[Q], gx[Q], gy[Q];
        int no_k = 0;
        if (valid) {
            hc[0] = h0;
            rd_f(A + tid, sa, hc);
            gradient_staged<NF, true, SPLIT3, GA>(d, geo, hc, code, ln, A, B, a_end, lg, gx, gy, bsave, bsave_k,
                                                  lstash + tid, T, sa);
            wr_g<GA>(A + tid, sa, gx, gy);
        }
        if constexpr (SPLIT3)
            if (validb) {
#pragma unroll
                for (int a = 0; a < Q; a++) hc[a] = f[a];   // (this wave loaded the cell's state)
                gradient_staged<NF, true, true, 1>(d, geo, hc, code, ln, A, B, a_end, lg, gx, gy, bsave, bsave_k,
                                                   lstash + ob, T, sa);
                wr_g<1>(A + ob, sa, gx, gy);
            }
        if (c1 >= 0) {
            hc[0] = hf0;
            rd_f(A + T + rj, sa, hc);
            if (SPLIT3 && halob) {
                gradient_staged<NF, false, false, 1>(d, hgeo, hc, hcode, hl, A, B, a_end, lg, gx, gy, hc, no_k,
                                                     nullptr, 0, sa);
                wr_g<1>(A + T + rj, sa, gx, gy);
            } else {
                gradient_staged<NF, false, false, GA>(d, hgeo, hc, hcode, hl, A, B, a_end, lg, gx, gy, hc, no_k,
                                                      nullptr, 0, sa);
                wr_g<GA>(A + T + rj, sa, gx, gy);
            }
        }
        for (int k = rin ? rj + RS : h1s; k < h1s; k += RS) {
            const int c = ldg(hidx, k);
            if (c < 0) continue;
            const uint2 hl2 = ldg(halo_code, (size_t)tile * h1s + k);
            int cc[NF];
#pragma unroll
            for (int s = 0; s < NF; s++) cc[s] = unpack16(s < 2 ? hl2.x : hl2.y, s & 1);
            CellGeo<NF> g2;
            g2.load(dxy, np, c);
            g2.invert(cc);
            {
                float t[Q];
                load_cell<STORE>(src, np, c, t, d.ref, 0, 1);
                hc[0] = t[0];
            }
            rd_f(A + T + k, sa, hc);
            if (SPLIT3 && halob) {
                gradient_staged<NF, false, false, 1>(d, g2, hc, cc, hl2, A, B, a_end, lg, gx, gy, hc, no_k, nullptr, 0,
                                                     sa);
                wr_g<1>(A + T + k, sa, gx, gy);
            } else {
                gradient_staged<NF, false, false, GA>(d, g2, hc, cc, hl2, A, B, a_end, lg, gx, gy, hc, no_k, nullptr,
                                                      0, sa);
                wr_g<GA>(A + T + k, sa, gx, gy);
            }
        }
    }
    __syncthreads();
    if (valid)
        tile_update<NF, STORE, M0, SPLIT3 ? 2 : -1, SPLIT3, SPLIT3>(d, i, h0, base, sep_base, code, ln, geo, cf,
                                                                    A + tid, A, sa, lg, bsave, bsave_k, lstash + tid,
                                                                    T, lneq + tid, cr);
    if constexpr (SPLIT3) {
        if (validb)
            tile_update<NF, STORE, M0, 4, true, true>(d, tile * T + ob, h0, base, sep_base, code, ln, geo, cf, A + ob,
                                                      A, sa, lg, bsave, bsave_k, lstash + ob, T, lneq + ob, cr);
        if (valid3 && halow)
            tile_update<NF, STORE, M0, 3, true, true>(d, i3, h0, base, sep_base, code, ln, geo, cf, A + rj, A, sa, lg,
                                                      bsave, -1, lstash + rj, T, lneq + rj, cr);
        if (valid3 && halob)
            tile_update<NF, STORE, M0, 5, true, true>(d, i3, h0, base, sep_base, code, ln, geo, cf, A + rj, A, sa, lg,
                                                      bsave, -1, lstash + rj, T, lneq + rj, cr);
    }
}

// DIRECT: one instance whose unit b is tile b, the bases and sizes its loads
// need passed as arguments; the first fourteen dwords (up to units_x) reach
// scalar registers with the wave, so no descriptor or argument load precedes
// the first loads (the ring-1 codes and the base are read one level later, as
// the halo values are); otherwise units are read from the table and everything
// from the descriptors.  units_x = 2 n_units + (XCD remap on), h12 = h1s + 2^16 h2s.
// M0: the stage is a base + coef RHS update (Euler, RK stages), fixed at compile
// time, so the update carries no mode tests; otherwise the mode is read from the
// descriptor (Adams-Bashforth, RHS output).
// (Arguments in the order the kernel needs them: the first sixteen dwords arrive in
// scalar registers.)
template <int NF, int STORE, int T, bool DIRECT, bool M0, bool RING>
__global__ void __launch_bounds__(max_tile_threads(T, STORE, RING)) k_tile(const int *hot_halo_idx, const void *hot_src, const uint2 *hot_lnbr,
                                            const float2 *hot_dxy, const float2 *hot_vxy, int hot_h12, int hot_np,
                                            int hot_n_cells, int units_x, const uint2 *hot_halo_code, const void *hot_base,
                                            const InstDesc *__restrict__ descs, int nA,
                                            const int2 *__restrict__ units, unsigned *) {
    extern __shared__ float4 lds4[];
    const int ub = remap_block(blockIdx.x, units_x >> 1, units_x & 1);
    const Hot hot{hot_src, hot_base, hot_halo_idx, hot_halo_code, hot_lnbr, hot_dxy, hot_vxy,
                  hot_np, hot_n_cells, hot_h12 & 0xffff, hot_h12 >> 16};
    // region-A records: T + h1s for a single instance (preloaded, so the first LDS
    // writes wait on no argument load), else the largest over the instances
    const int sa = DIRECT ? (T ? T : (int)blockDim.x) + (hot_h12 & 0xffff) : nA;
    tile_body<NF, STORE, T, DIRECT, M0, RING>(descs, (DIRECT || !units) ? make_int2(0, ub) : units[ub], hot, lds4,
                                             sa, lds4 + sa * RA);
}

// Work queue of the persistent form: XCD x owns units [x n / 8, (x + 1) n / 8)
// and a ticket counter of its own (one 128-byte line each, so the eight
// counters' atomics proceed in parallel and an XCD's units, contiguous in the
// cell order, share its L2), then a count of the workgroups that have left.
constexpr int QUEUE_STRIDE = 32;                 // uints between counters
constexpr int QUEUE_DONE = 8 * QUEUE_STRIDE;
__device__ inline int queue_lo(int n, int x) { return (int)((long long)n * x / 8); }

// The unit a ticket of XCD x's counter names, or -1 past the end of x's range.
__device__ inline int queue_unit(int n, int x, unsigned t) {
    const int lo = queue_lo(n, x), hi = queue_lo(n, x + 1);
    return t < (unsigned)(hi - lo) ? lo + (int)t : -1;
}

// A unit from any XCD's range once x's own is used up, or n when every range is:
// counters only grow, so one whose value is past its range is skipped without an
// atomic.
__device__ inline int queue_steal(unsigned *queue, int n, int x) {
    for (int k = 1; k < 8; k++) {
        const int y = (x + k) & 7;
        const unsigned seen = __hip_atomic_load(queue + y * QUEUE_STRIDE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (queue_unit(n, y, seen) < 0) continue;
        const int u = queue_unit(n, y, atomicAdd(queue + y * QUEUE_STRIDE, 1u));
        if (u >= 0) return u;
    }
    return n;
}

// Persistent form: a grid sized to the resident capacity takes units from the
// work queue above, so a workgroup starts its next unit as soon as it is done
// with one, and fast workgroups take more units than slow ones.  The ticket for
// the next unit is taken at the start of each unit and read at its end, so its
// round trip overlaps the unit.  A ticket is handed out once, so every unit is
// processed exactly once; every workgroup leaves once all ranges are used up,
// and the last to leave clears the queue for the next launch (launches on one
// queue never overlap: they are ordered on the solver's or batch's stream).
// Mode-0 stages only.
// DIRECT: a single instance (unit b is tile b) with its first-load values as
// arguments; else units from the table (null: a single instance).
template <int NF, int STORE, int T, bool DIRECT>
__global__ void __launch_bounds__(T ? T : 512) __attribute__((amdgpu_waves_per_eu(NF == 3 ? 4 : 1)))
k_tile_persistent(const int *hot_halo_idx, const void *hot_src, const uint2 *hot_lnbr, const float2 *hot_dxy,
                  const float2 *hot_vxy, int hot_h12, int hot_np, int hot_n_cells, int units_x,
                  const uint2 *hot_halo_code, const void *hot_base, const InstDesc *__restrict__ descs, int nA,
                  const int2 *__restrict__ units, unsigned *queue) {
    extern __shared__ float4 lds4[];
    __shared__ int next_unit;
    const Hot hot{hot_src, hot_base, hot_halo_idx, hot_halo_code, hot_lnbr, hot_dxy, hot_vxy,
                  hot_np, hot_n_cells, hot_h12 & 0xffff, hot_h12 >> 16};
    const int n_units = units_x >> 1;
    const int sa = DIRECT ? (T ? T : (int)blockDim.x) + (hot_h12 & 0xffff) : nA;
    // the XCD this workgroup runs on (hardware register XCC_ID)
    const int xcd = (int)(__builtin_amdgcn_s_getreg((15 << 11) | 20) & 7u);
    unsigned *own = queue + xcd * QUEUE_STRIDE;
    if (threadIdx.x == 0) {
        const int u = queue_unit(n_units, xcd, atomicAdd(own, 1u));
        next_unit = u >= 0 ? u : queue_steal(queue, n_units, xcd);
    }
    __syncthreads();
    int b = next_unit;
    while (b < n_units) {
        unsigned ticket = 0;
        if (threadIdx.x == 0) ticket = atomicAdd(own, 1u);
        tile_body<NF, STORE, T, DIRECT, true, false>(descs, (DIRECT || !units) ? make_int2(0, b) : units[b], hot,
                                                     lds4, sa, lds4 + sa * RA);
        if (threadIdx.x == 0) {      // (every wave read the last value before this unit's barriers)
            const int u = queue_unit(n_units, xcd, ticket);
            next_unit = u >= 0 ? u : queue_steal(queue, n_units, xcd);
        }
        __syncthreads();             // the next unit reuses the LDS records
        b = next_unit;
    }
    if (threadIdx.x == 0 && atomicAdd(queue + QUEUE_DONE, 1u) == gridDim.x - 1) {
        for (int x = 0; x < 8; x++) atomicExch(queue + x * QUEUE_STRIDE, 0u);
        atomicExch(queue + QUEUE_DONE, 0u);
    }
}

template <int NF, int STORE, int T>
const void *fn(bool persistent, bool direct, bool m0, bool ring) {
    if (!m0)    // runtime mode: one block per unit (the launchers never ask for persistence here)
        return direct ? reinterpret_cast<const void *>(&k_tile<NF, STORE, T, true, false, false>)
                      : reinterpret_cast<const void *>(&k_tile<NF, STORE, T, false, false, false>);
    if (persistent)
        return direct ? reinterpret_cast<const void *>(&k_tile_persistent<NF, STORE, T, true>)
                      : reinterpret_cast<const void *>(&k_tile_persistent<NF, STORE, T, false>);
    if constexpr (T != 0 && T <= 128)   // a ring wave: single instance, mode 0, tiles of 64 or 128 cells
        if (ring && direct) return reinterpret_cast<const void *>(&k_tile<NF, STORE, T, true, true, true>);
    return direct ? reinterpret_cast<const void *>(&k_tile<NF, STORE, T, true, true, false>)
                  : reinterpret_cast<const void *>(&k_tile<NF, STORE, T, false, true, false>);
}

template <int NF, int STORE>
const void *pick_t(int T, bool persistent, bool direct, bool m0, bool ring) {
    switch (T) {
    case 64: return fn<NF, STORE, 64>(persistent, direct, m0, ring);
    case 128: return fn<NF, STORE, 128>(persistent, direct, m0, ring);
    case 256: return fn<NF, STORE, 256>(persistent, direct, m0, ring);
    case 512: return fn<NF, STORE, 512>(persistent, direct, m0, ring);
    default: return fn<NF, STORE, 0>(persistent, direct, m0, ring);   // other multiples of 64: set at launch
    }
}

const void *pick(int nf, int storage, int T, bool persistent, bool direct, bool m0, bool ring) {
    if (nf == 3) {
        if (storage == FVLBM_STORE_FP32) return pick_t<3, FVLBM_STORE_FP32>(T, persistent, direct, m0, ring);
        if (storage == FVLBM_STORE_FP32_DEV) return pick_t<3, FVLBM_STORE_FP32_DEV>(T, persistent, direct, m0, ring);
        if (storage == FVLBM_STORE_I16_DEV) return pick_t<3, FVLBM_STORE_I16_DEV>(T, persistent, direct, m0, ring);
        return pick_t<3, FVLBM_STORE_FP16_DEV>(T, persistent, direct, m0, ring);
    }
    if (storage == FVLBM_STORE_FP32) return pick_t<4, FVLBM_STORE_FP32>(T, persistent, direct, m0, ring);
    if (storage == FVLBM_STORE_FP32_DEV) return pick_t<4, FVLBM_STORE_FP32_DEV>(T, persistent, direct, m0, ring);
    if (storage == FVLBM_STORE_I16_DEV) return pick_t<4, FVLBM_STORE_I16_DEV>(T, persistent, direct, m0, ring);
    return pick_t<4, FVLBM_STORE_FP16_DEV>(T, persistent, direct, m0, ring);
}

// Grid of a launch: one block per unit, or (persistent) the number of blocks
// the device holds at once, rounded down to a multiple of 8 (one per XCD).
int grid_blocks(const UnitTable &ut, int persistent, int nf, int storage, size_t lds, bool direct) {
    if (!persistent) return ut.n_units;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pick(nf, storage, ut.block, true, direct, true, false),
                                                     ut.block, lds) != hipSuccess)
        per_cu = 1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    int g = std::max(8, (per_cu > 0 ? per_cu : 1) * cus / 8 * 8);
    return std::min(g, (ut.n_units + 7) / 8 * 8);
}

}  // namespace

StageArgs stage_args(const InstDesc *descs_dev, const UnitTable &ut, int xcd_remap, int persistent, int h1max,
                     const InstDesc *host_desc) {
    StageArgs a{};
    a.d = descs_dev;
    a.u = ut.units;
    a.ux = 2 * ut.n_units + (xcd_remap ? 1 : 0);
    a.nA = ut.block + h1max;
    // (a single-instance launch sizes region A from its own ring-1 slot count)
    a.queue = ut.queue;
    a.direct = ut.direct && host_desc && a.nA == ut.block + host_desc->h1s;
    if (a.direct) {
        a.src = host_desc->src;
        a.base = host_desc->base;
        a.hidx = host_desc->halo_idx;
        a.hcode = host_desc->halo_code;
        a.lnbr = host_desc->lnbr;
        a.dxy = host_desc->dxy;
        a.vxy = host_desc->vxy;
        a.np = host_desc->np;
        a.nc = host_desc->n_cells;
        a.h12 = host_desc->h1s | (host_desc->h2s << 16);
    }
    return a;
}

size_t stage_lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        v = 65536;
    // less the staged group table, and the boundary stash (up to 4 slots x 2
    // float4), phase-3 geometry (5 float4) and collision terms (3 float4) of
    // 64-cell halo-wave tiles
    return (size_t)v - sizeof(GroupDev) * MAX_GROUPS - sizeof(float4) * 64 * (4 * 2 + 5 + 3);
}

size_t stage_lds_bytes(int T, int h2max, int h1max) {
    return ((size_t)(T + h1max) * RA + (size_t)h2max * RB) * sizeof(float4);
}

hipError_t launch_stage(const InstDesc *descs_dev, const UnitTable &ut, int nf, int storage,
                        int xcd_remap, int persistent, int h2max, int h1max, bool mode0, hipStream_t stream,
                        const InstDesc *host_desc) {
    if (ut.n_units == 0) return hipSuccess;
    const bool ring_form = persistent == 2;
    if (!mode0 || ring_form) persistent = 0;
    StageArgs a = stage_args(descs_dev, ut, xcd_remap, persistent, h1max, host_desc);
    const bool ring = ring_form && mode0 && a.direct && ut.block <= 128;
    void *args[] = {&a.hidx, &a.src, &a.lnbr, &a.dxy, &a.vxy, &a.h12, &a.np, &a.nc, &a.ux, &a.hcode, &a.base,
                    &a.d, &a.nA, &a.u, &a.queue};
    const size_t lds = stage_lds_bytes(ut.block, h2max, h1max);
    const void *fn_ptr = pick(nf, storage, ut.block, persistent, a.direct, mode0, ring);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn_ptr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipLaunchKernel(fn_ptr, dim3(grid_blocks(ut, persistent, nf, storage, lds, a.direct)),
                           dim3(tile_threads(ut.block, storage, ring, halo_waves(std::max(h1max, h2max)))),
                           args, lds, stream);
}

namespace {
// Kernel-node parameters of one stage launch (as launch_stage() would launch it).
// argbuf: caller-owned storage (a StageArgs block in argbuf[0], then one pointer per
// argument: argbuf[1..15]), alive until the node is added or set.
hipError_t stage_node_params(hipKernelNodeParams *p, const InstDesc *descs_dev, const UnitTable &ut, int nf,
                             int storage, int xcd_remap, int persistent, int h2max, int h1max, bool mode0,
                             void **argbuf, const InstDesc *host_desc) {
    const bool ring_form = persistent == 2;
    if (!mode0 || ring_form) persistent = 0;
    StageArgs *a = reinterpret_cast<StageArgs *>(argbuf[0]);
    *a = stage_args(descs_dev, ut, xcd_remap, persistent, h1max, host_desc);
    const bool ring = ring_form && mode0 && a->direct && ut.block <= 128;
    void **kp = argbuf + 1;
    kp[0] = &a->hidx; kp[1] = &a->src; kp[2] = &a->lnbr; kp[3] = &a->dxy; kp[4] = &a->vxy; kp[5] = &a->h12;
    kp[6] = &a->np; kp[7] = &a->nc; kp[8] = &a->ux; kp[9] = &a->hcode; kp[10] = &a->base; kp[11] = &a->d;
    kp[12] = &a->nA; kp[13] = &a->u; kp[14] = &a->queue;
    *p = hipKernelNodeParams{};
    const size_t lds = stage_lds_bytes(ut.block, h2max, h1max);
    p->func = const_cast<void *>(pick(nf, storage, ut.block, persistent, a->direct, mode0, ring));
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(p->func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    p->gridDim = dim3(grid_blocks(ut, persistent, nf, storage, lds, a->direct));
    p->blockDim = dim3(tile_threads(ut.block, storage, ring, halo_waves(std::max(h1max, h2max))));
    p->sharedMemBytes = (unsigned)lds;
    p->kernelParams = kp;
    p->extra = nullptr;
    return hipSuccess;
}
}  // namespace

hipError_t add_stage_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, int ndeps,
                          const InstDesc *descs_dev, const UnitTable &ut, int nf, int storage,
                          int xcd_remap, int persistent, int h2max, int h1max, bool mode0, void **argbuf,
                          const InstDesc *host_desc) {
    hipKernelNodeParams p;
    hipError_t e = stage_node_params(&p, descs_dev, ut, nf, storage, xcd_remap, persistent, h2max, h1max, mode0,
                                     argbuf, host_desc);
    if (e != hipSuccess) return e;
    return hipGraphAddKernelNode(node, g, deps, ndeps, &p);
}

hipError_t set_stage_node(hipGraphExec_t ex, hipGraphNode_t node, const InstDesc *descs_dev, const UnitTable &ut,
                          int nf, int storage, int xcd_remap, int persistent, int h2max, int h1max, bool mode0,
                          void **argbuf) {
    hipKernelNodeParams p;
    hipError_t e = stage_node_params(&p, descs_dev, ut, nf, storage, xcd_remap, persistent, h2max, h1max, mode0,
                                     argbuf, nullptr);
    if (e != hipSuccess) return e;
    return hipGraphExecKernelNodeSetParams(ex, node, &p);
}

}  // namespace fvlbm

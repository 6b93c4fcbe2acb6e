// Step 0 (equilibrium initialisation), Step 6 (macroscopic fields) and the
// FP64 reductions (mass, velocity residual of Eq. 32, non-finite flag), plus
// FP64 <-> storage conversions used by checkpoints and tests.
#include "fvlbm_internal.h"

namespace fvlbm {
namespace {

__device__ constexpr int EXd[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EYd[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr double WD[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
// the FP32 weights the step kernels use; the FP16 unit w S is formed as a float
// product on both sides so they agree bitwise
__device__ constexpr float WF[Q] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                                    1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
constexpr int RB = 256;   // reduction block

// the reference equilibrium f_eq(rho0, u_dev) as the step kernels see it (FP32)
__device__ inline double wref(int a, const RefDev &r) { return (double)r.fref[a]; }

// exact widening of cell i's stored values to the FP64 deviations h = f - f_ref
__device__ inline void load_cell_dev(const void *p, int storage, int np, int i, const RefDev &r, double h[Q]) {
    if (storage == FVLBM_STORE_I16_DEV) {             // h_a = q_a 2^(s - 142)
        const int sb = static_cast<const uint8_t *>(p)[(size_t)np * 18 + i];
        for (int a = 0; a < Q; a++)
            h[a] = sb ? ldexp((double)static_cast<const int16_t *>(p)[(size_t)a * np + i], sb - 142) : 0.0;
        return;
    }
    for (int a = 0; a < Q; a++) {
        const size_t idx = (size_t)a * np + i;
        if (storage == FVLBM_STORE_FP32) h[a] = (double)static_cast<const float *>(p)[idx] - wref(a, r);
        else if (storage == FVLBM_STORE_FP32_DEV) h[a] = (double)static_cast<const float *>(p)[idx];
        else h[a] = (double)__half2float(static_cast<const __half *>(p)[idx]) * (double)(WF[a] * r.scale);
    }
}

// FP16 storage: the cell's carried moment residual R (mass, momentum less the
// exact ones, units of S; 3 FP16 planes scaled by 2^20, as the step kernel
// writes them) taken out of the deviations as the equilibrium-shaped change
// -S w_a (R_0 + 3 e_a . R).
constexpr double CARRY_SCALE = 1048576.0;
__device__ inline void uncarry(const __half *carry, int np, int i, const RefDev &r, double h[Q]) {
    if (!carry) return;
    double R[3];
    for (int k = 0; k < 3; k++) R[k] = (double)__half2float(carry[(size_t)k * np + i]) / CARRY_SCALE;
    for (int a = 0; a < Q; a++) h[a] -= (double)r.scale * WD[a] * (R[0] + 3.0 * (EXd[a] * R[1] + EYd[a] * R[2]));
}

// round-to-nearest narrowing of FP64 deviations into cell i's storage (FP16
// storage with a carry: the rounding residual of the cell's mass and momentum
// is written to it)
__device__ inline void store_cell_dev(void *p, int storage, int np, int i, const double h[Q], const RefDev &r,
                                      __half *carry = nullptr) {
    if (storage == FVLBM_STORE_I16_DEV) {
        double m = 0.0;
        for (int a = 0; a < Q; a++) m = fmax(m, fabs(h[a]));
        // 2^(s - 127) just above m (taken from m as a float; one bit of headroom if that rounds up)
        const int sb = m > 0.0 ? min((int)((__float_as_uint((float)m) >> 23) & 0xffu) + 1, 254) : 0;
        for (int a = 0; a < Q; a++) {
            const double x = sb ? ldexp(h[a], 142 - sb) : 0.0;
            const int q = max(-32767, min(32767, (int)rint(x)));
            static_cast<int16_t *>(p)[(size_t)a * np + i] = (int16_t)q;
        }
        static_cast<uint8_t *>(p)[(size_t)np * 18 + i] = (uint8_t)sb;
        return;
    }
    double R[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < Q; a++) {
        const size_t idx = (size_t)a * np + i;
        if (storage == FVLBM_STORE_FP32) static_cast<float *>(p)[idx] = (float)(wref(a, r) + h[a]);
        else if (storage == FVLBM_STORE_FP32_DEV) static_cast<float *>(p)[idx] = (float)h[a];
        else {
            const __half q = __float2half_rn((float)(h[a] / (double)(WF[a] * r.scale)));
            static_cast<__half *>(p)[idx] = q;
            const double e = ((double)__half2float(q) * (double)(WF[a] * r.scale) - h[a]) / (double)r.scale;
            R[0] += e; R[1] += EXd[a] * e; R[2] += EYd[a] * e;
        }
    }
    if (carry && storage == FVLBM_STORE_FP16_DEV)
        for (int k = 0; k < 3; k++)
            carry[(size_t)k * np + i] = __float2half_rn((float)fmin(fmax(R[k] * CARRY_SCALE, -65504.0), 65504.0));
}

// Step 0: f = f_eq(rho, u) (Eq. 3), written as deviations from the reference equilibrium.
__global__ void k_init_eq(void *dst, int storage, int n, int np, RefDev ref,
                          const double *rho, const double *u, const int *perm, double rho_u, __half *carry) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = perm[i];
    double r = rho ? rho[c] : rho_u;
    double ux = u ? u[2 * c] : 0.0, uy = u ? u[2 * c + 1] : 0.0;
    double uu = ux * ux + uy * uy;
    double h[Q];
    for (int a = 0; a < Q; a++) {
        double eu = EXd[a] * ux + EYd[a] * uy;
        double feq = WD[a] * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        h[a] = feq - wref(a, ref);
    }
    store_cell_dev(dst, storage, np, i, h, ref, carry);
}

__global__ void k_get_f(const void *src, int storage, int n, int np, RefDev ref,
                        const int *perm, double *f) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = perm[i];
    double h[Q];
    load_cell_dev(src, storage, np, i, ref, h);
    for (int a = 0; a < Q; a++) f[(size_t)c * Q + a] = wref(a, ref) + h[a];
}

__global__ void k_set_f(void *dst, int storage, int n, int np, RefDev ref,
                        const int *perm, const double *f, __half *carry) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = perm[i];
    double h[Q];
    for (int a = 0; a < Q; a++) h[a] = f[(size_t)c * Q + a] - wref(a, ref);
    store_cell_dev(dst, storage, np, i, h, ref, carry);
}

__global__ void k_rhs_out(const float *rhs, int n, int np, const int *perm, double *out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = perm[i];
    for (int a = 0; a < Q; a++) out[(size_t)c * Q + a] = (double)rhs[(size_t)a * np + i];
}

// Block sum of two FP64 values in a fixed tree order (deterministic).
__device__ inline void block_sum2(double a, double b, double *partial) {
    __shared__ double sa[RB], sb[RB];
    sa[threadIdx.x] = a; sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) { sa[threadIdx.x] += sa[threadIdx.x + s]; sb[threadIdx.x] += sb[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = sa[0]; partial[2 * blockIdx.x + 1] = sb[0]; }
}

// Step 6 (Eq. 5) in FP64 from the stored state; mass = sum A rho; flag on non-finite values.
__global__ void k_macros(const void *src, int storage, int n, int np, RefDev ref, const __half *carry,
                         const double *area, const int *perm, double *rho_out, double *u_out,
                         double *partial, int *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double mass = 0.0;
    if (i < n) {
        double r = 0, mx = 0, my = 0, h[Q];
        load_cell_dev(src, storage, np, i, ref, h);
        uncarry(carry, np, i, ref, h);
        for (int a = 0; a < Q; a++) {
            double f = wref(a, ref) + h[a];
            r += f;
            mx += EXd[a] * f;
            my += EYd[a] * f;
        }
        double ux = mx / r, uy = my / r;
        if (!isfinite(r) || !isfinite(ux) || !isfinite(uy) || !(r > 0)) atomicOr(flag, 1);
        int c = perm[i];
        if (rho_out) rho_out[c] = r;
        if (u_out) { u_out[2 * c] = ux; u_out[2 * c + 1] = uy; }
        mass = area[i] * r;
    }
    block_sum2(mass, 0.0, partial);
}

// Velocity snapshot for the residual; partial sums of |u - u_old|^2 and |u_old|^2.
__global__ void k_snapshot(const void *src, int storage, int n, int np, RefDev ref, const __half *carry,
                           double *snap_new, const double *snap_old, double *partial) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double num = 0, den = 0;
    if (i < n) {
        double r = 0, mx = 0, my = 0, h[Q];
        load_cell_dev(src, storage, np, i, ref, h);
        uncarry(carry, np, i, ref, h);
        for (int a = 0; a < Q; a++) {
            double f = wref(a, ref) + h[a];
            r += f; mx += EXd[a] * f; my += EYd[a] * f;
        }
        double ux = mx / r, uy = my / r;
        snap_new[2 * i] = ux; snap_new[2 * i + 1] = uy;
        if (snap_old) {
            double du = ux - snap_old[2 * i], dv = uy - snap_old[2 * i + 1];
            num = du * du + dv * dv;
            den = snap_old[2 * i] * snap_old[2 * i] + snap_old[2 * i + 1] * snap_old[2 * i + 1];
        }
    }
    block_sum2(num, den, partial);
}

// Momentum flux through wall faces (FP64 from the stored state): per face k of
// border cell c, F = sum_a e_a (e_a . n dl) f_P,a with f_P = f_eq(rho_c, u_w) +
// f_c - f_eq(rho_c, u_c) (Eq. 18) and n dl the outward normal times the face
// length, from the cell's corner offsets.  Also p = rho_c / 3 per face.
__global__ void k_wall_force(const void *src, int storage, int np, RefDev ref, const int2 *faces, int n,
                             const float2 *vxy, int nf, double uwx, double uwy, double *partial, double *face_p) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    double fx = 0.0, fy = 0.0;
    if (j < n) {
        const int c = faces[j].x, k = faces[j].y;
        double h[Q], f[Q];
        load_cell_dev(src, storage, np, c, ref, h);
        double r = 0, mx = 0, my = 0;
        for (int a = 0; a < Q; a++) {
            f[a] = wref(a, ref) + h[a];
            r += f[a]; mx += EXd[a] * f[a]; my += EYd[a] * f[a];
        }
        const double ux = mx / r, uy = my / r;
        const float2 v0 = vxy[(size_t)k * np + c], v1 = vxy[(size_t)(k + 1 == nf ? 0 : k + 1) * np + c];
        // a triangle stored in a quad-slot mesh repeats corner 0 as its fourth corner
        const double nx = (double)v1.y - (double)v0.y, ny = -((double)v1.x - (double)v0.x);
        for (int a = 0; a < Q; a++) {
            const double ec = EXd[a] * ux + EYd[a] * uy, ew = EXd[a] * uwx + EYd[a] * uwy;
            const double feq_c = WD[a] * r * (1.0 + 3.0 * ec + 4.5 * ec * ec - 1.5 * (ux * ux + uy * uy));
            const double feq_w = WD[a] * r * (1.0 + 3.0 * ew + 4.5 * ew * ew - 1.5 * (uwx * uwx + uwy * uwy));
            const double fp = feq_w + f[a] - feq_c;
            const double en = EXd[a] * nx + EYd[a] * ny;
            fx += EXd[a] * en * fp;
            fy += EYd[a] * en * fp;
        }
        if (face_p) face_p[j] = r / 3.0;
    }
    block_sum2(fx, fy, partial);
}

// mode 0: out[0] = sum col0 (mass); mode 1: out[1] = sqrt(sum col0)/sqrt(sum col1) (residual);
// mode 2: out[0], out[1] = sum col0, sum col1
__global__ void k_finish(const double *partial, int nblk, double *out, int mode) {
    __shared__ double sa[RB], sb[RB];
    double a = 0, b = 0;
    for (int k = threadIdx.x; k < nblk; k += RB) { a += partial[2 * k]; b += partial[2 * k + 1]; }
    sa[threadIdx.x] = a; sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) { sa[threadIdx.x] += sa[threadIdx.x + s]; sb[threadIdx.x] += sb[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (mode == 0) out[0] = sa[0];
        else if (mode == 1) out[1] = sqrt(sa[0]) / sqrt(sb[0]);
        else { out[0] = sa[0]; out[1] = sb[0]; }
    }
}

// one thread clears n ints (a fill kernel, so that the clear can sit in a captured graph)
__global__ void k_zero_int(int *p, int n) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) p[k] = 0;
}

// dst[i] = *src[i]: one scalar from each of n solvers' buffers
__global__ void k_gather(const double *const *src, double *dst, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = *src[i];
}

// out[0] = 1 if the flag is set, else 0
__global__ void k_flag_out(const int *flag, double *out) {
    if (threadIdx.x == 0) out[0] = flag[0] ? 1.0 : 0.0;
}

inline dim3 grid(int n) { return dim3((n + RB - 1) / RB); }

}  // namespace

int reduce_blocks(int n) { return (n + RB - 1) / RB; }

RefDev make_ref(double rho0, double ux, double uy, double scale) {
    static const int ex[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int ey[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static const double w[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    RefDev r{};
    r.rho0 = (float)rho0;
    const double jx = rho0 * ux, jy = rho0 * uy;
    r.jx0 = (float)jx;
    r.jy0 = (float)jy;
    r.scale = (float)scale;
    const double uu = ux * ux + uy * uy;
    for (int a = 0; a < Q; a++) {
        const double eu = ex[a] * ux + ey[a] * uy;
        r.fref[a] = (float)(w[a] * rho0 * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
        // use the FP32 momentum so that the step kernels' deviation form is consistent
        const double ej = ex[a] * (double)r.jx0 + ey[a] * (double)r.jy0;
        const double jj = (double)r.jx0 * r.jx0 + (double)r.jy0 * r.jy0;
        r.c0[a] = (float)((4.5 * ej * ej - 1.5 * jj) / (double)r.rho0);
        r.inv_unit[a] = (float)(1.0 / (double)((float)w[a] * r.scale));
    }
    return r;
}

hipError_t launch_init_eq(void *dst, int storage, int n, int np, const RefDev &ref,
                          const double *rho_dev, const double *u_dev, const int *perm_dev,
                          double rho_u, __half *carry, hipStream_t stream) {
    hipLaunchKernelGGL(k_init_eq, grid(n), dim3(RB), 0, stream, dst, storage, n, np, ref, rho_dev, u_dev, perm_dev, rho_u,
                       carry);
    return hipGetLastError();
}

hipError_t launch_get_f(const void *src, int storage, int n, int np, const RefDev &ref,
                        const int *perm_dev, double *f_dev, hipStream_t stream) {
    hipLaunchKernelGGL(k_get_f, grid(n), dim3(RB), 0, stream, src, storage, n, np, ref, perm_dev, f_dev);
    return hipGetLastError();
}

hipError_t launch_set_f(void *dst, int storage, int n, int np, const RefDev &ref,
                        const int *perm_dev, const double *f_dev, __half *carry, hipStream_t stream) {
    hipLaunchKernelGGL(k_set_f, grid(n), dim3(RB), 0, stream, dst, storage, n, np, ref, perm_dev, f_dev, carry);
    return hipGetLastError();
}

hipError_t launch_rhs_out(const float *rhs32, int n, int np, const int *perm_dev, double *out_dev,
                          hipStream_t stream) {
    hipLaunchKernelGGL(k_rhs_out, grid(n), dim3(RB), 0, stream, rhs32, n, np, perm_dev, out_dev);
    return hipGetLastError();
}

hipError_t launch_macros(const void *src, int storage, int n, int np, const RefDev &ref, const __half *carry,
                         const double *area, const int *perm_dev, double *rho_out, double *u_out,
                         double *partial, int *flag, hipStream_t stream) {
    hipLaunchKernelGGL(k_macros, grid(n), dim3(RB), 0, stream, src, storage, n, np, ref, carry, area, perm_dev, rho_out,
                       u_out, partial, flag);
    return hipGetLastError();
}

hipError_t launch_wall_force(const void *src, int storage, int np, const RefDev &ref, const int2 *faces, int n,
                             const float2 *vxy, int nf, double uwx, double uwy, double *partial, double *face_p,
                             hipStream_t stream) {
    hipLaunchKernelGGL(k_wall_force, grid(n), dim3(RB), 0, stream, src, storage, np, ref, faces, n, vxy, nf, uwx, uwy,
                       partial, face_p);
    return hipGetLastError();
}

hipError_t launch_snapshot(const void *src, int storage, int n, int np, const RefDev &ref, const __half *carry,
                           double *snap_new, const double *snap_old, double *partial,
                           hipStream_t stream) {
    hipLaunchKernelGGL(k_snapshot, grid(n), dim3(RB), 0, stream, src, storage, n, np, ref, carry, snap_new, snap_old,
                       partial);
    return hipGetLastError();
}

hipError_t launch_zero_int(int *p, int n, hipStream_t stream) {
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_gather(const double *const *src, double *dst, int n, hipStream_t stream) {
    hipLaunchKernelGGL(k_gather, dim3(1), dim3(256), 0, stream, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_flag_out(const int *flag, double *out, hipStream_t stream) {
    hipLaunchKernelGGL(k_flag_out, dim3(1), dim3(64), 0, stream, flag, out);
    return hipGetLastError();
}

hipError_t launch_finish_sums(const double *partial, int nblk, double *out, int mode, hipStream_t stream) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(RB), 0, stream, partial, nblk, out, mode);
    return hipGetLastError();
}

}  // namespace fvlbm

// refine.hip -- variational refinement of each level's dense flow (the third
// stage of dense inverse search; EBOF_VAR_REFINE, stage calls).  After a
// level's inverse search, its dense flow U is formed (the densification, at
// every pixel of the level) and refined by a few fixed-point iterations of
// the linearised robust energy
//   delta Psi(E_c) + gamma Psi(E_g) + alpha Psi(|grad(u)|^2 + |grad(v)|^2),
// E_c the brightness-constancy and E_g the gradient-constancy residual of the
// increment (du, dv), Psi(s^2) = sqrt(s^2 + eps^2): per iteration the
// weights at the current increment, then red-black block SOR sweeps of the
// per-pixel 2x2 systems.  The next finer level starts from the refined flow.
// Images are taken on the 8-bit scale (x255), derivatives are central
// differences with replicated border.  Double precision: the smoothness
// weights reach 1000 alpha where the flow is smooth, and the systems' right
// sides difference neighbouring flows of order one, which single precision
// rounds to a visible part of a pixel.  Every sum that an axis swap would
// reorder is grouped so that it does not.
#include <hip/hip_runtime.h>

#include "ctx.h"
#include "dens_dev.h"

namespace ebof {

constexpr int kVarBlock = 256;
constexpr double kVarAlpha = 20.0, kVarGamma = 10.0, kVarDelta = 5.0, kVarOmega = 1.6;
constexpr int kVarOuter = 5, kVarInner = 5;
constexpr double kVarEps2 = 1e-6;

__device__ __forceinline__ int cl(int v, int n) { return clampi(v, 0, n - 1); }

// bilinear sample with replicated border, in double
__device__ __forceinline__ double bil(const float* __restrict__ I, int W, int H, int x, int y, double ux, double uy) {
    const double lim = (double)(W + H + 16);
    ux = fmin(fmax(ux, -lim), lim);
    uy = fmin(fmax(uy, -lim), lim);
    const double fx = floor(ux), fy = floor(uy);
    const int ix = (int)fx, iy = (int)fy;
    const double ax = ux - fx, ay = uy - fy;
    const int xa = cl(x + ix, W), xb = cl(x + ix + 1, W), ya = cl(y + iy, H), yb = cl(y + iy + 1, H);
    const double a = I[(size_t)ya * W + xa], b = I[(size_t)ya * W + xb];
    const double c = I[(size_t)yb * W + xa], d = I[(size_t)yb * W + xb];
    return (1.0 - ay) * ((1.0 - ax) * a + ax * b) + ay * ((1.0 - ax) * c + ax * d);
}

// the level's dense flow: the densification at every pixel (no mask)
__global__ __launch_bounds__(kVarBlock) void k_var_dense(int W, int H, int pnx, int pny, int s,
                                                         const float* __restrict__ I0, const float* __restrict__ I1,
                                                         const float2* __restrict__ pu, float* __restrict__ U) {
    const int64_t N = (int64_t)W * H;
    for (int64_t i = (int64_t)blockIdx.x * kVarBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVarBlock) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        const float inv_s = 1.0f / (float)s;
        const Cover cx = cover_of(x, W, pnx, s, inv_s), cy = cover_of(y, H, pny, s, inv_s);
        float sw, su, sv;
        dens_sums(I1, W, H, x, y, I0[i], pu, pnx, cx, cy, sw, su, sv);
        U[i] = su / sw;
        U[N + i] = sv / sw;
    }
}

// pass 1: the warped image, the average image and It (8-bit scale)
__global__ __launch_bounds__(kVarBlock) void k_var_prep1(int W, int H, const float* __restrict__ I0,
                                                         const float* __restrict__ I1, const float* __restrict__ U,
                                                         double* __restrict__ D) {
    const int64_t N = (int64_t)W * H;
    double* I1w = D;          // plane 0
    double* A = D + N;        // plane 1
    double* It = D + 2 * N;   // plane 2
    for (int64_t i = (int64_t)blockIdx.x * kVarBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVarBlock) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        const double w1 = 255.0 * bil(I1, W, H, x, y, (double)U[i], (double)U[N + i]);
        const double w0 = 255.0 * (double)I0[i];
        I1w[i] = w1;
        A[i] = 0.5 * (w0 + w1);
        It[i] = w1 - w0;
    }
}

template <class T>
__device__ __forceinline__ double dx_of(const T* f, int W, int H, int x, int y) {
    return 0.5 * ((double)f[(size_t)y * W + cl(x + 1, W)] - (double)f[(size_t)y * W + cl(x - 1, W)]);
}
template <class T>
__device__ __forceinline__ double dy_of(const T* f, int W, int H, int x, int y) {
    return 0.5 * ((double)f[(size_t)cl(y + 1, H) * W + x] - (double)f[(size_t)cl(y - 1, H) * W + x]);
}

// pass 2: first derivatives of the average (Ix, Iy) and the change of the
// gradient (Ixt, Iyt)
__global__ __launch_bounds__(kVarBlock) void k_var_prep2(int W, int H, const float* __restrict__ I0,
                                                         double* __restrict__ D) {
    const int64_t N = (int64_t)W * H;
    const double* I1w = D;
    const double* A = D + N;
    double* Ix = D + 3 * N;
    double* Iy = D + 4 * N;
    double* Ixt = D + 5 * N;
    double* Iyt = D + 6 * N;
    for (int64_t i = (int64_t)blockIdx.x * kVarBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVarBlock) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        Ix[i] = dx_of(A, W, H, x, y);
        Iy[i] = dy_of(A, W, H, x, y);
        const double gx0 = 255.0 * dx_of(I0, W, H, x, y), gy0 = 255.0 * dy_of(I0, W, H, x, y);
        Ixt[i] = dx_of(I1w, W, H, x, y) - gx0;
        Iyt[i] = dy_of(I1w, W, H, x, y) - gy0;
    }
}

// pass 3: second derivatives of the average (Ixx, Ixy symmetrised, Iyy)
__global__ __launch_bounds__(kVarBlock) void k_var_prep3(int W, int H, double* __restrict__ D) {
    const int64_t N = (int64_t)W * H;
    const double* Ix = D + 3 * N;
    const double* Iy = D + 4 * N;
    double* Ixx = D + 7 * N;
    double* Ixy = D + 8 * N;
    double* Iyy = D + 9 * N;
    for (int64_t i = (int64_t)blockIdx.x * kVarBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVarBlock) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        Ixx[i] = dx_of(Ix, W, H, x, y);
        Iyy[i] = dy_of(Iy, W, H, x, y);
        Ixy[i] = 0.5 * (dy_of(Ix, W, H, x, y) + dx_of(Iy, W, H, x, y));
    }
}

__device__ __forceinline__ double robust_w(double s2) { return 1.0 / sqrt(s2 + kVarEps2); }

// the weights at the current increment and the coefficients of the 2x2
// systems: a11, a12, a22, b1, b2 and the smoothness weight s
__global__ __launch_bounds__(kVarBlock) void k_var_coef(int W, int H, const double* __restrict__ D,
                                                        const float* __restrict__ U, const double* __restrict__ dU,
                                                        double* __restrict__ C) {
    const int64_t N = (int64_t)W * H;
    const double *It = D + 2 * N, *Ix = D + 3 * N, *Iy = D + 4 * N, *Ixt = D + 5 * N, *Iyt = D + 6 * N;
    const double *Ixx = D + 7 * N, *Ixy = D + 8 * N, *Iyy = D + 9 * N;
    const double *du = dU, *dv = dU + N;
    for (int64_t i = (int64_t)blockIdx.x * kVarBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVarBlock) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        const double c = It[i] + (Ix[i] * du[i] + Iy[i] * dv[i]);
        const double g1 = Ixt[i] + (Ixx[i] * du[i] + Ixy[i] * dv[i]);
        const double g2 = Iyt[i] + (Ixy[i] * du[i] + Iyy[i] * dv[i]);
        const double wc = kVarDelta * robust_w(c * c);
        const double wg = kVarGamma * robust_w(g1 * g1 + g2 * g2);
        C[i] = wc * Ix[i] * Ix[i] + wg * (Ixx[i] * Ixx[i] + Ixy[i] * Ixy[i]);
        C[N + i] = wc * (Ix[i] * Iy[i]) + wg * (Ixx[i] * Ixy[i] + Ixy[i] * Iyy[i]);
        C[2 * N + i] = wc * Iy[i] * Iy[i] + wg * (Ixy[i] * Ixy[i] + Iyy[i] * Iyy[i]);
        C[3 * N + i] = wc * Ix[i] * It[i] + wg * (Ixx[i] * Ixt[i] + Ixy[i] * Iyt[i]);
        C[4 * N + i] = wc * Iy[i] * It[i] + wg * (Ixy[i] * Ixt[i] + Iyy[i] * Iyt[i]);
        // smoothness of the refined flow u + du, v + dv
        const int xl = cl(x - 1, W), xr = cl(x + 1, W), yu = cl(y - 1, H), yd = cl(y + 1, H);
        const size_t pl = (size_t)y * W + xl, pr = (size_t)y * W + xr, pu_ = (size_t)yu * W + x,
                     pd = (size_t)yd * W + x;
        const double ux = 0.5 * (((double)U[pr] + du[pr]) - ((double)U[pl] + du[pl]));
        const double uy = 0.5 * (((double)U[pd] + du[pd]) - ((double)U[pu_] + du[pu_]));
        const double vx = 0.5 * (((double)U[N + pr] + dv[pr]) - ((double)U[N + pl] + dv[pl]));
        const double vy = 0.5 * (((double)U[N + pd] + dv[pd]) - ((double)U[N + pu_] + dv[pu_]));
        C[5 * N + i] = kVarAlpha * robust_w((ux * ux + vy * vy) + (uy * uy + vx * vx));
    }
}

// one half-sweep: the pixels with (x + y) % 2 == colour solve their 2x2
// systems with the other colour's current increments, relaxed by omega
__global__ __launch_bounds__(kVarBlock) void k_var_sor(int W, int H, int colour, const double* __restrict__ C,
                                                       const float* __restrict__ U, double* __restrict__ dU) {
    const int64_t N = (int64_t)W * H;
    const int half = (W + 1) / 2;
    const int64_t M = (int64_t)half * H;
    double *du = dU, *dv = dU + N;
    const double* s = C + 5 * N;
    for (int64_t j = (int64_t)blockIdx.x * kVarBlock + threadIdx.x; j < M; j += (int64_t)gridDim.x * kVarBlock) {
        const int y = (int)(j / half);
        const int x = 2 * (int)(j - (int64_t)y * half) + ((y + colour) & 1);
        if (x >= W) continue;
        const size_t p = (size_t)y * W + x;
        const int nx[4] = {x - 1, x + 1, x, x}, ny[4] = {y, y, y - 1, y + 1};
        double w[4], tu[4], tv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w[k] = tu[k] = tv[k] = 0.0;
            if (nx[k] >= 0 && nx[k] < W && ny[k] >= 0 && ny[k] < H) {
                const size_t q = (size_t)ny[k] * W + nx[k];
                w[k] = 0.5 * (s[p] + s[q]);
                tu[k] = w[k] * (((double)U[q] - (double)U[p]) + du[q]);
                tv[k] = w[k] * (((double)U[N + q] - (double)U[N + p]) + dv[q]);
            }
        }
        const double sw = (w[0] + w[1]) + (w[2] + w[3]);
        const double ru = (tu[0] + tu[1]) + (tu[2] + tu[3]);
        const double rv = (tv[0] + tv[1]) + (tv[2] + tv[3]);
        const double m11 = C[p] + sw, m12 = C[N + p], m22s = C[2 * N + p] + sw;
        const double r1 = ru - C[3 * N + p], r2 = rv - C[4 * N + p];
        const double det = m11 * m22s - m12 * m12;
        const double su = (m22s * r1 - m12 * r2) / det;
        const double sv = (m11 * r2 - m12 * r1) / det;
        du[p] = (1.0 - kVarOmega) * du[p] + kVarOmega * su;
        dv[p] = (1.0 - kVarOmega) * dv[p] + kVarOmega * sv;
    }
}

__global__ __launch_bounds__(kVarBlock) void k_var_zero(double* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kVarBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVarBlock)
        p[i] = 0.0;
}

__global__ __launch_bounds__(kVarBlock) void k_var_apply(int64_t N, float* __restrict__ U,
                                                         const double* __restrict__ dU) {
    for (int64_t i = (int64_t)blockIdx.x * kVarBlock + threadIdx.x; i < 2 * N; i += (int64_t)gridDim.x * kVarBlock)
        U[i] = (float)((double)U[i] + dU[i]);
}

// level 0: the refined flow to the outputs (masked as the densification does)
__global__ __launch_bounds__(kVarBlock) void k_var_output(int W, int H, const float* __restrict__ U,
                                                          const uint8_t* __restrict__ mask, uint32_t flags,
                                                          float* __restrict__ flow, float* __restrict__ keep,
                                                          uint8_t* __restrict__ mask_out) {
    const int64_t N = (int64_t)W * H;
    for (int64_t i = (int64_t)blockIdx.x * kVarBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVarBlock) {
        float fu = U[i], fv = U[N + i];
        if (keep) {
            keep[i] = fu;
            keep[N + i] = fv;
        }
        const uint8_t m = mask ? mask[i] : 1;
        if ((flags & EBOF_MASK_FLOW) && !m) fu = fv = 0.f;
        flow[i] = fu;
        flow[N + i] = fv;
        if (mask_out) mask_out[i] = m;
    }
}

static int var_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kVarBlock - 1) / kVarBlock, 4096)); }

// After level l's inverse search: its dense flow into d.ud (level l's part),
// refined; at level 0 also written to the outputs.  scratch: 10 N0 doubles of
// derivatives, 6 N0 of coefficients, 2 N0 of increments (N0 = level-0 pixels).
void launch_var_level(const WinDesc& d, int l, double* scratch, hipStream_t st) {
    const LevelGeom g = d.lv[l];
    const int W = g.w, H = g.h;
    const int64_t N = (int64_t)W * H, N0 = (int64_t)d.W * d.H;
    const float* I0 = d.pyr_prev + g.off;
    const float* I1 = d.pyr + g.off;
    float* U = d.ud + 2 * g.off;
    double* D = scratch;
    double* C = scratch + 10 * N0;
    double* dU = scratch + 16 * N0;
    const int gN = var_grid(N);
    hipLaunchKernelGGL(k_var_dense, dim3(gN), dim3(kVarBlock), 0, st, W, H, g.pnx, g.pny, d.stride, I0, I1,
                       (const float2*)(d.puv + g.poff), U);
    hipLaunchKernelGGL(k_var_prep1, dim3(gN), dim3(kVarBlock), 0, st, W, H, I0, I1, (const float*)U, D);
    hipLaunchKernelGGL(k_var_prep2, dim3(gN), dim3(kVarBlock), 0, st, W, H, I0, D);
    hipLaunchKernelGGL(k_var_prep3, dim3(gN), dim3(kVarBlock), 0, st, W, H, D);
    hipLaunchKernelGGL(k_var_zero, dim3(var_grid(2 * N)), dim3(kVarBlock), 0, st, dU, 2 * N);
    const int gH = var_grid((int64_t)((W + 1) / 2) * H);
    for (int o = 0; o < kVarOuter; ++o) {
        hipLaunchKernelGGL(k_var_coef, dim3(gN), dim3(kVarBlock), 0, st, W, H, (const double*)D, (const float*)U,
                           (const double*)dU, C);
        for (int it = 0; it < kVarInner; ++it)
            for (int colour = 0; colour < 2; ++colour)
                hipLaunchKernelGGL(k_var_sor, dim3(gH), dim3(kVarBlock), 0, st, W, H, colour, (const double*)C,
                                   (const float*)U, dU);
    }
    hipLaunchKernelGGL(k_var_apply, dim3(var_grid(2 * N)), dim3(kVarBlock), 0, st, N, U, (const double*)dU);
    if (l == 0)
        hipLaunchKernelGGL(k_var_output, dim3(gN), dim3(kVarBlock), 0, st, W, H, (const float*)U, d.mask, d.flags,
                           d.flow, d.flow_keep, d.mask_out);
}

}  // namespace ebof

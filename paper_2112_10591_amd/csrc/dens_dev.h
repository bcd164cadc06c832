// dens_dev.h -- device helpers of the densification (the covering patches of
// a pixel and their weighted mean), shared by the inverse search, the
// level-0 densification and the variational refinement.
#pragma once

#include <hip/hip_runtime.h>

#include "ebof_dev.h"

namespace ebof {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Patches of one axis that contain pixel p: the regular ones (origin k*s,
// k <= np-2, never clamped) with k*s <= p <= k*s+7, plus the last patch
// (origin n-8) when p >= n-8.
struct Cover {
    int lo, nreg, last, n;
};
// q / s for 0 <= q < 2^16 and 1 <= s <= 8, with inv_s = 1/s: (q + 1/2) / s
// lies at least 1/(2s) >= 1/16 from an integer, and the float product's
// relative error (2^-23) keeps it within 2^-7 of the exact quotient.
__device__ __forceinline__ int div_small(int q, float inv_s) { return (int)(((float)q + 0.5f) * inv_s); }

__device__ __forceinline__ Cover cover_of(int p, int n, int np, int s, float inv_s) {
    Cover c;
    c.lo = p >= kPatch - 1 ? div_small(p - (kPatch - 1) + s - 1, inv_s) : 0;
    const int hi = min(np - 2, div_small(p, inv_s));
    c.nreg = max(0, hi - c.lo + 1);
    c.last = np - 1;
    c.n = c.nreg + (p >= n - kPatch ? 1 : 0);
    return c;
}
__device__ __forceinline__ int cover_index(const Cover& c, int q) { return q < c.nreg ? c.lo + q : c.last; }

// Densification samples, single precision.  The sample position x + u is
// split exactly into an integer part and a fraction (floor of a float and
// the difference, both exact), so the fraction keeps full precision however
// wide the image; a position off the image samples the border whatever its
// distance.  Fetch and blend are separate so that several samples' loads can
// be in flight.
struct DensTap {
    float a, b, c, d, ax, ay;
};
__device__ __forceinline__ DensTap dens_fetch(const float* __restrict__ I, int W, int H, int x, int y, float ux,
                                              float uy) {
    const float lim = (float)(W + H + 16);
    ux = fminf(fmaxf(ux, -lim), lim);
    uy = fminf(fmaxf(uy, -lim), lim);
    const float fx = floorf(ux), fy = floorf(uy);
    const int ix = (int)fx, iy = (int)fy;
    const int xa = clampi(x + ix, 0, W - 1), xb = clampi(x + ix + 1, 0, W - 1);
    const int ya = clampi(y + iy, 0, H - 1), yb = clampi(y + iy + 1, 0, H - 1);
    return DensTap{I[(size_t)ya * W + xa], I[(size_t)ya * W + xb], I[(size_t)yb * W + xa], I[(size_t)yb * W + xb],
                   ux - fx, uy - fy};
}
__device__ __forceinline__ float dens_blend(const DensTap& t) {
    const float top = t.a + t.ax * (t.b - t.a);
    const float bot = t.c + t.ax * (t.d - t.c);
    return top + t.ay * (bot - top);
}
// 1 / max(1, 255 |d|) by the hardware reciprocal (1 ulp)
__device__ __forceinline__ float dens_weight_f(float dv) {
    return __builtin_amdgcn_rcpf(fmaxf(1.0f, 255.0f * fabsf(dv)));
}

constexpr int kDensChunk = 4;  // densification: covering patches loaded together

// Weighted sums over the patches (displacements pu, pnx per row) covering
// pixel (x, y) of an image I1 of W x H whose reference intensity is i0: the
// covering patches in row-major order, kDensChunk at a time, their
// displacements and then their samples loaded before any is used.
__device__ __forceinline__ void dens_sums(const float* __restrict__ I1, int W, int H, int x, int y, float i0,
                                          const float2* __restrict__ pu, int pnx, const Cover& cx, const Cover& cy,
                                          float& sw, float& su, float& sv) {
    sw = su = sv = 0.f;
    const int n = cx.n * cy.n;
    int qx = 0, qy = 0;
    for (int q0 = 0; q0 < n; q0 += kDensChunk) {
        float2 u[kDensChunk];
        DensTap tp[kDensChunk];
#pragma unroll
        for (int t = 0; t < kDensChunk; ++t) {
            if (q0 + t < n) u[t] = pu[(size_t)cover_index(cy, qy) * pnx + cover_index(cx, qx)];
            if (++qx == cx.n) {
                qx = 0;
                ++qy;
            }
        }
#pragma unroll
        for (int t = 0; t < kDensChunk; ++t)
            if (q0 + t < n) tp[t] = dens_fetch(I1, W, H, x, y, u[t].x, u[t].y);
#pragma unroll
        for (int t = 0; t < kDensChunk; ++t) {
            if (q0 + t < n) {
                const float w = dens_weight_f(dens_blend(tp[t]) - i0);
                sw += w;
                su += w * u[t].x;
                sv += w * u[t].y;
            }
        }
    }
}
}  // namespace ebof

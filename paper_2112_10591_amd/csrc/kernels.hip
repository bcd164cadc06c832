// kernels.hip -- gfx950 kernels of the per-window flow path.
//
// Every kernel runs 256-thread blocks over "work items" (a chunk of events, a
// tile, a row, a group of patches) and loops item = blockIdx.x, += gridDim.x,
// so one launch can cover one window or a whole batch of windows of mixed
// sizes (template parameter B: descriptor table + per-stage prefix sums).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebof_dev.h"

namespace ebof {

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------
template <bool B>
__device__ __forceinline__ const WinDesc* locate(const WinDesc& one, const BatchArgs& ba,
                                                 int32_t item, int32_t& local) {
    if constexpr (!B) {
        local = item;
        return &one;
    } else {
        int lo = 0, hi = ba.nwin - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ba.prefix[mid] <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        local = item - ba.prefix[lo];
        return ba.tab + lo;
    }
}

template <bool B>
__device__ __forceinline__ int32_t item_total(const BatchArgs& ba, int32_t total_arg) {
    if constexpr (B)
        return ba.prefix[ba.nwin];
    else
        return total_arg;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// 8-lane all-reduce (sum) within aligned groups of 8 lanes, by DPP:
// swap neighbours, swap pairs, then mirror the two quads of the half-row.
// Each step adds two values in an order that commutes, so all 8 lanes end
// with bit-identical sums.
template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                 0xF, 0xF, false));
}
__device__ __forceinline__ float red8(float v) {
    v += dppf<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dppf<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dppf<0x141>(v);  // row_half_mirror
    return v;
}

// Bilinear sample with replicated border (the four neighbour indices clamped
// into the image).  Offsets beyond the image all clamp to the border, so the
// position is limited first to keep the float-to-int conversion defined.
__device__ __forceinline__ float bilinear(const float* __restrict__ I, int W, int H, float sx,
                                          float sy) {
    const float lim = (float)(W + H + 16);
    sx = fminf(fmaxf(sx, -lim), lim);
    sy = fminf(fmaxf(sy, -lim), lim);
    const float fx = floorf(sx), fy = floorf(sy);
    const float ax = sx - fx, ay = sy - fy;
    const int x0 = (int)fx, y0 = (int)fy;
    const int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    const int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
    const float a = I[(size_t)ya * W + xa], b = I[(size_t)ya * W + xb];
    const float c = I[(size_t)yb * W + xa], d = I[(size_t)yb * W + xb];
    const float top = a + ax * (b - a);
    const float bot = c + ax * (d - c);
    return top + ay * (bot - top);
}

// Patches of one axis that contain pixel p: the regular ones (origin k*s,
// k <= np-2, never clamped) with k*s <= p <= k*s+7, plus the last patch
// (origin n-8) when p >= n-8.
struct Cover {
    int lo, nreg, last, n;
};
__device__ __forceinline__ Cover cover_of(int p, int n, int np, int s) {
    Cover c;
    c.lo = p >= kPatch - 1 ? (p - (kPatch - 1) + s - 1) / s : 0;
    const int hi = min(np - 2, p / s);
    c.nreg = max(0, hi - c.lo + 1);
    c.last = np - 1;
    c.n = c.nreg + (p >= n - kPatch ? 1 : 0);
    return c;
}
__device__ __forceinline__ int cover_index(const Cover& c, int q) { return q < c.nreg ? c.lo + q : c.last; }

// --------------------------------------------------------------------------
// zero the event staging image (done when the window stamp wraps)
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_zero(const WinDesc one, const BatchArgs ba, int32_t total_arg) {
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int64_t n = (int64_t)d->W * d->H;
        const int64_t base = (int64_t)local * kZeroBytesPerItem;
        const int64_t end = min(base + (int64_t)kZeroBytesPerItem, n);
        uint8_t* p = d->e_raw;
        for (int64_t i = base + threadIdx.x; i < end; i += kBlock) p[i] = 0;
    }
}

// --------------------------------------------------------------------------
// Sec. III-A: scatter the window's events into the staging image.  Every
// event of the window that lands on the sensor writes the window stamp at its
// pixel; concurrent writers of one pixel all store the same value, so no
// atomics are needed.  Polarity is not read.
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_scatter(const WinDesc one, const BatchArgs ba, int32_t total_arg) {
    __shared__ uint32_t s_drop[kBlock / 64];
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int64_t n = d->n_ev, t0 = d->t0, t1 = d->t1;
        const uint32_t W = (uint32_t)d->W, H = (uint32_t)d->H;
        const uint8_t stamp = (uint8_t)d->stamp;
        uint8_t* __restrict__ er = d->e_raw;
        const int64_t base = (int64_t)local * kEventsPerItem;
        uint32_t dropped = 0;
#pragma unroll
        for (int k = 0; k < kEventsPerItem / kBlock; ++k) {
            const int64_t e = base + k * kBlock + threadIdx.x;
            if (e < n) {
                const int64_t t = __builtin_nontemporal_load(d->et + e);
                const uint32_t x = __builtin_nontemporal_load(d->ex + e);
                const uint32_t y = __builtin_nontemporal_load(d->ey + e);
                if (t >= t0 && t < t1 && x < W && y < H)
                    er[(size_t)y * W + x] = stamp;
                else
                    ++dropped;
            }
        }
        if (d->n_dropped) {
            for (int off = 32; off > 0; off >>= 1) dropped += __shfl_down(dropped, off, 64);
            if ((threadIdx.x & 63) == 0) s_drop[threadIdx.x >> 6] = dropped;
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t s = 0;
                for (int w = 0; w < kBlock / 64; ++w) s += s_drop[w];
                if (s) atomicAdd(d->n_dropped, (unsigned long long)s);
            }
            __syncthreads();
        }
    }
}

// --------------------------------------------------------------------------
// Alg. 1 then Alg. 2 on one 64x64 tile.  The raw image is staged with a
// 2-pixel halo, the denoised image E_d is formed on the tile plus a 1-pixel
// halo (each pixel counts its 4 neighbours in E), then the fill forms E_df on
// the tile (counting neighbours in E_d).  Pixels off the image are non-edges.
// Optionally the tile's column bit masks (bit r of word (chunk, x) = E_df at
// row 64*chunk + r) are written for the distance transform.
// --------------------------------------------------------------------------
template <bool B, bool PACK>
__global__ __launch_bounds__(kBlock) void k_denoise_fill(const WinDesc one, const BatchArgs ba,
                                                         int32_t total_arg) {
    constexpr int R = kTile + 4;  // raw tile with 2-pixel halo
    constexpr int D = kTile + 2;  // denoised tile with 1-pixel halo
    __shared__ uint8_t sE[R][R + 4];
    __shared__ uint8_t sEd[D][D + 2];
    __shared__ uint16_t sBits[4][kTile];
    const int32_t total = item_total<B>(ba, total_arg);
    const int tid = threadIdx.x;
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int W = d->W, H = d->H;
        const int tiles_x = (W + kTile - 1) / kTile;
        const int tx = local % tiles_x, ty = local / tiles_x;
        const int x0 = tx * kTile, y0 = ty * kTile;
        const uint8_t stamp = (uint8_t)d->stamp;
        const uint8_t* __restrict__ er = d->e_raw;
        const int n_d = d->n_d, n_f = d->n_f;
        for (int i = tid; i < R * R; i += kBlock) {
            const int lx = i % R, ly = i / R;
            const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
            uint8_t v = 0;
            if (gx >= 0 && gx < W && gy >= 0 && gy < H) v = er[(size_t)gy * W + gx] == stamp;
            sE[ly][lx] = v;
        }
        __syncthreads();
        for (int i = tid; i < D * D; i += kBlock) {
            const int lx = i % D, ly = i / D;  // pixel (x0-1+lx, y0-1+ly) = sE[ly+1][lx+1]
            uint8_t v = sE[ly + 1][lx + 1];
            if (v) {
                const int nb = sE[ly][lx + 1] + sE[ly + 2][lx + 1] + sE[ly + 1][lx] + sE[ly + 1][lx + 2];
                v = nb >= n_d;
            }
            sEd[ly][lx] = v;
        }
        __syncthreads();
        const int c = tid & (kTile - 1), rg = tid / kTile;
        const int gx = x0 + c;
        uint32_t bits = 0;
        for (int r = 0; r < 16; ++r) {
            const int ly = rg * 16 + r;  // pixel (gx, y0+ly) = sEd[ly+1][c+1]
            const int gy = y0 + ly;
            uint8_t v = sEd[ly + 1][c + 1];
            if (!v) {
                const int nb = sEd[ly][c + 1] + sEd[ly + 2][c + 1] + sEd[ly + 1][c] + sEd[ly + 1][c + 2];
                v = nb >= n_f;
            }
            if (gx < W && gy < H) {
                d->e_df[(size_t)gy * W + gx] = v;
                bits |= (uint32_t)v << r;
            }
        }
        if constexpr (PACK) {
            sBits[rg][c] = (uint16_t)bits;
            __syncthreads();
            if (tid < kTile && x0 + tid < W) {
                const uint64_t m = (uint64_t)sBits[0][tid] | ((uint64_t)sBits[1][tid] << 16) |
                                   ((uint64_t)sBits[2][tid] << 32) | ((uint64_t)sBits[3][tid] << 48);
                d->colmask[(size_t)ty * W + x0 + tid] = m;
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// Column bit masks of an edge image (for edge images not produced by
// k_denoise_fill).  Item = 64 columns x 4 chunks; thread = (column, chunk).
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_pack_cols(const WinDesc one, const BatchArgs ba,
                                                      int32_t total_arg) {
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int W = d->W, H = d->H;
        const int bands = (W + 63) / 64, nch = (H + kChunk - 1) / kChunk;
        const int bx = local % bands, cg = local / bands;
        const int x = bx * 64 + (threadIdx.x & 63);
        const int ck = cg * 4 + (threadIdx.x >> 6);
        if (x < W && ck < nch) {
            const int rows = min(kChunk, H - ck * kChunk);
            const uint8_t* col = d->e_df + (size_t)ck * kChunk * W + x;
            uint64_t m = 0;
            for (int r = 0; r < rows; ++r) m |= (uint64_t)(col[(size_t)r * W] != 0) << r;
            d->colmask[(size_t)ck * W + x] = m;
        }
    }
}

// --------------------------------------------------------------------------
// Exact distance transform, column pass: g(x, y) = min |y - y'| over the edge
// pixels (x, y') of column x, or kGInf when the column has none.  Thread =
// (column, 64-row chunk): the nearest edges above and below the chunk come
// from the neighbouring chunks' masks, those inside it from bit scans.
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_edt_cols(const WinDesc one, const BatchArgs ba,
                                                     int32_t total_arg) {
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int W = d->W, H = d->H;
        const int bands = (W + 63) / 64, nch = (H + kChunk - 1) / kChunk;
        const int bx = local % bands, cg = local / bands;
        const int x = bx * 64 + (threadIdx.x & 63);
        const int ck = cg * 4 + (threadIdx.x >> 6);
        if (x < W && ck < nch) {
            const uint64_t* cm = d->colmask + x;
            const uint64_t m = cm[(size_t)ck * W];
            int prev = -1;  // last edge row above the chunk
            for (int c2 = ck - 1; c2 >= 0; --c2) {
                const uint64_t mm = cm[(size_t)c2 * W];
                if (mm) {
                    prev = c2 * kChunk + 63 - __clzll(mm);
                    break;
                }
            }
            int next = -1;  // first edge row below the chunk
            for (int c2 = ck + 1; c2 < nch; ++c2) {
                const uint64_t mm = cm[(size_t)c2 * W];
                if (mm) {
                    next = c2 * kChunk + __ffsll((unsigned long long)mm) - 1;
                    break;
                }
            }
            const int rows = min(kChunk, H - ck * kChunk);
            uint16_t* gcol = d->g + (size_t)ck * kChunk * W + x;
            for (int r = 0; r < rows; ++r) {
                const int y = ck * kChunk + r;
                const uint64_t rest = m >> r;
                if (rest & 1ull) prev = y;
                const int nxt = rest ? y + __ffsll((unsigned long long)rest) - 1 : next;
                int gv = 0x7fffffff;
                if (prev >= 0) gv = y - prev;
                if (nxt >= 0) gv = min(gv, nxt - y);
                gcol[(size_t)r * W] = gv == 0x7fffffff ? kGInf : (uint16_t)gv;
            }
        }
    }
}

// --------------------------------------------------------------------------
// Exact distance transform, row pass, fused with eq. (1).  One row per item:
// the row's g^2 is staged in LDS, then every pixel searches outwards,
// D2(x) = min_r r^2 + g(x +- r)^2, stopping once r^2 reaches the best value
// found (no later column can beat it), which gives the exact minimum.  The
// surface is looked up from the squared distance: lut[D2] below lut_n,
// exactly 1.0f from there on.
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_edt_rows(const WinDesc one, const BatchArgs ba,
                                                     int32_t total_arg) {
    __shared__ uint32_t sG2[EBOF_MAX_DIM];
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int W = d->W;
        const int y = local;
        const uint16_t* grow = d->g + (size_t)y * W;
        int any = 0;
        for (int x = threadIdx.x; x < W; x += kBlock) {
            const uint32_t gv = grow[x];
            any |= gv != kGInf;
            sG2[x] = gv == kGInf ? 0x7fffffffu : gv * gv;
        }
        any = __syncthreads_or(any);
        const int lut_n = d->lut_n;
        const float* __restrict__ lut = d->lut;
        int32_t* d2row = d->d2 ? d->d2 + (size_t)y * W : nullptr;
        float* srow = d->pyr + (size_t)y * W;
        for (int x = threadIdx.x; x < W; x += kBlock) {
            uint32_t best = 0x7fffffffu;
            if (any) {
                best = sG2[x];
                for (int r = 1;; ++r) {
                    const uint32_t r2 = (uint32_t)r * (uint32_t)r;
                    if (r2 >= best) break;
                    const bool lft = x - r >= 0, rgt = x + r < W;
                    if (!lft && !rgt) break;
                    if (lft) best = min(best, r2 + sG2[x - r]);
                    if (rgt) best = min(best, r2 + sG2[x + r]);
                }
            }
            const int32_t d2v = best >= 0x7fffffffu ? 0x7fffffff : (int32_t)best;
            if (d2row) d2row[x] = d2v;
            srow[x] = d2v < lut_n ? lut[d2v] : 1.0f;
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// Pyramid reduction level l-1 -> l: 5x5 binomial (separable [1 4 6 4 1]),
// reflect-101 border, even samples.  Sums are formed in double: the products
// of float samples by the small integer taps and their sums are exact there,
// so the single rounding to float at the end gives the correctly rounded
// value whatever the summation order.
// --------------------------------------------------------------------------
__device__ __forceinline__ int reflect101(int i, int n) {
    if (i < 0) i = -i;
    if (i >= n) i = 2 * n - 2 - i;
    return clampi(i, 0, n - 1);  // only reached for samples no output uses
}

template <bool B>
__global__ __launch_bounds__(kBlock) void k_pyr_down(const WinDesc one, const BatchArgs ba,
                                                     int32_t total_arg, int level) {
    constexpr int RH = 2 * kPyrTileH + 4, RW = 2 * kPyrTileW + 4;
    __shared__ float sIn[RH][RW];
    __shared__ double sH[RH][kPyrTileW];
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const LevelGeom gs = d->lv[level - 1], gd = d->lv[level];
        const float* __restrict__ src = d->pyr + gs.off;
        float* dst = d->pyr + gd.off;
        const int tiles_x = (gd.w + kPyrTileW - 1) / kPyrTileW;
        const int X0 = (local % tiles_x) * kPyrTileW, Y0 = (local / tiles_x) * kPyrTileH;
        for (int i = threadIdx.x; i < RH * RW; i += kBlock) {
            const int r = i / RW, c = i % RW;
            const int sy = reflect101(2 * Y0 - 2 + r, gs.h), sx = reflect101(2 * X0 - 2 + c, gs.w);
            sIn[r][c] = src[(size_t)sy * gs.w + sx];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < RH * kPyrTileW; i += kBlock) {
            const int r = i / kPyrTileW, X = i % kPyrTileW;
            const float* p = &sIn[r][2 * X];
            sH[r][X] = (double)p[0] + 4.0 * (double)p[1] + 6.0 * (double)p[2] + 4.0 * (double)p[3] +
                       (double)p[4];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kPyrTileH * kPyrTileW; i += kBlock) {
            const int Y = i / kPyrTileW, X = i % kPyrTileW;
            if (X0 + X < gd.w && Y0 + Y < gd.h) {
                const double v = sH[2 * Y][X] + 4.0 * sH[2 * Y + 1][X] + 6.0 * sH[2 * Y + 2][X] +
                                 4.0 * sH[2 * Y + 3][X] + sH[2 * Y + 4][X];
                dst[(size_t)(Y0 + Y) * gd.w + X0 + X] = (float)(v * (1.0 / 256.0));
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// Dense inverse search, one level.  A wave holds 8 patches; the 8 lanes of a
// patch each own one column of it (8 template pixels, their gradients).  Per
// iteration a lane reads the 9 rows of two adjacent columns of I1 around its
// column (all pixels of a patch share the sub-pixel offset), interpolates
// bilinearly, and the residual products are summed over the patch's 8 lanes.
// The initial displacement of a patch is twice the coarser level's densified
// flow at the pixel nearest the patch centre, computed here from the coarser
// patch displacements (only at that pixel).
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_dis_level(const WinDesc one, const BatchArgs ba,
                                                      int32_t total_arg, int level) {
    const int32_t total = item_total<B>(ba, total_arg);
    const int lane = threadIdx.x & 63;
    const int slot = (threadIdx.x >> 6) * 8 + (lane >> 3);
    const int c = lane & 7;
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const LevelGeom g = d->lv[level];
        const int Wl = g.w, Hl = g.h, pnx = g.pnx;
        const int npatch = g.pnx * g.pny;
        const int s = d->stride;
        const float lam = d->lambda;
        const float* __restrict__ I0 = d->pyr_prev + g.off;
        const float* __restrict__ I1 = d->pyr + g.off;
        const int pi = local * kPatchesPerItem + slot;
        const bool valid = pi < npatch;
        const int pic = valid ? pi : npatch - 1;
        const int kx = pic % pnx, ky = pic / pnx;
        const int ox = min(kx * s, Wl - kPatch), oy = min(ky * s, Hl - kPatch);
        const int x = ox + c;
        const int xm = max(x - 1, 0), xp = min(x + 1, Wl - 1);

        float T[kPatch], gxs[kPatch], gys[kPatch];
        float hxx = 0.f, hxy = 0.f, hyy = 0.f;
#pragma unroll
        for (int j = 0; j < kPatch; ++j) {
            const int y = oy + j;
            const int ym = max(y - 1, 0), yp = min(y + 1, Hl - 1);
            const float* row = I0 + (size_t)y * Wl;
            T[j] = row[x];
            gxs[j] = 0.5f * (row[xp] - row[xm]);
            gys[j] = 0.5f * (I0[(size_t)yp * Wl + x] - I0[(size_t)ym * Wl + x]);
            hxx += gxs[j] * gxs[j];
            hxy += gxs[j] * gys[j];
            hyy += gys[j] * gys[j];
        }
        hxx = red8(hxx);
        hxy = red8(hxy);
        hyy = red8(hyy);
        const float a = hxx + lam, cc = hyy + lam;
        const float det = a * cc - hxy * hxy;
        const float ia = cc / det, ib = -hxy / det, ic = a / det;

        float u0x = 0.f, u0y = 0.f;
        if (level < d->L - 1) {
            const LevelGeom gc = d->lv[level + 1];
            const float* __restrict__ C0 = d->pyr_prev + gc.off;
            const float* __restrict__ C1 = d->pyr + gc.off;
            const float2* __restrict__ cu = d->puv + gc.poff;
            const int px = min((ox + kPatch / 2) >> 1, gc.w - 1);
            const int py = min((oy + kPatch / 2) >> 1, gc.h - 1);
            const Cover cx = cover_of(px, gc.w, gc.pnx, s), cy = cover_of(py, gc.h, gc.pny, s);
            const float i0 = C0[(size_t)py * gc.w + px];
            float sw = 0.f, su = 0.f, sv = 0.f;
            for (int q = c; q < cx.n * cy.n; q += 8) {
                const int qx = cover_index(cx, q % cx.n), qy = cover_index(cy, q / cx.n);
                const float2 u = cu[(size_t)qy * gc.pnx + qx];
                const float dv = bilinear(C1, gc.w, gc.h, (float)px + u.x, (float)py + u.y) - i0;
                const float w = 1.0f / fmaxf(1.0f, 255.0f * fabsf(dv));
                sw += w;
                su += w * u.x;
                sv += w * u.y;
            }
            sw = red8(sw);
            su = red8(su);
            sv = red8(sv);
            u0x = 2.0f * (su / sw);
            u0y = 2.0f * (sv / sw);
        }

        float ux = u0x, uy = u0y;
        const float lim = (float)(Wl + Hl + 16);
        const int iters = d->iters;
        for (int it = 0; it < iters; ++it) {
            const float sx = fminf(fmaxf(ux, -lim), lim), sy = fminf(fmaxf(uy, -lim), lim);
            const float fx = floorf(sx), fy = floorf(sy);
            const float ax = sx - fx, ay = sy - fy;
            const int ix = (int)fx, iy = (int)fy;
            const int xa = clampi(x + ix, 0, Wl - 1), xb = clampi(x + ix + 1, 0, Wl - 1);
            float bx = 0.f, by = 0.f, hprev = 0.f;
#pragma unroll
            for (int j = 0; j <= kPatch; ++j) {
                const int yy = clampi(oy + j + iy, 0, Hl - 1);
                const float* row = I1 + (size_t)yy * Wl;
                const float A = row[xa], Bv = row[xb];
                const float h = A + ax * (Bv - A);
                if (j > 0) {
                    const float w = hprev + ay * (h - hprev);
                    const float r = w - T[j - 1];
                    bx += gxs[j - 1] * r;
                    by += gys[j - 1] * r;
                }
                hprev = h;
            }
            bx = red8(bx);
            by = red8(by);
            ux -= ia * bx + ib * by;
            uy -= ib * bx + ic * by;
        }
        const float mx = ux - u0x, my = uy - u0y;
        if (mx * mx + my * my > (float)(kPatch * kPatch)) {
            ux = u0x;
            uy = u0y;
        }
        if (valid && c == 0) d->puv[g.poff + pi] = make_float2(ux, uy);
    }
}

// --------------------------------------------------------------------------
// Densification at level 0: the flow of a pixel is the mean of the covering
// patches' displacements weighted by 1 / max(1, 255 |I1(x+u) - I0(x)|);
// optionally zero outside the reference window's edge pixels.
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_densify(const WinDesc one, const BatchArgs ba, int32_t total_arg) {
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const LevelGeom g = d->lv[0];
        const int W = g.w, H = g.h;
        const int tiles_x = (W + 63) / 64;
        const int x = (local % tiles_x) * 64 + (threadIdx.x & 63);
        const int y = (local / tiles_x) * kDensTileH + (threadIdx.x >> 6);
        if (x >= W || y >= H) continue;
        const int s = d->stride;
        const float* __restrict__ I0 = d->pyr_prev;
        const float* __restrict__ I1 = d->pyr;
        const float2* __restrict__ pu = d->puv + g.poff;
        const Cover cx = cover_of(x, W, g.pnx, s), cy = cover_of(y, H, g.pny, s);
        const float i0 = I0[(size_t)y * W + x];
        float sw = 0.f, su = 0.f, sv = 0.f;
        for (int qy = 0; qy < cy.n; ++qy) {
            const int ky = cover_index(cy, qy);
            for (int qx = 0; qx < cx.n; ++qx) {
                const int kx = cover_index(cx, qx);
                const float2 u = pu[(size_t)ky * g.pnx + kx];
                const float dv = bilinear(I1, W, H, (float)x + u.x, (float)y + u.y) - i0;
                const float w = 1.0f / fmaxf(1.0f, 255.0f * fabsf(dv));
                sw += w;
                su += w * u.x;
                sv += w * u.y;
            }
        }
        float fu = su / sw, fv = sv / sw;
        if ((d->flags & EBOF_MASK_FLOW) && d->mask && !d->mask[(size_t)y * W + x]) fu = fv = 0.f;
        d->flow[(size_t)y * W + x] = fu;
        d->flow[(size_t)W * H + (size_t)y * W + x] = fv;
    }
}

// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------
#define EBOF_LAUNCH(KERNEL, L, ...)                                                              \
    do {                                                                                         \
        if ((L).batch)                                                                           \
            hipLaunchKernelGGL(KERNEL<true>, dim3((L).grid), dim3(kBlock), 0, (L).stream, *(L).one, \
                               (L).ba, (L).total, ##__VA_ARGS__);                                \
        else                                                                                     \
            hipLaunchKernelGGL(KERNEL<false>, dim3((L).grid), dim3(kBlock), 0, (L).stream,        \
                               *(L).one, (L).ba, (L).total, ##__VA_ARGS__);                      \
    } while (0)

void launch_zero(const Launch& L) { EBOF_LAUNCH(k_zero, L); }
void launch_scatter(const Launch& L) { EBOF_LAUNCH(k_scatter, L); }
void launch_denoise_fill(const Launch& L, bool pack) {
    if (pack) {
        if (L.batch)
            hipLaunchKernelGGL((k_denoise_fill<true, true>), dim3(L.grid), dim3(kBlock), 0, L.stream, *L.one,
                               L.ba, L.total);
        else
            hipLaunchKernelGGL((k_denoise_fill<false, true>), dim3(L.grid), dim3(kBlock), 0, L.stream, *L.one,
                               L.ba, L.total);
    } else {
        if (L.batch)
            hipLaunchKernelGGL((k_denoise_fill<true, false>), dim3(L.grid), dim3(kBlock), 0, L.stream, *L.one,
                               L.ba, L.total);
        else
            hipLaunchKernelGGL((k_denoise_fill<false, false>), dim3(L.grid), dim3(kBlock), 0, L.stream,
                               *L.one, L.ba, L.total);
    }
}
void launch_pack_cols(const Launch& L) { EBOF_LAUNCH(k_pack_cols, L); }
void launch_edt_cols(const Launch& L) { EBOF_LAUNCH(k_edt_cols, L); }
void launch_edt_rows(const Launch& L) { EBOF_LAUNCH(k_edt_rows, L); }
void launch_pyr_down(const Launch& L, int level) { EBOF_LAUNCH(k_pyr_down, L, level); }
void launch_dis_level(const Launch& L, int level) { EBOF_LAUNCH(k_dis_level, L, level); }
void launch_densify(const Launch& L) { EBOF_LAUNCH(k_densify, L); }

// --------------------------------------------------------------------------
// per-window work items of each stage
// --------------------------------------------------------------------------
int32_t stage_items(const WinDesc& d, int stage, bool has_flow, bool zero) {
    const int64_t N = (int64_t)d.W * d.H;
    const int bands = (d.W + 63) / 64, nch = (d.H + kChunk - 1) / kChunk;
    if (stage == kStZero) return zero ? (int32_t)((N + kZeroBytesPerItem - 1) / kZeroBytesPerItem) : 0;
    if (stage == kStScatter) return (int32_t)((d.n_ev + kEventsPerItem - 1) / kEventsPerItem);
    if (stage == kStDenoise) return ((d.W + kTile - 1) / kTile) * ((d.H + kTile - 1) / kTile);
    if (stage == kStPack || stage == kStCols) return bands * ((nch + 3) / 4);
    if (stage == kStRows) return d.H;
    if (stage >= kStPyr && stage < kStPyr + kMaxLevels - 1) {
        const int l = stage - kStPyr + 1;
        if (l >= d.L) return 0;
        const LevelGeom& g = d.lv[l];
        return ((g.w + kPyrTileW - 1) / kPyrTileW) * ((g.h + kPyrTileH - 1) / kPyrTileH);
    }
    if (stage >= kStDis && stage < kStDis + kMaxLevels) {
        const int l = stage - kStDis;
        if (!has_flow || l >= d.L) return 0;
        const LevelGeom& g = d.lv[l];
        return (g.pnx * g.pny + kPatchesPerItem - 1) / kPatchesPerItem;
    }
    if (stage == kStDensify) return has_flow ? ((d.W + 63) / 64) * ((d.H + kDensTileH - 1) / kDensTileH) : 0;
    return 0;
}

}  // namespace ebof

// kernels.hip -- gfx950 kernels of the per-window flow path.
//
// Every kernel runs 256-thread blocks over "work items" (a chunk of events, a
// tile, a row, a group of patches) and loops item = blockIdx.x, += gridDim.x,
// so one launch can cover one window or a whole batch of windows of mixed
// sizes (template parameter B: descriptor table + per-stage prefix sums).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "ebof_dev.h"
#include "dens_dev.h"

// Patch displacements of the allocation-free flow call (ebof_flow_noalloc):
// a fixed array that each GPU the library runs on holds until the process
// ends.  In host code this name is a host-side stand-in, not a device
// address: host code passes the address noalloc_scratch() returns instead.
static __device__ __align__(256) float2 scratch[ebof::kNoAllocPatches];

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
        int lo = 0, hi = *ba.nwin - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ba.prefix[mid * kNumStages + ba.stage] <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        local = item - ba.prefix[lo * kNumStages + ba.stage];
        return ba.tab + lo;
    }
}

template <bool B>
__device__ __forceinline__ int32_t item_total(const BatchArgs& ba, int32_t total_arg) {
    if constexpr (B)
        return ba.prefix[*ba.nwin * kNumStages + ba.stage];
    else
        return total_arg;
}

// Work-groups are dispatched round-robin over the 8 XCDs (block b on XCD
// b mod 8), each with its own L2.  Neighbouring items share halo data, so
// block b takes item x*q + min(x, r) + b/8 (x = b mod 8, G = 8q + r): every
// XCD works through a contiguous run of items.  A bijection on [0, G).
constexpr int kXcds = 8;
__device__ __forceinline__ int32_t xcd_item(int32_t b, int32_t G) {
    const int32_t q = G / kXcds, r = G % kXcds, x = b % kXcds;
    return x * q + min(x, r) + b / kXcds;
}

// Copies an h x w window into LDS (row pitch w, or `pitch`): element (r, c) =
// src(r, c).
// Thread t takes elements t, t + kBlock, ...; it issues U of its loads before
// its first LDS write, so U global loads per thread are in flight instead of
// one (a load feeding an LDS store otherwise waits out the full memory
// latency before the next load issues).
template <int U, class T, class Src, int NT = kBlock>
__device__ __forceinline__ void stage_window(T* __restrict__ dst, int w, int h, Src src, int pitch = 0) {
    const int n = w * h;
    if (pitch == 0) pitch = w;
    int r = threadIdx.x / w, cc = threadIdx.x - r * w;
    const int dr = NT / w, dc = NT - dr * w;
    for (int base = 0; base < n; base += U * NT) {
        T v[U];
        int off[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            off[u] = r < h ? r * pitch + cc : -1;
            v[u] = r < h ? src(r, cc) : T(0);
            cc += dc;
            r += dr;
            if (cc >= w) {
                cc -= w;
                ++r;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (off[u] >= 0) dst[off[u]] = v[u];
    }
}

// --------------------------------------------------------------------------
// zero the event staging image (done when the window stamp wraps)
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_zero(const WinDesc one, const BatchArgs ba, int32_t total_arg) {
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = xcd_item(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
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
    for (int32_t item = xcd_item(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int64_t t0 = d->t0, t1 = d->t1;
        const uint32_t W = (uint32_t)d->W, H = (uint32_t)d->H;
        const uint8_t stamp = (uint8_t)d->stamp;
        uint8_t* __restrict__ er = d->e_raw;
        // a window by time, or an index range read from device memory (every
        // event in it belongs to the window)
        const bool by_range = d->range != nullptr;
        const int64_t r0 = by_range ? d->range[0] : 0;
        const int64_t n = by_range ? min(d->range[1], d->n_ev) : d->n_ev;  // n_ev: the arrays' length
        const int64_t base = r0 + (int64_t)local * kEventsPerItem;
        uint32_t dropped = 0;
#pragma unroll
        for (int k = 0; k < kEventsPerItem / kBlock; ++k) {
            const int64_t e = base + k * kBlock + threadIdx.x;
            if (e < n) {
                const int64_t t = by_range ? t0 : __builtin_nontemporal_load(d->et + e);
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
// Alg. 1 then Alg. 2 on one 64-wide, 32-tall tile.  The raw image is staged
// with a 2-pixel halo, the denoised image E_d is formed on the tile plus a
// 1-pixel halo (each pixel counts its 4 neighbours in E), then the fill forms
// E_df on the tile (counting neighbours in E_d).  Pixels off the image are
// non-edges.  Optionally the tile writes its half of the column bit masks
// (bit r of word (chunk, x) = E_df at row 64*chunk + r).
// --------------------------------------------------------------------------
template <bool B, bool PACK>
__global__ __launch_bounds__(kBlock) void k_denoise_fill(const WinDesc one, const BatchArgs ba,
                                                         int32_t total_arg) {
    constexpr int TW = kTile, TH = kTileH;
    constexpr int RW = TW + 4, RH = TH + 4;  // raw tile with 2-pixel halo
    constexpr int DW = TW + 2, DH = TH + 2;  // denoised tile with 1-pixel halo
    __shared__ uint8_t sE[RH][RW + 4];
    __shared__ uint8_t sEd[DH][DW + 2];
    __shared__ uint8_t sBits[4][TW];
    const int32_t total = item_total<B>(ba, total_arg);
    const int tid = threadIdx.x;
    for (int32_t item = xcd_item(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int W = d->W, H = d->H;
        const int tiles_x = (W + TW - 1) / TW;
        const int tx = local % tiles_x, ty = local / tiles_x;
        const int x0 = tx * TW, y0 = ty * TH;
        const uint8_t stamp = (uint8_t)d->stamp;
        const uint8_t* __restrict__ er = d->e_raw;
        const int n_d = d->n_d, n_f = d->n_f;
        {
            // staged with pitch RW into the padded rows of sE (pitch RW + 4)
            uint8_t raw[(RH * RW + kBlock - 1) / kBlock];
            int i = tid;
#pragma unroll
            for (int u = 0; u < (RH * RW + kBlock - 1) / kBlock; ++u, i += kBlock) {
                const int ly = i / RW, lx = i - ly * RW;
                const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
                raw[u] = (i < RH * RW && gx >= 0 && gx < W && gy >= 0 && gy < H) ? er[(size_t)gy * W + gx] : 0;
            }
            i = tid;
#pragma unroll
            for (int u = 0; u < (RH * RW + kBlock - 1) / kBlock; ++u, i += kBlock) {
                const int ly = i / RW, lx = i - ly * RW;
                if (i < RH * RW) sE[ly][lx] = raw[u] == stamp;  // stamps are 1..255: off-image 0 never matches
            }
        }
        __syncthreads();
        for (int i = tid; i < DH * DW; i += kBlock) {
            const int ly = i / DW, lx = i - ly * DW;  // pixel (x0-1+lx, y0-1+ly) = sE[ly+1][lx+1]
            uint8_t v = sE[ly + 1][lx + 1];
            if (v) {
                const int nb = sE[ly][lx + 1] + sE[ly + 2][lx + 1] + sE[ly + 1][lx] + sE[ly + 1][lx + 2];
                v = nb >= n_d;
            }
            sEd[ly][lx] = v;
        }
        __syncthreads();
        const int c = tid & (TW - 1), seg = tid / TW;  // 4 segments of 8 rows
        const int gx = x0 + c;
        uint32_t bits = 0;
#pragma unroll
        for (int r = 0; r < TH / 4; ++r) {
            const int ly = seg * (TH / 4) + r;  // pixel (gx, y0+ly) = sEd[ly+1][c+1]
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
            sBits[seg][c] = (uint8_t)bits;
            __syncthreads();
            if (tid < TW && x0 + tid < W) {
                const uint32_t m = (uint32_t)sBits[0][tid] | ((uint32_t)sBits[1][tid] << 8) |
                                   ((uint32_t)sBits[2][tid] << 16) | ((uint32_t)sBits[3][tid] << 24);
                // this tile is half `ty & 1` of chunk ty/2 (little endian words)
                uint32_t* half = (uint32_t*)(d->colmask + (size_t)(ty >> 1) * W + x0 + tid);
                half[ty & 1] = m;
                if (!(ty & 1) && y0 + TH >= H) half[1] = 0;  // no upper half tile
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// Column bit masks of an edge image (for edge images not produced by
// k_denoise_fill).  Item = one 64x64 tile; thread = (column, 16-row segment);
// the four 16-bit pieces of a column are joined in LDS.
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_pack_cols(const WinDesc one, const BatchArgs ba,
                                                      int32_t total_arg) {
    __shared__ uint16_t sBits[4][64];
    const int32_t total = item_total<B>(ba, total_arg);
    const int c = threadIdx.x & 63, seg = threadIdx.x >> 6;
    for (int32_t item = xcd_item(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int W = d->W, H = d->H;
        const int bands = (W + 63) / 64;
        const int bx = local % bands, ck = local / bands;
        const int x = bx * 64 + c;
        const int y0 = ck * kChunk + seg * 16;
        uint32_t bits = 0;
        if (x < W) {
            const uint8_t* col = d->e_df + (size_t)y0 * W + x;
            if (y0 + 16 <= H) {
#pragma unroll
                for (int r = 0; r < 16; ++r) bits |= (uint32_t)(col[(size_t)r * W] != 0) << r;
            } else {
                for (int r = 0; y0 + r < H; ++r) bits |= (uint32_t)(col[(size_t)r * W] != 0) << r;
            }
        }
        sBits[seg][c] = (uint16_t)bits;
        __syncthreads();
        if (seg == 0 && x < W)
            d->colmask[(size_t)ck * W + x] = (uint64_t)sBits[0][c] | ((uint64_t)sBits[1][c] << 16) |
                                             ((uint64_t)sBits[2][c] << 32) | ((uint64_t)sBits[3][c] << 48);
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// Exact distance transform, column pass: g(x, y) = min |y - y'| over the edge
// pixels (x, y') of column x, or kGInf when the column has none.  Item = one
// 64x64 tile; thread = (column, 16-row segment).  The nearest edges above and
// below the tile's chunk come from the neighbouring chunks' masks, those
// inside it from bit scans of the chunk's mask.
// --------------------------------------------------------------------------
template <bool B>
__global__ __launch_bounds__(kBlock) void k_edt_cols(const WinDesc one, const BatchArgs ba,
                                                     int32_t total_arg) {
    const int32_t total = item_total<B>(ba, total_arg);
    const int c = threadIdx.x & 63, seg = threadIdx.x >> 6;
    for (int32_t item = xcd_item(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int W = d->W, H = d->H;
        const int bands = (W + 63) / 64, nch = (H + kChunk - 1) / kChunk;
        const int bx = local % bands, ck = local / bands;
        const int x = bx * 64 + c;
        if (x >= W) continue;
        const uint64_t* cm = d->colmask + x;
        const uint64_t m = cm[(size_t)ck * W];
        // nearest edge rows above and below the chunk, from the neighbouring
        // chunks' masks read kScan at a time
        constexpr int kScan = 4;
        int above = -1, below = -1;
        for (int c2 = ck - 1; c2 >= 0 && above < 0; c2 -= kScan) {
            uint64_t mm[kScan];
#pragma unroll
            for (int u = 0; u < kScan; ++u) mm[u] = c2 - u >= 0 ? cm[(size_t)(c2 - u) * W] : 0;
#pragma unroll
            for (int u = 0; u < kScan; ++u)
                if (above < 0 && mm[u]) above = (c2 - u) * kChunk + 63 - __clzll(mm[u]);
        }
        for (int c2 = ck + 1; c2 < nch && below < 0; c2 += kScan) {
            uint64_t mm[kScan];
#pragma unroll
            for (int u = 0; u < kScan; ++u) mm[u] = c2 + u < nch ? cm[(size_t)(c2 + u) * W] : 0;
#pragma unroll
            for (int u = 0; u < kScan; ++u)
                if (below < 0 && mm[u]) below = (c2 + u) * kChunk + __ffsll((unsigned long long)mm[u]) - 1;
        }
        const int r0 = seg * 16;
        const int rows = min(16, H - ck * kChunk - r0);
        uint16_t* gcol = d->g + (size_t)(ck * kChunk + r0) * W + x;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (r < rows) {
                const int rr = r0 + r;  // row within the chunk
                const int y = ck * kChunk + rr;
                const uint64_t lo = rr == 63 ? m : (m & ((2ull << rr) - 1));  // bits <= rr
                const uint64_t hi = m >> rr;                                   // bits >= rr
                const int prev = lo ? ck * kChunk + 63 - __clzll(lo) : above;
                const int nxt = hi ? y + __ffsll((unsigned long long)hi) - 1 : below;
                int gv = 0x7fffffff;
                if (prev >= 0) gv = y - prev;
                if (nxt >= 0) gv = min(gv, nxt - y);
                gcol[(size_t)r * W] = gv == 0x7fffffff ? kGInf : (uint16_t)gv;
            }
        }
    }
}

// --------------------------------------------------------------------------
// Exact distance transform, row pass, fused with eq. (1).  Item = NR rows x
// a kRowSeg-pixel segment; thread = one column of the segment, which
// searches its rows together (independent LDS reads in flight).  Every pixel
// searches outwards, D2(x) = min_r r^2 + g(x +- r)^2, stopping once r^2
// reaches the best value found (no further column can beat it): the exact
// minimum.  The rows' g within kRowReach of the segment are staged in LDS; a
// search reaching further reads global memory.  The surface is looked up from
// the squared distance: lut[D2] below lut_n, exactly 1.0f from there on.  When
// D2 is not exported the search also stops at r^2 >= lut_n: a minimum of
// lut_n or more gives 1.0f whatever it is, and a smaller one is always found
// before that radius.  Such a window (edt_local) needs g only up to lut_r:
// the item forms its rows' column distances from the column masks (the
// chunk's word and its two neighbours, which reach 64 rows each way), capped
// at lut_r, over a band of lut_r rounded up to kRowUnroll columns each side,
// and there is no column pass.  Capping changes no candidate below lut_n: a
// squared distance under lut_n <= lut_r^2 comes from a column less than
// lut_r away whose g is less than lut_r, and every candidate that involves a
// capped g is at least lut_r^2.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t g_sq(uint32_t g) { return g == kGInf ? 0x7fffffffu : g * g; }
// the capped search's 16-bit pair for a column outside the image: above any
// candidate (g^2 and r^2 are at most 64^2 there), and with r^2 still below 2^15
constexpr uint32_t kFarPair = 0x3FFF3FFFu;

template <bool B, int NR>
__global__ __launch_bounds__(kBlock) void k_edt_rows(const WinDesc one, const BatchArgs ba,
                                                     int32_t total_arg) {
    constexpr int R = kRowReach;
    __shared__ uint32_t sG[NR * (kRowSeg + 2 * R)];  // g^2, 0x7fffffff = no edge in the column
    __shared__ float sLut[kLutLds];
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = xcd_item(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int W = d->W, H = d->H;
        const int nseg = (W + kRowSeg - 1) / kRowSeg;
        const int y0 = (local / nseg) * NR, x0 = (local - (local / nseg) * nseg) * kRowSeg;
        const int nrows = min(NR, H - y0);
        const bool exp_d2 = d->d2 != nullptr;
        const int lut_n = d->lut_n;
        const bool lut_lds = lut_n <= kLutLds;
        const int kind = d->surf_kind;
        const bool computed = kind == EBOF_SURFACE_LINEAR || kind == EBOF_SURFACE_LOG;
        const float sat = d->lut_sat;
        // (a surface that never saturates needs the exact distance everywhere)
        const uint32_t cap = (exp_d2 || computed) ? 0xffffffffu : (uint32_t)lut_n;
        const bool loc = edt_local(*d);
        const int band = loc ? (d->lut_r + kRowUnroll - 1) / kRowUnroll * kRowUnroll : R;
        // (the capped form stages its whole band, columns outside the image
        // included, so that its search reads without bounds checks)
        const int lo = loc ? x0 - band : max(0, x0 - band);
        const int hi = loc ? x0 + kRowSeg + band : min(W, x0 + kRowSeg + band);
        const int ww = hi - lo;
        const uint16_t* __restrict__ g = d->g + (size_t)y0 * W;
        const float* __restrict__ lut = d->lut;
        if (loc) {
            // the item's rows lie in one 64-row chunk (NR divides kChunk)
            const int ck = y0 / kChunk, nch = (H + kChunk - 1) / kChunk;
            const int rr0 = y0 - ck * kChunk, lr = d->lut_r;
            const uint64_t* __restrict__ cm = d->colmask + lo;
            for (int c = threadIdx.x; c < ww; c += kBlock) {
                if (lo + c < 0 || lo + c >= W) {  // outside the image: never the nearest
#pragma unroll
                    for (int k = 0; k < NR; ++k) {
                        if constexpr (NR % 2 == 0) {
                            if (!(k & 1)) sG[(k >> 1) * ww + c] = kFarPair;
                        } else {
                            sG[k * ww + c] = 0x7fffffffu;
                        }
                    }
                    continue;
                }
                const uint64_t m = cm[(size_t)ck * W + c];
                const uint64_t mp = ck > 0 ? cm[(size_t)(ck - 1) * W + c] : 0ull;
                const uint64_t mn = ck + 1 < nch ? cm[(size_t)(ck + 1) * W + c] : 0ull;
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const int rr = rr0 + k;  // row within the chunk
                    int gv = lr;
                    const uint64_t dn = m >> rr;                                     // bits >= rr
                    const uint64_t up = rr == 63 ? m : (m & ((2ull << rr) - 1));     // bits <= rr
                    if (dn)
                        gv = min(gv, __ffsll((unsigned long long)dn) - 1);
                    else if (mn)
                        gv = min(gv, kChunk - rr + __ffsll((unsigned long long)mn) - 1);
                    if (up)
                        gv = min(gv, rr - (63 - __clzll(up)));
                    else if (mp)
                        gv = min(gv, rr + 1 + __clzll(mp));
                    if constexpr (NR % 2 == 0) {
                        // rows 2j and 2j+1 as the halves of word j (row
                        // beyond the image: 0, so never searched)
                        const uint32_t v = k < nrows ? (uint32_t)(gv * gv) : 0u;
                        if (k & 1)
                            sG[(k >> 1) * ww + c] |= v << 16;
                        else
                            sG[(k >> 1) * ww + c] = v;
                    } else {
                        sG[k * ww + c] = k < nrows ? (uint32_t)(gv * gv) : 0x7fffffffu;
                    }
                }
            }
        } else {
            stage_window<8>(sG, ww, NR, [&](int r, int c) -> uint32_t {
                return r < nrows ? g_sq(g[(size_t)r * W + lo + c]) : 0x7fffffffu;
            });
        }
        if (lut_lds) {
            float lv[kLutLds / kBlock];
#pragma unroll
            for (int u = 0; u < kLutLds / kBlock; ++u) {
                const int i = threadIdx.x + u * kBlock;
                lv[u] = i < lut_n ? lut[i] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kLutLds / kBlock; ++u) sLut[threadIdx.x + u * kBlock] = lv[u];
        }
        __syncthreads();
        const int x = x0 + threadIdx.x;
        if constexpr (NR % 2 == 0) {
            if (loc) {
                // Capped search on 16-bit pairs: every value stays below
                // 2^15 (g^2 and r^2 at most 64^2 here; a column outside the
                // image holds kFarPair), so two rows take one packed add and one
                // packed min per candidate column.
                typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
                constexpr int NP = NR / 2;
                if (x < W) {
                    const uint32_t* row = sG - lo;  // rows 2j, 2j+1 at row + j * ww
                    u16x2 best[NP];
#pragma unroll
                    for (int j = 0; j < NP; ++j) best[j] = __builtin_bit_cast(u16x2, row[j * ww + x]);
                    constexpr int U = kRowUnroll;
                    for (int r = 1; r <= R; r += U) {
                        const uint32_t r2 = (uint32_t)(r * r);
                        bool live = false;
#pragma unroll
                        for (int j = 0; j < NP; ++j) live |= r2 < best[j].x || r2 < best[j].y;
                        if (!live || r2 >= (uint32_t)lut_n) break;
                        // (every radius read here lies in the staged band:
                        // r + 3 <= band whenever r * r < lut_n <= lut_r^2)
                        u16x2 cl[U][NP], cr[U][NP];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int rr = r + u;
#pragma unroll
                            for (int j = 0; j < NP; ++j) {
                                cl[u][j] = __builtin_bit_cast(u16x2, row[j * ww + x - rr]);
                                cr[u][j] = __builtin_bit_cast(u16x2, row[j * ww + x + rr]);
                            }
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const u16x2 rr2 = (u16x2)(unsigned short)((r + u) * (r + u));
#pragma unroll
                            for (int j = 0; j < NP; ++j)
                                best[j] = __builtin_elementwise_min(best[j],
                                                                    __builtin_elementwise_min(cl[u][j], cr[u][j]) + rr2);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < NR; ++k) {
                        if (k < nrows) {
                            const uint32_t b = (k & 1) ? best[k >> 1].y : best[k >> 1].x;
                            d->pyr[(size_t)(y0 + k) * W + x] = b < (uint32_t)lut_n ? (lut_lds ? sLut[b] : lut[b]) : sat;
                        }
                    }
                }
                __syncthreads();
                continue;
            }
        }
        if (x < W) {
            const uint32_t* row = sG - lo;  // row k at row + k * ww, columns lo .. hi-1
            uint32_t best[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) best[k] = k < nrows ? row[k * ww + x] : 0u;  // 0: nothing to search
            // radii in steps of kRowUnroll, the loads of a step issued
            // together; a radius past a row's stopping point only offers
            // candidates >= r^2 >= its best (or >= the cap), which change
            // neither D2 below the cap nor the surface
            constexpr int U = kRowUnroll;
            int r = 1;
            for (; r <= R; r += U) {
                const uint32_t r2 = (uint32_t)(r * r);
                bool live = false;
#pragma unroll
                for (int k = 0; k < NR; ++k) live |= r2 < best[k] && r2 < cap;
                if (!live || (x - r < 0 && x + r >= W)) break;
                uint32_t cl[U][NR], cr[U][NR];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int rr = r + u;
                    const bool lft = x - rr >= 0, rgt = x + rr < W;
#pragma unroll
                    for (int k = 0; k < NR; ++k) {
                        cl[u][k] = lft ? row[k * ww + x - rr] : 0x7fffffffu;
                        cr[u][k] = rgt ? row[k * ww + x + rr] : 0x7fffffffu;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t rr2 = (uint32_t)((r + u) * (r + u));
#pragma unroll
                    for (int k = 0; k < NR; ++k) best[k] = min(best[k], rr2 + min(cl[u][k], cr[u][k]));
                }
            }
            if (!loc && r > R) {  // beyond the staged columns (a capped search never gets here)
                for (;; ++r) {
                    const uint32_t r2 = (uint32_t)r * (uint32_t)r;
                    const bool lft = x - r >= 0, rgt = x + r < W;
                    if (!lft && !rgt) break;
                    bool live = false;
#pragma unroll
                    for (int k = 0; k < NR; ++k) {
                        if (r2 < best[k] && r2 < cap) {
                            live = true;
                            const uint16_t* gr = g + (size_t)k * W;
                            if (lft) best[k] = min(best[k], r2 + g_sq(gr[x - r]));
                            if (rgt) best[k] = min(best[k], r2 + g_sq(gr[x + r]));
                        }
                    }
                    if (!live) break;
                }
            }
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                if (k < nrows) {
                    const size_t pix = (size_t)(y0 + k) * W + x;
                    const uint32_t b = best[k];
                    if (exp_d2) d->d2[pix] = b >= 0x7fffffffu ? 0x7fffffff : (int32_t)b;
                    if (computed) {
                        // in double, rounded once, as the squared distance's
                        // table would hold it
                        const double dd = sqrt((double)b);
                        d->pyr[pix] = (float)(kind == EBOF_SURFACE_LINEAR ? dd : log(dd + 1.0));
                    } else {
                        d->pyr[pix] = b < (uint32_t)lut_n ? (lut_lds ? sLut[b] : lut[b]) : sat;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Copies the h x w window of img at (x0, y0) into LDS row-major with pitch
// p: element (r, c) at dst[r * p + c] takes img(map(y0 + r, H), map(x0 + c,
// W)), map placing positions outside the image (clamping for a replicated
// border, reflect-101 for the pyramid).  The block's NT / 64 waves take rows
// in turn and move each row in 64-column pieces straight from global memory
// into LDS (lane i of a piece lands at word i), so no registers hold the data
// and every load of the window is in flight at once.  The caller waits for
// the loads (lds_load_wait) and synchronises the block before reading.
template <int NT, class Map>
__device__ __forceinline__ void stage_rows_lds_map(float* __restrict__ dst, const float* __restrict__ img, int W,
                                                   int H, int x0, int y0, int w, int h, int p, Map map) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c0 = 0; c0 < w; c0 += 64) {
        const int gx = map(x0 + c0 + lane, W);
        if (c0 + lane < w) {
            for (int r = wave; r < h; r += NT / 64)
                __builtin_amdgcn_global_load_lds(img + (size_t)map(y0 + r, H) * W + gx,
                                                 (__attribute__((address_space(3))) void*)(dst + r * p + c0), 4, 0, 0);
        }
    }
}
// ... with indices clamped into the image (replicated border)
__device__ __forceinline__ void stage_rows_lds(float* __restrict__ dst, const float* __restrict__ img, int W, int H,
                                               int x0, int y0, int w, int h, int p) {
    stage_rows_lds_map<kBlock>(dst, img, W, H, x0, y0, w, h, p, [](int i, int n) { return clampi(i, 0, n - 1); });
}
// waits for this wave's loads into LDS (and everything else outstanding)
__device__ __forceinline__ void lds_load_wait() { __builtin_amdgcn_s_waitcnt(0); }

// --------------------------------------------------------------------------
// Pyramid: level l+1 = 5x5 binomial (separable [1 4 6 4 1]) of level l,
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

// One launch builds up to three levels below level `from`.  A block owns a
// kPyrTile x kPyrTile tile (8x8) of the deepest level it builds; it stages the
// region of level `from` that the tile depends on (85x85 for three levels)
// and computes each intermediate level over the region the next one needs,
// writing only its own part of every level.  Regions: R(deepest) = kPyrTile,
// R(k-1) = 2 R(k) + 3, origin o(k-1) = 2 o(k) - 2.
//
// Borders: a level's outputs read its source only within two pixels of the
// source image (positions -2 .. w+1), and reflect-101 maps those positions
// into the image.  So every region position in that band holds the value of
// its reflected position (staged from it, or computed at it), positions
// further out are never read, and every output takes its 25 taps at fixed
// offsets from one address.
template <int NT>
__device__ __forceinline__ void rc_init(int n, int& r, int& cc, int& dr, int& dc) {
    r = threadIdx.x / n;
    cc = threadIdx.x - r * n;
    dr = NT / n;
    dc = NT - dr * n;
}
__device__ __forceinline__ void rc_step(int n, int& r, int& cc, int dr, int dc) {
    cc += dc;
    r += dr;
    if (cc >= n) {
        cc -= n;
        ++r;
    }
}

// 5x5 binomial at q (top-left tap) of a region with row pitch P, in double
template <int P>
__device__ __forceinline__ float binom25(const float* q) {
    double acc = 0.0;
    constexpr double kw[5] = {1.0, 4.0, 6.0, 4.0, 1.0};
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const float* a = q + j * P;
        const double h = (double)a[0] + 4.0 * (double)a[1] + 6.0 * (double)a[2] + 4.0 * (double)a[3] + (double)a[4];
        acc += kw[j] * h;
    }
    return (float)(acc * (1.0 / 256.0));
}

template <bool B>
__global__ __launch_bounds__(kPyrBlock) void k_pyr_chain(const WinDesc one, const BatchArgs ba, int32_t total_arg,
                                                         int from) {
    // one array, three regions (R0 x R0 | R1 x R1 | R2 x R2: 85 | 41 | 19 for
    // 8x8 tiles); offsets rather than pointers keep every access in the LDS
    // address space
    constexpr int T = kPyrTile, R2c = 2 * T + 3, R1c = 2 * R2c + 3, R0c = 2 * R1c + 3;
    __shared__ float sP[R0c * R0c + R1c * R1c + R2c * R2c];
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = xcd_item(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const int nlev = min(kPyrChain, d->L - 1 - from);
        const LevelGeom gd = d->lv[from + nlev];
        const int tiles_x = (gd.w + T - 1) / T;
        const int tx = local % tiles_x, ty = local / tiles_x;
        int R[kPyrChain + 1], ox[kPyrChain + 1], oy[kPyrChain + 1];
        int buf[kPyrChain + 1];
        R[nlev] = T;
        ox[nlev] = T * tx;
        oy[nlev] = T * ty;
        for (int k = nlev - 1; k >= 0; --k) {
            R[k] = 2 * R[k + 1] + 3;
            ox[k] = 2 * ox[k + 1] - 2;
            oy[k] = 2 * oy[k + 1] - 2;
        }
        for (int k = 0; k <= nlev; ++k)
            buf[k] = (nlev - k == 1) ? R0c * R0c + R1c * R1c : (nlev - k == 2) ? R0c * R0c : 0;
        {
            // every position takes the value of its reflected position
            // (clamped as well: positions beyond the band are never read)
            const LevelGeom g0 = d->lv[from];
            stage_rows_lds_map<kPyrBlock>(sP + buf[0], d->pyr + g0.off, g0.w, g0.h, ox[0], oy[0], R[0], R[0], R[0],
                                          [](int i, int n) { return clampi(reflect101(i, n), 0, n - 1); });
            lds_load_wait();
        }
        __syncthreads();
        for (int k = 1; k <= nlev; ++k) {
            const LevelGeom gt = d->lv[from + k];
            const int in = buf[k - 1], outb = buf[k];
            const int Rin = R[k - 1], oxi = ox[k - 1], oyi = oy[k - 1];
            const int n = R[k];
            const int span = T << (nlev - k);
            const int cx0 = span * tx, cy0 = span * ty;
            float* dst = d->pyr + gt.off;
            int r, cc, dr, dc;
            rc_init<kPyrBlock>(n, r, cc, dr, dc);
            for (; r < n; rc_step(n, r, cc, dr, dc)) {
                const int X = ox[k] + cc, Y = oy[k] + r;
                // the band around the image feeds the next level; the deepest
                // level built here needs its image pixels only
                const int band = k < nlev ? 2 : 0;
                if (X < -band || X >= gt.w + band || Y < -band || Y >= gt.h + band) continue;
                const int Xr = reflect101(X, gt.w), Yr = reflect101(Y, gt.h);
                const float* q = sP + in + (2 * Yr - 2 - oyi) * Rin + (2 * Xr - 2 - oxi);
                const float v = Rin == R0c ? binom25<R0c>(q) : Rin == R1c ? binom25<R1c>(q) : binom25<R2c>(q);
                if (k < nlev) sP[outb + r * n + cc] = v;
                if (X == Xr && Y == Yr && X >= cx0 && X < cx0 + span && Y >= cy0 && Y < cy0 + span)
                    dst[(size_t)Y * gt.w + X] = v;
            }
            __syncthreads();
        }
    }
}

// --------------------------------------------------------------------------
// Dense inverse search.  The template gradients and the Hessian's sums are
// formed in single precision, the regularised Hessian's inverse in double
// (once per patch); the initial displacement from the coarser level is
// densified as at level 0 (single precision, exact sample split); the
// iterations run in single precision.
// With the Hessian regularised by lambda*I the step is bounded by
// |b| / lambda, so single-precision rounding of the residual sums (relative
// 2^-24 of sums of order one) moves a patch by far less than the endpoint
// tolerance of the flow.
// --------------------------------------------------------------------------
// (every lane is a valid source for these patterns: no old value needed)
template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

constexpr int kDisRW = 112;   // LDS search region, columns
constexpr int kDisRH = 68;    // LDS search region, rows
constexpr int kDisRP = 128;   // ... stored row-major with this pitch
constexpr int kDisMargin = kPatch + 6;   // around the initial windows: covers a patch
                                         // that drifts up to this far in an iteration
constexpr int kDisMargin0 = kPatch + 2;  // ... at level 0, where the initial displacement
                                         // (from a level of twice the resolution) drifts less


// sums over the LP lanes of a patch (LP = 8: quad swaps then the half-row
// mirror; LP = 4: the two quad swaps), result in every lane
template <int LP>
__device__ __forceinline__ float redf(float v) {
    v += dppf<0xB1>(v);
    v += dppf<0x4E>(v);
    if constexpr (LP == 8) v += dppf<0x141>(v);
    return v;
}

// One level.  LP lanes per patch, each owning 8/LP patch columns (LP = 8:
// one column per lane, the shortest dependent chain per iteration, for small
// levels; LP = 4: two columns per lane, the sample column between them read
// once and the per-iteration coordinate, reduction and update work shared by
// twice the pixels, for large levels).  Work item = 16 consecutive patches of
// 256/(16 LP) patch rows (256 lanes), a near-square block of the image, so
// that the spread of the patches' initial displacements, which sizes the
// search region, stays small.  The reference strip (rows oy-1 .. oy+8 of
// every patch row of the item) is staged in LDS for the template and its
// gradient; then the region of I1 covering every patch's search window at
// its initial displacement (plus a margin) is staged, row-major, and the
// iterations read it there (a patch whose window leaves the region reads
// global memory; both give the same clamped samples).  At level 0, when only
// the masked flow is wanted, the item's patches that hold a mask pixel are
// packed into its first waves and the others are not computed.
template <bool B, int LP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_dis_level(const WinDesc one, const BatchArgs ba, int32_t total_arg,
                                                      int level) {
    constexpr int CPL = kPatch / LP;                   // patch columns per lane
    constexpr int PR = kBlock / kPatchesPerItem / LP;  // patch rows per item
    constexpr int PPW = 64 / LP;                       // patches per wave
    constexpr int WPR = kPatchesPerItem / PPW;         // waves per patch row
    static_assert(WPR * PR == kBlock / 64, "the block's waves tile the item");
    // the reference strip at the largest stride (8) fits the buffer
    static_assert(((kPatchesPerItem - 1) * 8 + kPatch + 2) * ((PR - 1) * 8 + kPatch + 2) <= kDisRH * kDisRP,
                  "reference strip too large");
    __shared__ float sR[kDisRH * kDisRP];
    __shared__ int sBox[kBlock / 64][4];
    __shared__ int sCnt[kBlock / 64];        // needed patches per wave
    __shared__ int sList[kBlock / LP];       // the item's needed patches, packed
    const int32_t total = item_total<B>(ba, total_arg);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int prow = wave / WPR;                      // patch row within the item
    const int slot = (wave % WPR) * PPW + lane / LP;  // patch within the row segment
    const int cg = lane % LP;                         // the lane's column group
    for (int32_t item = xcd_item(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const LevelGeom g = d->lv[level];
        const int Wl = g.w, Hl = g.h, pnx = g.pnx, pny = g.pny;
        const int nseg = (pnx + kPatchesPerItem - 1) / kPatchesPerItem;
        const int kyi = local / nseg, seg = local - (local / nseg) * nseg;
        const int s = d->stride;
        const double lam = (double)d->lambda;
        const float* __restrict__ I0 = d->pyr_prev + g.off;
        const float* __restrict__ I1 = d->pyr + g.off;
        const int ky0 = kyi * PR, ky_last = min(ky0 + PR, pny) - 1;
        const int kx0 = seg * kPatchesPerItem;
        const int kx_last = min(kx0 + kPatchesPerItem, pnx) - 1;
        int ky = ky0 + prow, kx = kx0 + slot;
        bool valid = kx < pnx && ky < pny;
        // When only the masked flow is wanted, a level-0 patch with no pixel
        // on the mask is not needed: a pixel's flow reads only the patches
        // that contain it, and the densification skips pixels off the mask.
        // An item with no needed patch returns at once; the needed patches of
        // the others are packed, in item order, into the first waves, and the
        // waves left over (active false, the same for a whole wave) skip the
        // initial displacement, the template and the iterations.  A needed
        // patch runs the same arithmetic wherever it is packed.
        const bool mask_only = level == 0 && (d->flags & EBOF_MASK_FLOW) && d->mask && !d->flow_keep && !d->ud;
        bool active = true;
        if (mask_only) {
            const int ox = min(min(kx, kx_last) * s, Wl - kPatch), oy = min(min(ky, ky_last) * s, Hl - kPatch);
            const uint8_t* __restrict__ mp = d->mask + (size_t)oy * Wl + ox + cg * CPL;
            uint32_t mb = 0;
#pragma unroll
            for (int j = 0; j < kPatch; ++j)
#pragma unroll
                for (int c = 0; c < CPL; ++c) mb |= mp[(size_t)j * Wl + c];
            const bool need = valid && redf<LP>(mb ? 1.f : 0.f) > 0.f;  // any lane of the patch
            const uint64_t bal = __ballot(need && cg == 0);
            if (lane == 0) sCnt[wave] = __popcll(bal);
            const int n = __syncthreads_count(need && cg == 0);
            if (n == 0) continue;
            int base = 0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) base += w < wave ? sCnt[w] : 0;
            if (need && cg == 0) sList[base + __popcll(bal & ((1ull << lane) - 1ull))] = prow * kPatchesPerItem + slot;
            __syncthreads();
            const int ci = wave * PPW + lane / LP;  // this lane's packed patch
            const int q = sList[ci < n ? ci : 0];
            ky = ky0 + q / kPatchesPerItem;
            kx = kx0 + q % kPatchesPerItem;
            valid = ci < n;
            active = wave * PPW < n;
        }
        const int kxc = min(kx, kx_last), kyc = min(ky, ky_last);
        const int ox = min(kxc * s, Wl - kPatch), oy = min(kyc * s, Hl - kPatch);
        const int x = ox + cg * CPL;  // the lane's first column

        // ---- the reference strip: its loads are issued first and complete
        // while the initial displacement is formed
        const int oyA = min(ky0 * s, Hl - kPatch), oyB = min(ky_last * s, Hl - kPatch);
        const int sh = oyB - oyA + kPatch + 2;
        const int sx0 = min(kx0 * s, Wl - kPatch) - 1;
        const int sw = min(kx_last * s, Wl - kPatch) + kPatch + 1 - sx0;
        stage_rows_lds(sR, I0, Wl, Hl, sx0, oyA - 1, sw, sh, sw);

        // ---- initial displacement: twice the coarser dense flow at the
        // pixel nearest the patch centre, densified there from the coarser
        // level's patch displacements as in the densification
        double u0x = 0.0, u0y = 0.0;
        if (!active) {
            // (a wave with no patch to compute)
        } else if (level == d->L - 1 && d->flow_init) {
            // warm start: the previous pair's level-0 flow at the pixel under
            // the patch centre, in pixels of this level (a power-of-two
            // scale, exact)
            const int W0 = d->W, H0 = d->H;
            const int px = min((ox + kPatch / 2) << level, W0 - 1);
            const int py = min((oy + kPatch / 2) << level, H0 - 1);
            const double sc = 1.0 / (double)(1 << level);
            const size_t q = (size_t)py * W0 + px;
            u0x = (double)d->flow_init[q] * sc;
            u0y = (double)d->flow_init[(size_t)W0 * H0 + q] * sc;
        } else if (level < d->L - 1 && d->ud) {
            // the coarser level's refined dense flow at the pixel nearest the
            // patch centre
            const LevelGeom gc = d->lv[level + 1];
            const int px = min((ox + kPatch / 2) >> 1, gc.w - 1);
            const int py = min((oy + kPatch / 2) >> 1, gc.h - 1);
            const float* Uc = d->ud + 2 * gc.off;
            const size_t q = (size_t)py * gc.w + px;
            u0x = 2.0 * (double)Uc[q];
            u0y = 2.0 * (double)Uc[(size_t)gc.w * gc.h + q];
        } else if (level < d->L - 1) {
            const LevelGeom gc = d->lv[level + 1];
            const float* __restrict__ C0 = d->pyr_prev + gc.off;
            const float* __restrict__ C1 = d->pyr + gc.off;
            const int px = min((ox + kPatch / 2) >> 1, gc.w - 1);
            const int py = min((oy + kPatch / 2) >> 1, gc.h - 1);
            const float inv_s = 1.0f / (float)s;
            const Cover cx = cover_of(px, gc.w, gc.pnx, s, inv_s), cy = cover_of(py, gc.h, gc.pny, s, inv_s);
            float sw_, su, sv;
            // (the densification's weighted mean at the patch centre:) the
            // covering patches shared out over four lane slots (slot q % 4,
            // in order), the slots' sums added as one tree (lanes ^ 1, then
            // ^ 2 within a quad); with 8 lanes per patch lanes 4..7 repeat
            // 0..3, so both lane counts form the same bits
            {
                const float c0v = C0[(size_t)py * gc.w + px];
                const float2* __restrict__ pu = d->puv + gc.poff;
                const int n = cx.n * cy.n;
                sw_ = su = sv = 0.f;
                for (int q = cg & 3; q < n; q += 4) {
                    const int qy = q / cx.n, qx = q - qy * cx.n;
                    const float2 uq = pu[(size_t)cover_index(cy, qy) * gc.pnx + cover_index(cx, qx)];
                    const float w = dens_weight_f(dens_blend(dens_fetch(C1, gc.w, gc.h, px, py, uq.x, uq.y)) - c0v);
                    sw_ += w;
                    su += w * uq.x;
                    sv += w * uq.y;
                }
                sw_ += dppf<0xB1>(sw_);
                su += dppf<0xB1>(su);
                sv += dppf<0xB1>(sv);
                sw_ += dppf<0x4E>(sw_);
                su += dppf<0x4E>(su);
                sv += dppf<0x4E>(sv);
            }
            u0x = 2.0 * (double)(su / sw_);
            u0y = 2.0 * (double)(sv / sw_);
        }

        // ---- template and gradient from the staged reference strip
        lds_load_wait();
        __syncthreads();
        // The residual sum of an iteration, sum_j g_j (I1(x_j + u) - T_j), is
        // split as sum_j g_j I1(x_j + u) - c with c = sum_j g_j T_j fixed for
        // the patch; the first part is formed from the corner sums of u's
        // integer cell (below).  Every sum over the patch is formed per patch
        // column (rows in order), then the columns are added as a binary
        // tree (a lane's two columns first, then the lanes by DPP), so both
        // lane counts give the same bits and the launch shape never changes
        // a result.
        float fgx[CPL][kPatch], fgy[CPL][kPatch];
        double hxx = 1.0, hxy = 0.0, hyy = 1.0;
        float fcx = 0.f, fcy = 0.f;
        if (active) {
            float tf[CPL][kPatch];
            // gradients in single precision (the difference of two floats
            // rounded once: the value a double difference rounded to float
            // would give), the Hessian's sums too (relative error ~1e-6 of
            // sums of order one; the inverse below is formed in double)
            float fxx = 0.f, fxy = 0.f, fyy = 0.f;
            const float* base = sR + (oy - oyA + 1) * sw + (x - sx0);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                float sxx = 0.f, sxy = 0.f, syy = 0.f;
#pragma unroll
                for (int j = 0; j < kPatch; ++j) {
                    const float* q = base + j * sw + c;
                    tf[c][j] = q[0];
                    const float gx = 0.5f * (q[1] - q[-1]);
                    const float gy = 0.5f * (q[sw] - q[-sw]);
                    sxx += gx * gx;
                    sxy += gx * gy;
                    syy += gy * gy;
                    fgx[c][j] = gx;
                    fgy[c][j] = gy;
                }
                fxx = c ? fxx + sxx : sxx;
                fxy = c ? fxy + sxy : sxy;
                fyy = c ? fyy + syy : syy;
            }
            hxx = (double)redf<LP>(fxx);
            hxy = (double)redf<LP>(fxy);
            hyy = (double)redf<LP>(fyy);
            // c by the same single-precision chain, in the same order, as
            // the corner sum SA: at an integer u where I1 equals the template
            // the residual is exactly 0, so a patch that does not move stays
            // exactly in place
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                float cx_ = 0.f, cy_ = 0.f;
#pragma unroll
                for (int j = 0; j < kPatch; ++j) {
                    cx_ += fgx[c][j] * tf[c][j];
                    cy_ += fgy[c][j] * tf[c][j];
                }
                fcx = c ? fcx + cx_ : cx_;
                fcy = c ? fcy + cy_ : cy_;
            }
            fcx = redf<LP>(fcx);
            fcy = redf<LP>(fcy);
        }
        const double ha = hxx + lam, hc = hyy + lam;
        const double det = ha * hc - hxy * hxy;
        const double idet = 1.0 / det;
        // a lane that holds no needed patch (the tail of the last packed
        // wave) keeps its initial displacement: a zero update, and its cell
        // fixed from the start (below), so it never makes its wave form
        // corner sums
        const bool live = !mask_only || valid;
        const float fia = live ? (float)(hc * idet) : 0.f, fib = live ? (float)(-hxy * idet) : 0.f,
                    fic = live ? (float)(ha * idet) : 0.f;

        // ---- stage the search region of I1: the box of the patches'
        // initial windows, reduced over each wave's lanes, then over the
        // waves through LDS
        const double lim = (double)(Wl + Hl + 16);
        int bx0 = INT32_MAX, bx1 = INT32_MIN, by0 = INT32_MAX, by1 = INT32_MIN;
        if (valid) {
            bx0 = bx1 = ox + (int)floor(fmin(fmax(u0x, -lim), lim));
            by0 = by1 = oy + (int)floor(fmin(fmax(u0y, -lim), lim));
        }
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            bx0 = min(bx0, __shfl_xor(bx0, m));
            bx1 = max(bx1, __shfl_xor(bx1, m));
            by0 = min(by0, __shfl_xor(by0, m));
            by1 = max(by1, __shfl_xor(by1, m));
        }
        if (lane == 0) {
            sBox[wave][0] = bx0;
            sBox[wave][1] = bx1;
            sBox[wave][2] = by0;
            sBox[wave][3] = by1;
        }
        __syncthreads();  // also ends the reads of the reference strip
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            bx0 = min(bx0, sBox[w][0]);
            bx1 = max(bx1, sBox[w][1]);
            by0 = min(by0, sBox[w][2]);
            by1 = max(by1, sBox[w][3]);
        }
        const int mg = level == 0 ? kDisMargin0 : kDisMargin;
        const int RX0 = bx0 - mg, RY0 = by0 - mg;
        const int RW = min(bx1 + kPatch + 1 + mg - RX0, kDisRW);
        const int RH = min(by1 + kPatch + 1 + mg - RY0, kDisRH);
        // row-major: every read of an iteration is an immediate offset from
        // one address
        stage_rows_lds(sR, I1, Wl, Hl, RX0, RY0, RW, RH, kDisRP);
        lds_load_wait();
        __syncthreads();

        // ---- inverse-compositional iterations (single precision).  The
        // residual sum is bilinear in the fraction (ax, ay) of u within its
        // integer cell n = floor(u): with the cell's corner sums
        // SA = sum_j g_j I1(x_j + n), SB at n + (1, 0), SC at n + (0, 1),
        // SD at n + (1, 1), it is (SA + ax (SB - SA)) + ay ((SC + ax (SD -
        // SC)) - (SA + ax (SB - SA))) - c, formed as P + ay (Q - P) with
        // P = (SA - c) + ax (SB - SA) and Q = (SC - c) + ax (SD - SC).  The
        // corner sums and their differences depend on the cell only, so a
        // patch forms them when u enters a cell and reuses them while u
        // stays there (the usual case once it converges).
        const float flim = (float)lim;
        float ux = (float)u0x, uy = (float)u0y;
        const int iters = d->iters;
        float S[8] = {};  // SA, SB, SC, SD for the x gradient, then for the y gradient
        float D[4] = {};  // SB - SA, SD - SC (x), then (y): formed with the sums
        int cix = INT32_MIN, ciy = INT32_MIN;
        if (!live) {
            cix = (int)floorf(__builtin_amdgcn_fmed3f(ux, -flim, flim));
            ciy = (int)floorf(__builtin_amdgcn_fmed3f(uy, -flim, flim));
        }
        // (a wave whose patches are all kept skips the iterations)
        for (int it = __ballot(live) ? 0 : iters; it < iters; ++it) {
            // (med3 clamps in one instruction, the same value as min(max()))
            const float sxu = __builtin_amdgcn_fmed3f(ux, -flim, flim), syu = __builtin_amdgcn_fmed3f(uy, -flim, flim);
            const float fx = floorf(sxu), fy = floorf(syu);
            const float ax = sxu - fx, ay = syu - fy;
            const int ix = (int)fx, iy = (int)fy;
            if (ix != cix || iy != ciy) {  // the same for every lane of a patch
                cix = ix;
                ciy = iy;
                float A[kPatch + 1][CPL + 1];  // samples rows 0..8, columns 0..CPL
                const int rx = x + ix - RX0, ry = oy + iy - RY0;
                if ((unsigned)rx < (unsigned)(RW - CPL) && (unsigned)ry < (unsigned)(RH - kPatch)) {
                    const float* q = sR + ry * kDisRP + rx;
#pragma unroll
                    for (int j = 0; j <= kPatch; ++j)
#pragma unroll
                        for (int c = 0; c <= CPL; ++c) A[j][c] = q[j * kDisRP + c];
                } else {
                    // off the staged region: clamped samples from global
                    // memory, all loaded before the first is used
                    int xs[CPL + 1];
#pragma unroll
                    for (int c = 0; c <= CPL; ++c) xs[c] = clampi(x + ix + c, 0, Wl - 1);
#pragma unroll
                    for (int j = 0; j <= kPatch; ++j) {
                        const float* row = I1 + (size_t)clampi(oy + j + iy, 0, Hl - 1) * Wl;
#pragma unroll
                        for (int c = 0; c <= CPL; ++c) A[j][c] = row[xs[c]];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                // per patch column, rows in order; then the columns as one
                // binary tree (a lane's columns, then the lanes)
#pragma unroll
                for (int k = 0; k < 8; ++k) S[k] = 0.f;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    float t[8] = {};
#pragma unroll
                    for (int j = 0; j < kPatch; ++j) {
                        t[0] += fgx[c][j] * A[j][c];
                        t[1] += fgx[c][j] * A[j][c + 1];
                        t[2] += fgx[c][j] * A[j + 1][c];
                        t[3] += fgx[c][j] * A[j + 1][c + 1];
                        t[4] += fgy[c][j] * A[j][c];
                        t[5] += fgy[c][j] * A[j][c + 1];
                        t[6] += fgy[c][j] * A[j + 1][c];
                        t[7] += fgy[c][j] * A[j + 1][c + 1];
                    }
#pragma unroll
                    for (int k = 0; k < 8; ++k) S[k] = c ? S[k] + t[k] : t[k];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) S[k] = redf<LP>(S[k]);
#pragma unroll
                for (int k = 0; k < 4; ++k) D[k] = S[2 * k + 1] - S[2 * k];
                // c taken off the sums at the cell's corners y = 0 and 1 (b
                // is still exactly 0 where I1 equals the template at an
                // integer u)
                S[0] -= fcx;
                S[2] -= fcx;
                S[4] -= fcy;
                S[6] -= fcy;
            }
            const float px_ = S[0] + ax * D[0], qx_ = S[2] + ax * D[1];
            const float py_ = S[4] + ax * D[2], qy_ = S[6] + ax * D[3];
            const float bx = px_ + ay * (qx_ - px_);
            const float by = py_ + ay * (qy_ - py_);
            ux = fmaf(-fib, by, fmaf(-fia, bx, ux));
            uy = fmaf(-fic, by, fmaf(-fib, bx, uy));
        }
        // outlier reset: back to the initial displacement when the patch
        // moved more than its size
        double rux = ux, ruy = uy;
        const double mx = rux - u0x, my = ruy - u0y;
        if (sqrt(mx * mx + my * my) > (double)kPatch) {
            rux = u0x;
            ruy = u0y;
        }
        // (exact in float: u is a float, and u0 twice a float quotient)
        if (valid && cg == 0) d->puv[g.poff + (size_t)ky * pnx + kx] = make_float2((float)rux, (float)ruy);
        __syncthreads();  // the next item restages sR
    }
}

// --------------------------------------------------------------------------
// Densification at level 0: the flow of a pixel is the mean of the covering
// patches' displacements weighted by 1 / max(1, 255 |I1(x+u) - I0(x)|)
// (single precision: a weight's relative error of a few ulp moves the mean
// by that fraction of the spread of the displacements); optionally zero
// outside the reference window's edge pixels.
// --------------------------------------------------------------------------
template <bool B, int TW>
__global__ __launch_bounds__(kBlock) void k_densify(const WinDesc one, const BatchArgs ba, int32_t total_arg) {
    constexpr int TH = kBlock / TW;  // tile TW x TH pixels, one per thread
    const int32_t total = item_total<B>(ba, total_arg);
    for (int32_t item = xcd_item(blockIdx.x, gridDim.x); item < total; item += gridDim.x) {
        int32_t local;
        const WinDesc* d = locate<B>(one, ba, item, local);
        const LevelGeom g = d->lv[0];
        const int W = g.w, H = g.h;
        const int tiles_x = (W + TW - 1) / TW;
        const int x = (local % tiles_x) * TW + (int)(threadIdx.x % TW);
        const int y = (local / tiles_x) * TH + (int)(threadIdx.x / TW);
        if (x >= W || y >= H) continue;
        const size_t pix = (size_t)y * W + x;
        if (d->zero_out) {  // first window of a served stream: no flow yet
            d->flow[pix] = 0.f;
            d->flow[(size_t)W * H + pix] = 0.f;
            if (d->mask_out) d->mask_out[pix] = 0;
            continue;
        }
        // a pixel off the mask gets 0 without its sums, unless the flow
        // before masking is wanted too
        const uint8_t m = d->mask ? d->mask[pix] : 1;
        const bool off = (d->flags & EBOF_MASK_FLOW) && !m;
        if (off && !d->flow_keep) {
            d->flow[pix] = 0.f;
            d->flow[(size_t)W * H + pix] = 0.f;
            if (d->mask_out) d->mask_out[pix] = m;
            continue;
        }
        const int s = d->stride;
        const float* __restrict__ I0 = d->pyr_prev;
        const float* __restrict__ I1 = d->pyr;
        const float2* __restrict__ pu = d->puv + g.poff;
        const float inv_s = 1.0f / (float)s;
        const Cover cx = cover_of(x, W, g.pnx, s, inv_s), cy = cover_of(y, H, g.pny, s, inv_s);
        const float i0 = I0[pix];
        float sw, su, sv;
        dens_sums(I1, W, H, x, y, i0, pu, g.pnx, cx, cy, sw, su, sv);
        float fu = su / sw, fv = sv / sw;
        if (d->flow_keep) {
            d->flow_keep[pix] = fu;
            d->flow_keep[(size_t)W * H + pix] = fv;
        }
        if (off) fu = fv = 0.f;
        d->flow[pix] = fu;
        d->flow[(size_t)W * H + pix] = fv;
        if (d->mask_out) d->mask_out[pix] = m;
    }
}

// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------
// Every launch goes through here; with timing events attached they are
// recorded on the stream right before and right after the kernel.
template <typename K, typename... Args>
static void klaunch(const Launch& L, K kernel, int block, Args... args) {
    if (L.ev_start) (void)hipEventRecord(L.ev_start, L.stream);
    hipLaunchKernelGGL(kernel, dim3(L.grid), dim3(block), 0, L.stream, args...);
    if (L.ev_stop) (void)hipEventRecord(L.ev_stop, L.stream);
}
#define EBOF_LAUNCH(KERNEL, L, ...)                                                        \
    do {                                                                                   \
        if ((L).batch)                                                                     \
            klaunch((L), KERNEL<true>, kBlock, *(L).one, (L).ba, (L).total, ##__VA_ARGS__);  \
        else                                                                               \
            klaunch((L), KERNEL<false>, kBlock, *(L).one, (L).ba, (L).total, ##__VA_ARGS__); \
    } while (0)

void launch_zero(const Launch& L) { EBOF_LAUNCH(k_zero, L); }
void launch_scatter(const Launch& L) { EBOF_LAUNCH(k_scatter, L); }
void launch_denoise_fill(const Launch& L, bool pack) {
    if (pack) {
        if (L.batch)
            klaunch(L, k_denoise_fill<true, true>, kBlock, *L.one, L.ba, L.total);
        else
            klaunch(L, k_denoise_fill<false, true>, kBlock, *L.one, L.ba, L.total);
    } else {
        if (L.batch)
            klaunch(L, k_denoise_fill<true, false>, kBlock, *L.one, L.ba, L.total);
        else
            klaunch(L, k_denoise_fill<false, false>, kBlock, *L.one, L.ba, L.total);
    }
}
void launch_pack_cols(const Launch& L) { EBOF_LAUNCH(k_pack_cols, L); }
void launch_edt_cols(const Launch& L) { EBOF_LAUNCH(k_edt_cols, L); }
#define EBOF_LAUNCH_T(KERNEL, T, L)                                               \
    do {                                                                          \
        if ((L).batch)                                                            \
            klaunch((L), KERNEL<true, T>, kBlock, *(L).one, (L).ba, (L).total);   \
        else                                                                      \
            klaunch((L), KERNEL<false, T>, kBlock, *(L).one, (L).ba, (L).total);  \
    } while (0)

void launch_edt_rows(const Launch& L, int rows_nr) {
    switch (rows_nr) {
        case 1: EBOF_LAUNCH_T(k_edt_rows, 1, L); break;
        case 2: EBOF_LAUNCH_T(k_edt_rows, 2, L); break;
        case 8: EBOF_LAUNCH_T(k_edt_rows, 8, L); break;
        default: EBOF_LAUNCH_T(k_edt_rows, 4, L); break;
    }
}
void launch_pyr_chain(const Launch& L, int from) {
    if (L.batch)
        klaunch(L, k_pyr_chain<true>, kPyrBlock, *L.one, L.ba, L.total, from);
    else
        klaunch(L, k_pyr_chain<false>, kPyrBlock, *L.one, L.ba, L.total, from);
}
void launch_dis_level(const Launch& L, int level, int lanes) {
    if (lanes == 4) {
        if (L.batch)
            klaunch(L, k_dis_level<true, 4>, kBlock, *L.one, L.ba, L.total, level);
        else
            klaunch(L, k_dis_level<false, 4>, kBlock, *L.one, L.ba, L.total, level);
    } else {
        if (L.batch)
            klaunch(L, k_dis_level<true, 8>, kBlock, *L.one, L.ba, L.total, level);
        else
            klaunch(L, k_dis_level<false, 8>, kBlock, *L.one, L.ba, L.total, level);
    }
}
void launch_densify(const Launch& L, int tile_w) {
    switch (tile_w) {
        case 16: EBOF_LAUNCH_T(k_densify, 16, L); break;
        case 128: EBOF_LAUNCH_T(k_densify, 128, L); break;
        case 256: EBOF_LAUNCH_T(k_densify, 256, L); break;
        default: EBOF_LAUNCH_T(k_densify, 64, L); break;
    }
}

// --------------------------------------------------------------------------
// the fixed scratch array's device address, per device
// --------------------------------------------------------------------------
int noalloc_scratch(float2** out) {
    static std::mutex mu;
    static float2* addr[kNoAllocMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(e));
        return EBOF_E_DEVICE;
    }
    if (dev < 0 || dev >= kNoAllocMaxDevices) {
        set_error("device %d out of range for the fixed scratch", dev);
        return EBOF_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return EBOF_E_DEVICE;
        }
        addr[dev] = (float2*)p;
    }
    *out = addr[dev];
    return EBOF_OK;
}

// --------------------------------------------------------------------------
// per-window work items of each stage
// --------------------------------------------------------------------------
int32_t stage_items(const WinDesc& d, int stage, bool has_flow, bool zero, const Tune& t) {
    const int64_t N = (int64_t)d.W * d.H;
    const int bands = (d.W + 63) / 64, nch = (d.H + kChunk - 1) / kChunk;
    if (stage == kStZero) return zero ? (int32_t)((N + kZeroBytesPerItem - 1) / kZeroBytesPerItem) : 0;
    if (stage == kStScatter) return (int32_t)((d.n_ev + kEventsPerItem - 1) / kEventsPerItem);
    if (stage == kStDenoise) return ((d.W + kTile - 1) / kTile) * ((d.H + kTileH - 1) / kTileH);
    if (stage == kStPack) return bands * nch;
    if (stage == kStCols) return edt_local(d) ? 0 : bands * nch;
    if (stage == kStRows) return ((d.H + t.rows_nr - 1) / t.rows_nr) * ((d.W + kRowSeg - 1) / kRowSeg);
    if (stage >= kStPyr && stage < kStPyr + kMaxLevels - 1) {
        const int from = (stage - kStPyr) * kPyrChain;
        if (from >= d.L - 1) return 0;
        const LevelGeom& g = d.lv[from + std::min(kPyrChain, d.L - 1 - from)];
        return ((g.w + kPyrTile - 1) / kPyrTile) * ((g.h + kPyrTile - 1) / kPyrTile);
    }
    if (stage >= kStDis && stage < kStDis + kMaxLevels) {
        const int l = stage - kStDis;
        if (!has_flow || l >= d.L) return 0;
        const LevelGeom& g = d.lv[l];
        const int pr = kBlock / kPatchesPerItem / t.dis_lanes[l];  // patch rows per item
        return ((g.pny + pr - 1) / pr) * ((g.pnx + kPatchesPerItem - 1) / kPatchesPerItem);
    }
    if (stage == kStDensify)
        return (has_flow || d.zero_out)
                   ? ((d.W + t.dens_tw - 1) / t.dens_tw) * ((d.H + kBlock / t.dens_tw - 1) / (kBlock / t.dens_tw))
                   : 0;
    return 0;
}

}  // namespace ebof

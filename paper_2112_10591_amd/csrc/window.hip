// window.hip -- adaptive windows (the adaptive accumulation time the
// Conclusion proposes, with the area event count as the rule): where a window
// of a time-ordered event stream ends.  The sensor is tiled by squares of
// `area` pixels; scanning from event i0, every on-sensor event counts for its
// square, and the window ends right after the event that brings some square to
// k_events.  Three passes over chunks of the stream: per-chunk square
// histograms; per square, the chunk where its count reaches k_events and the
// rank of that event inside the chunk; in the earliest such chunk, the exact
// event (a block scan per candidate square).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ctx.h"

namespace ebof {

constexpr int kWinBlock = 256;
constexpr int kWinMaxChunks = 1024;
constexpr int kWinMinChunk = 4096;
constexpr int kWinMaxAreas = 8192;

__global__ __launch_bounds__(kWinBlock) void k_area_hist(const uint16_t* __restrict__ x,
                                                         const uint16_t* __restrict__ y, int64_t n, int64_t i0,
                                                         int64_t S, int W, int H, int area, int ax, int M,
                                                         uint32_t* __restrict__ hist, uint32_t* __restrict__ cmin) {
    extern __shared__ uint32_t cnt[];
    if (blockIdx.x == 0 && threadIdx.x == 0) *cmin = 0xffffffffu;  // for the next pass
    for (int m = threadIdx.x; m < M; m += kWinBlock) cnt[m] = 0;
    __syncthreads();
    const int64_t b = i0 + (int64_t)blockIdx.x * S, e = min(n, b + S);
    for (int64_t i = b + threadIdx.x; i < e; i += kWinBlock) {
        const int xe = x[i], ye = y[i];
        if (xe < W && ye < H) atomicAdd(&cnt[(ye / area) * ax + xe / area], 1u);
    }
    __syncthreads();
    uint32_t* h = hist + (size_t)blockIdx.x * M;
    for (int m = threadIdx.x; m < M; m += kWinBlock) h[m] = cnt[m];
}

// per square: first chunk where the running count reaches k (C when none)
// and the rank (1-based) of that event among the square's events in it
__global__ __launch_bounds__(kWinBlock) void k_area_first(const uint32_t* __restrict__ hist, int C, int M,
                                                          int k, uint32_t* __restrict__ first,
                                                          uint32_t* __restrict__ rank, uint32_t* __restrict__ cmin) {
    const int m = blockIdx.x * kWinBlock + threadIdx.x;
    if (m >= M) return;
    uint32_t cum = 0;
    int c = 0;
    uint32_t r = 0;
    for (; c < C; ++c) {
        const uint32_t h = hist[(size_t)c * M + m];
        if (cum + h >= (uint32_t)k) {
            r = (uint32_t)k - cum;
            break;
        }
        cum += h;
    }
    first[m] = (uint32_t)c;
    rank[m] = r;
    if (c < C) atomicMin(cmin, (uint32_t)c);
}

__global__ __launch_bounds__(kWinBlock) void k_area_locate(const uint16_t* __restrict__ x,
                                                           const uint16_t* __restrict__ y, int64_t n, int64_t i0,
                                                           int64_t S, int W, int H, int area, int ax, int M, int C,
                                                           const uint32_t* __restrict__ first,
                                                           const uint32_t* __restrict__ rank,
                                                           const uint32_t* __restrict__ cmin,
                                                           int64_t* __restrict__ range) {
    __shared__ uint32_t s_pre[kWinBlock];
    __shared__ int s_cand[kWinMaxAreas];
    __shared__ int s_nc;
    __shared__ int64_t s_best;
    const uint32_t c = C > 0 ? *cmin : 0xffffffffu;
    if (c >= (uint32_t)C) {  // no square reaches k: the window takes every event
        if (threadIdx.x == 0) {
            range[0] = i0;
            range[1] = n;
        }
        return;
    }
    // the squares that reach k in chunk c (their order does not matter: the
    // end is the earliest of their k-th events)
    if (threadIdx.x == 0) {
        s_nc = 0;
        s_best = INT64_MAX;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += kWinBlock)
        if (first[m] == c) s_cand[atomicAdd(&s_nc, 1)] = m;
    __syncthreads();
    const int nc = s_nc;
    const int64_t b = i0 + (int64_t)c * S, e = min(n, b + S);
    const int64_t per = (e - b + kWinBlock - 1) / kWinBlock;
    const int64_t lo = min(e, b + threadIdx.x * per), hi = min(e, lo + per);
    for (int q = 0; q < nc; ++q) {
        const int m0 = s_cand[q];
        const uint32_t r = rank[m0];
        uint32_t mine = 0;
        for (int64_t i = lo; i < hi; ++i) {
            const int xe = x[i], ye = y[i];
            if (xe < W && ye < H && (ye / area) * ax + xe / area == m0) ++mine;
        }
        // exclusive prefix over the threads, in thread order
        s_pre[threadIdx.x] = mine;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (int t = 0; t < kWinBlock; ++t) {
                const uint32_t v = s_pre[t];
                s_pre[t] = run;
                run += v;
            }
        }
        __syncthreads();
        const uint32_t before = s_pre[threadIdx.x];
        if (before < r && r <= before + mine) {  // one thread: the one holding the r-th event
            uint32_t seen = before;
            for (int64_t i = lo; i < hi; ++i) {
                const int xe = x[i], ye = y[i];
                if (xe < W && ye < H && (ye / area) * ax + xe / area == m0 && ++seen == r) {
                    if (i + 1 < s_best) s_best = i + 1;
                    break;
                }
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        range[0] = i0;
        range[1] = s_best;
    }
}

}  // namespace ebof

using namespace ebof;

extern "C" {

int ebof_window_end(ebof_ctx* ctx, int32_t width, int32_t height, const uint16_t* x, const uint16_t* y, int64_t n,
                    int64_t i0, int32_t area, int32_t k_events, int64_t* range_dev, void* hip_stream) {
    if (!ctx || !range_dev || width < 1 || height < 1 || width > EBOF_MAX_DIM || height > EBOF_MAX_DIM ||
        area < 1 || k_events < 1 || i0 < 0 || n < i0 || (n > i0 && (!x || !y))) {
        set_error("ebof_window_end: bad arguments");
        return EBOF_E_INVAL;
    }
    if (ctx->failed) return EBOF_E_DEVICE;
    const int ax = (width + area - 1) / area, ay = (height + area - 1) / area;
    const int64_t M = (int64_t)ax * ay;
    if (M > kWinMaxAreas) {
        set_error("ebof_window_end: %lld squares of %d px exceed %d", (long long)M, area, kWinMaxAreas);
        return EBOF_E_INVAL;
    }
    const int64_t events = n - i0;
    const int64_t S = std::max<int64_t>(kWinMinChunk, (events + kWinMaxChunks - 1) / kWinMaxChunks);
    const int C = (int)((events + S - 1) / S);
    hipStream_t st = (hipStream_t)hip_stream;
    uint32_t* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->window_scratch.find((uintptr_t)st);
        if (it == ctx->window_scratch.end()) {
            const size_t bytes = ((size_t)kWinMaxChunks * kWinMaxAreas + 2 * (size_t)kWinMaxAreas + 64) * 4;
            void* p = ctx->arena.alloc(bytes);
            if (!p) {
                set_error("arena full: window-end scratch of %zu bytes", bytes);
                return EBOF_E_NOMEM;
            }
            it = ctx->window_scratch.emplace((uintptr_t)st, p).first;
        }
        base = (uint32_t*)it->second;
    }
    uint32_t* hist = base;
    uint32_t* first = hist + (size_t)kWinMaxChunks * kWinMaxAreas;
    uint32_t* rank = first + kWinMaxAreas;
    uint32_t* cmin = rank + kWinMaxAreas;
    if (C > 0) {
        hipLaunchKernelGGL(k_area_hist, dim3(C), dim3(kWinBlock), (size_t)M * 4, st, x, y, n, i0, S, (int)width,
                           (int)height, (int)area, ax, (int)M, hist, cmin);
        hipLaunchKernelGGL(k_area_first, dim3((unsigned)((M + kWinBlock - 1) / kWinBlock)), dim3(kWinBlock), 0, st,
                           (const uint32_t*)hist, C, (int)M, (int)k_events, first, rank, cmin);
    }
    hipLaunchKernelGGL(k_area_locate, dim3(1), dim3(kWinBlock), 0, st, x, y, n, i0, S, (int)width, (int)height,
                       (int)area, ax, (int)M, C, (const uint32_t*)first, (const uint32_t*)rank,
                       (const uint32_t*)cmin, range_dev);
    return check_hip(ctx, hipGetLastError(), "kernel launch");
}

}  // extern "C"

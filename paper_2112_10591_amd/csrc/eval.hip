// eval.hip -- the evaluation kit of Sec. IV on the GPU: endpoint errors of a
// flow against a ground truth (average endpoint error, outlier rate) and the
// flow warp loss of one window's events.  Reductions are two-pass with
// per-block partial sums added in a fixed order, so results do not depend on
// scheduling.  The per-pixel and per-event arithmetic is double precision
// without contraction, as the definitions are written.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "ctx.h"

namespace ebof {

constexpr int kEvalBlock = 256;
constexpr int kEvalParts = 1024;             // blocks (partial sums) per reduction
constexpr double kVoteScale = 4294967296.0;  // fixed-point votes: 2^-32 px units

struct ErrPart {
    double sum;
    unsigned long long cnt, out;
};

// sum over the block in a fixed order: each wave by shuffles, then the waves
template <class T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    T s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kEvalBlock / 64; ++i) s += sh[i];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(kEvalBlock) void k_flow_err(const float* __restrict__ u, const float* __restrict__ v,
                                                         const uint8_t* __restrict__ mask, int64_t n,
                                                         ErrPart* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double shd[kEvalBlock / 64];
    __shared__ unsigned long long shc[kEvalBlock / 64];
    double s = 0.0;
    unsigned long long c = 0, o = 0;
    for (int64_t i = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kEvalBlock) {
        if (mask && !mask[i]) continue;
        const double vx = v[i], vy = v[n + i];
        const double ex = vx - (double)u[i], ey = vy - (double)u[n + i];
        const double e = sqrt(ex * ex + ey * ey);
        const double m = sqrt(vx * vx + vy * vy);
        s += e;
        ++c;
        if (e > 3.0 && e > 0.05 * m) ++o;
    }
    s = block_sum(s, shd);
    c = block_sum(c, shc);
    o = block_sum(o, shc);
    if (threadIdx.x == 0) part[blockIdx.x] = ErrPart{s, c, o};
}

__global__ __launch_bounds__(kEvalBlock) void k_flow_err_final(const ErrPart* __restrict__ part, int nparts,
                                                               double* __restrict__ out) {
    __shared__ double shd[kEvalBlock / 64];
    __shared__ unsigned long long shc[kEvalBlock / 64];
    double s = 0.0;
    unsigned long long c = 0, o = 0;
    for (int i = threadIdx.x; i < nparts; i += kEvalBlock) {
        s += part[i].sum;
        c += part[i].cnt;
        o += part[i].out;
    }
    s = block_sum(s, shd);
    c = block_sum(c, shc);
    o = block_sum(o, shc);
    if (threadIdx.x == 0) {
        out[0] = c ? s / (double)c : 0.0;
        out[1] = c ? (double)o / (double)c : 0.0;
        out[2] = (double)c;
    }
}

__global__ __launch_bounds__(kEvalBlock) void k_fill64(long long* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kEvalBlock)
        p[i] = 0;
}

// Votes of one window's events: at their own pixel (uncompensated) and, moved
// back to the window start by the flow at their pixel, bilinearly into the
// four pixels around the moved position (compensated).  Votes are fixed
// point (2^-32) so that their sums do not depend on the order of the atomics.
__global__ __launch_bounds__(kEvalBlock) void k_fwl_vote(int W, int H, const uint16_t* __restrict__ x,
                                                         const uint16_t* __restrict__ y,
                                                         const int64_t* __restrict__ t,
                                                         const int8_t* __restrict__ pol, int64_t n, int64_t t0,
                                                         int64_t dt, const float* __restrict__ flow,
                                                         long long* __restrict__ Ic, long long* __restrict__ Iu) {
#pragma clang fp contract(off)
    const int64_t N = (int64_t)W * H;
    for (int64_t e = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kEvalBlock) {
        const int64_t te = t[e];
        const int xe = x[e], ye = y[e];
        if (te < t0 || te >= t0 + dt || xe >= W || ye >= H) continue;
        const double w = pol ? (pol[e] < 0 ? -1.0 : 1.0) : 1.0;
        const int64_t p = (int64_t)ye * W + xe;
        atomicAdd((unsigned long long*)&Iu[p], (unsigned long long)(long long)llrint(w * kVoteScale));
        const double tau = (double)(te - t0) / (double)dt;
        const double sx = (double)xe - (double)flow[p] * tau, sy = (double)ye - (double)flow[N + p] * tau;
        const double fx = floor(sx), fy = floor(sy);
        const double ax = sx - fx, ay = sy - fy;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const double X = fx + i, Y = fy + j;
                if (X < 0.0 || X >= (double)W || Y < 0.0 || Y >= (double)H) continue;
                const double b = (i ? ax : 1.0 - ax) * (j ? ay : 1.0 - ay);
                const long long q = llrint(w * b * kVoteScale);
                if (q) atomicAdd((unsigned long long*)&Ic[(int64_t)Y * W + (int64_t)X], (unsigned long long)q);
            }
    }
}

// pass 1: sums of both images; pass 2 (mean given): sums of squared deviations
__global__ __launch_bounds__(kEvalBlock) void k_img_moments(const long long* __restrict__ Ic,
                                                            const long long* __restrict__ Iu, int64_t N,
                                                            const double* __restrict__ mean, double* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double shd[kEvalBlock / 64];
    const double mc = mean ? mean[0] : 0.0, mu = mean ? mean[1] : 0.0;
    double sc = 0.0, su = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kEvalBlock) {
        const double a = (double)Ic[i] / kVoteScale, b = (double)Iu[i] / kVoteScale;
        if (mean) {
            sc += (a - mc) * (a - mc);
            su += (b - mu) * (b - mu);
        } else {
            sc += a;
            su += b;
        }
    }
    sc = block_sum(sc, shd);
    su = block_sum(su, shd);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sc;
        part[2 * blockIdx.x + 1] = su;
    }
}

// adds the partials in a fixed order; stage 0: the means into out[0..1];
// stage 1: the variances and their ratio into res[0..2] (fwl, comp, uncomp)
__global__ __launch_bounds__(kEvalBlock) void k_img_final(const double* __restrict__ part, int nparts, int64_t N,
                                                          int stage, double* __restrict__ mean,
                                                          double* __restrict__ res) {
    __shared__ double shd[kEvalBlock / 64];
    double sc = 0.0, su = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kEvalBlock) {
        sc += part[2 * i];
        su += part[2 * i + 1];
    }
    sc = block_sum(sc, shd);
    su = block_sum(su, shd);
    if (threadIdx.x == 0) {
        const double vc = sc / (double)N, vu = su / (double)N;
        if (stage == 0) {
            mean[0] = vc;
            mean[1] = vu;
        } else {
            res[0] = vu > 0.0 ? vc / vu : 0.0;
            res[1] = vc;
            res[2] = vu;
        }
    }
}

static int grid_for(int64_t n) {
    const int64_t b = (n + kEvalBlock - 1) / kEvalBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kEvalParts));
}

// per-(size, stream) scratch of the evaluation calls, in the arena
static int eval_scratch(ebof_ctx* ctx, int64_t N, hipStream_t st, EvalScratch** out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto key = std::make_pair(N, (uintptr_t)st);
    auto it = ctx->eval_scratch.find(key);
    if (it != ctx->eval_scratch.end()) {
        *out = &it->second;
        return EBOF_OK;
    }
    EvalScratch s;
    s.img = (long long*)ctx->arena.alloc((size_t)N * 16);
    s.part = (char*)ctx->arena.alloc(kEvalParts * sizeof(ErrPart) + 256);
    if (!s.img || !s.part) {
        ctx->arena.free(s.img);
        ctx->arena.free(s.part);
        set_error("arena full: evaluation scratch of %lld bytes", (long long)(N * 16));
        return EBOF_E_NOMEM;
    }
    *out = &(ctx->eval_scratch[key] = s);
    return EBOF_OK;
}

}  // namespace ebof

using namespace ebof;

extern "C" {

int ebof_flow_errors(ebof_ctx* ctx, int32_t width, int32_t height, const float* flow, const float* gt,
                     const uint8_t* mask, double* out_dev, void* hip_stream) {
    if (!ctx || !flow || !gt || !out_dev || width < 1 || height < 1 || width > EBOF_MAX_DIM ||
        height > EBOF_MAX_DIM) {
        set_error("ebof_flow_errors: NULL buffer or size out of range");
        return EBOF_E_INVAL;
    }
    if (ctx->failed) return EBOF_E_DEVICE;
    const int64_t N = (int64_t)width * height;
    hipStream_t st = (hipStream_t)hip_stream;
    EvalScratch* s;
    int rc = eval_scratch(ctx, N, st, &s);
    if (rc) return rc;
    const int g = grid_for(N);
    ErrPart* part = (ErrPart*)s->part;
    hipLaunchKernelGGL(k_flow_err, dim3(g), dim3(kEvalBlock), 0, st, flow, gt, mask, N, part);
    hipLaunchKernelGGL(k_flow_err_final, dim3(1), dim3(kEvalBlock), 0, st, part, g, out_dev);
    return check_hip(ctx, hipGetLastError(), "kernel launch");
}

int ebof_fwl(ebof_ctx* ctx, const ebof_params* p, const uint16_t* x, const uint16_t* y, const int64_t* t,
             const int8_t* pol, int64_t n, int64_t t0_us, const float* flow, double* out_dev, void* hip_stream) {
    if (!ctx || !flow || !out_dev || n < 0 || (n > 0 && (!x || !y || !t))) {
        set_error("ebof_fwl: NULL buffer or negative n");
        return EBOF_E_INVAL;
    }
    if (ctx->failed) return EBOF_E_DEVICE;
    int rc = validate_params(p);
    if (rc) return rc;
    if (t0_us > INT64_MAX - p->dt_us) {
        set_error("ebof_fwl: t0 + dt overflows");
        return EBOF_E_INVAL;
    }
    const int64_t N = (int64_t)p->width * p->height;
    hipStream_t st = (hipStream_t)hip_stream;
    EvalScratch* s;
    if ((rc = eval_scratch(ctx, N, st, &s))) return rc;
    long long* Ic = s->img;
    long long* Iu = s->img + N;
    double* part = (double*)s->part;
    double* mean = part + 2 * kEvalParts;
    hipLaunchKernelGGL(k_fill64, dim3(grid_for(2 * N)), dim3(kEvalBlock), 0, st, s->img, 2 * N);
    if (n > 0)
        hipLaunchKernelGGL(k_fwl_vote, dim3(grid_for(n)), dim3(kEvalBlock), 0, st, p->width, p->height, x, y, t, pol,
                           n, t0_us, p->dt_us, flow, Ic, Iu);
    const int g = grid_for(N);
    hipLaunchKernelGGL(k_img_moments, dim3(g), dim3(kEvalBlock), 0, st, Ic, Iu, N, (const double*)nullptr, part);
    hipLaunchKernelGGL(k_img_final, dim3(1), dim3(kEvalBlock), 0, st, part, g, N, 0, mean, out_dev);
    hipLaunchKernelGGL(k_img_moments, dim3(g), dim3(kEvalBlock), 0, st, Ic, Iu, N, (const double*)mean, part);
    hipLaunchKernelGGL(k_img_final, dim3(1), dim3(kEvalBlock), 0, st, part, g, N, 1, mean, out_dev);
    return check_hip(ctx, hipGetLastError(), "kernel launch");
}

}  // extern "C"

// filter.hip -- the update-prediction flow filter: the kind of flow block
// Sec. III-D selects (a predictive filter that carries the flow from one
// window to the next and refines it per pyramid layer, each layer with its
// own regularisation weight and smoothing iterations, Sec. IV-A).  The
// reading the library implements is stated with ebof_flow_filter in ebof.h.
//
// Per layer, coarse to fine: one pass forms the prediction (the layer's
// previous flow gathered at x - U(x), plus the coarser layer's innovation at
// the parent pixel) and the regularised brightness-constancy update, one
// thread per pixel; then the Jacobi smoothing runs kFfSteps iterations per
// launch on 32x32 tiles held in LDS with a halo of kFfSteps pixels (each
// launch recomputes the halo, so the tile's centre is exact after its
// iterations); the last launch of a layer writes the new state, the
// innovation and, at layer 0, the output flow.  Single precision.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "ctx.h"

namespace ebof {

constexpr int kFfBlock = 256;
constexpr int kFfTile = 32;                      // smoothing: output tile edge
constexpr int kFfSteps = 8;                      // smoothing: iterations per launch (= halo)
constexpr int kFfEdge = kFfTile + 2 * kFfSteps;  // smoothing: tile edge with its halo
constexpr int kFfCells = kFfEdge * kFfEdge / kFfBlock;  // smoothing: cells per thread
constexpr int kFfMaxSmooth = 1000;

__device__ __forceinline__ int ff_clamp(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ float ff_at(const float* __restrict__ I, int W, int H, int x, int y) {
    return I[(size_t)ff_clamp(y, 0, H - 1) * W + ff_clamp(x, 0, W - 1)];
}

// bilinear sample at (sx, sy), replicated border; the integer part is
// limited first (any index beyond the border reads the border), which also
// keeps a non-finite position's indices in range
__device__ __forceinline__ float ff_bilinear(const float* __restrict__ I, int W, int H, float sx, float sy) {
    float fx = floorf(sx), fy = floorf(sy);
    const float ax = sx - fx, ay = sy - fy;
    fx = fminf(fmaxf(fx, -2.0f), (float)W + 2.0f);
    fy = fminf(fmaxf(fy, -2.0f), (float)H + 2.0f);
    const int x0 = (int)fx, y0 = (int)fy;
    const float i00 = ff_at(I, W, H, x0, y0), i10 = ff_at(I, W, H, x0 + 1, y0);
    const float i01 = ff_at(I, W, H, x0, y0 + 1), i11 = ff_at(I, W, H, x0 + 1, y0 + 1);
    return (1.0f - ay) * ((1.0f - ax) * i00 + ax * i10) + ay * ((1.0f - ax) * i01 + ax * i11);
}

// Prediction and update of one layer (w x h).  U: the layer's previous flow
// (two planes); Dc: the coarser layer's innovation (wc x hc, two planes) or
// NULL at the top layer.  Writes the updated flow to A and the prediction to
// Q (two planes each).
__global__ __launch_bounds__(kFfBlock) void k_ff_update(const float* __restrict__ I0, const float* __restrict__ I1,
                                                        const float* __restrict__ U, const float* __restrict__ Dc,
                                                        int w, int h, int wc, int hc, float gamma,
                                                        float* __restrict__ A, float* __restrict__ Q) {
    const int64_t N = (int64_t)w * h;
    const int64_t i = (int64_t)blockIdx.x * kFfBlock + threadIdx.x;
    if (i >= N) return;
    const int y = (int)(i / w), x = (int)(i - (int64_t)y * w);
    const float sx = (float)x - U[i], sy = (float)y - U[N + i];
    float pu = ff_bilinear(U, w, h, sx, sy);
    float pv = ff_bilinear(U + N, w, h, sx, sy);
    if (Dc) {
        const int64_t Nc = (int64_t)wc * hc;
        const int64_t q = (int64_t)min(y / 2, hc - 1) * wc + min(x / 2, wc - 1);
        pu += 2.0f * Dc[q];
        pv += 2.0f * Dc[Nc + q];
    }
    const float gx = 127.5f * (ff_at(I0, w, h, x + 1, y) - ff_at(I0, w, h, x - 1, y));
    const float gy = 127.5f * (ff_at(I0, w, h, x, y + 1) - ff_at(I0, w, h, x, y - 1));
    const float r = 255.0f * (ff_bilinear(I1, w, h, (float)x + pu, (float)y + pv) - I0[i]);
    const float k = r / (gx * gx + gy * gy + gamma);
    A[i] = pu - gx * k;
    A[N + i] = pv - gy * k;
    Q[i] = pu;
    Q[N + i] = pv;
}

// `iters` (<= kFfSteps) Jacobi iterations of the five-point mean on both
// planes of src (w x h), one 32x32 output tile per block.  Not finishing:
// the result goes to dst.  Finishing (dst NULL): the result is the layer's
// new flow, written to U, with the innovation (result - Q) to D and, when
// flow is not NULL, the output flow (zero where mask is given and 0).
__global__ __launch_bounds__(kFfBlock) void k_ff_smooth(const float* __restrict__ src, int w, int h, int iters,
                                                        float* __restrict__ dst, const float* __restrict__ Q,
                                                        float* __restrict__ U, float* __restrict__ D,
                                                        float* __restrict__ flow, const uint8_t* __restrict__ mask) {
    __shared__ float buf[2][2][kFfEdge * kFfEdge];
    const int64_t N = (int64_t)w * h;
    const int tilesx = (w + kFfTile - 1) / kFfTile;
    const int X0 = (int)(blockIdx.x % tilesx) * kFfTile - kFfSteps;
    const int Y0 = (int)(blockIdx.x / tilesx) * kFfTile - kFfSteps;
    for (int idx = threadIdx.x; idx < kFfEdge * kFfEdge; idx += kFfBlock) {
        const int gx = X0 + idx % kFfEdge, gy = Y0 + idx / kFfEdge;
        const bool in = gx >= 0 && gx < w && gy >= 0 && gy < h;
        const int64_t g = (int64_t)gy * w + gx;
        buf[0][0][idx] = in ? src[g] : 0.0f;
        buf[0][1][idx] = in ? src[N + g] : 0.0f;
    }
    __syncthreads();
    // Each thread owns kFfCells cells of the tile.  A cell's neighbour is the
    // pixel's own index clamped into the image (the replicated border), then
    // into the tile (cells that reach past the tile are in the halo and
    // their values are not used at the end): one bit per side says whether
    // the neighbour is a different cell, one whether the cell is on the image.
    static_assert(kFfEdge * kFfEdge == kFfCells * kFfBlock, "the tile's cells are spread evenly");
    int side[kFfCells];
#pragma unroll
    for (int k = 0; k < kFfCells; ++k) {
        const int idx = threadIdx.x + k * kFfBlock;
        const int lx = idx % kFfEdge, ly = idx / kFfEdge;
        const int gx = X0 + lx, gy = Y0 + ly;
        const bool in = gx >= 0 && gx < w && gy >= 0 && gy < h;
        side[k] = (in ? 16 : 0) | (gx > 0 && lx > 0 ? 1 : 0) | (gx < w - 1 && lx < kFfEdge - 1 ? 2 : 0) |
                  (gy > 0 && ly > 0 ? 4 : 0) | (gy < h - 1 && ly < kFfEdge - 1 ? 8 : 0);
    }
    for (int it = 0; it < iters; ++it) {
        const int cur = it & 1;
#pragma unroll
        for (int k = 0; k < kFfCells; ++k) {
            const int m = side[k];
            if (!(m & 16)) continue;
            const int idx = threadIdx.x + k * kFfBlock;
            const int l = (m & 1) ? idx - 1 : idx, r = (m & 2) ? idx + 1 : idx;
            const int u = (m & 4) ? idx - kFfEdge : idx, d = (m & 8) ? idx + kFfEdge : idx;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const float* b = buf[cur][p];
                buf[cur ^ 1][p][idx] = ((((b[idx] + b[l]) + b[r]) + b[u]) + b[d]) * 0.2f;
            }
        }
        __syncthreads();
    }
    const int fin = iters & 1;
    for (int idx = threadIdx.x; idx < kFfTile * kFfTile; idx += kFfBlock) {
        const int lx = kFfSteps + idx % kFfTile, ly = kFfSteps + idx / kFfTile;
        const int gx = X0 + lx, gy = Y0 + ly;
        if (gx >= w || gy >= h) continue;
        const int64_t g = (int64_t)gy * w + gx;
        const float vu = buf[fin][0][ly * kFfEdge + lx], vv = buf[fin][1][ly * kFfEdge + lx];
        if (dst) {
            dst[g] = vu;
            dst[N + g] = vv;
        } else {
            U[g] = vu;
            U[N + g] = vv;
            D[g] = vu - Q[g];
            D[N + g] = vv - Q[N + g];
            if (flow) {
                const bool off = mask && !mask[g];
                flow[g] = off ? 0.0f : vu;
                flow[N + g] = off ? 0.0f : vv;
            }
        }
    }
}

// Work memory of one (sensor, layer count, stream): A, B (two planes of
// level 0 each, the smoothing's ping-pong), Q (the prediction) and the
// innovation of every layer.
static int64_t ff_scratch_floats(const Geom& g, int layers) {
    const int64_t N0 = (int64_t)g.W * g.H;
    int64_t n = 6 * N0;
    for (int l = 0; l < layers; ++l) n += 2 * (int64_t)g.lv[l].w * g.lv[l].h;
    return n;
}

static int ff_scratch(ebof_ctx* ctx, const Geom& g, int layers, hipStream_t st, float** out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const auto key = std::make_tuple(g.W, g.H, (int32_t)layers, (uintptr_t)st);
    auto it = ctx->filter_scratch.find(key);
    if (it != ctx->filter_scratch.end()) {
        *out = it->second;
        return EBOF_OK;
    }
    const size_t bytes = (size_t)ff_scratch_floats(g, layers) * sizeof(float);
    float* p = (float*)ctx->arena.alloc(bytes);
    if (!p) {
        set_error("arena full: the flow filter needs %zu bytes of work memory, %zu free", bytes,
                  ctx->arena.bytes_free());
        return EBOF_E_NOMEM;
    }
    *out = ctx->filter_scratch[key] = p;
    return EBOF_OK;
}

static int ff_validate(const ebof_params* p, const ebof_filter_params* fp) {
    int rc = validate_params(p);
    if (rc) return rc;
    if (!fp) {
        set_error("filter params is NULL");
        return EBOF_E_INVAL;
    }
    if (fp->layers < 1 || fp->layers > p->levels) {
        set_error("filter layers %d outside [1, %d] (the pyramid's levels)", fp->layers, p->levels);
        return EBOF_E_INVAL;
    }
    for (int l = 0; l < fp->layers; ++l) {
        if (!std::isfinite(fp->gamma[l]) || !(fp->gamma[l] > 0.0f)) {
            set_error("filter layer %d: weight %g is not finite and positive", l, (double)fp->gamma[l]);
            return EBOF_E_INVAL;
        }
        if (fp->smooth[l] < 0 || fp->smooth[l] > kFfMaxSmooth) {
            set_error("filter layer %d: %d smoothing iterations outside [0, %d]", l, fp->smooth[l], kFfMaxSmooth);
            return EBOF_E_INVAL;
        }
    }
    return EBOF_OK;
}

}  // namespace ebof

using namespace ebof;

extern "C" {

int ebof_filter_params_default(int32_t width, int32_t height, ebof_filter_params* out) {
    if (!out) {
        set_error("ebof_filter_params_default: out is NULL");
        return EBOF_E_INVAL;
    }
    std::memset(out, 0, sizeof(*out));
    out->layers = 3;
    const bool low = (int64_t)width * height <= 346 * 260;
    const float g_low[3] = {500.0f, 250.0f, 50.0f};
    const int32_t s_low[3] = {5, 25, 50};
    for (int l = 0; l < 3; ++l) {
        out->gamma[l] = low ? g_low[l] : 500.0f;
        out->smooth[l] = low ? s_low[l] : 20;
    }
    return EBOF_OK;
}

int64_t ebof_filter_state_floats(const ebof_params* p, const ebof_filter_params* fp) {
    if (ff_validate(p, fp)) return -1;
    const Geom g = make_geom(*p);
    int64_t n = 0;
    for (int l = 0; l < fp->layers; ++l) n += 2 * (int64_t)g.lv[l].w * g.lv[l].h;
    return n;
}

int ebof_flow_filter(ebof_ctx* ctx, const ebof_params* p, const ebof_filter_params* fp, const float* pyr_prev,
                     const float* pyr_curr, const uint8_t* mask, float* state, float* flow_out, void* hip_stream) {
    if (!ctx) {
        set_error("ctx is NULL");
        return EBOF_E_INVAL;
    }
    if (ctx->failed) {
        set_error("context failed earlier (device error)");
        return EBOF_E_DEVICE;
    }
    int rc = ff_validate(p, fp);
    if (rc) return rc;
    if (!pyr_prev || !pyr_curr || !state || !flow_out) {
        set_error("ebof_flow_filter: NULL pyramid, state or flow_out");
        return EBOF_E_INVAL;
    }
    const hipStream_t st = (hipStream_t)hip_stream;
    const Geom g = make_geom(*p);
    float* work;
    if ((rc = ff_scratch(ctx, g, fp->layers, st, &work))) return rc;
    const int64_t N0 = (int64_t)g.W * g.H;
    float* A = work;
    float* B = A + 2 * N0;
    float* Q = B + 2 * N0;
    float* Dbase = Q + 2 * N0;
    int64_t soff[kMaxLevels], doff[kMaxLevels];
    int64_t so = 0;
    for (int l = 0; l < fp->layers; ++l) {
        soff[l] = doff[l] = so;
        so += 2 * (int64_t)g.lv[l].w * g.lv[l].h;
    }
    const bool masked = (p->flags & EBOF_MASK_FLOW) && mask;
    for (int l = fp->layers - 1; l >= 0; --l) {
        const LevelGeom& lv = g.lv[l];
        const int64_t N = (int64_t)lv.w * lv.h;
        const float* I0 = pyr_prev + lv.off;
        const float* I1 = pyr_curr + lv.off;
        float* U = state + soff[l];
        const bool top = l == fp->layers - 1;
        const float* Dc = top ? nullptr : Dbase + doff[l + 1];
        const int wc = top ? 1 : g.lv[l + 1].w, hc = top ? 1 : g.lv[l + 1].h;
        hipLaunchKernelGGL(k_ff_update, dim3((unsigned)((N + kFfBlock - 1) / kFfBlock)), dim3(kFfBlock), 0, st, I0,
                           I1, U, Dc, lv.w, lv.h, wc, hc, fp->gamma[l], A, Q);
        const int n = fp->smooth[l];
        const int launches = n == 0 ? 1 : (n + kFfSteps - 1) / kFfSteps;
        const unsigned tiles =
            (unsigned)(((lv.w + kFfTile - 1) / kFfTile) * (int64_t)((lv.h + kFfTile - 1) / kFfTile));
        float* src = A;
        float* dst = B;
        for (int j = 0; j < launches; ++j) {
            const int it = n == 0 ? 0 : std::min(kFfSteps, n - j * kFfSteps);
            const bool last = j == launches - 1;
            hipLaunchKernelGGL(k_ff_smooth, dim3(tiles), dim3(kFfBlock), 0, st, src, lv.w, lv.h, it,
                               last ? nullptr : dst, Q, U, Dbase + doff[l], l == 0 ? flow_out : nullptr,
                               masked ? mask : nullptr);
            std::swap(src, dst);
        }
    }
    return check_hip(ctx, hipGetLastError(), "kernel launch");
}

}  // extern "C"

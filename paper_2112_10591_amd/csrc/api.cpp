// api.cpp -- the C ABI: parameters, context, stage calls, batched runs and
// kernel timing.  Argument checking happens here; kernels assume valid
// descriptors.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "ctx.h"

namespace ebof {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

int check_hip(ebof_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return EBOF_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    if (ctx) ctx->failed = true;
    return EBOF_E_DEVICE;
}

// ---------------------------------------------------------------- params
// The value a saturating surface takes from some squared distance on: 1 for
// eq. (1), d_sat = alpha ln 255 for the bounded distance; the others grow
// without bound and use no table.
static bool surface_saturates(int32_t kind) { return kind == EBOF_SURFACE_EXP || kind == EBOF_SURFACE_BOUNDED; }
static float surface_sat(float alpha, int32_t kind) {
    return kind == EBOF_SURFACE_BOUNDED ? (float)((double)alpha * std::log(255.0)) : 1.0f;
}

static int64_t lut_entries(float alpha, int32_t kind, std::vector<float>* out) {
    // squared distances whose surface value is below the saturation value
    if (!surface_saturates(kind)) return 0;
    const double a = (double)alpha;
    const float sat = surface_sat(alpha, kind);
    const int64_t cap = int64_t(1) << 22;
    for (int64_t i = 0; i < cap; ++i) {
        const double d = std::sqrt((double)i);
        const float s = kind == EBOF_SURFACE_BOUNDED ? (float)std::min(d, (double)a * std::log(255.0))
                                                     : (float)(1.0 - std::exp(-d / a));
        if (s == sat) return i;
        if (out) out->push_back(s);
    }
    return -1;
}

static int validate(const ebof_params* p) {
    if (!p) {
        set_error("params is NULL");
        return EBOF_E_INVAL;
    }
    if (p->struct_size != sizeof(ebof_params)) {
        set_error("params.struct_size is %u, expected %zu", p->struct_size, sizeof(ebof_params));
        return EBOF_E_INVAL;
    }
    if (p->width < EBOF_MIN_DIM || p->width > EBOF_MAX_DIM || p->height < EBOF_MIN_DIM ||
        p->height > EBOF_MAX_DIM) {
        set_error("sensor size %dx%d outside [%d, %d]", p->width, p->height, EBOF_MIN_DIM, EBOF_MAX_DIM);
        return EBOF_E_INVAL;
    }
    if (p->levels < 1 || p->levels > EBOF_MAX_LEVELS) {
        set_error("levels %d outside [1, %d]", p->levels, EBOF_MAX_LEVELS);
        return EBOF_E_INVAL;
    }
    int32_t w = p->width, h = p->height;
    for (int l = 0; l < p->levels; ++l) {
        if (w < EBOF_PATCH || h < EBOF_PATCH) {
            set_error("pyramid level %d is %dx%d, smaller than the %d-pixel patch", l, w, h, EBOF_PATCH);
            return EBOF_E_INVAL;
        }
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    if (p->n_d < 0 || p->n_d > 5 || p->n_f < 0 || p->n_f > 5) {
        set_error("n_d %d / n_f %d outside [0, 5]", p->n_d, p->n_f);
        return EBOF_E_INVAL;
    }
    if (!(std::isfinite(p->alpha) && p->alpha > 0.f && p->alpha < 100.f)) {
        set_error("alpha %g must be finite, > 0 and < 100", (double)p->alpha);
        return EBOF_E_INVAL;
    }
    if (!(std::isfinite(p->lambda_reg) && p->lambda_reg > 0.f)) {
        set_error("lambda_reg %g must be finite and > 0", (double)p->lambda_reg);
        return EBOF_E_INVAL;
    }
    if (p->patch != EBOF_PATCH) {
        set_error("patch %d: only %d is supported", p->patch, EBOF_PATCH);
        return EBOF_E_INVAL;
    }
    if (p->stride < 1 || p->stride > EBOF_PATCH) {
        set_error("stride %d outside [1, %d]", p->stride, EBOF_PATCH);
        return EBOF_E_INVAL;
    }
    if (p->iters < 0 || p->iters > 1024) {
        set_error("iters %d outside [0, 1024]", p->iters);
        return EBOF_E_INVAL;
    }
    if (p->dt_us <= 0) {
        set_error("dt_us %lld must be > 0", (long long)p->dt_us);
        return EBOF_E_INVAL;
    }
    if (p->surface < EBOF_SURFACE_EXP || p->surface > EBOF_SURFACE_LOG) {
        set_error("surface %d is not one of EBOF_SURFACE_*", p->surface);
        return EBOF_E_INVAL;
    }
    if (p->flags & ~(EBOF_MASK_FLOW | EBOF_CHAIN_ALWAYS | EBOF_WARM_START | EBOF_VAR_REFINE)) {
        set_error("unknown flags 0x%x", p->flags);
        return EBOF_E_INVAL;
    }
    return EBOF_OK;
}

Geom make_geom(const ebof_params& p) {
    Geom g{};
    g.W = p.width;
    g.H = p.height;
    g.L = p.levels;
    g.stride = p.stride;
    int32_t w = p.width, h = p.height;
    int64_t off = 0, poff = 0;
    for (int l = 0; l < kMaxLevels; ++l) {
        LevelGeom& lv = g.lv[l];
        if (l < p.levels) {
            lv.w = w;
            lv.h = h;
            lv.pnx = (w - kPatch + p.stride - 1) / p.stride + 1;
            lv.pny = (h - kPatch + p.stride - 1) / p.stride + 1;
            lv.off = off;
            lv.poff = poff;
            off += (int64_t)w * h;
            poff += (int64_t)lv.pnx * lv.pny;
            w = (w + 1) / 2;
            h = (h + 1) / 2;
        } else {
            lv = LevelGeom{0, 0, 0, 0, off, poff};
        }
    }
    g.pyr_floats = off;
    g.patches = poff;
    return g;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static size_t scratch_bytes(const Geom& g) {
    const size_t N = (size_t)g.W * g.H;
    const size_t nch = (size_t)(g.H + kChunk - 1) / kChunk;
    return align256(N) + align256(nch * g.W * 8) + align256(N * 2) + align256((size_t)g.patches * 8);
}

// ---------------------------------------------------------------- ctx helpers
int lut_for(ebof_ctx* ctx, float alpha, int32_t kind, Lut* out) {
    for (const Lut& l : ctx->luts)
        if (std::memcmp(&l.alpha, &alpha, sizeof(float)) == 0 && l.kind == kind) {
            *out = l;
            return EBOF_OK;
        }
    std::vector<float> v;
    const int64_t n = lut_entries(alpha, kind, &v);
    if (n < 0) {
        set_error("alpha %g needs a lookup table over 2^22 entries", (double)alpha);
        return EBOF_E_INVAL;
    }
    Lut l;
    l.alpha = alpha;
    l.kind = kind;
    l.sat = surface_sat(alpha, kind);
    l.n = (int32_t)n;
    l.dev = (float*)ctx->arena.alloc(std::max<size_t>(4, v.size() * 4));
    if (!l.dev) {
        set_error("arena full (lookup table of %lld floats)", (long long)n);
        return EBOF_E_NOMEM;
    }
    if (!v.empty()) {
        int rc = check_hip(ctx, hipMemcpy(l.dev, v.data(), v.size() * 4, hipMemcpyHostToDevice), "hipMemcpy(lut)");
        if (rc) return rc;
    }
    ctx->luts.push_back(l);
    *out = l;
    return EBOF_OK;
}

int scratch_alloc(ebof_ctx* ctx, const Geom& g, Scratch* s, hipStream_t) {
    const size_t N = (size_t)g.W * g.H;
    const size_t nch = (size_t)(g.H + kChunk - 1) / kChunk;
    Scratch t;
    t.W = g.W;
    t.H = g.H;
    t.L = g.L;
    t.stride = g.stride;
    t.e_raw = (uint8_t*)ctx->arena.alloc(N);
    t.colmask = (uint64_t*)ctx->arena.alloc(nch * g.W * 8);
    t.g = (uint16_t*)ctx->arena.alloc(N * 2);
    t.puv = (float2*)ctx->arena.alloc((size_t)g.patches * 8);
    if (!t.e_raw || !t.colmask || !t.g || !t.puv) {
        scratch_free(ctx, &t);
        set_error("arena full: window scratch needs %zu bytes, %zu free", scratch_bytes(g),
                  ctx->arena.bytes_free());
        return EBOF_E_NOMEM;
    }
    t.stamp = 0;
    t.needs_zero = true;
    *s = t;
    return EBOF_OK;
}

void scratch_free(ebof_ctx* ctx, Scratch* s) {
    ctx->arena.free(s->var);
    ctx->arena.free(s->ud);
    ctx->arena.free(s->e_raw);
    ctx->arena.free(s->colmask);
    ctx->arena.free(s->g);
    ctx->arena.free(s->puv);
    *s = Scratch();
}

void fill_desc(const ebof_params& p, const Geom& g, const Lut& lut, const Scratch& s, WinDesc* d) {
    std::memset(d, 0, sizeof(*d));
    d->W = p.width;
    d->H = p.height;
    d->L = p.levels;
    d->n_d = p.n_d;
    d->n_f = p.n_f;
    d->stride = p.stride;
    d->iters = p.iters;
    d->flags = p.flags;
    d->lambda = p.lambda_reg;
    d->lut_n = lut.n;
    d->lut_r = 0;
    while ((int64_t)d->lut_r * d->lut_r < lut.n) ++d->lut_r;
    d->lut = lut.dev;
    d->surf_kind = p.surface;
    d->lut_sat = lut.sat;
    d->e_raw = s.e_raw;
    d->colmask = s.colmask;
    d->g = s.g;
    d->puv = s.puv;
    for (int l = 0; l < kMaxLevels; ++l) d->lv[l] = g.lv[l];
}

static Scratch* stage_scratch(ebof_ctx* ctx, const Geom& g, hipStream_t st, int* rc) {
    auto key = std::make_tuple(g.W, g.H, g.L, g.stride, (uintptr_t)st);
    auto it = ctx->stage_scratch.find(key);
    if (it != ctx->stage_scratch.end()) return &it->second;
    Scratch s;
    *rc = scratch_alloc(ctx, g, &s, st);
    if (*rc) return nullptr;
    return &(ctx->stage_scratch[key] = s);
}

// ---------------------------------------------------------------- timing
// Kernel timing: while timed() runs f for a selected kernel, every launch
// built (one_launch, batch_launch) takes an event pair recorded right before
// and right after it on its stream.  In span mode the launches f makes (one
// stream) are only counted, and one pair recorded around f brackets them all.
struct TimingScope {
    ebof_ctx* ctx = nullptr;
    int kid = -1;
    bool span = false;
    int launches = 0;
};
static thread_local TimingScope tl_timing;

static bool take_pair(ebof_ctx* ctx, TimedPair& tp) {  // under timing_mu
    for (hipEvent_t* e : {&tp.a, &tp.b}) {
        if (!ctx->event_pool.empty()) {
            *e = ctx->event_pool.back();
            ctx->event_pool.pop_back();
        } else if (hipEventCreate(e) != hipSuccess) {
            if (e == &tp.b) ctx->event_pool.push_back(tp.a);
            return false;  // untimed launches rather than failed ones
        }
    }
    return true;
}

static void attach_timing(Launch& L) {
    ebof_ctx* ctx = tl_timing.ctx;
    if (!ctx) return;
    if (tl_timing.span) {
        ++tl_timing.launches;
        return;
    }
    TimedPair tp;
    tp.launches = 1;
    std::lock_guard<std::mutex> lk(ctx->timing_mu);
    if (!take_pair(ctx, tp)) return;
    ctx->timed[tl_timing.kid].push_back(tp);
    L.ev_start = tp.a;
    L.ev_stop = tp.b;
}

template <class F>
static void timed(ebof_ctx* ctx, int kid, hipStream_t st, F&& f) {
    if (!(ctx->timing_mask.load(std::memory_order_relaxed) & (1u << kid))) {
        f();
        return;
    }
    const bool span = ctx->timing_span.load(std::memory_order_relaxed);
    TimedPair tp{};
    if (span) {
        std::lock_guard<std::mutex> lk(ctx->timing_mu);
        if (!take_pair(ctx, tp)) {
            f();
            return;
        }
    }
    if (span && hipEventRecord(tp.a, st) != hipSuccess) {
        std::lock_guard<std::mutex> lk(ctx->timing_mu);
        ctx->event_pool.push_back(tp.a);
        ctx->event_pool.push_back(tp.b);
        f();
        return;
    }
    tl_timing = TimingScope{ctx, kid, span, 0};
    f();
    const int n = tl_timing.launches;
    tl_timing = TimingScope{};
    if (!span) return;
    const bool ok = hipEventRecord(tp.b, st) == hipSuccess;
    std::lock_guard<std::mutex> lk(ctx->timing_mu);
    if (ok && n > 0) {
        tp.launches = n;
        ctx->timed[kid].push_back(tp);
    } else {
        ctx->event_pool.push_back(tp.a);
        ctx->event_pool.push_back(tp.b);
    }
}

// stage calls launch one block per item with the default tile shapes
static const Tune kStageTune{};

static Launch one_launch(const WinDesc* d, int32_t total, hipStream_t st) {
    Launch L;
    L.one = d;
    L.ba = BatchArgs{nullptr, nullptr, nullptr, 0, 0};
    L.batch = false;
    L.total = total;
    L.grid = std::max(1, total);
    L.stream = st;
    attach_timing(L);
    return L;
}

static int ctx_ok(ebof_ctx* ctx) {
    if (!ctx) {
        set_error("ctx is NULL");
        return EBOF_E_INVAL;
    }
    if (ctx->failed) {
        set_error("context failed earlier (device error)");
        return EBOF_E_DEVICE;
    }
    return EBOF_OK;
}

static int launch_status(ebof_ctx* ctx) { return check_hip(ctx, hipGetLastError(), "kernel launch"); }

// ---------------------------------------------------------------- batched
static std::string layout_key(const std::vector<WinDesc>& d, const std::vector<char>& flow) {
    std::string k;
    char buf[64];
    for (size_t i = 0; i < d.size(); ++i) {
        snprintf(buf, sizeof buf, "%d,%d,%d,%d,%d,%d;", d[i].W, d[i].H, d[i].L, d[i].stride, (int)flow[i],
                 (int)d[i].zero_out);
        k += buf;
    }
    return k;
}

static size_t prefix_bytes(int32_t n) { return sizeof(int32_t) * (size_t)kNumStages * (n + 1); }
static size_t table_desc_offset() { return align256(kTableHeader + prefix_bytes(EBOF_MAX_BATCH)); }

void runner_release(BatchRunner& br) {
    for (auto& kv : br.graphs)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    br.graphs.clear();
    if (br.capture) (void)hipStreamDestroy(br.capture);
    br.capture = nullptr;
    for (auto& pb : br.pinned) {
        if (pb.host) (void)hipHostFree(pb.host);
        if (pb.done) (void)hipEventDestroy(pb.done);
    }
    br.pinned.clear();
}

static int runner_init(ebof_ctx* ctx, BatchRunner& br) {
    if (br.table_dev) return EBOF_OK;
    br.table_bytes = table_desc_offset() + sizeof(WinDesc) * EBOF_MAX_BATCH;
    br.table_dev = (char*)ctx->arena.alloc(br.table_bytes);
    if (!br.table_dev) {
        set_error("arena full (batch table of %zu bytes)", br.table_bytes);
        return EBOF_E_NOMEM;
    }
    int rc0 = check_hip(ctx, hipStreamCreateWithFlags(&br.capture, hipStreamNonBlocking), "hipStreamCreate(capture)");
    if (rc0) return rc0;
    br.pinned.resize(4);
    for (auto& pb : br.pinned) {
        int rc = check_hip(ctx, hipHostMalloc((void**)&pb.host, br.table_bytes, hipHostMallocDefault), "hipHostMalloc");
        if (rc) return rc;
        rc = check_hip(ctx, hipEventCreateWithFlags(&pb.done, hipEventDisableTiming), "hipEventCreate");
        if (rc) return rc;
    }
    return EBOF_OK;
}

// ---------------------------------------------------------------- launch shapes
// The stages of a batch in pipeline order: binning, denoise/fill, EDT,
// pyramid chains from the finest, then the inverse search from the coarsest
// level to the finest (each level starts from the coarser one), then the
// densification.
static std::vector<int> pipeline_order(int lmax) {
    std::vector<int> o{kStZero, kStScatter, kStDenoise, kStCols, kStRows};
    for (int c = 0; c * kPyrChain < lmax - 1; ++c) o.push_back(kStPyr + c);
    for (int l = lmax - 1; l >= 0; --l) o.push_back(kStDis + l);
    o.push_back(kStDensify);
    return o;
}
static int stage_kernel_id(int s) {
    if (s == kStZero) return -1;
    if (s == kStScatter) return EBOF_K_SCATTER;
    if (s == kStDenoise) return EBOF_K_DENOISE_FILL;
    if (s == kStCols) return EBOF_K_EDT_COLS;
    if (s == kStRows) return EBOF_K_EDT_ROWS;
    if (s >= kStPyr && s < kStDis) return EBOF_K_PYR_DOWN;
    if (s >= kStDis && s < kStDensify) return EBOF_K_DIS_LEVEL;
    return EBOF_K_DENSIFY;
}
// Default persistent grids of the universal graph (any batch), and of the
// stages whose item counts vary between batches of one layout (event counts).
static int32_t stage_cap(int s) {
    if (s == kStZero) return 512;
    if (s >= kStPyr && s < kStDis) return 1024;
    return 2048;
}
static int32_t stage_grid(int s, int32_t total, const Tune& t, int mode) {
    if (t.grid[s] > 0) return t.grid[s];
    if (mode == kGraphUniversal || s == kStZero || s == kStScatter) return stage_cap(s);
    return std::max(1, std::min(total, 1 << 20));
}
static Launch batch_launch(BatchRunner& br, const WinDesc* first, int s, int32_t total, int32_t grid,
                           hipStream_t st) {
    Launch L;
    L.one = first;
    L.ba = BatchArgs{(const WinDesc*)(br.table_dev + table_desc_offset()),
                     (const int32_t*)(br.table_dev + kTableHeader), (const int32_t*)br.table_dev, s, 0};
    L.batch = true;
    L.total = total;
    L.grid = grid;
    L.stream = st;
    attach_timing(L);
    return L;
}
static void launch_stage(const Launch& L, int s, const Tune& t) {
    if (s == kStZero)
        launch_zero(L);
    else if (s == kStScatter)
        launch_scatter(L);
    else if (s == kStDenoise)
        launch_denoise_fill(L, true);
    else if (s == kStCols)
        launch_edt_cols(L);
    else if (s == kStRows)
        launch_edt_rows(L, t.rows_nr);
    else if (s >= kStPyr && s < kStDis)
        launch_pyr_chain(L, (s - kStPyr) * kPyrChain);
    else if (s >= kStDis && s < kStDensify)
        launch_dis_level(L, s - kStDis, t.dis_lanes[s - kStDis]);
    else
        launch_densify(L, t.dens_tw);
}

// prefix sums, window-major: prefix[i * kNumStages + s]
static int build_prefix(const std::vector<WinDesc>& descs, const std::vector<char>& flow,
                        const std::vector<char>& zero, const Tune& t, std::vector<int32_t>* prefix,
                        int32_t* totals) {
    const int32_t n = (int32_t)descs.size();
    prefix->assign((size_t)kNumStages * (n + 1), 0);
    for (int s = 0; s < kNumStages; ++s) {
        int64_t run = 0;
        for (int32_t i = 0; i < n; ++i) {
            (*prefix)[(size_t)i * kNumStages + s] = (int32_t)run;
            run += stage_items(descs[i], s, flow[i], zero[i], t);
        }
        if (run > INT32_MAX) {
            set_error("batch too large: stage %d has %lld work items", s, (long long)run);
            return EBOF_E_INVAL;
        }
        (*prefix)[(size_t)n * kNumStages + s] = (int32_t)run;
        totals[s] = (int32_t)run;
    }
    return EBOF_OK;
}

// Copies [nwin | prefix sums] and the descriptors to the device table through
// the next pinned staging buffer, ordered on st.
static int upload_table(ebof_ctx* ctx, BatchRunner& br, const std::vector<WinDesc>& descs,
                        const std::vector<int32_t>& prefix, hipStream_t st) {
    const int32_t n = (int32_t)descs.size();
    auto& pb = br.pinned[br.pinned_next];
    br.pinned_next = (br.pinned_next + 1) % (int)br.pinned.size();
    int rc;
    if (pb.used && (rc = check_hip(ctx, hipEventSynchronize(pb.done), "hipEventSynchronize"))) return rc;
    const size_t doff = table_desc_offset();
    std::memcpy(pb.host, &n, sizeof(int32_t));
    std::memcpy(pb.host + kTableHeader, prefix.data(), prefix_bytes(n));
    std::memcpy(pb.host + doff, descs.data(), sizeof(WinDesc) * n);
    if ((rc = check_hip(ctx,
                        hipMemcpyAsync(br.table_dev, pb.host, kTableHeader + prefix_bytes(n), hipMemcpyHostToDevice,
                                       st),
                        "hipMemcpyAsync(prefix)")))
        return rc;
    if ((rc = check_hip(ctx,
                        hipMemcpyAsync(br.table_dev + doff, pb.host + doff, sizeof(WinDesc) * n,
                                       hipMemcpyHostToDevice, st),
                        "hipMemcpyAsync(table)")))
        return rc;
    if ((rc = check_hip(ctx, hipEventRecord(pb.done, st), "hipEventRecord"))) return rc;
    pb.used = true;
    return EBOF_OK;
}

// The autotuner.  For a new batch layout it runs the batch once with default
// shapes (so every stage's inputs exist), then times each stage alone for
// each candidate shape (the persistent grid; the rows per item of the EDT row
// pass; the tile width of the densification), stage by stage in pipeline
// order, keeping the fastest.  Every stage is idempotent given its inputs
// and the candidates change no window's arithmetic, so the outputs are the
// same whatever is chosen.  The tuning copy of the table counts no dropped
// events; the caller's run that follows does.
static int autotune(ebof_ctx* ctx, BatchRunner& br, const std::vector<WinDesc>& descs, const std::vector<char>& flow,
                    const std::vector<char>& zero, int lmax, hipStream_t st, Tune* out) {
    std::vector<WinDesc> td = descs;
    for (auto& d : td) d.n_dropped = nullptr;
    Tune best;
    resolve_dis_lanes(best, td.data(), (int)td.size());
    std::vector<int32_t> prefix;
    int32_t totals[kNumStages];
    int rc;
    // the previous batch on st may still read the table
    if ((rc = check_hip(ctx, hipStreamSynchronize(st), "hipStreamSynchronize"))) return rc;
    auto upload = [&](const Tune& t) -> int {
        int r = build_prefix(td, flow, zero, t, &prefix, totals);
        if (!r) r = upload_table(ctx, br, td, prefix, st);
        return r;
    };
    if ((rc = upload(best))) return rc;
    for (int s : pipeline_order(lmax))
        if (totals[s])
            launch_stage(batch_launch(br, &td[0], s, totals[s], stage_grid(s, totals[s], best, kGraphLayout), st), s,
                         best);
    if ((rc = launch_status(ctx))) return rc;
    hipEvent_t e0, e1;
    if ((rc = check_hip(ctx, hipEventCreate(&e0), "hipEventCreate"))) return rc;
    if ((rc = check_hip(ctx, hipEventCreate(&e1), "hipEventCreate"))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    auto time_stage = [&](int s, const Tune& t, float* ms) -> int {
        int r = upload(t);
        if (r) return r;
        if (!totals[s]) {
            *ms = 0.f;
            return EBOF_OK;
        }
        const Launch L = batch_launch(br, &td[0], s, totals[s], stage_grid(s, totals[s], t, kGraphLayout), st);
        launch_stage(L, s, t);  // warm
        if ((r = check_hip(ctx, hipEventRecord(e0, st), "hipEventRecord"))) return r;
        for (int rep = 0; rep < 3; ++rep) launch_stage(L, s, t);
        if ((r = check_hip(ctx, hipEventRecord(e1, st), "hipEventRecord"))) return r;
        if ((r = launch_status(ctx))) return r;
        if ((r = check_hip(ctx, hipEventSynchronize(e1), "hipEventSynchronize"))) return r;
        return check_hip(ctx, hipEventElapsedTime(ms, e0, e1), "hipEventElapsedTime");
    };
    static const int32_t kGrids[] = {0, 256, 512, 1024, 2048, 4096};
    for (int s : pipeline_order(lmax)) {
        if (rc) break;
        if (s == kStZero) continue;
        const bool dis = s >= kStDis && s < kStDensify;
        std::vector<int> shapes{0};
        if (s == kStRows) shapes = {1, 2, 4, 8};
        if (s == kStDensify) shapes = {16, 64, 128, 256};
        if (dis) shapes = {8, 4};
        float best_ms = -1.f;
        Tune win = best;
        for (int shape : shapes) {
            Tune t = best;
            if (s == kStRows) t.rows_nr = shape;
            if (s == kStDensify) t.dens_tw = shape;
            if (dis) t.dis_lanes[s - kStDis] = shape;
            if ((rc = build_prefix(td, flow, zero, t, &prefix, totals))) break;
            for (int32_t g : kGrids) {
                if (g == 0 && s == kStScatter) continue;  // its item count varies: a fixed grid
                if (g > 0 && g >= totals[s]) continue;    // no more blocks than items
                t.grid[s] = g;
                float ms = 0.f;
                if ((rc = time_stage(s, t, &ms))) break;
                if (best_ms < 0.f || ms < best_ms) {
                    best_ms = ms;
                    win = t;
                }
            }
            if (rc) break;
        }
        best = win;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *out = best;
    return EBOF_OK;
}

// Appends one tuned layout to the cache file, if one is set.
static void save_tune(ebof_ctx* ctx, const std::string& key, const Tune& t) {
    if (ctx->tune_path.empty()) return;
    FILE* f = std::fopen(ctx->tune_path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s\t%d %d", key.c_str(), t.rows_nr, t.dens_tw);
    for (int l = 0; l < kMaxLevels; ++l) std::fprintf(f, " %d", t.dis_lanes[l]);
    for (int s = 0; s < kNumStages; ++s) std::fprintf(f, " %d", t.grid[s]);
    std::fprintf(f, "\n");
    std::fclose(f);
}

// Reads a cache file written by save_tune (or by hand); EBOF_E_INVAL names
// the first malformed line.
static int load_tunes(const char* path, std::map<std::string, Tune>* out) {
    FILE* f = std::fopen(path, "r");
    if (!f) return EBOF_OK;  // nothing tuned yet
    char line[1 << 14];
    int lineno = 0, rc = EBOF_OK;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        std::string l(line), key;
        if (l.find_first_not_of(" \r\n") == std::string::npos) continue;
        std::vector<int> v;
        Tune t;
        bool ok = parse_tune_line(l, 2 + kMaxLevels + kNumStages, &key, &v);
        if (ok) {
            t.rows_nr = v[0];
            t.dens_tw = v[1];
            for (int lv = 0; lv < kMaxLevels; ++lv) t.dis_lanes[lv] = v[2 + lv];
            for (int s = 0; s < kNumStages; ++s) t.grid[s] = v[2 + kMaxLevels + s];
            ok = tune_valid(t);
        }
        if (!ok) {
            set_error("tuning cache %s: malformed line %d", path, lineno);
            rc = EBOF_E_INVAL;
            break;
        }
        (*out)[key] = t;
    }
    std::fclose(f);
    return rc;
}

// Runs n windows, one launch per stage.  scr[i] is window i's scratch (its
// geometry must match the window's parameters).  graph_mode: kGraphNone
// launches directly; kGraphLayout captures one graph per batch layout with
// exact grids; kGraphUniversal captures one graph per maximum level count
// with fixed persistent grids, valid for any batch (every count is read from
// the uploaded table).
int run_batch_impl(ebof_ctx* ctx, BatchRunner& br, const ebof_window* w, const WinExtra* extra, int32_t n,
                   hipStream_t st, Scratch* const* scr, int graph_mode,
                   const std::function<int(hipStream_t)>* between) {
    if (!w || n < 1 || n > EBOF_MAX_BATCH) {
        set_error("batch of %d windows outside [1, %d]", n, EBOF_MAX_BATCH);
        return EBOF_E_INVAL;
    }
    for (int32_t i = 0; i < n; ++i) {
        int rc = validate(w[i].params);
        if (rc) return rc;
        if (w[i].params->flags & EBOF_VAR_REFINE) {
            set_error("window %d: the variational refinement runs in the stage calls only", i);
            return EBOF_E_INVAL;
        }
        const bool zero_out = extra && extra[i].zero_out;
        if (w[i].n < 0 || (w[i].n > 0 && (!w[i].x || !w[i].y || !w[i].t)) || !w[i].edge_out || !w[i].pyr_out ||
            ((w[i].pyr_prev || zero_out) && !w[i].flow_out)) {
            set_error("window %d: missing buffer or negative event count", i);
            return EBOF_E_INVAL;
        }
        if (w[i].t0_us > INT64_MAX - w[i].params->dt_us) {
            set_error("window %d: t0 + dt overflows", i);
            return EBOF_E_INVAL;
        }
        const Scratch& s = *scr[i];
        if (s.W != w[i].params->width || s.H != w[i].params->height || s.L != w[i].params->levels ||
            s.stride != w[i].params->stride) {
            set_error("window %d: scratch geometry does not match its parameters", i);
            return EBOF_E_INVAL;
        }
    }
    int rc = runner_init(ctx, br);
    if (rc) return rc;
    std::vector<WinDesc> descs(n);
    std::vector<char> flow(n), zero(n);
    int32_t lmax = 1;
    for (int32_t i = 0; i < n; ++i) {
        const ebof_params& p = *w[i].params;
        const Geom g = make_geom(p);
        Lut lut;
        if ((rc = lut_for(ctx, p.alpha, p.surface, &lut))) return rc;
        Scratch& s = *scr[i];
        WinDesc& d = descs[i];
        fill_desc(p, g, lut, s, &d);
        d.ex = w[i].x;
        d.ey = w[i].y;
        d.et = w[i].t;
        d.n_ev = w[i].n;
        d.t0 = w[i].t0_us;
        d.t1 = w[i].t0_us + p.dt_us;
        d.stamp = s.next_stamp();
        zero[i] = s.needs_zero;
        s.needs_zero = false;
        d.e_df = w[i].edge_out;
        d.d2 = w[i].d2_out;
        d.pyr = w[i].pyr_out;
        d.pyr_prev = w[i].pyr_prev;
        d.mask = w[i].mask;
        d.flow = w[i].flow_out;
        d.flow_init = w[i].pyr_prev ? w[i].flow_init : nullptr;
        d.flow_keep = w[i].pyr_prev ? w[i].flow_dense_out : nullptr;
        d.n_dropped = (unsigned long long*)w[i].n_dropped_dev;
        if (extra) {
            d.mask_out = extra[i].mask_out;
            d.zero_out = (!w[i].pyr_prev && extra[i].zero_out) ? 1u : 0u;
        }
        flow[i] = w[i].pyr_prev != nullptr;
        lmax = std::max(lmax, p.levels);
    }
    const bool universal = graph_mode == kGraphUniversal;
    const std::string key = universal ? "U" + std::to_string(lmax) : layout_key(descs, flow);
    // launch shapes: defaults for the universal graph, else this layout's
    // tuned shapes (timed now if the layout is new and tuning is on)
    Tune tune;
    if (!universal) {
        auto ti = br.tunes.find(key);
        if (ti != br.tunes.end()) {
            tune = ti->second;
        } else if (ctx->tune_mode == EBOF_TUNE_AUTO) {
            // (not while the caller captures the stream: tuning synchronises it)
            hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
            if (st && (rc = check_hip(ctx, hipStreamIsCapturing(st, &cst), "hipStreamIsCapturing"))) return rc;
            if (cst == hipStreamCaptureStatusNone) {
                if ((rc = autotune(ctx, br, descs, flow, zero, lmax, st, &tune))) return rc;
                br.tunes[key] = tune;
                save_tune(ctx, key, tune);
            }
        }
    }
    // One universal graph serves batches of any composition, so its launch
    // shapes must not depend on the batch: by level only, 4 lanes per patch
    // at level 0 (many patches: throughput) and 8 above (a layout's shapes
    // are fixed by the layout itself).
    if (universal) {
        for (int l = 0; l < kMaxLevels; ++l) tune.dis_lanes[l] = l == 0 ? 4 : 8;
        tune.dens_tw = 16;  // square tiles: waves off the mask skip their sums
    }
    resolve_dis_lanes(tune, descs.data(), n);
    std::vector<int32_t> prefix;
    int32_t totals[kNumStages];
    if ((rc = build_prefix(descs, flow, zero, tune, &prefix, totals))) return rc;
    // upload through a pinned staging buffer: [nwin | prefix sums] and the descriptors
    if ((rc = upload_table(ctx, br, descs, prefix, st))) return rc;

    const int mode = (ctx->timing_mask == 0 && ctx->use_graphs) ? graph_mode : kGraphNone;
    // part: 0 every stage, 1 the preprocessing stages, 2 the flow stages;
    // ls: the stream the launches go to (the capture stream while capturing)
    auto run_all = [&](bool all, int part, hipStream_t ls) {
        // consecutive launches of one kernel (pyramid chains, search levels)
        // form one group
        std::vector<int> order;
        for (int s : pipeline_order(lmax))
            if ((all || totals[s]) && (part == 0 || (part == 1) == (s < kStDis))) order.push_back(s);
        for (size_t i = 0; i < order.size();) {
            const int kid = stage_kernel_id(order[i]);
            size_t j = i + 1;
            while (j < order.size() && stage_kernel_id(order[j]) == kid) ++j;
            auto launch_group = [&] {
                for (size_t q = i; q < j; ++q) {
                    const int s = order[q];
                    launch_stage(batch_launch(br, &descs[0], s, totals[s], stage_grid(s, totals[s], tune, mode), ls),
                                 s, tune);
                }
            };
            if (kid < 0)
                launch_group();
            else
                timed(ctx, kid, st, launch_group);
            i = j;
        }
    };
    const int parts[2] = {between ? 1 : 0, 2};
    for (int pi = 0; pi < (between ? 2 : 1); ++pi) {
        const int part = parts[pi];
        if (part == 2 && (rc = (*between)(st))) return rc;
        if (mode == kGraphNone) {
            run_all(false, part, st);
            if ((rc = launch_status(ctx))) return rc;
            continue;
        }
        const std::string gkey = key + (part == 0 ? "" : part == 1 ? "/pre" : "/flow");
        auto it = br.graphs.find(gkey);
        if (it == br.graphs.end()) {
            hipStreamCaptureStatus cst;
            if ((rc = check_hip(ctx, hipStreamIsCapturing(st, &cst), "hipStreamIsCapturing"))) return rc;
            if (cst != hipStreamCaptureStatusNone || st == nullptr) {
                // the stream cannot be captured here: launch directly
                run_all(false, part, st);
                if ((rc = launch_status(ctx))) return rc;
                continue;
            }
            hipGraph_t graph;
            if ((rc = check_hip(ctx, hipStreamBeginCapture(br.capture, hipStreamCaptureModeThreadLocal),
                                "hipStreamBeginCapture")))
                return rc;
            run_all(universal || mode == kGraphLayout, part, br.capture);
            if ((rc = check_hip(ctx, hipStreamEndCapture(br.capture, &graph), "hipStreamEndCapture"))) return rc;
            hipGraphExec_t exec = nullptr;
            rc = check_hip(ctx, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            (void)hipGraphDestroy(graph);
            if (rc) return rc;
            it = br.graphs.emplace(gkey, exec).first;
        }
        if ((rc = check_hip(ctx, hipGraphLaunch(it->second, st), "hipGraphLaunch"))) return rc;
    }
    return EBOF_OK;
}

int validate_params(const ebof_params* p) { return validate(p); }

// A stream with a CU mask covering every compute unit, which the HIP runtime
// backs with a hardware queue of its own.
int queue_stream_create(ebof_ctx* ctx, hipStream_t* out) {
    int ncu = 0;
    int rc = check_hip(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device),
                       "hipDeviceGetAttribute");
    if (rc) return rc;
    std::vector<uint32_t> mask((size_t)(ncu + 31) / 32, 0xffffffffu);
    return check_hip(ctx, hipExtStreamCreateWithCUMask(out, (uint32_t)mask.size(), mask.data()),
                     "hipExtStreamCreateWithCUMask");
}

}  // namespace ebof

using namespace ebof;

// ============================================================== C ABI
extern "C" {

const char* ebof_version(void) { return "ebof 0.1 gfx950"; }

int ebof_params_default(int32_t width, int32_t height, ebof_params* out) {
    if (!out) {
        set_error("out is NULL");
        return EBOF_E_INVAL;
    }
    ebof_params p;
    std::memset(&p, 0, sizeof p);
    p.struct_size = sizeof(ebof_params);
    p.width = width;
    p.height = height;
    p.dt_us = 10000;
    const bool low = (int64_t)width * height <= 100000;
    p.n_d = low ? 1 : 2;
    p.n_f = low ? 4 : 3;
    p.alpha = 1.08f;
    p.levels = low ? 3 : 4;
    p.patch = EBOF_PATCH;
    p.stride = 4;
    p.iters = 16;
    p.lambda_reg = 0.3f;
    p.flags = 0;
    p.surface = EBOF_SURFACE_EXP;
    // fewer levels for small sensors so that every level holds a patch
    while (p.levels > 1) {
        int32_t w = width, h = height;
        bool ok = true;
        for (int l = 0; l < p.levels; ++l) {
            if (w < EBOF_PATCH || h < EBOF_PATCH) ok = false;
            w = (w + 1) / 2;
            h = (h + 1) / 2;
        }
        if (ok) break;
        --p.levels;
    }
    int rc = validate(&p);
    if (rc) return rc;
    *out = p;
    return EBOF_OK;
}

int ebof_validate(const ebof_params* p) { return validate(p); }

int64_t ebof_pyramid_floats(const ebof_params* p) {
    if (validate(p)) return -1;
    return make_geom(*p).pyr_floats;
}

int64_t ebof_window_scratch_bytes(const ebof_params* p) {
    if (validate(p)) return -1;
    return (int64_t)scratch_bytes(make_geom(*p));
}

int ebof_create(int device, void* arena, size_t arena_bytes, ebof_ctx** out) {
    if (!out || !arena || arena_bytes < 4096 || ((uintptr_t)arena & 255)) {
        set_error("ebof_create: need out, a 256-byte aligned arena and arena_bytes >= 4096");
        return EBOF_E_INVAL;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        set_error("ebof_create: device %d not available (%d devices)", device, count);
        return EBOF_E_INVAL;
    }
    if (check_hip(nullptr, hipSetDevice(device), "hipSetDevice")) return EBOF_E_DEVICE;
    ebof_ctx* c = new ebof_ctx();
    c->device = device;
    c->arena.init((char*)arena, arena_bytes);
    *out = c;
    set_error("");
    return EBOF_OK;
}

namespace {
// Signal memory is never freed: the command processor reads it, and a
// process keeps the few words it ever allocated for reuse by later contexts.
std::mutex g_signal_pool_mu;
std::vector<uint32_t*> g_signal_pool;

int signal_slot(ebof_ctx* ctx, int32_t slot, uint32_t** out) {
    if (slot < 0 || slot >= EBOF_SIGNAL_SLOTS) {
        set_error("signal slot out of range");
        return EBOF_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->signal_mu);
    if (!ctx->signals[slot]) {
        uint32_t* p = nullptr;
        {
            std::lock_guard<std::mutex> pk(g_signal_pool_mu);
            if (!g_signal_pool.empty()) {
                p = g_signal_pool.back();
                g_signal_pool.pop_back();
            }
        }
        if (!p) {
            void* v = nullptr;
            int rc = check_hip(ctx, hipExtMallocWithFlags(&v, 8, hipMallocSignalMemory), "hipExtMallocWithFlags(signal)");
            if (rc) return rc;
            p = (uint32_t*)v;
        }
        *(volatile uint32_t*)p = 0u;  // host-visible memory; no stream has used it yet
        ctx->signals[slot] = p;
    }
    *out = ctx->signals[slot];
    return EBOF_OK;
}
}  // namespace

int ebof_stream_signal(ebof_ctx* ctx, int32_t slot, uint32_t value, void* hip_stream) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    uint32_t* p = nullptr;
    if ((rc = signal_slot(ctx, slot, &p))) return rc;
    return check_hip(ctx, hipStreamWriteValue32((hipStream_t)hip_stream, p, value, 0), "hipStreamWriteValue32");
}

int ebof_stream_wait(ebof_ctx* ctx, int32_t slot, uint32_t value, void* hip_stream) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    uint32_t* p = nullptr;
    if ((rc = signal_slot(ctx, slot, &p))) return rc;
    return check_hip(ctx,
                     hipStreamWaitValue32((hipStream_t)hip_stream, p, value, hipStreamWaitValueGte, 0xffffffffu),
                     "hipStreamWaitValue32");
}

int ebof_signal_read(ebof_ctx* ctx, int32_t slot, uint32_t* value) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    if (!value) {
        set_error("ebof_signal_read: NULL output");
        return EBOF_E_INVAL;
    }
    uint32_t* p = nullptr;
    if ((rc = signal_slot(ctx, slot, &p))) return rc;
    *value = *(volatile uint32_t*)p;
    return EBOF_OK;
}

// The pipelined plain driver: the per-window stage calls of one camera
// stream, window k on stream k mod n_streams, ordered by the counters.  A
// flow j is known complete once window j + n_streams (issued after it on
// the same stream) has stored its counter value.
int ebof_run_sequence(ebof_ctx* ctx, const ebof_params* p, const ebof_window_events* win, int64_t k_lo, int64_t k_hi,
                      const ebof_ring_slot* ring, int32_t n_ring, void* const* streams, int32_t n_streams,
                      int32_t slot0) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    if (!p || !win || !ring || !streams || n_streams < 1 || n_ring <= n_streams || k_lo < 0 || k_hi < k_lo ||
        slot0 < 0 || slot0 > EBOF_SIGNAL_SLOTS - n_streams || 2 * k_hi + 1 > (int64_t)UINT32_MAX) {
        set_error("ebof_run_sequence: NULL array, n_ring <= n_streams, bad window range or slots out of range");
        return EBOF_E_INVAL;
    }
    std::vector<uint32_t> seen((size_t)n_streams, 0u);
    auto flow_done = [&](int64_t j) {
        const int f = (int)(j % n_streams);
        const uint32_t need = (uint32_t)(2 * (j + n_streams) + 1);
        if (seen[f] < need) {
            uint32_t v = 0;
            if (ebof_signal_read(ctx, slot0 + f, &v) == EBOF_OK) seen[f] = v;
        }
        return seen[f] >= need;
    };
    for (int64_t k = k_lo; k < k_hi; ++k) {
        const int i = (int)(k % n_streams);
        void* st = streams[i];
        // the flows that last read ring slot k mod n_ring (one on this stream
        // is ordered before window k already)
        for (int64_t j = k - n_ring; j <= k - n_ring + 1; ++j) {
            if (j < std::max<int64_t>(1, k_lo) || j % n_streams == i || flow_done(j)) continue;
            if ((rc = ebof_stream_wait(ctx, slot0 + (int)(j % n_streams), (uint32_t)(2 * (j + n_streams) + 1), st)))
                return rc;
        }
        const ebof_window_events& e = win[k - k_lo];
        const ebof_ring_slot& b = ring[k % n_ring];
        if ((rc = ebof_window_surface(ctx, p, e.x, e.y, e.t, e.n, e.t0_us, b.edge, nullptr, nullptr, b.pyr, st)))
            return rc;
        if ((rc = ebof_stream_signal(ctx, slot0 + i, (uint32_t)(2 * k + 1), st))) return rc;
        if (k > 0) {
            if (k - 1 >= k_lo && (rc = ebof_stream_wait(ctx, slot0 + (int)((k - 1) % n_streams), (uint32_t)(2 * k - 1), st)))
                return rc;
            const ebof_ring_slot& bp = ring[(k - 1) % n_ring];
            if ((rc = ebof_flow(ctx, p, bp.pyr, b.pyr, bp.edge, b.flow, st))) return rc;
        }
    }
    return EBOF_OK;
}

int ebof_stream_create(ebof_ctx* ctx, void** hip_stream) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    if (!hip_stream) {
        set_error("ebof_stream_create: NULL output");
        return EBOF_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->signal_mu);
    if (ctx->owned_streams.size() >= (size_t)EBOF_MAX_OWNED_STREAMS) {
        set_error("ebof_stream_create: the context owns the maximum number of streams");
        return EBOF_E_STATE;
    }
    hipStream_t st = nullptr;
    if ((rc = queue_stream_create(ctx, &st))) return rc;
    ctx->owned_streams.push_back(st);
    *hip_stream = (void*)st;
    return EBOF_OK;
}

int ebof_destroy(ebof_ctx* ctx) {
    if (!ctx) return EBOF_OK;
    serve_shutdown(ctx);
    (void)hipDeviceSynchronize();
    for (hipStream_t st : ctx->owned_streams) (void)hipStreamDestroy(st);
    ctx->owned_streams.clear();
    {
        std::lock_guard<std::mutex> pk(g_signal_pool_mu);
        for (uint32_t*& p : ctx->signals)
            if (p) {
                g_signal_pool.push_back(p);
                p = nullptr;
            }
    }
    runner_release(ctx->batch);
    for (auto& v : ctx->timed)
        for (auto& tp : v) {
            (void)hipEventDestroy(tp.a);
            (void)hipEventDestroy(tp.b);
        }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    delete ctx;
    return EBOF_OK;
}

const char* ebof_last_error(const ebof_ctx*) { return g_err; }

// Binning and denoising/filling of one window (Sec. III-A, III-B) on a stage
// scratch: validates, takes the scratch's next stamp and launches the zeroing
// (when the stamp wrapped), the scatter and the denoise/fill; with pack, the
// fill also writes the column masks the distance transform starts from, and
// the descriptor carries the surface table.  *out: the window's descriptor.
static int bin_impl(ebof_ctx* ctx, const ebof_params* p, const uint16_t* x, const uint16_t* y, const int64_t* t,
                    int64_t n, int64_t t0_us, uint8_t* edge_out, uint64_t* n_dropped_dev, hipStream_t st, bool pack,
                    const char* who, WinDesc* out, const int64_t* range = nullptr) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    if ((rc = validate(p))) return rc;
    if (n < 0 || (n > 0 && (!x || !y || (!t && !range))) || !edge_out) {
        set_error("%s: NULL buffer or negative n", who);
        return EBOF_E_INVAL;
    }
    if ((n + kEventsPerItem - 1) / kEventsPerItem > INT32_MAX) {
        set_error("%s: too many events", who);
        return EBOF_E_INVAL;
    }
    if (t0_us > INT64_MAX - p->dt_us) {
        set_error("%s: t0 + dt overflows", who);
        return EBOF_E_INVAL;
    }
    const Geom g = make_geom(*p);
    Scratch scr;
    Lut lut{p->alpha, p->surface, 0, 1.0f, nullptr};
    uint32_t stamp;
    bool zero;
    {  // the lock covers the context's maps; launches run outside it
        std::lock_guard<std::mutex> lk(ctx->mu);
        Scratch* s = stage_scratch(ctx, g, st, &rc);
        if (!s) return rc;
        if (pack && (rc = lut_for(ctx, p->alpha, p->surface, &lut))) return rc;
        stamp = s->next_stamp();
        zero = s->needs_zero;
        s->needs_zero = false;
        scr = *s;
    }
    WinDesc& d = *out;
    fill_desc(*p, g, lut, scr, &d);
    d.ex = x;
    d.ey = y;
    d.et = t;
    d.n_ev = n;
    d.t0 = t0_us;
    d.t1 = t0_us + p->dt_us;
    d.stamp = stamp;
    d.e_df = edge_out;
    d.n_dropped = (unsigned long long*)n_dropped_dev;
    d.range = range;
    if (zero) launch_zero(one_launch(&d, stage_items(d, kStZero, false, true, kStageTune), st));
    if (n > 0) timed(ctx, EBOF_K_SCATTER, st, [&] { launch_scatter(one_launch(&d, stage_items(d, kStScatter, false, false, kStageTune), st)); });
    timed(ctx, EBOF_K_DENOISE_FILL, st,
          [&] { launch_denoise_fill(one_launch(&d, stage_items(d, kStDenoise, false, false, kStageTune), st), pack); });
    return EBOF_OK;
}

// The distance transform, surface and pyramid (Sec. III-C) of the edge image
// d.e_df into d.d2 / d.pyr; the column masks are packed first unless the
// fill already wrote them.  A saturating surface with no squared distance
// exported skips the column pass (edt_local).
static void surface_impl(ebof_ctx* ctx, const ebof_params* p, const WinDesc& d, hipStream_t st, bool packed) {
    if (!packed)
        timed(ctx, EBOF_K_PACK_COLS, st, [&] { launch_pack_cols(one_launch(&d, stage_items(d, kStPack, false, false, kStageTune), st)); });
    if (!edt_local(d))
        timed(ctx, EBOF_K_EDT_COLS, st, [&] { launch_edt_cols(one_launch(&d, stage_items(d, kStCols, false, false, kStageTune), st)); });
    timed(ctx, EBOF_K_EDT_ROWS, st, [&] { launch_edt_rows(one_launch(&d, stage_items(d, kStRows, false, false, kStageTune), st), kStageTune.rows_nr); });
    if (p->levels > 1)
        timed(
            ctx, EBOF_K_PYR_DOWN, st,
            [&] {
                for (int from = 0; from < p->levels - 1; from += kPyrChain)
                    launch_pyr_chain(
                        one_launch(&d, stage_items(d, kStPyr + from / kPyrChain, false, false, kStageTune), st), from);
            });
}

int ebof_bin_events(ebof_ctx* ctx, const ebof_params* p, const uint16_t* x, const uint16_t* y, const int64_t* t,
                    int64_t n, int64_t t0_us, uint8_t* edge_out, uint64_t* n_dropped_dev, void* hip_stream) {
    WinDesc d;
    int rc = bin_impl(ctx, p, x, y, t, n, t0_us, edge_out, n_dropped_dev, (hipStream_t)hip_stream, false,
                      "ebof_bin_events", &d);
    return rc ? rc : launch_status(ctx);
}

int ebof_edt_surface(ebof_ctx* ctx, const ebof_params* p, const uint8_t* edge, int32_t* d2_out, float* pyr_out,
                     void* hip_stream) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    if ((rc = validate(p))) return rc;
    if (!edge || !pyr_out) {
        set_error("ebof_edt_surface: NULL edge or pyr_out");
        return EBOF_E_INVAL;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    const Geom g = make_geom(*p);
    Scratch scr;
    Lut lut;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        Scratch* s = stage_scratch(ctx, g, st, &rc);
        if (!s) return rc;
        if ((rc = lut_for(ctx, p->alpha, p->surface, &lut))) return rc;
        scr = *s;
    }
    WinDesc d;
    fill_desc(*p, g, lut, scr, &d);
    d.e_df = const_cast<uint8_t*>(edge);  // read only by these kernels
    d.d2 = d2_out;
    d.pyr = pyr_out;
    surface_impl(ctx, p, d, st, false);
    return launch_status(ctx);
}

int ebof_window_surface(ebof_ctx* ctx, const ebof_params* p, const uint16_t* x, const uint16_t* y, const int64_t* t,
                        int64_t n, int64_t t0_us, uint8_t* edge_out, uint64_t* n_dropped_dev, int32_t* d2_out,
                        float* pyr_out, void* hip_stream) {
    if (ctx && !pyr_out) {
        set_error("ebof_window_surface: NULL pyr_out");
        return EBOF_E_INVAL;
    }
    const hipStream_t st = (hipStream_t)hip_stream;
    WinDesc d;
    int rc = bin_impl(ctx, p, x, y, t, n, t0_us, edge_out, n_dropped_dev, st, true, "ebof_window_surface", &d);
    if (rc) return rc;
    d.d2 = d2_out;
    d.pyr = pyr_out;
    surface_impl(ctx, p, d, st, true);
    return launch_status(ctx);
}

// The inverse search, level by level, and the densification of window
// descriptor d (timed per kernel when ctx has timing on).
static void flow_launches(ebof_ctx* ctx, const ebof_params* p, const WinDesc& d, hipStream_t st,
                          double* var = nullptr) {
    Tune tune = kStageTune;
    resolve_dis_lanes(tune, &d, 1);
    if (var) {  // each level refined before the next starts from it
        for (int l = p->levels - 1; l >= 0; --l) {
            auto dis = [&] {
                launch_dis_level(one_launch(&d, stage_items(d, kStDis + l, true, false, tune), st), l,
                                 tune.dis_lanes[l]);
            };
            if (ctx)
                timed(ctx, EBOF_K_DIS_LEVEL, st, dis);
            else
                dis();
            launch_var_level(d, l, var, st);
        }
        return;
    }
    auto dis = [&] {
        for (int l = p->levels - 1; l >= 0; --l)
            launch_dis_level(one_launch(&d, stage_items(d, kStDis + l, true, false, tune), st), l, tune.dis_lanes[l]);
    };
    // masked output without the flow before masking: square 16x16 tiles, so
    // that whole waves (16x4 pixels) lie off the edge pixels and skip the sums
    Tune dt = kStageTune;
    if ((d.flags & EBOF_MASK_FLOW) && d.mask && !d.flow_keep) dt.dens_tw = 16;
    auto dens = [&] { launch_densify(one_launch(&d, stage_items(d, kStDensify, true, false, dt), st), dt.dens_tw); };
    if (ctx) {
        timed(ctx, EBOF_K_DIS_LEVEL, st, dis);
        timed(ctx, EBOF_K_DENSIFY, st, dens);
    } else {
        dis();
        dens();
    }
}

int ebof_window_surface_range(ebof_ctx* ctx, const ebof_params* p, const uint16_t* x, const uint16_t* y, int64_t n,
                              const int64_t* range_dev, uint8_t* edge_out, uint64_t* n_dropped_dev, int32_t* d2_out,
                              float* pyr_out, void* hip_stream) {
    if (ctx && (!pyr_out || !range_dev)) {
        set_error("ebof_window_surface_range: NULL pyr_out or range_dev");
        return EBOF_E_INVAL;
    }
    const hipStream_t st = (hipStream_t)hip_stream;
    WinDesc d;
    // (no time test: t0 = 0 and every event reads as t = 0, inside [0, dt))
    int rc = bin_impl(ctx, p, x, y, nullptr, n, 0, edge_out, n_dropped_dev, st, true, "ebof_window_surface_range", &d,
                      range_dev);
    if (rc) return rc;
    d.d2 = d2_out;
    d.pyr = pyr_out;
    surface_impl(ctx, p, d, st, true);
    return launch_status(ctx);
}

int ebof_flow(ebof_ctx* ctx, const ebof_params* p, const float* pyr_prev, const float* pyr_curr, const uint8_t* mask,
              float* flow_out, void* hip_stream) {
    return ebof_flow_warm(ctx, p, pyr_prev, pyr_curr, mask, nullptr, flow_out, nullptr, hip_stream);
}

int ebof_flow_warm(ebof_ctx* ctx, const ebof_params* p, const float* pyr_prev, const float* pyr_curr,
                   const uint8_t* mask, const float* flow_init, float* flow_out, float* flow_dense_out,
                   void* hip_stream) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    if ((rc = validate(p))) return rc;
    if (!pyr_prev || !pyr_curr || !flow_out) {
        set_error("ebof_flow: NULL pyramid or flow_out");
        return EBOF_E_INVAL;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    const Geom g = make_geom(*p);
    const bool refine = (p->flags & EBOF_VAR_REFINE) != 0;
    const size_t N0 = (size_t)g.W * g.H;
    Scratch scr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        Scratch* s = stage_scratch(ctx, g, st, &rc);
        if (!s) return rc;
        if (refine && !s->var) {
            const size_t bv = (size_t)kVarScratchPerPixel * N0 * sizeof(double);
            const size_t bu = 2 * (size_t)g.pyr_floats * sizeof(float);
            s->var = (double*)ctx->arena.alloc(bv);
            s->ud = (float*)ctx->arena.alloc(bu);
            if (!s->var || !s->ud) {
                ctx->arena.free(s->var);
                ctx->arena.free(s->ud);
                s->var = nullptr;
                s->ud = nullptr;
                set_error("arena full: variational refinement needs %zu bytes", bv + bu);
                return EBOF_E_NOMEM;
            }
        }
        scr = *s;
    }
    Lut lut{p->alpha, p->surface, 0, 1.0f, nullptr};
    WinDesc d;
    fill_desc(*p, g, lut, scr, &d);
    d.pyr = const_cast<float*>(pyr_curr);  // read only by these kernels
    d.pyr_prev = pyr_prev;
    d.mask = mask;
    d.flow = flow_out;
    d.flow_init = flow_init;
    d.flow_keep = flow_dense_out;
    if (refine) d.ud = scr.ud;
    flow_launches(ctx, p, d, st, refine ? scr.var : nullptr);
    return launch_status(ctx);
}

int ebof_flow_noalloc(const ebof_params* p, const float* pyr_prev, const float* pyr_curr, const uint8_t* mask,
                      float* flow_out, void* hip_stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!pyr_prev || !pyr_curr || !flow_out) {
        set_error("ebof_flow_noalloc: NULL pyramid or flow_out");
        return EBOF_E_INVAL;
    }
    const Geom g = make_geom(*p);
    if (p->flags & EBOF_VAR_REFINE) {
        set_error("ebof_flow_noalloc: the variational refinement needs scratch (use ebof_flow)");
        return EBOF_E_INVAL;
    }
    if (g.patches > kNoAllocPatches) {
        set_error("ebof_flow_noalloc: %lld patches exceed the fixed scratch of %lld", (long long)g.patches,
                  (long long)kNoAllocPatches);
        return EBOF_E_NOMEM;
    }
    Scratch scr;
    if ((rc = noalloc_scratch(&scr.puv))) return rc;
    scr.W = g.W;
    scr.H = g.H;
    scr.L = g.L;
    scr.stride = g.stride;
    Lut lut{p->alpha, p->surface, 0, 1.0f, nullptr};
    WinDesc d;
    fill_desc(*p, g, lut, scr, &d);
    d.pyr = const_cast<float*>(pyr_curr);  // read only by these kernels
    d.pyr_prev = pyr_prev;
    d.mask = mask;
    d.flow = flow_out;
    flow_launches(nullptr, p, d, (hipStream_t)hip_stream);
    return check_hip(nullptr, hipGetLastError(), "kernel launch");
}

int ebof_set_tuning(ebof_ctx* ctx, int mode, const char* cache_path) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    if (mode != EBOF_TUNE_OFF && mode != EBOF_TUNE_AUTO) {
        set_error("tuning mode %d is neither EBOF_TUNE_OFF nor EBOF_TUNE_AUTO", mode);
        return EBOF_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    std::map<std::string, Tune> loaded;
    if (cache_path && (rc = load_tunes(cache_path, &loaded))) return rc;
    // graphs were captured with the shapes in effect then
    if (ctx->batch.table_dev && (rc = check_hip(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize"))) return rc;
    for (auto& kv : ctx->batch.graphs)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    ctx->batch.graphs.clear();
    for (auto& kv : loaded) ctx->batch.tunes[kv.first] = kv.second;
    ctx->tune_mode = mode;
    ctx->tune_path = cache_path ? cache_path : "";
    return EBOF_OK;
}

int ebof_run_batch(ebof_ctx* ctx, const ebof_window* w, int32_t n, void* hip_stream) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    if (!w || n < 1 || n > EBOF_MAX_BATCH) {
        set_error("batch of %d windows outside [1, %d]", n, EBOF_MAX_BATCH);
        return EBOF_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    // scratch per batch position, reallocated when the geometry changes
    if ((int32_t)ctx->batch_slots.size() < n) ctx->batch_slots.resize(n);
    std::vector<Scratch*> scr(n);
    for (int32_t i = 0; i < n; ++i) {
        if ((rc = validate(w[i].params))) return rc;
        const Geom g = make_geom(*w[i].params);
        Scratch& s = ctx->batch_slots[i];
        if (s.W != g.W || s.H != g.H || s.L != g.L || s.stride != g.stride) {
            scratch_free(ctx, &s);
            if ((rc = scratch_alloc(ctx, g, &s, st))) return rc;
        }
        scr[i] = &s;
    }
    return run_batch_impl(ctx, ctx->batch, w, nullptr, n, st, scr.data(), kGraphLayout);
}

int ebof_timing_enable(ebof_ctx* ctx, uint32_t kernel_mask) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    ctx->timing_span = (kernel_mask & EBOF_TIMING_SPAN) != 0;
    ctx->timing_mask = kernel_mask & ((1u << EBOF_K_COUNT) - 1);
    return EBOF_OK;
}

int ebof_timing_read(ebof_ctx* ctx, int32_t kernel_id, double* total_ms, int64_t* launches) {
    int rc = ctx_ok(ctx);
    if (rc) return rc;
    if (kernel_id < 0 || kernel_id >= EBOF_K_COUNT || !total_ms || !launches) {
        set_error("ebof_timing_read: bad kernel id or NULL output");
        return EBOF_E_INVAL;
    }
    std::vector<TimedPair> pairs;
    {
        std::lock_guard<std::mutex> lk(ctx->timing_mu);
        pairs.swap(ctx->timed[kernel_id]);
    }
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto& tp : pairs) {
        if (!rc) rc = check_hip(ctx, hipEventSynchronize(tp.b), "hipEventSynchronize");
        float ms = 0.f;
        if (!rc) rc = check_hip(ctx, hipEventElapsedTime(&ms, tp.a, tp.b), "hipEventElapsedTime");
        tot += ms;
        cnt += tp.launches;
    }
    {
        std::lock_guard<std::mutex> lk(ctx->timing_mu);
        for (auto& tp : pairs) {
            ctx->event_pool.push_back(tp.a);
            ctx->event_pool.push_back(tp.b);
        }
    }
    if (rc) return rc;
    *total_ms = tot;
    *launches = cnt;
    return EBOF_OK;
}

}  // extern "C"

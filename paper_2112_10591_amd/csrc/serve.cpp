// serve.cpp -- serving runtime.
//
// A served stream keeps its recent windows' pyramids and edge images
// resident in the arena (one more than the compute lanes, in turn), one
// scratch per lane (in turn) and, with EBOF_WARM_START, its previous flow
// before masking; opening a stream is admitted only while the arena can hold
// that state.  Submitted windows are queued; their host events are copied
// into a pinned ring and sent asynchronously (copy stream) into a device ring
// in the arena.  A batch-former thread takes whatever is queued (at most one
// window per stream per batch, in submission order) as soon as a compute
// lane is free, and runs it as one launch per stage (two captured graphs,
// replayed for every batch: the preprocessing stages, then the flow stages)
// on that lane's HIP stream.  Batches go to the lanes in turn and overlap:
// a batch's flow stages wait only for the newest batch of every other lane
// to finish its preprocessing (a stream's window k+1 reads window k's
// pyramid), or to finish entirely when a window starts from its stream's
// previous flow; a lane's own batches are ordered by its stream, so that
// covers every earlier batch.  Up to one window per lane of a stream is in
// flight at once, so lanes + 1 pyramid buffers keep what a window's
// preprocessing writes apart from what earlier windows' flows read.  A
// completion thread waits for the batches in the order they were issued and
// timestamps their windows.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <set>

#include "ctx.h"

namespace ebof {

static int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr int kLanes = 3;             // compute streams; batches go to them in turn
constexpr int kMaxInflight = kLanes;  // batches on the GPU at once
// Batches of different lanes overlap (up to kLanes in flight), so a stream's
// window k+j (j < kLanes) may be preprocessed while window k's flow runs:
// kLanes + 1 resident pyramids and edge images, kLanes scratches.
constexpr int kPyrBufs = kLanes + 1;
constexpr int kServeMaxBatch = 256;   // windows per batch
constexpr size_t kPinnedRing = size_t(128) << 20;
constexpr size_t kDevRingMax = size_t(1) << 30;

static size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

struct ServeStream {
    ebof_params p;
    Geom g;
    Scratch scr[kLanes];  // scratch of consecutive windows, in turn
    int scr_next = 0;
    float* pyr[kPyrBufs] = {};
    uint8_t* edge[kPyrBufs] = {};
    float* flow = nullptr;  // EBOF_WARM_START: the newest flow before masking
    int cur = 0;  // buffer of the newest window taken into a batch
    bool has_prev = false;
    bool has_flow = false;  // the newest window computed a flow (flow is valid)
    int64_t last_t0 = 0;
    bool closing = false;
    int queued = 0;  // submitted and not completed
};

struct Pending {
    uint64_t ticket;
    int32_t sid;
    const uint16_t* x;
    const uint16_t* y;
    const int64_t* t;
    int64_t n, t0;
    bool dev_ring;     // events live in the device ring at dev_off
    size_t dev_off;
    hipEvent_t copied; // copy into the device ring (null for caller's device events)
    float* flow_out;
    uint8_t* mask_out;
};

struct TicketInfo {
    int32_t status = EBOF_E_AGAIN;
    bool done = false;
    int64_t t_submit = 0, t_done = 0;
};

struct Batch {
    hipEvent_t done = nullptr;
    hipEvent_t pre_done = nullptr;  // its preprocessing (pyramids) complete
    bool warm = false;              // a window starts from its stream's previous flow
    std::vector<uint64_t> tickets;
    std::vector<int32_t> status;
    std::vector<int32_t> sids;
    std::vector<size_t> dev_offs;  // device ring ranges to release
    std::vector<hipEvent_t> copy_events;
};

struct ServeState {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread former, reaper;
    bool stop = false;
    hipStream_t copy_stream = nullptr;
    std::map<int32_t, ServeStream> streams;
    int32_t next_sid = 1;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, TicketInfo> tickets;
    uint64_t next_ticket = 1;
    char* pinned = nullptr;
    Ring pin_ring;
    std::deque<std::pair<size_t, hipEvent_t>> pin_live;  // (offset, copy event)
    char* dev_ring = nullptr;
    size_t dev_ring_bytes = 0;
    Ring dev_ring_alloc;
    std::vector<hipEvent_t> event_pool;
    std::deque<Batch> inflight;
    hipStream_t lane[kLanes] = {};
    BatchRunner runner[kLanes];
    int next_lane = 0;
    hipEvent_t lane_done[kLanes] = {};  // completion of each lane's newest batch
    hipEvent_t lane_pre[kLanes] = {};   // ... and of its preprocessing
    int forming = 0;                 // batches taken from the queue, not yet in flight
    int32_t error = EBOF_OK;
};

static hipEvent_t get_event(ServeState* S) {
    if (!S->event_pool.empty()) {
        hipEvent_t e = S->event_pool.back();
        S->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// pinned ranges whose copy has finished go back to the ring
static void reclaim_pinned(ServeState* S) {
    while (!S->pin_live.empty()) {
        auto& f = S->pin_live.front();
        if (hipEventQuery(f.second) != hipSuccess) break;
        S->pin_ring.release(f.first);
        S->event_pool.push_back(f.second);
        S->pin_live.pop_front();
    }
}

static void former_loop(ebof_ctx* ctx, ServeState* S) {
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        S->cv_work.wait(lk, [&] { return S->stop || (!S->queue.empty() && (int)S->inflight.size() < kMaxInflight); });
        if (S->stop) break;
        std::vector<Pending> take =
            take_one_per_stream(S->queue, kServeMaxBatch, [](const Pending& q) { return q.sid; });
        const int n = (int)take.size();
        std::vector<ebof_window> win(n);
        std::vector<WinExtra> ext(n);
        std::vector<Scratch*> scr(n);
        Batch b;
        for (int i = 0; i < n; ++i) {
            const Pending& q = take[i];
            ServeStream& s = S->streams[q.sid];
            if (s.has_prev && !(s.p.flags & EBOF_CHAIN_ALWAYS) && q.t0 != s.last_t0 + s.p.dt_us)
                s.has_prev = s.has_flow = false;  // gap in time: start over
            const int nb = s.has_prev ? (s.cur + 1) % kPyrBufs : s.cur;
            const bool warm = (s.p.flags & EBOF_WARM_START) != 0;
            ebof_window& w = win[i];
            std::memset(&w, 0, sizeof w);
            w.params = &s.p;
            w.x = q.x;
            w.y = q.y;
            w.t = q.t;
            w.n = q.n;
            w.t0_us = q.t0;
            w.edge_out = s.edge[nb];
            w.pyr_out = s.pyr[nb];
            w.pyr_prev = s.has_prev ? s.pyr[s.cur] : nullptr;
            w.mask = s.has_prev ? s.edge[s.cur] : nullptr;
            w.flow_out = q.flow_out;
            // (the coarsest search level reads the previous flow before the
            // densification overwrites it: one buffer serves both)
            w.flow_dense_out = (warm && s.has_prev) ? s.flow : nullptr;
            w.flow_init = (warm && s.has_prev && s.has_flow) ? s.flow : nullptr;
            b.warm = b.warm || w.flow_init != nullptr;
            ext[i].mask_out = q.mask_out;
            ext[i].zero_out = !s.has_prev;
            scr[i] = &s.scr[s.scr_next];
            s.scr_next = (s.scr_next + 1) % kLanes;
            b.tickets.push_back(q.ticket);
            b.status.push_back(s.has_prev ? EBOF_OK : EBOF_NO_FLOW);
            b.sids.push_back(q.sid);
            if (q.dev_ring) b.dev_offs.push_back(q.dev_off);
            if (q.copied) b.copy_events.push_back(q.copied);
            s.has_flow = s.has_prev;
            s.cur = nb;
            s.has_prev = true;
            s.last_t0 = q.t0;
        }
        // launched without the serving lock, so that submissions and polls
        // are not held up behind the launches (this thread alone forms and
        // launches batches, in order)
        const int li = S->next_lane;
        S->next_lane = (li + 1) % kLanes;
        hipStream_t st = S->lane[li];
        // The flow stages read pyramids that earlier batches wrote, and a
        // warm start the flows they wrote: they wait for the newest batch of
        // every other lane, its preprocessing or all of it (a lane's older
        // batches precede it on its stream).
        std::vector<hipEvent_t> prev;
        for (int x = 0; x < kLanes; ++x)
            if (x != li && (b.warm ? S->lane_done[x] : S->lane_pre[x]))
                prev.push_back(b.warm ? S->lane_done[x] : S->lane_pre[x]);
        b.done = get_event(S);
        b.pre_done = get_event(S);
        S->lane_done[li] = b.done;
        S->lane_pre[li] = b.pre_done;
        ++S->forming;
        lk.unlock();
        // the batch's event copies were queued in order on the copy stream:
        // waiting for the last one covers all of them
        int rc = EBOF_OK;
        if (!b.copy_events.empty())
            rc = check_hip(ctx, hipStreamWaitEvent(st, b.copy_events.back(), 0), "hipStreamWaitEvent");
        // between this batch's preprocessing and its flow stages: mark the
        // preprocessing done, then wait for the previous batch's part this
        // flow reads (unless that has completed already)
        const std::function<int(hipStream_t)> after_prev = [&](hipStream_t s_) {
            int r = b.pre_done ? check_hip(ctx, hipEventRecord(b.pre_done, s_), "hipEventRecord") : EBOF_OK;
            for (hipEvent_t e : prev)
                if (!r && hipEventQuery(e) != hipSuccess)
                    r = check_hip(ctx, hipStreamWaitEvent(s_, e, 0), "hipStreamWaitEvent");
            return r;
        };
        if (rc == EBOF_OK) {
            std::lock_guard<std::mutex> g(ctx->mu);
            rc = run_batch_impl(ctx, S->runner[li], win.data(), ext.data(), n, st, scr.data(), kGraphUniversal,
                                &after_prev);
        }
        if (rc == EBOF_OK && b.done) rc = check_hip(ctx, hipEventRecord(b.done, st), "hipEventRecord");
        lk.lock();
        if (rc != EBOF_OK || !b.done || !b.pre_done) {
            if (rc == EBOF_OK) rc = EBOF_E_DEVICE;
            for (auto& st_ : b.status) st_ = rc;
            S->error = rc;
        }
        S->inflight.push_back(std::move(b));
        --S->forming;
        S->cv_done.notify_all();
    }
}

static void reaper_loop(ServeState* S) {
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        S->cv_done.wait(lk, [&] { return S->stop || !S->inflight.empty(); });
        if (S->inflight.empty()) {
            if (S->stop) break;
            continue;
        }
        hipEvent_t ev = S->inflight.front().done;
        lk.unlock();
        bool failed = !ev || hipEventSynchronize(ev) != hipSuccess;
        const int64_t t = now_ns();
        lk.lock();
        Batch b = std::move(S->inflight.front());
        S->inflight.pop_front();
        for (size_t i = 0; i < b.tickets.size(); ++i) {
            auto it = S->tickets.find(b.tickets[i]);
            if (it != S->tickets.end()) {
                it->second.done = true;
                it->second.status = failed ? EBOF_E_DEVICE : b.status[i];
                it->second.t_done = t;
            }
            auto st = S->streams.find(b.sids[i]);
            if (st != S->streams.end()) --st->second.queued;
        }
        for (size_t off : b.dev_offs) S->dev_ring_alloc.release(off);
        for (hipEvent_t e : b.copy_events) S->event_pool.push_back(e);
        // (a completed batch needs no more waiting on: its events go back to
        // the pool, and the lanes forget them)
        for (int x = 0; x < kLanes; ++x) {
            if (S->lane_done[x] == b.done) S->lane_done[x] = nullptr;
            if (S->lane_pre[x] == b.pre_done) S->lane_pre[x] = nullptr;
        }
        if (b.done) S->event_pool.push_back(b.done);
        if (b.pre_done) S->event_pool.push_back(b.pre_done);
        if (failed) S->error = EBOF_E_DEVICE;
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
}

static int serve_init(ebof_ctx* ctx) {
    if (ctx->serve) return EBOF_OK;
    auto* S = new ServeState();
    int rc = EBOF_OK;
    for (int i = 0; i < kLanes && !rc; ++i) rc = queue_stream_create(ctx, &S->lane[i]);
    if (!rc) rc = check_hip(ctx, hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking), "hipStreamCreate");
    if (!rc) rc = check_hip(ctx, hipHostMalloc((void**)&S->pinned, kPinnedRing, hipHostMallocDefault), "hipHostMalloc");
    if (!rc) {
        std::lock_guard<std::mutex> g(ctx->mu);
        S->dev_ring_bytes = std::min(kDevRingMax, (ctx->arena.bytes_free() / 4) & ~size_t(255));
        S->dev_ring = S->dev_ring_bytes ? (char*)ctx->arena.alloc(S->dev_ring_bytes) : nullptr;
        if (!S->dev_ring) {
            set_error("arena too small for the serving event ring");
            rc = EBOF_E_NOMEM;
        }
    }
    if (rc) {
        for (hipStream_t l : S->lane)
            if (l) (void)hipStreamDestroy(l);
        if (S->copy_stream) (void)hipStreamDestroy(S->copy_stream);
        if (S->pinned) (void)hipHostFree(S->pinned);
        delete S;
        return rc;
    }
    S->pin_ring.init(kPinnedRing);
    S->dev_ring_alloc.init(S->dev_ring_bytes);
    ctx->serve = S;
    S->former = std::thread(former_loop, ctx, S);
    S->reaper = std::thread(reaper_loop, S);
    return EBOF_OK;
}

void serve_shutdown(ebof_ctx* ctx) {
    ServeState* S = ctx->serve;
    if (!S) return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->queue.empty() && S->inflight.empty() && S->forming == 0; });
        S->stop = true;
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
    S->former.join();
    S->reaper.join();
    for (hipStream_t l : S->lane) (void)hipStreamSynchronize(l);
    (void)hipStreamSynchronize(S->copy_stream);
    for (BatchRunner& r : S->runner) runner_release(r);
    for (auto& pl : S->pin_live) (void)hipEventDestroy(pl.second);
    for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
    for (hipStream_t l : S->lane) (void)hipStreamDestroy(l);
    (void)hipStreamDestroy(S->copy_stream);
    (void)hipHostFree(S->pinned);
    delete S;
    ctx->serve = nullptr;
}

static void free_stream(ebof_ctx* ctx, ServeStream& s) {
    std::lock_guard<std::mutex> g(ctx->mu);
    for (int i = 0; i < kPyrBufs; ++i) {
        ctx->arena.free(s.pyr[i]);
        ctx->arena.free(s.edge[i]);
        s.pyr[i] = nullptr;
        s.edge[i] = nullptr;
    }
    ctx->arena.free(s.flow);
    s.flow = nullptr;
    for (Scratch& sc : s.scr) scratch_free(ctx, &sc);
}

}  // namespace ebof

using namespace ebof;

extern "C" {

int ebof_stream_open(ebof_ctx* ctx, const ebof_params* p, int32_t* stream_id) {
    if (!ctx || !stream_id) {
        set_error("ebof_stream_open: NULL ctx or stream_id");
        return EBOF_E_INVAL;
    }
    if (ctx->failed) return EBOF_E_DEVICE;
    int rc = validate_params(p);
    if (rc) return rc;
    if (p->flags & EBOF_VAR_REFINE) {
        set_error("ebof_stream_open: the variational refinement runs in the stage calls only");
        return EBOF_E_INVAL;
    }
    if ((rc = serve_init(ctx))) return rc;
    ServeState* S = ctx->serve;
    ServeStream s;
    s.p = *p;
    s.g = make_geom(*p);
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        Lut lut;
        if ((rc = lut_for(ctx, p->alpha, p->surface, &lut))) return rc;
        const size_t N = (size_t)p->width * p->height;
        const bool warm = (p->flags & EBOF_WARM_START) != 0;
        bool ok = true;
        for (int i = 0; i < kPyrBufs; ++i) {
            s.pyr[i] = (float*)ctx->arena.alloc(s.g.pyr_floats * sizeof(float));
            s.edge[i] = (uint8_t*)ctx->arena.alloc(N);
            ok = ok && s.pyr[i] && s.edge[i];
        }
        if (warm) {
            s.flow = (float*)ctx->arena.alloc(2 * N * sizeof(float));
            ok = ok && s.flow;
        }
        for (Scratch& sc : s.scr)
            if (ok) ok = scratch_alloc(ctx, s.g, &sc, nullptr) == EBOF_OK;
        if (!ok) {
            for (int i = 0; i < kPyrBufs; ++i) {
                ctx->arena.free(s.pyr[i]);
                ctx->arena.free(s.edge[i]);
            }
            ctx->arena.free(s.flow);
            for (Scratch& sc : s.scr) scratch_free(ctx, &sc);
            set_error("arena full: a %dx%d stream needs %zu bytes of resident state, %zu free", p->width, p->height,
                      kPyrBufs * ((size_t)s.g.pyr_floats * 4 + N) + (warm ? 8 * N : 0) +
                          kLanes * (size_t)ebof_window_scratch_bytes(p),
                      ctx->arena.bytes_free());
            return EBOF_E_NOMEM;
        }
    }
    std::lock_guard<std::mutex> lk(S->mu);
    const int32_t sid = S->next_sid++;
    S->streams[sid] = s;
    *stream_id = sid;
    return EBOF_OK;
}

int ebof_stream_close(ebof_ctx* ctx, int32_t stream_id) {
    if (!ctx || !ctx->serve) {
        set_error("ebof_stream_close: no served stream");
        return EBOF_E_NOTFOUND;
    }
    ServeState* S = ctx->serve;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->streams.find(stream_id);
    if (it == S->streams.end()) {
        set_error("ebof_stream_close: unknown stream %d", stream_id);
        return EBOF_E_NOTFOUND;
    }
    it->second.closing = true;
    S->cv_done.wait(lk, [&] {
        auto j = S->streams.find(stream_id);
        return j->second.queued == 0;
    });
    ServeStream s = it->second;
    S->streams.erase(stream_id);
    lk.unlock();
    free_stream(ctx, s);
    return EBOF_OK;
}

int ebof_submit(ebof_ctx* ctx, int32_t stream_id, const uint16_t* x, const uint16_t* y, const int64_t* t, int64_t n,
                int64_t t0_us, int events_on_device, float* flow_out_dev, uint8_t* mask_out_dev, uint64_t* ticket) {
    if (!ctx || !ctx->serve || !ticket || !flow_out_dev || n < 0 || (n > 0 && (!x || !y || !t))) {
        set_error("ebof_submit: bad arguments");
        return (!ctx || !ctx->serve) ? EBOF_E_STATE : EBOF_E_INVAL;
    }
    ServeState* S = ctx->serve;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->error) {
        set_error("serving failed earlier (device error)");
        return S->error;
    }
    auto it = S->streams.find(stream_id);
    if (it == S->streams.end()) {
        set_error("ebof_submit: unknown stream %d", stream_id);
        return EBOF_E_NOTFOUND;
    }
    ServeStream& s = it->second;
    if (s.closing) {
        set_error("ebof_submit: stream %d is closing", stream_id);
        return EBOF_E_STATE;
    }
    if (t0_us > INT64_MAX - s.p.dt_us) {
        set_error("ebof_submit: t0 + dt overflows");
        return EBOF_E_INVAL;
    }
    Pending q;
    std::memset(&q, 0, sizeof q);
    q.sid = stream_id;
    q.n = n;
    q.t0 = t0_us;
    q.flow_out = flow_out_dev;
    q.mask_out = mask_out_dev;
    if (events_on_device || n == 0) {
        q.x = x;
        q.y = y;
        q.t = t;
    } else {
        // host events: pinned ring -> device ring, asynchronously
        reclaim_pinned(S);
        const size_t bx = a256(2 * (size_t)n), bt = a256(8 * (size_t)n);
        const size_t len = 2 * bx + bt;
        size_t doff, poff;
        if (len > S->dev_ring_bytes || len > kPinnedRing) {
            set_error("ebof_submit: %lld events (%zu bytes staged) exceed the event ring (%zu bytes device, %zu "
                      "pinned)",
                      (long long)n, len, S->dev_ring_bytes, kPinnedRing);
            return EBOF_E_NOMEM;
        }
        if (!S->dev_ring_alloc.alloc(len, &doff)) {
            set_error("ebof_submit: device event ring full");
            return EBOF_E_AGAIN;
        }
        if (!S->pin_ring.alloc(len, &poff)) {
            S->dev_ring_alloc.release(doff);
            set_error("ebof_submit: pinned staging full");
            return EBOF_E_AGAIN;
        }
        char* hp = S->pinned + poff;
        std::memcpy(hp, x, 2 * (size_t)n);
        std::memcpy(hp + bx, y, 2 * (size_t)n);
        std::memcpy(hp + 2 * bx, t, 8 * (size_t)n);
        char* dp = S->dev_ring + doff;
        hipEvent_t ev = get_event(S);
        hipEvent_t ev_pin = get_event(S);
        int rc = EBOF_OK;
        if (!ev || !ev_pin) rc = check_hip(ctx, hipErrorOutOfMemory, "hipEventCreate");
        if (!rc) rc = check_hip(ctx, hipMemcpyAsync(dp, hp, len, hipMemcpyHostToDevice, S->copy_stream), "hipMemcpyAsync");
        if (!rc) rc = check_hip(ctx, hipEventRecord(ev, S->copy_stream), "hipEventRecord");
        if (!rc) rc = check_hip(ctx, hipEventRecord(ev_pin, S->copy_stream), "hipEventRecord");
        if (rc) {
            S->dev_ring_alloc.release(doff);
            S->pin_ring.release(poff);
            return rc;
        }
        S->pin_live.push_back({poff, ev_pin});
        q.x = (const uint16_t*)dp;
        q.y = (const uint16_t*)(dp + bx);
        q.t = (const int64_t*)(dp + 2 * bx);
        q.dev_ring = true;
        q.dev_off = doff;
        q.copied = ev;
    }
    q.ticket = S->next_ticket++;
    TicketInfo ti;
    ti.t_submit = now_ns();
    S->tickets[q.ticket] = ti;
    ++s.queued;
    S->queue.push_back(q);
    *ticket = q.ticket;
    S->cv_work.notify_all();
    return EBOF_OK;
}

int ebof_poll(ebof_ctx* ctx, uint64_t ticket, int32_t* status, int64_t* latency_ns) {
    if (!ctx || !ctx->serve || !status) {
        set_error("ebof_poll: bad arguments");
        return EBOF_E_NOTFOUND;
    }
    ServeState* S = ctx->serve;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) {
        set_error("ebof_poll: unknown ticket %llu", (unsigned long long)ticket);
        return EBOF_E_NOTFOUND;
    }
    if (!it->second.done) return EBOF_E_AGAIN;
    *status = it->second.status;
    if (latency_ns) *latency_ns = it->second.t_done - it->second.t_submit;
    S->tickets.erase(it);
    return EBOF_OK;
}

int ebof_drain(ebof_ctx* ctx) {
    if (!ctx) return EBOF_E_INVAL;
    ServeState* S = ctx->serve;
    if (!S) return EBOF_OK;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->queue.empty() && S->inflight.empty() && S->forming == 0; });
    return S->error;
}

}  // extern "C"

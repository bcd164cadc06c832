// ctx.h -- host-side context of the library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ebof_dev.h"
#include "hostlogic.h"

namespace ebof {

void set_error(const char* fmt, ...);

// Geometry of one parameter set.
struct Geom {
    int32_t W, H, L, stride;
    LevelGeom lv[kMaxLevels];
    int64_t pyr_floats;
    int64_t patches;
};
Geom make_geom(const ebof_params& p);

// Scratch of one window (staging image, column masks, column distances,
// patch displacements) in the arena.
struct Scratch {
    int32_t W = 0, H = 0, L = 0, stride = 0;
    uint8_t* e_raw = nullptr;
    uint64_t* colmask = nullptr;
    uint16_t* g = nullptr;
    float2* puv = nullptr;
    double* var = nullptr;  // variational refinement: working planes (allocated on first use)
    float* ud = nullptr;    // ... and every level's refined dense flow
    uint32_t stamp = 0;
    bool needs_zero = true;
    // next stamp; sets needs_zero when the counter wraps
    uint32_t next_stamp() {
        if (++stamp > 255) {
            stamp = 1;
            needs_zero = true;
        }
        return stamp;
    }
};

struct Lut {
    float alpha;
    int32_t kind;  // EBOF_SURFACE_*
    int32_t n;     // entries (0: the surface does not saturate, no table)
    float sat;     // value from squared distance n on
    float* dev;
};

struct TimedPair {
    hipEvent_t a, b;  // stamped before and after the launches they bracket
    int launches;     // one, or in span mode those of one call
};

// Device descriptor table + pinned staging ring + captured graphs of one
// batched launcher (the public batch call and the server each own one).
struct BatchRunner {
    char* table_dev = nullptr;
    size_t table_bytes = 0;
    // graphs are captured on this non-blocking stream and launched on the
    // caller's: a capture on a blocking stream would fail other threads'
    // work on the legacy stream meanwhile
    hipStream_t capture = nullptr;
    struct Pinned {
        char* host = nullptr;
        hipEvent_t done = nullptr;
        bool used = false;
    };
    std::vector<Pinned> pinned;
    int pinned_next = 0;
    std::map<std::string, hipGraphExec_t> graphs;
    std::map<std::string, Tune> tunes;  // launch shapes per batch layout (autotuner)
};

// Scratch of the evaluation calls: two int64 images and the partial sums.
struct EvalScratch {
    long long* img = nullptr;
    char* part = nullptr;
};

// Extra per-window outputs of the served form.
struct WinExtra {
    uint8_t* mask_out = nullptr;
    bool zero_out = false;
};

enum GraphMode { kGraphNone = 0, kGraphLayout = 1, kGraphUniversal = 2 };

struct ServeState;  // serving runtime (serve.cpp)

}  // namespace ebof

struct ebof_ctx {
    int device = 0;
    ebof::Arena arena;
    bool failed = false;
    std::mutex mu;  // guards arena, luts, scratch maps against the server thread

    std::vector<ebof::Lut> luts;
    // stage-call scratch per (W, H, levels, stride, HIP stream): calls on
    // different streams may overlap, calls on one stream are ordered by it
    std::map<std::tuple<int, int, int, int, uintptr_t>, ebof::Scratch> stage_scratch;
    // evaluation-call scratch per (pixels, HIP stream)
    std::map<std::pair<int64_t, uintptr_t>, ebof::EvalScratch> eval_scratch;
    // update-prediction filter work memory per (width, height, layers, stream)
    std::map<std::tuple<int32_t, int32_t, int32_t, uintptr_t>, float*> filter_scratch;
    // adaptive-window scratch per HIP stream
    std::map<uintptr_t, void*> window_scratch;

    // batched form
    std::vector<ebof::Scratch> batch_slots;
    ebof::BatchRunner batch;
    bool use_graphs = true;
    int tune_mode = EBOF_TUNE_AUTO;  // batched launch shapes: defaults or timed candidates
    std::string tune_path;           // cache file of tuned shapes ("" = none)

    // timing
    std::atomic<uint32_t> timing_mask{0};
    std::atomic<bool> timing_span{false};  // one pair per call, not per launch
    std::mutex timing_mu;  // guards timed[] and event_pool (launches happen outside mu)
    std::vector<ebof::TimedPair> timed[EBOF_K_COUNT];
    std::vector<hipEvent_t> event_pool;

    ebof::ServeState* serve = nullptr;  // owned; released by serve_shutdown

    // cross-stream ordering counters (signal memory, taken lazily from a
    // process-wide pool and returned to it by ebof_destroy)
    std::mutex signal_mu;
    uint32_t* signals[EBOF_SIGNAL_SLOTS] = {};
    std::vector<hipStream_t> owned_streams;  // ebof_stream_create (guarded by signal_mu)
};

namespace ebof {
// helpers shared by api.cpp and serve.cpp
int lut_for(ebof_ctx* ctx, float alpha, int32_t kind, Lut* out);
int scratch_alloc(ebof_ctx* ctx, const Geom& g, Scratch* s, hipStream_t stream);
void scratch_free(ebof_ctx* ctx, Scratch* s);
void fill_desc(const ebof_params& p, const Geom& g, const Lut& lut, const Scratch& s, WinDesc* d);
// between: when not null, called with the stream after the batch's
// preprocessing stages and before its flow stages (to order the flow after
// other work); the two parts are then launched (or captured) separately.
int run_batch_impl(ebof_ctx* ctx, BatchRunner& br, const ebof_window* w, const WinExtra* extra, int32_t n,
                   hipStream_t stream, Scratch* const* scr, int graph_mode,
                   const std::function<int(hipStream_t)>* between = nullptr);
void runner_release(BatchRunner& br);
int validate_params(const ebof_params* p);
int queue_stream_create(ebof_ctx* ctx, hipStream_t* out);
int check_hip(ebof_ctx* ctx, hipError_t e, const char* what);
void serve_shutdown(ebof_ctx* ctx);
}  // namespace ebof

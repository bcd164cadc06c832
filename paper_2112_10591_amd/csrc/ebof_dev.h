// ebof_dev.h -- descriptors shared by the HIP kernels and the host side of
// the library.  One WinDesc describes one window of one stream: its
// parameters, its input events and every buffer its stages read or write.
// A kernel launch either carries a single WinDesc by value (the stage calls)
// or reads a device table of them (the batched form), in which case each
// launch covers every window of the batch and a block finds its window by a
// binary search over the stage's prefix sum of per-window work items.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ebof.h"

namespace ebof {

constexpr int kMaxLevels = EBOF_MAX_LEVELS;
constexpr int kPatch = EBOF_PATCH;
constexpr uint16_t kGInf = 0xFFFF;  // "no edge pixel in this column"
constexpr int kBlock = 256;         // threads per block of every kernel but the pyramid's
#ifndef EBOF_PYR_TILE
#define EBOF_PYR_TILE 8
#endif
constexpr int kPyrTile = EBOF_PYR_TILE;               // pyramid: deepest level's tile edge per block
constexpr int kPyrBlock = kPyrTile >= 8 ? 512 : 256;  // threads per block of the pyramid chain

// work-item granularity of each stage
constexpr int kEventsPerItem = 512;   // scatter: events per block
constexpr int kTile = 64;             // denoise/fill: 64 wide ...
constexpr int kTileH = 32;            // ... and 32 tall per block
constexpr int kChunk = 64;            // column-mask chunk: 64 rows per word
constexpr int kPyrChain = 3;          // pyramid: levels built per launch
constexpr int kPatchesPerItem = 16;   // inverse search: patches per item row
constexpr int kZeroBytesPerItem = 4096;
constexpr int kRowSeg = 256;          // EDT row pass: pixels per item row
constexpr int kRowReach = 64;         // EDT row pass: columns staged each side of a segment
constexpr int kRowUnroll = 4;         // EDT row pass: radii per search step (divides kRowReach)
constexpr int kLutLds = 1024;         // EDT row pass: surface tables up to this size sit in LDS

// Allocation-free flow call: its patch displacements live in a fixed device
// array of this many float2 (8 MiB; 3840x2160 at stride 4 with 4 levels needs
// about 690k).
constexpr int64_t kNoAllocPatches = EBOF_NOALLOC_MAX_PATCHES;
constexpr int kNoAllocMaxDevices = 64;

struct LevelGeom {
    int32_t w, h;      // level size
    int32_t pnx, pny;  // patch grid
    int64_t off;       // first float of the level in a pyramid
    int64_t poff;      // first patch of the level in the patch-flow array
};

struct WinDesc {
    int32_t W, H, L;
    int32_t n_d, n_f;
    int32_t stride, iters;
    uint32_t flags;
    float lambda;
    int32_t lut_n;      // squared distances below lut_n read lut[], others lut_sat
    int32_t lut_r;      // smallest r with r*r >= lut_n
    int32_t surf_kind;  // EBOF_SURFACE_*: LINEAR and LOG are computed, not looked up
    float lut_sat;
    const float* lut;
    // events of the window, SoA, and the half-open window [t0, t1)
    const uint16_t* ex;
    const uint16_t* ey;
    const int64_t* et;
    int64_t n_ev, t0, t1;
    const int64_t* range;  // device [i0, i1): bin these events, no time test (n_ev: the arrays' length)
    uint32_t stamp;     // value marking this window's pixels in e_raw
    uint32_t pad0;
    // buffers
    uint8_t* e_raw;     // W*H staging of the scattered events (stamps)
    uint8_t* e_df;      // W*H denoised and filled edge image (0/1)
    uint64_t* colmask;  // ceil(H/64) x W column bit masks of e_df
    uint16_t* g;        // W*H distance to the nearest edge in the column
    int32_t* d2;        // W*H squared distance, or null
    float* pyr;         // this window's pyramid (level 0 = surface)
    const float* pyr_prev;  // reference pyramid for the flow, or null
    const uint8_t* mask;    // reference edge image for EBOF_MASK_FLOW, or null
    float* flow;            // 2*W*H output flow
    uint8_t* mask_out;      // W*H copy of the reference edge image, or null
    uint32_t zero_out;      // no reference window: flow and mask_out written as 0
    uint32_t pad1;
    float2* puv;            // patch displacements (u, v), all levels
    const float* flow_init; // level-0 flow of the previous pair (2*W*H): the
                            // coarsest level's start, or null (start at 0)
    float* flow_keep;       // 2*W*H copy of the flow before masking, or null
    float* ud;              // variational refinement: every level's refined dense flow
                            // (level l's u and v planes at 2 * lv[l].off), or null
    unsigned long long* n_dropped;  // optional counter
    LevelGeom lv[kMaxLevels];
};

// A window whose squared distance is not exported and whose surface is
// looked up (it saturates from lut_n on) needs column distances only up to
// lut_r: the row pass then forms them itself from the column bit masks,
// capped at lut_r, and the column pass has no work (k_edt_rows).
__host__ __device__ inline bool edt_local(const WinDesc& d) {
    return d.d2 == nullptr && d.surf_kind != EBOF_SURFACE_LINEAR && d.surf_kind != EBOF_SURFACE_LOG &&
           d.lut_n > 0 && d.lut_r <= kRowReach;
}

// Stages of the batched pipeline; each has a prefix sum of work items.
enum Stage : int32_t {
    kStZero = 0,
    kStScatter = 1,
    kStDenoise = 2,
    kStPack = 3,
    kStCols = 4,
    kStRows = 5,
    kStPyr = 6,                      // + chain index (levels 1-3, 4-6, 7)
    kStDis = kStPyr + kMaxLevels - 1,  // + l, levels 0 .. 7
    kStDensify = kStDis + kMaxLevels,
    kNumStages = kStDensify + 1
};

// Batched launch arguments (device table form).  The table holds the window
// count, then per window i (and i = nwin) the running sums of every stage's
// items (prefix[i * kNumStages + stage]), then the descriptors.  Reading the
// count from memory lets one captured graph serve batches of any size.
struct BatchArgs {
    const WinDesc* tab;     // descriptors
    const int32_t* prefix;  // prefix[i * kNumStages + stage]
    const int32_t* nwin;    // number of windows
    int32_t stage;
    int32_t pad;
};
constexpr size_t kTableHeader = 256;  // bytes before the prefix sums

// Host-side launch description.
struct Launch {
    const WinDesc* one;  // single window (host copy, passed by value)
    BatchArgs ba;        // used when batch is true
    bool batch;
    int32_t total;       // items (single-window form)
    int32_t grid;        // blocks
    hipStream_t stream;
    hipEvent_t ev_start = nullptr;  // when set: events recorded right before
    hipEvent_t ev_stop = nullptr;   // and right after the kernel
};

// Launch shapes the autotuner chooses among.  None of them changes what a
// window computes: they decide how work is cut into items and how many
// blocks a batched launch runs.
struct Tune {
    int32_t rows_nr = 4;    // k_edt_rows: rows per item (1, 2, 4 or 8)
    int32_t dens_tw = 64;   // k_densify: tile width (16, 64, 128 or 256), kBlock / dens_tw rows
    int32_t dis_lanes[kMaxLevels] = {};  // k_dis_level: lanes per patch (8 or 4; 0: by size)
    int32_t grid[kNumStages] = {};       // batched launch blocks per stage (0: the default)
};
inline bool tune_valid(const Tune& t) {
    const bool nr = t.rows_nr == 1 || t.rows_nr == 2 || t.rows_nr == 4 || t.rows_nr == 8;
    const bool tw = t.dens_tw == 16 || t.dens_tw == 64 || t.dens_tw == 128 || t.dens_tw == 256;
    for (int l = 0; l < kMaxLevels; ++l)
        if (t.dis_lanes[l] != 0 && t.dis_lanes[l] != 4 && t.dis_lanes[l] != 8) return false;
    for (int s = 0; s < kNumStages; ++s)
        if (t.grid[s] < 0 || t.grid[s] > (1 << 20)) return false;
    return nr && tw;
}
// A level with at least this many patches in one launch uses 4 lanes per
// patch by default (throughput), a smaller one 8 (latency).
constexpr int64_t kDisWideMinPatches = 16384;
// Resolves dis_lanes left at 0 from the level's patch count over the windows
// (one launch per level serves them all, so one choice per level).
inline void resolve_dis_lanes(Tune& t, const WinDesc* d, int n) {
    for (int l = 0; l < kMaxLevels; ++l) {
        if (t.dis_lanes[l]) continue;
        int64_t patches = 0;
        for (int i = 0; i < n; ++i)
            if (l < d[i].L) patches += (int64_t)d[i].lv[l].pnx * d[i].lv[l].pny;
        t.dis_lanes[l] = patches >= kDisWideMinPatches ? 4 : 8;
    }
}

// Work items of one stage for one window (0 when the stage does not apply).
int32_t stage_items(const WinDesc& d, int stage, bool has_flow, bool zero, const Tune& t);

// stage item counts of a window described by d
inline bool desc_has_flow(const WinDesc& d) { return d.pyr_prev != nullptr; }

void launch_zero(const Launch& L);
void launch_scatter(const Launch& L);
void launch_denoise_fill(const Launch& L, bool pack);
void launch_pack_cols(const Launch& L);
void launch_edt_cols(const Launch& L);
void launch_edt_rows(const Launch& L, int rows_nr);
void launch_pyr_chain(const Launch& L, int from);
void launch_dis_level(const Launch& L, int level, int lanes);
void launch_densify(const Launch& L, int tile_w);
// variational refinement of level l (single window, after its inverse search)
void launch_var_level(const WinDesc& d, int l, double* scratch, hipStream_t st);
constexpr int kVarScratchPerPixel = 18;  // doubles per level-0 pixel

// Device address, on the current HIP device, of the fixed patch-displacement
// array of the allocation-free flow call (kNoAllocPatches float2); looked up
// once per device.  EBOF_OK, or EBOF_E_DEVICE with the error set.
int noalloc_scratch(float2** out);
void set_error(const char* fmt, ...);

}  // namespace ebof

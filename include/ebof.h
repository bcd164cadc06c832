/*
 * ebof.h -- C ABI of the MI355X (gfx950) event-based optical-flow hot path.
 *
 * The method is the one of Brebion, Moreau and Davoine, "Real-Time Optical
 * Flow for Vehicular Perception with Low- and High-Resolution Event Cameras"
 * (arXiv 2112.10591): events of one time window become a binary edge image
 * (Sec. III-A), which is denoised and filled (Sec. III-B, Alg. 1 and 2); the
 * exact Euclidean distance to the closest edge pixel turns it into the
 * inverse exponential distance surface (Sec. III-C, eq. 1-3); a frame-based
 * dense flow then runs between consecutive surfaces and is restricted to the
 * edge pixels (Sec. III-D).  The frame-based flow here is dense inverse
 * search (coarse-to-fine patch inverse search with Lucas-Kanade refinement
 * and patch densification), which Sec. III-D allows in place of the paper's
 * own choice.
 *
 * Conventions
 *   - Every pointer argument named *_dev or documented "device" is device
 *     memory of the context's GPU, owned by the caller; the library never
 *     frees it.  Stage calls are asynchronous on the caller's HIP stream
 *     (passed as void*, NULL = the null stream): inputs must stay alive and
 *     outputs untouched until that stream reaches the work.
 *   - Images are row-major with pitch = width: pixel (x, y) is element
 *     y*width + x.  x grows to the right, y downwards.
 *   - A pyramid of L levels is one float array: level 0 (width x height)
 *     first, then level 1 ((width+1)/2 x (height+1)/2), and so on, each
 *     level tightly packed.  ebof_pyramid_floats() gives its length P.
 *   - A flow is two float planes, u (along +x) then v (along +y), each
 *     width*height, in pixels of level 0.
 *   - Every call returns a status (EBOF_OK or a negative EBOF_E_*); nothing
 *     throws across the ABI.  On failure ebof_last_error() describes it.
 *   - All library-owned device memory comes from the caller's arena given to
 *     ebof_create(); the library calls no device allocator after that,
 *     except for pinned host staging of the serving calls.
 */
#ifndef EBOF_H
#define EBOF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define EBOF_OK 0
#define EBOF_NO_FLOW 1      /* served window accepted, no previous window yet */
#define EBOF_E_INVAL (-1)   /* bad argument or parameter                      */
#define EBOF_E_NOMEM (-2)   /* the arena cannot hold what the call needs      */
#define EBOF_E_AGAIN (-3)   /* not done yet / queue full: try again later     */
#define EBOF_E_NOTFOUND (-4)/* unknown stream id or ticket                    */
#define EBOF_E_DEVICE (-5)  /* a HIP call failed; the context is unusable     */
#define EBOF_E_STATE (-6)   /* call not allowed in the current state          */

/* ---- limits ------------------------------------------------------------ */
#define EBOF_MAX_DIM 8192   /* width and height are at most this            */
#define EBOF_MIN_DIM 8      /* and at least the patch size                  */
#define EBOF_MAX_LEVELS 8
#define EBOF_PATCH 8        /* the only supported patch size                */
#define EBOF_MAX_BATCH 1024 /* windows per ebof_run_batch call              */

/* ---- flags of ebof_params.flags ------------------------------------------ */
#define EBOF_MASK_FLOW 1u   /* write 0 flow outside the mask (Sec. III-D)   */
#define EBOF_CHAIN_ALWAYS 2u /* served stream: a window always pairs with the
                                stream's previous window, whatever its t0 (by
                                default a t0 other than previous t0 + dt_us
                                starts the stream over, EBOF_NO_FLOW)       */
#define EBOF_WARM_START 4u  /* served stream: the coarsest level starts from
                                the stream's previous flow (kept resident),
                                as ebof_flow_warm does, instead of from 0   */
#define EBOF_VAR_REFINE 8u  /* stage calls (ebof_flow, ebof_flow_warm): each
                                level's dense flow is refined variationally
                                before the next level starts (the third stage
                                of dense inverse search; see ebof_flow)      */

typedef struct ebof_ctx ebof_ctx; /* opaque, library-owned */

/* Parameters of one sensor / stream.  Plain data; struct_size must be
 * sizeof(ebof_params) (lets the struct grow). */
typedef struct {
    uint32_t struct_size;
    int32_t width, height; /* sensor size in pixels                        */
    int64_t dt_us;         /* window length Delta-T (Sec. III-A)             */
    int32_t n_d;           /* denoising threshold N_d, Alg. 1; 0 disables   */
    int32_t n_f;           /* filling threshold N_f, Alg. 2; 5 disables     */
    float alpha;           /* spreading parameter of eq. (1), > 0           */
    int32_t levels;        /* pyramid levels L, 1..EBOF_MAX_LEVELS           */
    int32_t patch;         /* patch size, must be EBOF_PATCH                 */
    int32_t stride;        /* patch grid stride, 1..8                        */
    int32_t iters;         /* inverse-search iterations per patch, 0..1024   */
    float lambda_reg;      /* Tikhonov term added to the patch Hessian, > 0  */
    uint32_t flags;        /* EBOF_MASK_FLOW | EBOF_CHAIN_ALWAYS | EBOF_WARM_START
                              | EBOF_VAR_REFINE */
    int32_t surface;       /* EBOF_SURFACE_*: the distance surface (Sec. IV-B) */
} ebof_params;

/* Distance surfaces of ebof_params.surface, from the squared distance D2 with
 * d = sqrt(D2), each rounded once to float (the ablations of Sec. IV-B):
 * eq. (1), the proposed one, 1 - exp(-d / alpha); DS_L, d; DS_LB, min(d,
 * d_sat) with d_sat = alpha ln 255 (eq. 3: 6 px in the paper); DS_Log,
 * ln(d + 1).  The no-edge value D2 = INT32_MAX goes through the same
 * formula. */
#define EBOF_SURFACE_EXP 0
#define EBOF_SURFACE_LINEAR 1
#define EBOF_SURFACE_BOUNDED 2
#define EBOF_SURFACE_LOG 3

/* Defaults of Sec. IV-A for a sensor of the given size: N_d = 1, N_f = 4 up to
 * 100k pixels (the 346x260 setting), N_d = 2, N_f = 3 above (1280x720);
 * alpha = 1.08 (d_sat = 6 px, eq. 3); dt = 10 ms; levels = 3 up to 100k
 * pixels, else 4 (each level at least 8 px); patch 8, stride 4, 16 iterations,
 * lambda_reg 0.3, no flags, surface EBOF_SURFACE_EXP.  Returns EBOF_E_INVAL for a size out of range. */
int ebof_params_default(int32_t width, int32_t height, ebof_params *out);

/* EBOF_OK when the parameters are usable, else EBOF_E_INVAL.  Checks: sizes
 * in [EBOF_MIN_DIM, EBOF_MAX_DIM], every pyramid level at least the patch
 * size, n_d and n_f in [0, 5], alpha and lambda_reg finite and > 0, alpha
 * small enough for a squared-distance lookup table of at most 2^22 entries,
 * patch == 8, stride in [1, 8], iters in [0, 1024], dt_us > 0, surface one
 * of EBOF_SURFACE_*. */
int ebof_validate(const ebof_params *p);

/* Length P (in floats) of the pyramid of p, or -1 if p is invalid. */
int64_t ebof_pyramid_floats(const ebof_params *p);

/* Arena bytes the context needs for the scratch of one window of p (edge
 * staging, column masks, column distances, patch flows), or -1. */
int64_t ebof_window_scratch_bytes(const ebof_params *p);

/* ---- context ------------------------------------------------------------- */
/* Creates a context on HIP device `device`.  `arena` is caller-owned device
 * memory of arena_bytes bytes (256-byte aligned) from which the library takes
 * every device buffer it needs (lookup tables, scratch, per-stream state); it
 * must outlive the context.  Returns EBOF_E_INVAL for a NULL/misaligned arena
 * or a bad device. */
int ebof_create(int device, void *arena, size_t arena_bytes, ebof_ctx **out);

/* Waits for the context's own work, releases its host resources.  The arena
 * is not touched. */
int ebof_destroy(ebof_ctx *ctx);

/* Description of the last failure of a call on ctx made by this thread
 * (never NULL; "" when none). */
const char *ebof_last_error(const ebof_ctx *ctx);

/* ---- stage calls (one window, caller's stream) --------------------------
 * The context keeps one scratch per parameter set and HIP stream (held until
 * ebof_destroy): calls on different streams may run concurrently, also from
 * different host threads (the context's lock covers only its bookkeeping,
 * not the launches); calls on one stream are ordered by it and must be made
 * in that order.  Only the caller's own buffers carry data
 * from one call to the next (edge image, pyramid), so a window's stages may
 * run on one stream and the flow that reads its pyramid on another, ordered
 * by a HIP event or the context's stream counters (below). */

/* Sec. III-A + III-B: bins the events with t0_us <= t < t0_us + dt_us into a
 * binary edge image (polarity is not an input; events off the sensor or off
 * the window are not binned), then applies Alg. 1 (N_d) and Alg. 2 (N_f) in
 * that order.  x, y, t: n device values (SoA); n may be 0.  edge_out: device
 * width*height bytes, receives the denoised and filled image E_df as 0/1.
 * n_dropped_dev: NULL, or a device uint64 to which the number of events not
 * binned is ADDED (the caller zeroes it). */
int ebof_bin_events(ebof_ctx *ctx, const ebof_params *p, const uint16_t *x,
                    const uint16_t *y, const int64_t *t, int64_t n,
                    int64_t t0_us, uint8_t *edge_out,
                    uint64_t *n_dropped_dev, void *hip_stream);

/* Sec. III-C, eq. (1): from a 0/1 edge image (device, width*height bytes),
 * the exact squared Euclidean distance D2 to the closest edge pixel (int32;
 * INT32_MAX everywhere when the image has no edge pixel), the surface
 * S = 1 - exp(-sqrt(D2)/alpha) rounded once to float, and its Gaussian
 * pyramid: each level is the 5x5 binomial ([1 4 6 4 1]/16 per axis,
 * reflect-101 border) of the level above, sampled at even pixels.
 * d2_out: NULL or device width*height int32.  pyr_out: device P floats;
 * level 0 is S. */
int ebof_edt_surface(ebof_ctx *ctx, const ebof_params *p,
                     const uint8_t *edge, int32_t *d2_out, float *pyr_out,
                     void *hip_stream);

/* Sec. III-A to III-C in one call: ebof_bin_events into edge_out followed by
 * ebof_edt_surface of edge_out, with the same arguments, outputs and errors,
 * on one stream; the column masks the distance transform starts from are
 * formed while the edge image is written (one launch and one call fewer
 * than the two calls). */
int ebof_window_surface(ebof_ctx *ctx, const ebof_params *p, const uint16_t *x,
                        const uint16_t *y, const int64_t *t, int64_t n,
                        int64_t t0_us, uint8_t *edge_out,
                        uint64_t *n_dropped_dev, int32_t *d2_out,
                        float *pyr_out, void *hip_stream);

/* Adaptive windows (the Conclusion proposes an accumulation time that adapts
 * to the scene instead of a fixed Delta-T; the rule here is the area event
 * count): the sensor of width x height is tiled from (0, 0) by squares of
 * `area` pixels; scanning the time-ordered events x, y (device, n each) from
 * index i0, every event on the sensor counts for its square, and the window
 * ends right after the event that brings some square to k_events (or at n
 * when none does).  A square as large as the sensor makes windows of
 * k_events events.  range_dev: device int64[2] receiving [i0, end) on the
 * stream, for ebof_window_surface_range.  EBOF_E_INVAL for bad sizes, area
 * < 1, k_events < 1, i0 outside [0, n], more than 8192 squares or NULL
 * arrays.  Scratch (32 MiB per HIP stream) comes from the arena. */
int ebof_window_end(ebof_ctx *ctx, int32_t width, int32_t height,
                    const uint16_t *x, const uint16_t *y, int64_t n, int64_t i0,
                    int32_t area, int32_t k_events, int64_t *range_dev,
                    void *hip_stream);

/* ebof_window_surface for the events of the index range range_dev (device
 * int64[2], [i0, i1), e.g. from ebof_window_end, read on the stream): every
 * event of the range is binned, with no time test; x, y: device arrays of n
 * events (indices at or past n are never read, whatever the range holds;
 * the launch covers n events from i0).  Outputs and errors as
 * ebof_window_surface. */
int ebof_window_surface_range(ebof_ctx *ctx, const ebof_params *p,
                              const uint16_t *x, const uint16_t *y, int64_t n,
                              const int64_t *range_dev, uint8_t *edge_out,
                              uint64_t *n_dropped_dev, int32_t *d2_out,
                              float *pyr_out, void *hip_stream);

/* Sec. III-D: dense flow from the surface pyramid of window k-1 (pyr_prev,
 * the reference) to that of window k (pyr_curr), both device, P floats, by
 * dense inverse search: for levels L-1 .. 0, a grid of 8x8 patches at the
 * given stride (origins k*stride, the last clamped to the border) each runs
 * `iters` inverse-compositional Lucas-Kanade steps (bilinear sampling with
 * replicated border, central-difference template gradient, Hessian plus
 * lambda_reg*I), returns to its initial displacement when it moved more than
 * the patch size, and the per-pixel flow is the mean of the covering patch
 * displacements weighted by 1/max(1, 255*|I1(x+u)-I0(x)|).  A patch starts
 * from twice the coarser level's flow at the pixel nearest its centre, from 0
 * at the coarsest level.  flow_out: device 2*width*height floats.  mask: NULL,
 * or device width*height bytes (the edge image of window k-1); with
 * EBOF_MASK_FLOW set the flow is written as 0 where the mask is 0.
 * With EBOF_VAR_REFINE, each level's dense flow (the densification at every
 * pixel) is refined before the next level starts from it (at the pixel
 * nearest a patch centre, doubled): 5 fixed-point iterations, each weighting
 * the linearised brightness-constancy residual (weight 5), the
 * gradient-constancy residuals (weight 10) and the refined flow's smoothness
 * (weight 20) by the robust penalty's derivative 1 / sqrt(s^2 + 1e-6) at the
 * current increment, then 5 red-black block SOR sweeps (relaxation 1.6) of
 * the per-pixel 2x2 systems; images on the 8-bit scale (x255), derivatives
 * by central differences with replicated border (Ix, Iy, Ixx, Ixy, Iyy of the
 * average of the reference and the warped image, It and the gradient change
 * between them), in double precision.  The context then also holds 18
 * doubles per pixel of scratch and the dense flow of every level.  Stage calls only: batched and
 * served windows with EBOF_VAR_REFINE are refused (EBOF_E_INVAL). */
int ebof_flow(ebof_ctx *ctx, const ebof_params *p, const float *pyr_prev,
              const float *pyr_curr, const uint8_t *mask, float *flow_out,
              void *hip_stream);

/* Sec. III-D (the temporal propagation the paper values in its flow method,
 * reduced to a prediction of constant motion): ebof_flow with the coarsest
 * level warm-started from the previous window pair's flow.  flow_init: NULL
 * (then exactly ebof_flow) or device 2*width*height floats, the dense flow
 * k-2 -> k-1 before masking; a patch of the coarsest level l = L-1 starts
 * from flow_init at the level-0 pixel under its centre,
 * (min((o_x + 4) * 2^l, width-1), min((o_y + 4) * 2^l, height-1)), divided
 * by 2^l (a level-0 displacement spans 2^l times fewer pixels there); finer
 * levels start from the coarser level as in ebof_flow.  flow_dense_out: NULL
 * or device 2*width*height floats receiving the flow before masking (what a
 * later call takes as its flow_init; equal to flow_out without
 * EBOF_MASK_FLOW).  Same errors as ebof_flow. */
int ebof_flow_warm(ebof_ctx *ctx, const ebof_params *p, const float *pyr_prev,
                   const float *pyr_curr, const uint8_t *mask,
                   const float *flow_init, float *flow_out,
                   float *flow_dense_out, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation and results as ebof_flow, with no context.  It allocates
 * nothing: the patch displacements live in a fixed device array of
 * EBOF_NOALLOC_MAX_PATCHES (float2, 8 MiB) that each GPU the library runs on
 * holds until the process ends; its address on a device is looked up on the
 * first call made with that device current.  The call runs on the current
 * HIP device; hip_stream must belong to it.  Every call on one GPU shares
 * that GPU's array, which keeps the last call's contents (nothing in it needs
 * clearing: each level writes its patches before the next reads them), so
 * calls that overlap on one GPU (other streams, other threads) race; order
 * them.  The pyramid's patch count summed over levels must not exceed
 * EBOF_NOALLOC_MAX_PATCHES (3840x2160 at stride 4 with 4 levels fits):
 * EBOF_E_NOMEM otherwise.  EBOF_E_INVAL for bad parameters or NULL buffers,
 * EBOF_E_DEVICE when a HIP call fails.  Errors are read with
 * ebof_last_error(NULL). */
#define EBOF_NOALLOC_MAX_PATCHES (1 << 20)
int ebof_flow_noalloc(const ebof_params *p, const float *pyr_prev,
                      const float *pyr_curr, const uint8_t *mask,
                      float *flow_out, void *hip_stream);

/* ---- batched form ---------------------------------------------------------
 * One descriptor per window; every stage of every window of the batch runs
 * in one kernel launch per stage (one per pyramid level for the pyramid and
 * the flow).  Windows may have different parameters (sizes, levels). */
typedef struct {
    const ebof_params *params;
    const uint16_t *x;      /* device, n events                           */
    const uint16_t *y;
    const int64_t *t;
    int64_t n;
    int64_t t0_us;
    uint8_t *edge_out;      /* device W*H bytes: E_df of this window      */
    int32_t *d2_out;        /* device W*H int32, or NULL                  */
    float *pyr_out;         /* device P floats: this window's pyramid     */
    const float *pyr_prev;  /* device P floats of window k-1, or NULL     */
    const uint8_t *mask;    /* E_df of window k-1 for EBOF_MASK_FLOW      */
    float *flow_out;        /* device 2*W*H floats, used if pyr_prev      */
    uint64_t *n_dropped_dev;/* NULL or device counter (added to)          */
    const float *flow_init; /* NULL, or the previous pair's flow: warm start
                               of the coarsest level as in ebof_flow_warm  */
    float *flow_dense_out;  /* NULL, or device 2*W*H: flow before masking  */
} ebof_window;

/* Runs n (1..EBOF_MAX_BATCH) windows on the caller's stream.  Window i's
 * results are the same as the stage calls would give for it alone.  Scratch
 * is per batch slot; consecutive batches must be ordered on one stream.  The
 * first call for a given batch layout records a HIP graph that later calls
 * with the same layout (number of windows, maximum level count, which windows
 * compute flow) replay. */
int ebof_run_batch(ebof_ctx *ctx, const ebof_window *w, int32_t n,
                   void *hip_stream);

/* ---- launch-shape tuning (batched form) ----------------------------------
 * The batched runner times candidate launch shapes the first time it sees a
 * batch layout and keeps the fastest: the block count of each stage's
 * launch, the rows per item of the EDT row pass (1, 2, 4, 8), the tile width
 * of the densification (64, 128, 256 pixels) and, per pyramid level, the
 * lanes per patch of the inverse search (8 or 4).  No candidate changes any
 * window's results.  Timing a new layout synchronises the stream and
 * runs each stage a few times (milliseconds, once per layout).
 * mode: EBOF_TUNE_AUTO (the default) or EBOF_TUNE_OFF (default shapes for
 * layouts not tuned yet).  cache_path: NULL, or a text file from which tuned
 * layouts are read now and to which newly tuned ones are appended, one line
 * per layout: "<layout>\t<rows> <tile_w> <l_0> ... <l_7> <g_0> ... <g_21>",
 * where <layout>
 * is "W,H,levels,stride,flow,first;" for each window in batch order (flow: 1
 * when the window computes flow; first: 1 for a served stream's first
 * window), l_k the lanes per patch at level k (0: by the level's size) and
 * g_s the block count of internal stage s (0: default).
 * Serving launches keep the default shapes.  Returns EBOF_E_INVAL for a bad
 * mode or a malformed cache line (nothing is changed then).  Captured
 * graphs are released. */
#define EBOF_TUNE_OFF 0
#define EBOF_TUNE_AUTO 1
int ebof_set_tuning(ebof_ctx *ctx, int mode, const char *cache_path);

/* ---- serving ----------------------------------------------------------------
 * A served stream keeps its previous window's pyramid, edge image and flow
 * (before masking) in the arena; with EBOF_WARM_START in its parameters the
 * coarsest level of each flow starts from that previous flow (ebof_flow_warm),
 * from the stream's third window on (the second has no previous flow).  Windows are admitted while their arena bytes fit, batched as they
 * arrive, and run on the context's own HIP stream; each submitted window
 * yields the flow from the stream's previous window (EBOF_NO_FLOW for the
 * first window after open). */
int ebof_stream_open(ebof_ctx *ctx, const ebof_params *p, int32_t *stream_id);

/* Closes a stream after its submitted windows complete. */
int ebof_stream_close(ebof_ctx *ctx, int32_t stream_id);

/* Queues one window of a stream.  Host event arrays (events_on_device = 0)
 * are copied into pinned staging before the call returns; device arrays
 * (events_on_device = 1) must stay alive until the ticket completes.
 * flow_out_dev (2*W*H floats) and mask_out_dev (W*H bytes, the reference
 * window's E_df) are device buffers written when the window completes; they
 * must stay alive until ebof_poll reports completion.  Returns EBOF_E_AGAIN
 * when the event staging is full for now (retry once earlier windows
 * complete), EBOF_E_NOMEM when the window's host events (12 bytes each) can
 * never fit the staging rings, whatever completes. */
int ebof_submit(ebof_ctx *ctx, int32_t stream_id, const uint16_t *x,
                const uint16_t *y, const int64_t *t, int64_t n, int64_t t0_us,
                int events_on_device, float *flow_out_dev,
                uint8_t *mask_out_dev, uint64_t *ticket);

/* Non-blocking.  *status becomes EBOF_OK (flow written), EBOF_NO_FLOW (first
 * window of the stream, or first after a gap in time: outputs zeroed) or a
 * negative error; the call returns EBOF_E_AGAIN while the window is pending,
 * EBOF_E_NOTFOUND for an unknown or already-reported ticket, EBOF_OK once
 * reported.  latency_ns: NULL, or receives the time from ebof_submit to the
 * completion of the window's batch (host steady clock). */
int ebof_poll(ebof_ctx *ctx, uint64_t ticket, int32_t *status, int64_t *latency_ns);

/* Blocks until every submitted window has completed. */
int ebof_drain(ebof_ctx *ctx);

/* ---- cross-stream ordering ----------------------------------------------------
 * For callers that pipeline stage calls over several HIP streams (binning
 * and the distance surface of window k on one stream, the flow k-1 -> k on
 * another, after both pyramids are ready; the blocks of Fig. 1 running
 * concurrently).  A context owns EBOF_SIGNAL_SLOTS 32-bit counters in
 * host-visible signal memory, all 0 at creation.
 *
 * ebof_stream_signal: enqueues on hip_stream the store of value into counter
 * slot; it takes effect after all work issued to that stream before it has
 * completed (that work's results are then visible to any stream).
 * ebof_stream_wait: work issued to hip_stream after this call starts only
 * once counter slot holds a value >= value (unsigned).  The caller owns the
 * protocol: a value waited for must be stored by a signal already issued (or
 * issued later on a stream that does not itself wait on this one); a wait
 * for a value that is never stored blocks the stream for good.  Values
 * stored into a slot must not decrease.
 * ebof_signal_read: the counter's value as the host sees it now (a wait on a
 * value <= it would not block, so a caller may skip issuing it).
 * Each call is one stream operation (host cost a few us, a fraction of an
 * event record plus a cross-stream event wait).  EBOF_E_INVAL for a slot out
 * of range or a NULL output.  Streams using the counters must be idle before
 * ebof_destroy. */
#define EBOF_SIGNAL_SLOTS 64
int ebof_stream_signal(ebof_ctx *ctx, int32_t slot, uint32_t value, void *hip_stream);
int ebof_stream_wait(ebof_ctx *ctx, int32_t slot, uint32_t value, void *hip_stream);
int ebof_signal_read(ebof_ctx *ctx, int32_t slot, uint32_t *value);

/* Creates a HIP stream for such pipelining, owned by the context (destroyed
 * by ebof_destroy; at most EBOF_MAX_OWNED_STREAMS per context), and stores
 * it in *hip_stream.  The stream is created with a CU mask covering every
 * compute unit, which the HIP runtime backs with a hardware queue of its
 * own: streams that share a hardware queue run one after the other, and a
 * stream wait at the head of a shared queue also holds up the other
 * streams' work behind it.  EBOF_E_INVAL for a NULL output, EBOF_E_STATE
 * when the context owns the maximum already. */
#define EBOF_MAX_OWNED_STREAMS 16
int ebof_stream_create(ebof_ctx *ctx, void **hip_stream);

/* ---- pipelined plain driver ------------------------------------------------------
 * One camera stream's consecutive windows through the per-window path
 * (Sec. III, Fig. 1: binning, denoising and filling, distance surface and
 * pyramid of window k, then the flow from window k-1 to window k), issued
 * natively and pipelined over n_streams HIP streams with the counters above,
 * so that consecutive windows' blocks run concurrently.  Window k's
 * ebof_window_surface runs on streams[k mod n_streams], then counter
 * slot0 + (k mod n_streams) is set to 2k + 1; its ebof_flow (the previous
 * window's pyramid as reference, masked to the previous window's E_df when
 * p asks for it) follows on the same stream once counter
 * slot0 + ((k-1) mod n_streams) reaches 2k - 1.
 *
 * win[i]: the events of window k_lo + i (device arrays, as for
 * ebof_window_surface), for k_lo <= k < k_hi.  ring: n_ring > n_streams slots
 * of caller-owned device buffers; window k writes its edge image (E_df) and
 * pyramid into ring[k mod n_ring] and its flow into ring[k mod n_ring].flow
 * (2 * width * height floats).  A slot is reused by window k + n_ring only
 * after the flows that read it (k + 1's) and the one that writes its flow
 * (k's) have completed: the host reads the counters and otherwise makes the
 * stream wait, so the call never blocks on the device.  Asynchronous: it
 * returns once everything is issued; the caller synchronises the streams
 * before reading the outputs.
 *
 * Calls may continue a sequence: with k_lo > 0, ring[(k_lo - 1) mod n_ring]
 * must hold window k_lo - 1's edge image and pyramid and all work of the
 * earlier calls must have completed.  The counters only grow: window indices
 * must increase across calls that share slots (a new sequence from k = 0
 * takes other slots or another context), and 2 k_hi + 1 must fit in 32 bits.
 * Window 0 gets no flow (its ring slot's flow is not written).
 * Errors: EBOF_E_INVAL for NULL arrays, n_streams < 1, n_ring <= n_streams,
 * k_hi < k_lo, k_lo < 0 or slots out of range; the first error of a stage
 * call is returned as is (work issued before it stays issued). */
typedef struct {
    const uint16_t *x;
    const uint16_t *y;
    const int64_t *t;
    int64_t n;
    int64_t t0_us;
} ebof_window_events;

typedef struct {
    uint8_t *edge;
    float *pyr;
    float *flow;
} ebof_ring_slot;

int ebof_run_sequence(ebof_ctx *ctx, const ebof_params *p, const ebof_window_events *win, int64_t k_lo,
                      int64_t k_hi, const ebof_ring_slot *ring, int32_t n_ring, void *const *streams,
                      int32_t n_streams, int32_t slot0);

/* ---- evaluation (Sec. IV, evaluation metrics) -----------------------------------
 * Asynchronous on hip_stream; results land in device memory (out_dev) when
 * the stream reaches them.  Scratch comes from the context's arena, one per
 * image size and stream. */

/* Average endpoint error and outlier rate of flow against a ground truth gt
 * (both device, 2*width*height floats, u plane then v plane) over the pixels
 * where mask != 0 (device width*height bytes; NULL = every pixel): AEE =
 * mean |gt - flow|; a pixel is an outlier when |gt - flow| > 3 px and > 5 %
 * of |gt|.  Per-pixel arithmetic in double.  out_dev: device 3 doubles, AEE,
 * outlier fraction, pixels counted (0 and 0 when none).  EBOF_E_INVAL for
 * NULL buffers or a size outside [1, EBOF_MAX_DIM]. */
int ebof_flow_errors(ebof_ctx *ctx, int32_t width, int32_t height,
                     const float *flow, const float *gt, const uint8_t *mask,
                     double *out_dev, void *hip_stream);

/* Flow warp loss (Sec. IV) of the events of the window [t0_us, t0_us +
 * p->dt_us) on the sensor of p under flow (device 2*W*H floats, pixels per
 * dt_us): the events are accumulated at their own pixel (uncompensated) and,
 * moved back to the window start by the flow at their pixel scaled by their
 * time in the window (x - u (t - t0) / dt), bilinearly into the four pixels
 * around the moved position (compensated; votes off the sensor are lost).
 * Each event votes its polarity (pol: device n int8, <0 is -1, else +1) or
 * 1 when pol is NULL.  Votes are summed in fixed point (2^-32), so the
 * result does not depend on scheduling.  out_dev: device 3 doubles, the FWL
 * var(compensated) / var(uncompensated) (0 when the latter is 0), and the
 * two variances over all W*H pixels. */
int ebof_fwl(ebof_ctx *ctx, const ebof_params *p, const uint16_t *x,
             const uint16_t *y, const int64_t *t, const int8_t *pol, int64_t n,
             int64_t t0_us, const float *flow, double *out_dev,
             void *hip_stream);

/* ---- update-prediction flow filter --------------------------------------------
 * The kind of flow block Sec. III-D selects: a predictive filter whose state
 * is the flow itself, carried from one window to the next (its memory effect)
 * and refined by an update per pyramid layer, each layer with its own
 * regularisation weight and number of smoothing iterations (the parameters of
 * Sec. IV-A).  The paper gives no equations; per window pair, for every layer
 * l from the coarsest (layers-1) to the finest (0), on pyramid level l
 * (W_l x H_l) of both windows' pyramids (I0: window k-1, I1: window k):
 *   prediction  Psi = U_l(x - U_l(x)): the layer's previous flow carried along
 *               itself (bilinear, replicated border); below the top layer
 *               plus twice the coarser layer's innovation at the parent pixel
 *               (x/2, y/2);
 *   update      Phi = Psi - g r / (|g|^2 + gamma_l) with g = 255 grad I0
 *               (central differences, replicated border) and
 *               r = 255 (I1(x + Psi) - I0(x)) (bilinear): the minimiser of
 *               (g.(Phi - Psi) + r)^2 + gamma_l |Phi - Psi|^2;
 *   smoothing   smooth_l Jacobi iterations of the five-point mean of both
 *               planes (replicated border);
 *   U_l <- Phi; the innovation Phi - Psi goes to the next finer layer.
 * The output flow is U_0 (pixels per window), zero off the edge pixels of
 * mask when p->flags has EBOF_MASK_FLOW and mask is not NULL.  Single
 * precision. */
typedef struct {
    int32_t layers;                  /* filter layers, 1 .. p->levels                */
    float gamma[EBOF_MAX_LEVELS];    /* layer l's regularisation weight (l = 0 the
                                        finest), finite and > 0                     */
    int32_t smooth[EBOF_MAX_LEVELS]; /* layer l's smoothing iterations, 0 .. 1000    */
} ebof_filter_params;

/* Sec. IV-A's settings: 3 layers; for sensors up to 346x260 weights 500, 250
 * and 50 with 5, 25 and 50 smoothing iterations (finest layer first: the
 * paper lists the layers from the coarsest), for larger ones 500 and 20 at
 * every layer.  EBOF_E_INVAL when out is NULL. */
int ebof_filter_params_default(int32_t width, int32_t height, ebof_filter_params *out);

/* Floats of a filter state: 2 * sum over the layers of W_l * H_l; -1 (with the
 * error set) when p or fp is invalid. */
int64_t ebof_filter_state_floats(const ebof_params *p, const ebof_filter_params *fp);

/* One filter step from pyramid pyr_prev (window k-1) to pyr_curr (window k),
 * both of p->levels levels (device, ebof_pyramid_floats floats each).
 * state: device, ebof_filter_state_floats floats, layer 0 first, each layer
 * its u plane then its v plane (row-major W_l x H_l); on entry the previous
 * step's flows (zeros before the first step), on return this step's.
 * flow_out: device 2*W*H floats (u plane, v plane).  mask: NULL or device
 * W*H bytes (E_df of window k-1).  Work memory comes from the context's
 * arena, per sensor size, layer count and stream; calls on one stream are
 * ordered, calls on different streams use different work memory.  Returns
 * EBOF_E_INVAL on bad arguments, EBOF_E_NOMEM when the arena cannot hold the
 * work memory (about 8.7 W*H floats for 3 layers). */
int ebof_flow_filter(ebof_ctx *ctx, const ebof_params *p, const ebof_filter_params *fp,
                     const float *pyr_prev, const float *pyr_curr, const uint8_t *mask,
                     float *state, float *flow_out, void *hip_stream);

/* ---- measurement -------------------------------------------------------------
 * Kernel timing: when enabled, every launch of a selected kernel is
 * bracketed by a pair of HIP events recorded on its stream right before and
 * right after it (the pair itself adds a fixed cost, which a caller can
 * measure with an empty pair); ebof_timing_read waits for them and returns
 * the total milliseconds and the launch count accumulated since the last
 * read (then resets).  Timing disables graph capture of the batched form.
 * With EBOF_TIMING_SPAN or-ed into the mask, the launches of a selected
 * kernel that one call makes back to back on one stream (the inverse
 * search's levels of ebof_flow) share one pair, recorded before the first
 * and after the last, so that the kernels' own dispatch gaps, not a pair's
 * wait for each launch, separate them; the launch count still counts each
 * launch.  A pair's events come from a pool the context owns (created on
 * demand, destroyed with it); if an event cannot be created, the launches
 * run untimed. */
#define EBOF_K_SCATTER 0
#define EBOF_K_DENOISE_FILL 1
#define EBOF_K_PACK_COLS 2
#define EBOF_K_EDT_COLS 3
#define EBOF_K_EDT_ROWS 4
#define EBOF_K_PYR_DOWN 5
#define EBOF_K_DIS_LEVEL 6
#define EBOF_K_DENSIFY 7
#define EBOF_K_COUNT 8
#define EBOF_TIMING_SPAN 0x80000000u
int ebof_timing_enable(ebof_ctx *ctx, uint32_t kernel_mask);
int ebof_timing_read(ebof_ctx *ctx, int32_t kernel_id, double *total_ms,
                     int64_t *launches);

/* Library version string. */
const char *ebof_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EBOF_H */

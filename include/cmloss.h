/*
 * cmloss.h -- C ABI of the MI355X (gfx950) contrast-maximization loss library.
 *
 * The library computes the multi-reference contrast-maximization (CM) loss of
 * one or many windows of events and its gradient with respect to per-pixel
 * inverse depth and 6-DoF ego-motion, entirely in HIP kernels.
 *
 * Paper (arXiv 2412.06359): the loss is Eq. 1 of Sec. 3.1 (iterative warp of
 * every event to all reference times, bilinear splatting into per-polarity
 * images of warped events, active-pixel normalisation, masking of events that
 * leave the image); the flow comes from inverse depth and ego-motion through
 * Eq. 2 of Sec. 3.2 (by default in its first-order, motion-field form; the
 * exact reprojection is a per-window option); the gradient is the analytic
 * backward of Sec. 3.3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pixel centres sit at integer coordinates; the image domain is the closed
 *    box [0, width-1] x [0, height-1].  Row-major images: pixel (x, y) is at
 *    index y * width + x.
 *  - Events are structure-of-arrays in device memory: x, y, t float32, p int8
 *    (p > 0 positive polarity, anything else negative).  t is the timestamp
 *    normalised to the window, expected in [0, 1].
 *  - inv_depth: float32 [F][height * width] device array, rho = 1/depth (any
 *    common scale, Eq. 2 fixes depth only up to scale).
 *  - ego: float32 [F][6] device array (v_x, v_y, v_z, w_x, w_y, w_z):
 *    translation and rotation (exponential coordinates) of the camera over the
 *    window; flow is in pixels per window.
 *  - Flow sets (Sec. 3.1 concatenates the flows of consecutive slices of the
 *    event stream): F = 1 warps the whole window with one flow.  Otherwise F
 *    is the number of segments between consecutive knots {0, 1} U refs and
 *    segment f (in time order) has its own inverse depth and ego-motion; a warp
 *    step samples the flow of the segment it crosses.  Gradients have the same
 *    [F] layout.
 *  - Loss: L = (1/R) sum_r [sum_x sum_p (S_p/(C_p+eps))^2] / (N_r + eps), with
 *    C_p / S_p the bilinear splat of the surviving events' weights / weights
 *    times (1 - |r - t_k|), and N_r the number of pixels with C_+ + C_- > 0.
 *  - Memory: the caller allocates every buffer (device memory for all arrays
 *    unless stated otherwise); the library never frees caller memory.  The
 *    handle owns nothing that a call writes, so calls on different streams
 *    with different state buffers may overlap.
 *  - Streams: every call is asynchronous on `stream` (a hipStream_t; NULL is
 *    the null stream).  No host synchronisation happens inside a call.
 *  - Errors: every function returns a cm_status and never aborts.  Invalid
 *    arguments detected on the host return CM_ERR_INVALID_ARG with nothing
 *    enqueued.  Data errors in device arrays are not reported: an event with a
 *    non-finite coordinate, a timestamp outside [0, 1] or a start position off
 *    the image is masked like an event that leaves the image.
 */
#ifndef CMLOSS_H
#define CMLOSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cm_handle_s* cm_handle;

typedef enum {
    CM_OK = 0,
    CM_ERR_INVALID_ARG = -1,
    CM_ERR_OOM = -2,
    CM_ERR_HIP = -3,
    CM_ERR_UNSUPPORTED = -4,
    CM_ERR_BUDGET = -5
} cm_status;

/* Splat modes.  ATOMIC: floating-point atomic accumulation, results vary in
 * the last bits from run to run.  DETERMINISTIC: the warped positions are
 * sorted stably (event order) into 32x32-tile bins and each tile accumulates
 * them in a fixed order (records in event order, 64 at a time, per tap slot,
 * equal pixels in lane order), the backward walks the valid events in the
 * order of their reference-0 bins and bins its records the same way, and
 * every reduction uses a fixed tree: results are bit-identical from run to run
 * and between a window alone and in a batch.
 * It always takes the tiled path (CM_ERR_UNSUPPORTED where that path does not
 * apply) and is slower. */
enum { CM_MODE_ATOMIC = 0, CM_MODE_DETERMINISTIC = 1 };

#define CM_MAX_REFS 16

/* One window's geometry and loss settings (host memory). */
typedef struct {
    int32_t width, height;          /* sensor size, > 0 */
    float fx, fy, cx, cy;           /* pinhole intrinsics, fx, fy > 0 */
    int32_t n_refs;                 /* R, 1 <= R <= CM_MAX_REFS */
    float refs[CM_MAX_REFS];        /* reference times, strictly increasing, in [0, 1] */
    int32_t mode;                   /* CM_MODE_* */
    float eps;                      /* regulariser of Eq. 1's ratios, finite and > 0 (1e-9 by default) */
    int32_t n_flows;                /* F: 0 or 1 (one flow), or the number of segments between
                                       consecutive knots {0, 1} U refs */
    int32_t flow_model;             /* CM_FLOW_* */
} cm_window_desc;

/* How Eq. 2 turns inverse depth and ego-motion into a flow (pixels per
 * window).  FIRST_ORDER: the motion field, linear in (v, w) and in rho
 * (u = A(x) w + rho B(x) v).  EXACT: the pixel is back-projected with depth
 * 1/rho, moved by the rigid motion (rotation exp([w]x) by Rodrigues' formula,
 * then translation v) and projected again; u = projection - pixel, and a point
 * that lands on or behind the camera plane (z <= 0) has zero flow and no
 * gradient.  The two agree to first order in (v, w). */
enum { CM_FLOW_FIRST_ORDER = 0, CM_FLOW_EXACT = 1 };

/* Create a handle bound to HIP device `device`.  *h receives the handle. */
cm_status cm_create(cm_handle* h, int device);

/* Destroy a handle (NULL is accepted).  No call may be in flight on it. */
cm_status cm_destroy(cm_handle h);

/* Human-readable name of a status code (static string). */
const char* cm_status_string(cm_status s);

/* Bytes of the per-window `state` buffer for a window of n_events events: the
 * splatted images C and S per reference and polarity (32 * R * width * height
 * bytes, FP64), per-reference sums, reduction scratch and, where the tiled
 * path applies, its workspace (binned records, at most 32 * R bytes per event,
 * a 16-byte source record and a 1-byte mask per event, per-tile buffers).  The forward and
 * backward of one window must be called with the same n_events.  0 if `d` is
 * invalid or n_events < 0. */
size_t cm_state_bytes(const cm_window_desc* d, int64_t n_events);

/* Kernel path used by a handle.  AUTO picks per window: the direct path
 * (floating-point atomics straight into the images) for small windows, the
 * tiled path (warped positions binned by 32x32 tile and accumulated in LDS,
 * each pixel written at most once) for large ones where the sensor allows
 * it.  The two compute the same quantities; TILED fails with CM_ERR_UNSUPPORTED where
 * it does not apply (more than 16384 reference-tile bins).  The forward and
 * the backward on one state must take the same path: the tiled backward walks
 * per-event source records that only the tiled forward writes, and on a state
 * the direct forward filled it returns NaN in grad_ego. */
enum { CM_PATH_AUTO = 0, CM_PATH_DIRECT = 1, CM_PATH_TILED = 2 };
cm_status cm_set_path(cm_handle h, int path);

/* Launch tuning of a handle (the project's autotuner searches it; see
 * paper_2412_06359_amd/autotune.py).  Zero fields keep the defaults.
 *   event_blocks      : event blocks a batch's count / scatter / sweep
 *                       kernels aim for (sets events per lane), 256..65536,
 *                       default 4096
 *   tile_threads      : threads of the forward tile kernel, 256 or 512,
 *                       default 512
 *   tiled_min_records : CM_PATH_AUTO takes the tiled path for single windows
 *                       with at least this many event-reference records,
 *                       >= 1, default 131072
 *   tile_w, tile_h    : the tiled path's tile size, 32 x 32 (default),
 *                       64 x 32, 32 x 16 or 16 x 16; a plan whose windows
 *                       would need more than 16384 bins at that size takes
 *                       32 x 32
 * event_blocks, tile_threads and the tile size apply to batch plans created
 * after the call, in the atomic mode only (the deterministic mode's launch
 * geometry and 32 x 32 tiles define its operation order and are fixed);
 * single-window calls keep the default geometry, which cm_state_bytes sizes.
 * Results in the atomic mode agree across tunings within rounding.
 * CM_ERR_INVALID_ARG for values out of range, with the handle unchanged. */
typedef struct {
    int32_t event_blocks;
    int32_t tile_threads;
    int64_t tiled_min_records;
    int32_t tile_w;
    int32_t tile_h;
} cm_tuning;
cm_status cm_set_tuning(cm_handle h, const cm_tuning* t);
cm_status cm_get_tuning(cm_handle h, cm_tuning* out);

/* Forward (paper Sec. 3.1 Eq. 1 with Sec. 3.2 Eq. 2; Sec. 3.3 per-event
 * forward).
 *   ev_x, ev_y, ev_t, ev_p : n_events events (device; may be NULL if n_events == 0)
 *   inv_depth, ego         : as above (device)
 *   loss                   : float32 [1] (device), receives L
 *   state                  : cm_state_bytes(d, n_events) bytes (device), written; the
 *                            backward reads it, so keep it and the inputs
 *                            unchanged until the backward has run.
 * n_events == 0 gives L = 0. */
cm_status cm_loss_forward(cm_handle h, const cm_window_desc* d,
                          const float* ev_x, const float* ev_y, const float* ev_t,
                          const int8_t* ev_p, int64_t n_events,
                          const float* inv_depth, const float* ego,
                          float* loss, void* state, void* stream);

/* Backward (paper Sec. 3.3: analytic gradient; here the exact adjoint of the
 * forward with the active-pixel count and the event mask held fixed, computed
 * by re-running each event's warp instead of storing it).
 *   state          : the buffer the forward wrote for the same inputs; its
 *                    scratch tail is overwritten, the images are only read.
 *   grad_loss      : float32 [1] (device), dOut/dL from the caller
 *   grad_inv_depth : float32 [F][height * width] (device), overwritten with
 *                    grad_loss * dL/d(inv_depth)
 *   grad_ego       : float32 [F][6] (device), overwritten with grad_loss * dL/d(ego) */
cm_status cm_loss_backward(cm_handle h, const cm_window_desc* d,
                           const float* ev_x, const float* ev_y, const float* ev_t,
                           const int8_t* ev_p, int64_t n_events,
                           const float* inv_depth, const float* ego,
                           void* state, const float* grad_loss,
                           float* grad_inv_depth, float* grad_ego, void* stream);

/* Forward without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and result as cm_loss_forward, without
 * `state`: the window's whole forward state lives in a file-scope device array
 * of the library (CM_NOALLOC_MAX_STATE_BYTES bytes, one per device, held
 * until the process ends), so the call allocates nothing and no backward can
 * follow it.  The caller passes the inputs and `loss` (device float32 [1]).
 * The array is shared by every call on a device and keeps the last call's
 * contents (the forward clears what it accumulates into): calls that overlap
 * on one device, on any streams or handles, race and give wrong results.
 * CM_ERR_BUDGET, with nothing enqueued, if cm_state_bytes(d, n_events)
 * exceeds CM_NOALLOC_MAX_STATE_BYTES (e.g. 640x480 with 3 references and 100k
 * events fits; 1280x720 with 8 references does not).  Profiling
 * (cm_profile_enable) does not record this call. */
#define CM_NOALLOC_MAX_STATE_BYTES (128u * 1024u * 1024u)
cm_status cm_loss_forward_noalloc(cm_handle h, const cm_window_desc* d,
                                  const float* ev_x, const float* ev_y, const float* ev_t,
                                  const int8_t* ev_p, int64_t n_events,
                                  const float* inv_depth, const float* ego,
                                  float* loss, void* stream);

/* Diagnostics of the last forward on `state` (device -> host copy; this call
 * synchronises `stream`).  out[0] = loss (FP64), out[1] = number of valid
 * (unmasked) events, out[2 + r] = numerator of reference r, out[2 + R + r] =
 * N_r.  `out` is host memory of 2 + 2R doubles. */
cm_status cm_state_diagnostics(const cm_window_desc* d, const void* state, double* out,
                               void* stream);

/* Batches (the tiled path over many windows in one launch sequence).
 *
 * A plan fixes a batch's shape: n_windows descriptors (host memory, all with
 * the same mode and flow model) and their event counts.  Events of all windows are packed in
 * flat device arrays, window w at [event_offsets[w], event_offsets[w+1]), in
 * window order; inverse depth and d inverse depth likewise at
 * [pixel_offsets[w], pixel_offsets[w+1]) (F * height * width floats each);
 * ego and d ego hold 6 floats per flow set, window w's sets starting at set
 * set_offsets[w] (cm_batch_flow_offsets; w * 6 floats when every window has
 * one flow); loss and grad_loss are [n_windows].  Each window's
 * loss and gradient equal those of a single-window call on the same data.
 * A plan holds host memory only: each call copies the per-window metadata into
 * the caller's state buffer (cm_batch_state_bytes) on the call's stream, so
 * plans are cheap to create and destroy per batch (a serving loop does).  With
 * graphs enabled (cm_batch_set_graph allocates a device copy of the metadata
 * and a capture stream), the first call with a given set of buffers captures
 * the launch sequence into a hipGraph and later calls with the same buffers
 * replay it.  A plan is used by one host thread at a time.  Windows that
 * exceed the tiled path's limits (more than 16384 reference-tile bins, or 2^31
 * records in the batch) make cm_batch_create fail with CM_ERR_UNSUPPORTED. */
typedef struct cm_batch_s* cm_batch;
cm_status cm_batch_create(cm_handle h, int32_t n_windows, const cm_window_desc* descs,
                          const int64_t* n_events, cm_batch* out);
cm_status cm_batch_destroy(cm_batch b);
size_t cm_batch_state_bytes(cm_batch b);
/* Host arrays of n_windows + 1 entries each (either may be NULL). */
cm_status cm_batch_offsets(cm_batch b, int64_t* event_offsets, int64_t* pixel_offsets);
/* First flow set of each window (host array of n_windows + 1 entries): ego and
 * d ego of window w are floats [6 * set_offsets[w], 6 * set_offsets[w+1]). */
cm_status cm_batch_flow_offsets(cm_batch b, int64_t* set_offsets);
cm_status cm_batch_set_graph(cm_batch b, int enable);
cm_status cm_loss_forward_batched(cm_batch b, const float* ev_x, const float* ev_y,
                                  const float* ev_t, const int8_t* ev_p, const float* inv_depth,
                                  const float* ego, float* loss, void* state, void* stream);
cm_status cm_loss_backward_batched(cm_batch b, const float* ev_x, const float* ev_y,
                                   const float* ev_t, const int8_t* ev_p, const float* inv_depth,
                                   const float* ego, void* state, const float* grad_loss,
                                   float* grad_inv_depth, float* grad_ego, void* stream);
/* Per-window (loss, valid events) of the last batched forward, host array of
 * 2 * n_windows doubles; synchronises `stream`. */
cm_status cm_batch_diagnostics(cm_batch b, const void* state, double* out, void* stream);
/* Per window, the bytes of splat image held by its occupied (reference,
 * 32x32 tile) bins after the last batched forward on `state`: 32 bytes per
 * pixel of every tile that some warped position falls in (the other tiles
 * hold only zeros and are not written; inside an occupied tile only the
 * pixels some tap reached are).  Host array of n_windows doubles; call
 * between the forward and the backward; synchronises `stream`.  A
 * measurement aid. */
cm_status cm_batch_occupied_image_bytes(cm_batch b, const void* state, double* out, void* stream);
/* Per window and reference, N_r (pixels with C_+ + C_- > 0) of the last
 * batched forward on `state`: host array of n_windows * CM_MAX_REFS doubles,
 * window w's at [w * CM_MAX_REFS, w * CM_MAX_REFS + R), zeros after;
 * synchronises `stream`.  The splat images hold their non-zero values at
 * these pixels only: the backward's gathers read 32 bytes at each. */
cm_status cm_batch_active_pixels(cm_batch b, const void* state, double* out, void* stream);

/* Geometry consistency and the full loss (paper Sec. 3.2 Eq. 3, Eq. 4).
 *
 * For a window with F >= 2 flow sets, consecutive sets f and f+1 form a pair.
 * Set f's pixel x (depth D_f = 1/rho_f(x)) moves with segment f's motion --
 * rotation Exp(Delta_f w_f), translation Delta_f v_f, Delta_f the segment's
 * length in window time -- giving the forward-projected depth D_{0->1}(x)
 * (the moved point's z) and, at the moved point's projection x', the bilinear
 * interpolation D'_1(x) of D_{f+1}.  V: pixels with rho_f > 0 whose point
 * stays in front of the camera, with x' inside the image and rho_{f+1} > 0 at
 * x''s on-sensor taps.  L_geo = mean over the F-1 pairs of
 * mean over V of |D_{0->1} - D'_1| / (D_{0->1} + D'_1) (an empty V counts
 * 0); a window with one flow set has L_geo = 0.  The full loss is
 * L = L_CM + lambda L_geo (the paper trains with lambda = 0.05).
 *
 * inv_depth and ego are laid out as for the CM loss.  `state` is a caller
 * buffer of cm_geo_state_bytes (cm_batch_geo_state_bytes) bytes, separate from
 * the CM state; the backward reads what the forward on the same state and
 * inputs wrote.  The first batched call on a plan allocates a device copy of
 * the plan's metadata (as cm_batch_set_graph does), freed with the plan.
 * Results are deterministic in both modes (fixed-order
 * reductions; in the deterministic mode the scatter of d rho_{f+1} is summed
 * in 64-bit fixed point, so d inv_depth is bit-identical from run to run).
 *
 * Forward: loss_geo (device, [1] or [n_windows]) receives L_geo; if loss_total
 * is not NULL it receives loss_cm + lambda L_geo, loss_cm (device, may be NULL
 * for 0) being the CM loss of the same windows.  lambda must be finite.
 * Backward: ACCUMULATES grad_loss * lambda * dL_geo/d(inv_depth, ego) into
 * grad_inv_depth and grad_ego, so that after cm_loss_backward (which writes
 * them) they hold the gradient of L = L_CM + lambda L_geo; grad_loss (device,
 * [1] or [n_windows]) is dE/dL of the caller's objective E.  |V| is held
 * constant in the derivative and d|d|/dd = sign(d), sign(0) = 0. */
size_t cm_geo_state_bytes(const cm_window_desc* d);
cm_status cm_geo_forward(cm_handle h, const cm_window_desc* d, const float* inv_depth,
                         const float* ego, float lambda, const float* loss_cm, float* loss_geo,
                         float* loss_total, void* state, void* stream);
cm_status cm_geo_backward(cm_handle h, const cm_window_desc* d, const float* inv_depth,
                          const float* ego, float lambda, void* state, const float* grad_loss,
                          float* grad_inv_depth, float* grad_ego, void* stream);
size_t cm_batch_geo_state_bytes(cm_batch b);
cm_status cm_geo_forward_batched(cm_batch b, const float* inv_depth, const float* ego,
                                 float lambda, const float* loss_cm, float* loss_geo,
                                 float* loss_total, void* state, void* stream);
cm_status cm_geo_backward_batched(cm_batch b, const float* inv_depth, const float* ego,
                                  float lambda, void* state, const float* grad_loss,
                                  float* grad_inv_depth, float* grad_ego, void* stream);

/* Phase timing (diagnostics, not part of the method).  While enabled on a
 * handle, each call records a pair of HIP events on its stream around every
 * kernel it launches.  cm_profile_read waits for the recorded events, writes
 * the accumulated milliseconds and launch counts per phase (host arrays of
 * CM_N_PHASES entries) and clears them.  A handle that profiles must be used
 * from one host thread at a time. */
enum {
    CM_PHASE_ZERO = 0,          /* clear the splat images (forward) */
    CM_PHASE_SPLAT = 1,         /* warp + splat, or the tiled path's per-tile splat (forward) */
    CM_PHASE_REDUCE = 2,        /* per-reference sums, or the tiled path's halo merge (forward) */
    CM_PHASE_FINALIZE = 3,      /* loss (forward) */
    CM_PHASE_GRAD_ZERO = 4,     /* clear d inv_depth (backward) */
    CM_PHASE_ADJOINT = 5,       /* recompute warp + adjoint sweep (backward) */
    CM_PHASE_GRAD_FINALIZE = 6, /* d ego (backward) */
    CM_PHASE_COUNT = 7,         /* tiled path: bin the warped positions (forward) */
    CM_PHASE_SCAN = 8,          /* tiled path: bin offsets (forward) */
    CM_PHASE_SCATTER = 9,       /* tiled path: write the binned records (forward) */
    CM_PHASE_GRAD_COUNT = 10,   /* tiled path: bin the flow-sampling positions (backward) */
    CM_PHASE_GRAD_SCAN = 11,    /* tiled path: bin offsets (backward) */
    CM_PHASE_GRAD_TILE = 12,    /* tiled path: dL/du per tile -> d inv_depth, d ego (backward) */
    CM_N_PHASES = 13
};
cm_status cm_profile_enable(cm_handle h, int enable);
cm_status cm_profile_read(cm_handle h, double* ms, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* CMLOSS_H */

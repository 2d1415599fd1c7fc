/*
 * vgr.h - C ABI of libvgr, an MI355X (gfx950) implementation of the hot path
 * of "Volumetrically Consistent 3D Gaussian Rasterization" (arXiv 2412.03378).
 *
 * What is computed.  A scene is a mixture of 3D Gaussians with density
 * sigma(x) = sum_i kappa_i G_i(x) (Sec. 3.2, eq. gauss_mixture).  For the ray
 * o + t d through a pixel centre (|d| = 1), each Gaussian's full-line
 * integral is x_i = kappa_i sqrt(2 pi) beta_i G_i(o + gamma_i d) with
 * beta_i = (d^T Sigma_i^-1 d)^(-1/2) (Sec. 4.2, eq. betagamma and the boxed
 * eq. our_trans_final), its opacity alpha_i = 1 - exp(-x_i), and colour mode
 * composites C = sum_i c_i alpha_i prod_{j<i}(1 - alpha_j) front to back
 * (Sec. 4.1, eq. our_alpha_blend).  X-ray mode returns I = sum_i x_i
 * (Sec. 6.2, Beer-Lambert line integral).  The rules the paper leaves open
 * (thresholds, order of ties, colour model) are fields of vgr_settings and are
 * documented there.
 *
 * Conventions shared by every entry point.
 *   - Return value: VGR_OK (0) or a negative VGR_ERR_* code; the message of
 *     the last failure is returned by vgr_last_error().  Nothing is thrown.
 *   - Pointers are DEVICE pointers (HIP, the context's device) to contiguous
 *     FP32 row-major arrays owned by the caller, unless marked "host".  The
 *     library never frees caller memory.
 *   - All GPU work is enqueued on the context's stream (vgr_set_stream) and
 *     the calls return without waiting for it, except where noted.
 *   - A context is not thread safe; use one context per host thread / stream.
 *   - The context owns its workspace (device memory that only grows) and the
 *     state the last forward saved for the backward.
 */
#ifndef VGR_H
#define VGR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VGR_OK = 0,
    VGR_ERR_INVALID_ARG = -1,   /* a null pointer, bad size or bad setting */
    VGR_ERR_HIP = -2,           /* a HIP runtime call failed */
    VGR_ERR_OOM = -3,           /* workspace allocation failed */
    VGR_ERR_CAPACITY = -4,      /* a fixed-capacity (graph) run overflowed */
    VGR_ERR_NOT_CAPTURED = -5,  /* vgr_graph_launch without a captured graph */
    VGR_ERR_NO_FORWARD = -6     /* backward / aux query without a forward */
};

/* Pinhole camera (host struct).  World -> view: x_v = R x_w + t, OpenCV axes
 * (x right, y down, z forward).  Pixel (px, py) has its centre at
 * (px + 0.5, py + 0.5); its view-space ray direction is proportional to
 * ((px + 0.5 - cx)/fx, (py + 0.5 - cy)/fy, 1).  Gaussians whose view-space
 * mean depth is <= znear are not rendered. */
typedef struct {
    float R[9];          /* row-major rotation */
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    float znear;
    int32_t reserved;
} vgr_camera;

enum { VGR_MODE_COLOR = 0, VGR_MODE_XRAY = 1 };
enum { VGR_ACT_CLAMP0 = 0, VGR_ACT_SOFTPLUS10 = 1 };
enum { VGR_DENSITY_KAPPA = 0, VGR_DENSITY_THETA = 1 };
enum { VGR_ALPHA_VOLUMETRIC = 0, VGR_ALPHA_SPLAT = 1 };
enum { VGR_KERNEL_GAUSSIAN = 0, VGR_KERNEL_EPANECHNIKOV = 1 };

/* Largest per-pixel re-sorting window (vgr_settings.pixel_window). */
#define VGR_MAX_PIXEL_WINDOW 32

/* Rendering rules.  Defaults in brackets (vgr_default_settings).
 *   mode        colour compositing or X-ray line integrals [COLOR]
 *   sh_degree   0..3, real spherical harmonics with the Condon-Shortley
 *               phase, basis index k = l^2 + l + m [0]
 *   alpha_min   a Gaussian with alpha < alpha_min is skipped for that pixel
 *               [1/255]
 *   alpha_max   alpha is clamped to alpha_max, with zero gradient [0.99]
 *   T_min       compositing stops before the Gaussian that would take the
 *               transmittance below T_min; it is not blended [1e-4]
 *   x_min_xray  X-ray mode drops terms x_i < x_min_xray [1e-6]
 *   bg          background colour, C += T_final * bg [0,0,0]
 *   act         colour c = act(sum_k sh_k Y_k(v) + 0.5), v the unit vector
 *               from the camera centre to the mean; max(.,0) or
 *               softplus(10 y)/10 (Supp. D) [CLAMP0]
 *   tile_w/h    screen tile in pixels, one of 8x8, 16x8, 16x16, 32x8;
 *               0 = tuned: vgr_autotune's choice for the call's workload class
 *               (total pixels and Gaussians in powers of two, mode,
 *               alpha_model, kernel, tile_resort, near_segment), else the
 *               context's last tuned shape (8x8 until vgr_autotune) [0, 0]
 *   batch       records staged in LDS per rasteriser batch (the block
 *               shape), 32 or 64; 0 = tuned as tile_w/h (64 until
 *               vgr_autotune).  Never changes the result [0]
 *   density     what the `dens` input holds: KAPPA, the density kappa >= 0
 *               itself, or THETA, the paper's density parameter theta, with
 *               kappa = -ln(1 - 0.99 theta) (1/s_x + 1/s_y + 1/s_z) / 3
 *               computed inside the preprocess (Sec. 5, eq. density_reparam);
 *               theta is clamped to its range [0, 1], with zero gradient
 *               outside it [KAPPA]
 *   alpha_model VOLUMETRIC: the paper's opacity from the ray integral (above).
 *               SPLAT: the 3DGS splatting opacity the paper compares against
 *               (Sec. 3, eq. 3dgs_alpha, eq. affine_approx), for A/B runs on
 *               the same pipeline: alpha = o exp(-1/2 dp^T Sigma'^-1 dp) with
 *               dp = pixel centre - projected mean, Sigma' = J W Sigma W^T J^T
 *               (W the world-to-view rotation, J the pinhole Jacobian at the
 *               view-space mean) and o = `dens` read as the peak opacity,
 *               clamped to [0, 1]; the same skip, clamp, stop and background
 *               rules; tiles from the exact alpha >= alpha_min ellipse; the
 *               backward returns d_dens = dL/do (zero where o was clamped).
 *               Colour mode with density KAPPA only [VOLUMETRIC]
 *   near_segment 0: each Gaussian's integral covers the whole line (the
 *               boxed result of Sec. 4.2).  1: it starts where the pixel's ray
 *               crosses the near plane z = znear, x = kappa sqrt(2 pi) beta
 *               G(o + gamma d) Phi((gamma - t_n) / beta) with Phi the standard
 *               normal distribution function (the finite-limit erf form of
 *               Sec. 4.2), so Gaussians straddling the plane lose the part
 *               behind it.  Evaluated only for records whose bound reaches
 *               within 6 standard deviations of the plane (elsewhere Phi = 1 to
 *               FP32 precision).  VOLUMETRIC only [0]
 *   tile_resort 0: every tile composites in the depth order of the means.
 *               1: within each tile, in ascending depth of each Gaussian's
 *               maximum along the ray through the tile's centre (the
 *               per-tile level of the re-sorting the paper points to against
 *               popping, Sec. 7, Limitations; ties by mean depth, then index).  The image
 *               then depends on the tile shape (also on the one vgr_autotune
 *               picks when tile_w = tile_h = 0).  Costs one more 32-bit sort
 *               of the instances.  Colour mode, VOLUMETRIC [0]
 *   kernel      the primitive's density profile along Sigma (VOLUMETRIC
 *               only).  GAUSSIAN: kappa exp(-r^2/2), r^2 = (x-mu)^T Sigma^-1
 *               (x-mu), the paper's primitive.  EPANECHNIKOV: the compact
 *               kernel the paper names as future work (Sec. 8, compact
 *               primitives), kappa max(0, 1 - r^2), whose support is the
 *               ellipsoid with semi-axes s; its line integral is
 *               x = (4/3) kappa beta (1 - D^2)^(3/2) for D^2 < 1 and 0 beyond
 *               (the same beta and D^2 as the Gaussian's), and the tiles come
 *               from the same dual-conic box with D2max = 1 - (3 tau /
 *               (4 kappa beta_max))^(2/3).  Not with the near-plane segment
 *               [GAUSSIAN]
 *   pixel_window W > 0 (needs tile_resort): the per-pixel level of the
 *               re-sorting (Sec. 7, Limitations).  At each pixel the Gaussians
 *               that reach alpha_min, in the per-tile order, pass through a
 *               window of W entries ordered by the depth of each maximum on
 *               the pixel's own ray (ties by list position); when the window
 *               is full its smallest entry is composited, at the end of the
 *               list the rest in order; termination ends the pixel, leaving
 *               what the window still holds.  W = 1 is the per-tile order; a
 *               W at least the number of such Gaussians sorts each pixel
 *               exactly.  At most VGR_MAX_PIXEL_WINDOW; 8x8 tiles and
 *               64-record batches (tile_w/h and batch 0 or those values).
 *               The forward keeps, per (tile pixel, list entry), the
 *               compositing sequence and 8 bytes for the backward's replay:
 *               16 bytes x 64 per instance of workspace.  Pair counters
 *               (vgr_set_counting) stay zero [0]
 * Without tile_resort, Gaussians are composited in ascending order of the
 * FP32 view-space depth of their mean, z = fmaf(R20, mx, fmaf(R21, my,
 * fmaf(R22, mz, t2))); ties keep the input index order.  The result then
 * does not depend on the tile size:
 * tiles only bound, conservatively, where alpha >= alpha_min can occur. */
typedef struct {
    int32_t mode;
    int32_t sh_degree;
    float alpha_min, alpha_max, T_min, x_min_xray;
    float bg[3];
    int32_t act;
    int32_t tile_w, tile_h;
    int32_t density;
    int32_t alpha_model;
    int32_t near_segment;
    int32_t tile_resort;
    int32_t kernel;
    int32_t batch;
    int32_t pixel_window;
} vgr_settings;

/* Counters of the last forward (host struct). */
typedef struct {
    int64_t instances;       /* (Gaussian, tile) pairs emitted, all views */
    int64_t capacity;        /* instance capacity of the workspace */
    int64_t visible;         /* (Gaussian, view) pairs that survived culling */
    int64_t pairs_tested;    /* filled when pair counting is on: (pixel,     */
    int64_t pairs_full;      /*   Gaussian) pairs visited, pairs evaluated   */
    int64_t pairs_blended;   /*   past the cheap bound test, pairs blended   */
    int64_t visits;          /* wave-level: (Gaussian, pixel slot of a wave)  */
    int64_t visits_full;     /*   steps, and those that took the evaluation   */
                             /*   branch (some pixel passed the bound test)   */
    int64_t bwd_pairs_tested;   /* the same five counts for the backward   */
    int64_t bwd_pairs_full;     /*   rasteriser of the last backward (no    */
                                /*   pairs tested, and visits = evaluation */
                                /*   steps, where it reuses the forward's  */
                                /*   bound-test masks: colour mode, or one */
                                /*   pixel per lane).  With 8x8 tiles each */
                                /*   4x4 quarter walks its own Gaussians:  */
                                /*   bwd_visits counts wave steps (up to   */
                                /*   four Gaussians each), bwd_visits_full */
                                /*   (Gaussian, quarter) visits            */
    int64_t bwd_pairs_blended;
    int64_t bwd_visits;
    int64_t bwd_visits_full;
    int32_t overflow;        /* 1 if a fixed-capacity run dropped instances */
    int32_t tile_w, tile_h;  /* tile used */
    int32_t n_views;
    double load_balance_fwd; /* after a forward timed by vgr_set_counting bit */
    double load_balance_bwd; /*   1: per compute unit, the summed durations  */
                             /*   of its raster workgroups, max over mean    */
                             /*   (1 = balanced; 0 if not timed)             */
    int32_t emit_mismatch;   /* (Gaussian, view) items whose emitted tiles did */
                             /*   not number exactly the tile count the       */
                             /*   preprocess gave them (0 expected; a nonzero */
                             /*   value is a library defect)                  */
    int32_t _pad;
} vgr_stats;

typedef struct vgr_ctx vgr_ctx;

/* Fill *s with the defaults listed above. */
void vgr_default_settings(vgr_settings *s);

/* Create a context on HIP device `device` (the null stream until
 * vgr_set_stream).  *out receives the handle.  Allocates a small amount of
 * host pinned and device memory.  VGR_ERR_INVALID_ARG, VGR_ERR_HIP. */
int vgr_create(vgr_ctx **out, int device);

/* Release the context and all its memory; waits for its stream first.
 * NULL is accepted. */
void vgr_destroy(vgr_ctx *ctx);

/* Enqueue all later work on `hip_stream` (a hipStream_t; NULL = null
 * stream). */
int vgr_set_stream(vgr_ctx *ctx, void *hip_stream);

/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *vgr_last_error(const vgr_ctx *ctx);

/* Forward render of n Gaussians into n_views views (Sec. 4.1-4.2, Sec. 6.2).
 *   means  n x 3, world-space mean mu_i
 *   quats  n x 4, rotation (w, x, y, z); normalised inside, need not be unit
 *   scales n x 3, standard deviations along the rotated axes, > 0
 *          (Sigma_i = R_i diag(s_i^2) R_i^T)
 *   dens   n, density kappa_i >= 0 (units 1/length), or theta_i in [0, 1]
 *          (settings->density)
 *   sh     n x (sh_degree+1)^2 x 3 colour coefficients (COLOR); may be NULL
 *          in XRAY mode
 *   cams   host array of n_views cameras (1 <= n_views <= 64)
 *   out    host array of n_views device pointers: view v receives
 *          3 x H_v x W_v (COLOR, channel-major) or H_v x W_v (XRAY)
 * The state needed by vgr_render_backward (sorted lists, per-pixel final
 * transmittance and last contributor) is kept in ctx until the next forward.
 * Waits once on the host, for an event recorded right after the preprocess
 * (the instance count that sizes the lists), while the depth sort proceeds.
 * Errors: VGR_ERR_INVALID_ARG (bad sizes, settings or null pointers),
 * VGR_ERR_OOM, VGR_ERR_HIP. */
int vgr_render_forward(vgr_ctx *ctx, const vgr_settings *settings, int64_t n,
                       const float *means, const float *quats, const float *scales,
                       const float *dens, const float *sh, int32_t n_views,
                       const vgr_camera *cams, float *const *out);

/* Backward of the last forward on this context: given dL/d(out) (host array
 * of n_views device pointers, same shapes as `out`), the gradients with
 * respect to d_means (n x 3), d_quats (n x 4), d_scales (n x 3), d_dens (n)
 * and d_sh (same shape as sh; may be NULL in XRAY mode); d_dens is the
 * gradient with respect to the forward's `dens` input (kappa or theta, and
 * with theta the scales receive the path through kappa too).  accumulate = 1:
 * ADD them to the arrays; accumulate = 0: overwrite every element (the
 * arrays are not read, so they need no zeroing).  Gradients flow through the
 * quaternion normalisation; clamped, skipped and unblended (Gaussian, pixel)
 * pairs contribute zero.  The parameter arrays given to the forward must
 * still hold the same values.  Errors: VGR_ERR_NO_FORWARD,
 * VGR_ERR_INVALID_ARG, VGR_ERR_HIP. */
int vgr_render_backward(vgr_ctx *ctx, const float *const *dL_dout, float *d_means,
                        float *d_quats, float *d_scales, float *d_dens, float *d_sh,
                        int32_t accumulate);

/* Densification statistics (Supp. D: the paper thresholds the world-space
 * positional gradient of each Gaussian to decide where to densify).  After
 * this call every backward on the context, and every replay of a graph
 * captured after it (the eager steps that vgr_graph_capture and vgr_autotune
 * run included), ADDS for each Gaussian i
 *   grad_norm_sum[i] += sum over the call's views v of |dL_v/dmu_i|, the
 *                       Euclidean norm of view v's share of d_means[i];
 *   view_count[i]    += the number of those views in which Gaussian i was
 *                       handed to the rasteriser (at least one tile).
 * Both are device arrays owned by the caller (n floats, n int32), either may
 * be NULL; both NULL turns the statistics off.  `capacity` is their length:
 * a later backward with n > capacity fails with VGR_ERR_INVALID_ARG.  The
 * caller clears them (e.g. at each densification step).  A captured graph
 * keeps the arrays (and the on/off state) that were set when it was
 * captured; re-capture after changing them.  Adds one pass over
 * the per-view tile counts (4 bytes per Gaussian and view) to the backward.
 * VGR_ERR_INVALID_ARG for a negative capacity. */
int vgr_set_densify_stats(vgr_ctx *ctx, float *grad_norm_sum, int32_t *view_count,
                          int64_t capacity);

/* Per-pixel state of view `view` of the last forward, copied (on the
 * stream) into caller arrays of H x W: final transmittance T_final (may be
 * NULL) and the index of the last blended Gaussian, -1 if none (may be NULL;
 * in XRAY mode the number of terms summed).  VGR_ERR_NO_FORWARD,
 * VGR_ERR_INVALID_ARG. */
int vgr_get_aux(vgr_ctx *ctx, int32_t view, float *T_final, int32_t *last_index);

/* Counters of the last forward.  Waits for the stream.  When counting is on
 * (vgr_set_counting) the pair counters of the rasteriser are filled. */
int vgr_get_stats(vgr_ctx *ctx, vgr_stats *out);

/* Bit 0: pair counting in the rasterisers (separate instrumented kernel
 * variants; timing runs keep it off).  Bit 1: the rasterisers of eager calls
 * record each workgroup's duration and compute unit, for the load balance in
 * vgr_stats (the production kernels, two clock reads and one store per
 * workgroup).  0 turns both off. */
int vgr_set_counting(vgr_ctx *ctx, int enable);

/* Stage timing with HIP events recorded on the context's stream around each
 * stage (preprocess, sorts, emission, ranges, rasterisers, preprocess
 * backward) of every forward and backward call made since
 * vgr_set_timing(ctx, 1) (which waits for the stream and starts a new
 * series).  vgr_get_timing waits for the stream and writes, for up to `cap`
 * stages, the stage name (static strings) and its mean duration in ms over
 * those calls; *count receives the number of stages written. */
int vgr_set_timing(vgr_ctx *ctx, int enable);
int vgr_get_timing(vgr_ctx *ctx, int32_t cap, const char **names, float *ms, int32_t *count);

/* Capture one whole training step - the forward of all n_views views and the
 * backward - into a HIP graph, for callers that replay the same step (same
 * pointers, sizes and cameras; new values in the arrays) without per-call
 * host work.  Arguments are those of vgr_render_forward and
 * vgr_render_backward together; zero_grads = 1 makes the backward overwrite
 * the gradient arrays (accumulate = 0), 0 makes it add to them.  The
 * pointers are recorded and must stay valid while the graph is used.
 * The call first runs the step once eagerly (its results are valid), then
 * captures with instance lists of capacity_factor (>= 1; default 1.25) times
 * the instance count measured there: graph replays never wait on the host,
 * so a replay whose scene needs more instances than that drops the surplus
 * and raises a device flag that vgr_graph_check reports.  A later call that
 * grows the context's workspace invalidates the graph.  The stream is the
 * context's stream (a private non-blocking stream when that is the null
 * stream).  Errors: as forward/backward, VGR_ERR_HIP on capture failure. */
int vgr_graph_capture(vgr_ctx *ctx, const vgr_settings *settings, int64_t n,
                      const float *means, const float *quats, const float *scales,
                      const float *dens, const float *sh, int32_t n_views,
                      const vgr_camera *cams, float *const *out, const float *const *dL_dout,
                      float *d_means, float *d_quats, float *d_scales, float *d_dens,
                      float *d_sh, float capacity_factor, int32_t zero_grads);

/* Largest number of calls one captured graph holds. */
#define VGR_MAX_GRAPH_CALLS 16

/* Capture several forward + backward calls into one HIP graph: call k renders
 * the views_per_call[k] (host array, each in [1, 64]) cameras that follow the
 * previous calls' in cams / out / dL_dout (host arrays over all views), and
 * its backward adds to the same gradient arrays (call 0 overwrites them when
 * zero_grads is set).  This is the multi-view training step that does not
 * fit one call (more than 64 views, or a working set split on purpose), as
 * one replayable graph.  The calls share the context's workspace one after
 * the other; the instance capacity is capacity_factor times the largest
 * call's count.  Otherwise as vgr_graph_capture.  n_calls in
 * [1, VGR_MAX_GRAPH_CALLS]. */
int vgr_graph_capture_calls(vgr_ctx *ctx, const vgr_settings *settings, int64_t n,
                            const float *means, const float *quats, const float *scales,
                            const float *dens, const float *sh, int32_t n_calls,
                            const int32_t *views_per_call, const vgr_camera *cams,
                            float *const *out, const float *const *dL_dout, float *d_means,
                            float *d_quats, float *d_scales, float *d_dens, float *d_sh,
                            float capacity_factor, int32_t zero_grads);

/* Enqueue one replay of the captured graph.  VGR_ERR_NOT_CAPTURED if there is
 * none or it was invalidated; otherwise returns without waiting. */
int vgr_graph_launch(vgr_ctx *ctx);

/* Wait for the replays enqueued so far.  Returns VGR_ERR_CAPACITY (and
 * clears the flag) if any of them overflowed its instance lists since the
 * last check - their outputs are then incomplete and the caller re-captures
 * - else VGR_OK.  *instances (may be NULL) receives the last replay's
 * instance count. */
int vgr_graph_check(vgr_ctx *ctx, int64_t *instances);

/* Number of launch shapes vgr_autotune times. */
#define VGR_TUNE_CANDIDATES 8

/* Time the step (forward, plus backward when dL_dout is not NULL) for each
 * launch shape: tile 8x8, 16x8, 16x16, 32x8 with 64-record batches, then the
 * same tiles with 32-record batches (candidates 0..7), with HIP events over
 * `iters` calls after one warm-up call.  The fastest becomes the context's
 * shape for calls of the same workload class that leave tile_w = tile_h = 0
 * or batch = 0 (the class: total pixels and Gaussians in powers of two, mode,
 * alpha_model, kernel, tile_resort, near_segment), and its last tuned shape
 * for other classes.  Reports it in *best_tile_w, *best_tile_h, *best_batch
 * and the mean ms of each candidate in ms_per_candidate[VGR_TUNE_CANDIDATES]
 * (any may be NULL).  The gradient arrays receive the sum of all the
 * backward passes run.  The per-class choices persist through
 * vgr_tune_export / vgr_tune_import. */
int vgr_autotune(vgr_ctx *ctx, const vgr_settings *settings, int64_t n, const float *means,
                 const float *quats, const float *scales, const float *dens, const float *sh,
                 int32_t n_views, const vgr_camera *cams, float *const *out,
                 const float *const *dL_dout, float *d_means, float *d_quats,
                 float *d_scales, float *d_dens, float *d_sh, int32_t iters,
                 int32_t *best_tile_w, int32_t *best_tile_h, int32_t *best_batch,
                 float *ms_per_candidate);

/* The context's tuned shapes as text (host buffer of cap bytes, NUL
 * terminated; *len receives the size needed, also when buf is NULL): one line
 * per workload class, "pix_log2 n_log2 mode alpha_model kernel tile_resort
 * near_segment tile_w tile_h batch ms".  VGR_ERR_INVALID_ARG if cap is too
 * small. */
int vgr_tune_export(vgr_ctx *ctx, char *buf, int64_t cap, int64_t *len);

/* Merge tuned shapes written by vgr_tune_export (host text) into the
 * context's cache; lines of a class already present replace it.  A malformed
 * line (wrong field count, unsupported tile or batch) rejects the whole text
 * with VGR_ERR_INVALID_ARG and changes nothing. */
int vgr_tune_import(vgr_ctx *ctx, const char *text);

/* Stable LSD radix sort of n (key, value) pairs on the low `bits` bits of
 * key, in place (keys, vals: device u32 arrays of n).  This is the sort the
 * rasteriser uses to order (tile, depth); exposed for testing.  Equal keys
 * keep their input order.  VGR_ERR_INVALID_ARG, VGR_ERR_OOM, VGR_ERR_HIP. */
int vgr_sort_pairs(vgr_ctx *ctx, uint32_t *keys, uint32_t *vals, int64_t n, int32_t bits);

/* Largest n of vgr_sort_pairs_static. */
#define VGR_STATIC_SORT_MAX (1 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sort of
 * vgr_sort_pairs with the same arguments, results and stream, that allocates
 * nothing.  Its scratch (ping-pong halves and radix tables, 9 MiB) is a
 * static device array of the library, one copy per device, set up by
 * vgr_create; n is limited to VGR_STATIC_SORT_MAX (VGR_ERR_INVALID_ARG above
 * it, before anything is enqueued).  Every call on a device shares that
 * device's copy, so calls that can overlap on one GPU (several contexts or
 * streams) race and must be serialised by the caller.  Does not touch the
 * context's saved forward.  VGR_ERR_INVALID_ARG, VGR_ERR_HIP. */
int vgr_sort_pairs_static(vgr_ctx *ctx, uint32_t *keys, uint32_t *vals, int64_t n, int32_t bits);

#ifdef __cplusplus
}
#endif

#endif /* VGR_H */

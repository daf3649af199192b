/*
 * gsr.h -- C ABI of the MI355X (gfx950) differentiable Gaussian rasterizer.
 *
 * The paper this library serves (On-the-fly Large-scale 3D Reconstruction
 * from Multi-Camera Rigs) optimises a set of 3D Gaussians -- position, scale,
 * rotation, opacity and spherical-harmonic colour -- jointly by gradient steps
 * through a differentiable renderer (Sec. 3.3, "Optimization"), drawing the
 * frames of several rig cameras and a window of keyframes per iteration
 * (Sec. 3.3, "Frequency-based Scheduling").  The renderer is the tile-based
 * rasterizer of 3D Gaussian Splatting, which the paper inherits without
 * restating.  This library is that per-iteration hot path: EWA projection,
 * (view | tile | depth) binning with an LDS radix sort, front-to-back alpha
 * compositing, the reverse-order adjoint, an L1 photometric loss and a fused
 * Adam step, for a batch of views of arbitrary resolutions in one launch per
 * stage.
 *
 * Conventions shared by every entry point:
 *  - Array pointers are DEVICE pointers owned by the caller, unless a comment
 *    says HOST.  Floating-point arrays are float32, structure-of-arrays,
 *    C-contiguous, at least 16-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Render, loss and optimiser calls only enqueue work on it: they never
 *    synchronise, allocate or copy to the host, so a caller may capture them
 *    in a hipGraph.  gsr_plan, gsr_check, gsr_required_capacity and
 *    gsr_autotune synchronise.
 *  - Errors are returned as gsr_status; gsr_last_error() holds a message.
 *    Invalid arguments are rejected before any work is enqueued.
 *  - A context is not thread-safe; use one per stream.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsr_ctx gsr_ctx;

typedef enum {
  GSR_OK = 0,
  GSR_ERR_INVALID_ARG = -1, /* a pointer, size or option is invalid                    */
  GSR_ERR_CAPACITY = -2,    /* visible records or tile pairs exceeded the plan's capacity */
  GSR_ERR_HIP = -3,         /* a HIP runtime call failed                                 */
  GSR_ERR_UNSUPPORTED = -4, /* a value the library does not handle (e.g. SH degree > 3)  */
  GSR_ERR_NOT_PLANNED = -5  /* render called before gsr_plan, or with other sizes        */
} gsr_status;

/* Gaussian parameters (Sec. 3.3 optimises all of them), n Gaussians:
 *   mean          [3][n]   world position x, y, z
 *   log_scale     [3][n]   log of the per-axis standard deviation (s = exp)
 *   quat          [4][n]   rotation (w, x, y, z); normalised inside the
 *                          renderer, gradient taken through the normalisation;
 *                          a zero quaternion culls the Gaussian
 *   opacity_logit [n]      opacity = sigmoid(opacity_logit)
 *   sh            [K][3][n] colour coefficients, K = (sh_degree+1)^2, real
 *                          orthonormal SH basis ordered l^2 + l + m; colour =
 *                          max(0, sum_k sh_k Y_k(d) + 0.5), d the unit vector
 *                          from the camera centre to the mean.            */
typedef struct {
  int64_t n;
  int32_t sh_degree; /* 0..3 */
  const float *mean;
  const float *log_scale;
  const float *quat;
  const float *opacity_logit;
  const float *sh;
} gsr_gaussians;

/* Pinhole camera, world -> camera x_c = R x_w + t, R row-major, OpenCV axes
 * (x right, y down, z forward).  Pixel (i, j) has its centre at
 * (i + 0.5, j + 0.5).  72 bytes; arrays of these are passed to render calls
 * in DEVICE memory so poses can change between graph replays.            */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} gsr_camera;

typedef struct {
  int32_t tile_size;        /* 8, 16 or 32; 0 = the context's tuning (16 unless set by
                               gsr_set_tuning or gsr_autotune)                         */
  int64_t capacity_records; /* visible (view, Gaussian) records; 0 = n_views * n (exact) */
  int64_t capacity_pairs;   /* (record, tile) pairs; 0 = 8 * n_views * n                 */
  float bg[3];              /* background colour                                       */
} gsr_plan_options;

/* Forward outputs, flat over views: view v starts at pixel offset pix_off[v]
 * (from gsr_plan).  image is planar per view: view v occupies
 * image[3*pix_off[v] .. 3*pix_off[v+1]) as [3][H_v][W_v].                   */
typedef struct {
  float *image;        /* [3 * total_pixels]                                      */
  float *t_final;      /* [total_pixels] transmittance after the last composite    */
  uint32_t *last_pos;  /* [total_pixels] one past the last composited position in
                          the pixel's tile list (0 if none); read by the backward */
  uint32_t *n_contrib; /* [total_pixels] number of composited Gaussians            */
} gsr_fwd_out;

/* Parameter gradients, same layouts as gsr_gaussians; every entry is written
 * (invisible Gaussians get zeros).
 *  camera  optional (NULL: not computed): [n_views][12] pose gradient of
 *          each view, dL/dR (row-major, R taken as a general 3x3 matrix) then
 *          dL/dt of x_c = R mu + t, through the projection geometry only --
 *          the paper updates camera parameters jointly with the Gaussians and
 *          detaches the SH colour from that update (Sec. 3.3, "Optimization").
 *          Summed per view in a fixed order (deterministic).  gsr_adam_step
 *          ignores it.                                                      */
typedef struct {
  float *mean, *log_scale, *quat, *opacity_logit, *sh;
  float *camera;
} gsr_grads;

/* Create / destroy a context.  The context owns a few device words (status
 * flags, counters) allocated here.                                          */
gsr_status gsr_create(gsr_ctx **out);
void gsr_destroy(gsr_ctx *ctx);

/* Plan a batch: n_views cameras (HOST array; only width/height and the
 * intrinsics' image extents are used here), n Gaussians of degree sh_degree.
 * Fixes the tile grid of every view, the workspace layout and capacities.
 * Outputs: *workspace_bytes, the size of the caller-allocated DEVICE workspace
 * each render call needs; pix_off (HOST, n_views + 1 entries) the per-view
 * pixel offsets.  Synchronises (uploads the per-view tile table).
 * The plan also fixes the context's current work split (gsr_tuning).
 * Errors: INVALID_ARG for n_views < 1, n < 0, a non-positive image size, a
 * tile size other than 0/8/16/32, or sizes beyond the 32-bit index range;
 * UNSUPPORTED for sh_degree outside 0..3.                                   */
gsr_status gsr_plan(gsr_ctx *ctx, const gsr_camera *cams_host, int32_t n_views, int64_t n,
                    int32_t sh_degree, const gsr_plan_options *opt, size_t *workspace_bytes,
                    int64_t *pix_off);

/* Forward render of every planned view (the 3DGS image model the paper
 * renders with, Sec. 3.3): projection, binning, per-tile sort, compositing.
 * cams: DEVICE array of n_views gsr_camera (same sizes as planned).  The
 * workspace keeps the binning state that gsr_render_backward and
 * gsr_debug_binning read; it must not be modified in between.  If the visible
 * records or pairs exceed the capacity, the kernels skip the excess work and
 * set a device flag that gsr_check reports as GSR_ERR_CAPACITY.            */
gsr_status gsr_render_forward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams,
                              int32_t n_views, void *workspace, size_t workspace_bytes,
                              const gsr_fwd_out *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * gsr_render_forward with its workspace in the library's own device scratch
 * instead of a caller buffer -- a fixed array of GSR_NOALLOC_SCRATCH_BYTES
 * (64 MiB), one per GPU, held from the first gsr_create on that GPU until
 * the process ends.  The call allocates nothing and enqueues only; the
 * caller still passes the inputs and the outputs (as for gsr_render_forward,
 * whose outputs it reproduces bit for bit).  The context's plan must need a
 * workspace of at most GSR_NOALLOC_SCRATCH_BYTES (gsr_plan's
 * workspace_bytes), else GSR_ERR_CAPACITY; the current device must be the
 * one the context was created on, else GSR_ERR_INVALID_ARG.  Every context
 * on a GPU shares that GPU's scratch, which keeps the last call's contents
 * (the forward clears what it needs): calls that may overlap on one GPU
 * (other streams, other host threads) race and must be serialised by the
 * caller, and only the last forward's state is there for gsr_check and
 * gsr_required_capacity, which read it when passed workspace = NULL.     */
#define GSR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
gsr_status gsr_render_forward_noalloc(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams,
                                      int32_t n_views, const gsr_fwd_out *out, void *stream);

/* L1 photometric loss over n_elems image values (all views, channels, pixels):
 * loss = sum |image - target| / n_elems, written to loss_out (DEVICE, 1
 * float); dL_dimage[i] = sign(image[i] - target[i]) / n_elems.  Deterministic
 * (fixed-order reduction).                                                  */
gsr_status gsr_l1_loss(gsr_ctx *ctx, const float *image, const float *target, int64_t n_elems,
                       float *loss_out, float *dL_dimage, void *stream);

/* gsr_render_forward with the L1 loss of gsr_l1_loss fused into the
 * compositing epilogue: target (same layout as the image, all planned
 * pixels), *loss_out (DEVICE float), dL_dimage (same layout).  dL_dimage is
 * bit for bit that of gsr_l1_loss; the loss is summed per wave and then in a
 * fixed order (deterministic, and equal to gsr_l1_loss up to the order of
 * the float additions).  The image and the fwd outputs are as for
 * gsr_render_forward.                                                       */
gsr_status gsr_render_forward_l1(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                 void *workspace, size_t workspace_bytes, const gsr_fwd_out *out,
                                 const float *target, float *loss_out, float *dL_dimage, void *stream);

/* Reverse-order adjoint of gsr_render_forward: from dL/dimage (same layout as
 * the image) to gradients of every Gaussian parameter.  Reads the forward's
 * workspace state and the fwd outputs t_final / last_pos.  Overwrites grads
 * (accumulate = 0) or adds to them (accumulate = 1).  Deterministic: no
 * floating-point atomics.                                                   */
gsr_status gsr_render_backward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams,
                               int32_t n_views, void *workspace, size_t workspace_bytes,
                               const gsr_fwd_out *fwd, const float *dL_dimage,
                               const gsr_grads *grads, int32_t accumulate, void *stream);

/* Adam hyper-parameters: one learning rate per group, in this order:
 * mean, log_scale, quat, opacity_logit, sh degree 0 (the first 3n sh
 * entries), sh higher degrees.                                              */
typedef struct {
  float lr[6];
  float beta1, beta2, eps;
} gsr_adam_config;

/* Optimizer state in the gsr_grads layout (first and second moments). */
typedef struct {
  float *mean, *log_scale, *quat, *opacity_logit, *sh;
} gsr_adam_moments;

/* One dense Adam step with bias correction over all parameters (the paper's
 * joint gradient update, Sec. 3.3), in one launch.  params are updated in
 * place (the gsr_gaussians pointers, cast to writable).  step_dev: DEVICE
 * int32 step counter, incremented on the device before use, so a captured
 * graph replays correctly.                                                  */
gsr_status gsr_adam_step(gsr_ctx *ctx, const gsr_grads *params, const gsr_grads *grads,
                         const gsr_adam_moments *m, const gsr_adam_moments *v,
                         const gsr_adam_config *cfg, int32_t *step_dev, int64_t n,
                         int32_t sh_degree, void *stream);

/* Backward and Adam fused: the per-Gaussian backward applies the Adam update
 * directly, without writing gradients (grads_out may be NULL) -- same result
 * as gsr_render_backward followed by gsr_adam_step with grads zeroed first.
 * grads_out, if given, receives the gradients too: its five Gaussian
 * pointers all set or all NULL, its camera pointer as in gsr_grads (the
 * pose gradient for a separate camera update).  params may be the arrays
 * of g (updated in place) or other arrays; params, m, v and grads_out must
 * not overlap one another.                                                 */
gsr_status gsr_render_backward_adam(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams,
                                    int32_t n_views, void *workspace, size_t workspace_bytes,
                                    const gsr_fwd_out *fwd, const float *dL_dimage,
                                    const gsr_grads *params, const gsr_adam_moments *m,
                                    const gsr_adam_moments *v, const gsr_adam_config *cfg,
                                    int32_t *step_dev, const gsr_grads *grads_out, void *stream);

/* Export the binning of the last forward for parity checks: keys[M] =
 * (global tile) << 32 | depth bits, vals[M] = Gaussian index, sorted
 * ascending by (key, value); tile_csr[T_total + 1] the list offsets.  Buffers
 * are DEVICE, sized from gsr_required_capacity.                            */
gsr_status gsr_debug_binning(gsr_ctx *ctx, void *workspace, uint64_t *keys, uint32_t *vals,
                             uint32_t *tile_csr, void *stream);

/* Compositing work of the last forward, for roofline accounting: writes to
 * *evals (DEVICE, one uint64) the number of (pixel, list entry) pairs with
 * the entry in front of the pixel's stop position fwd->last_pos and the
 * pixel inside the entry's binning box (Sec. 3.3 compositing order), summed
 * over all pixels of all views.  These are the evaluations the backward
 * performs; the forward performs the same plus the entries between a
 * pixel's last composited Gaussian and its stop.  Reads the workspace and
 * fwd->last_pos only; the count is 0 after a capacity overflow.            */
gsr_status gsr_count_evaluations(gsr_ctx *ctx, void *workspace, const gsr_fwd_out *fwd, uint64_t *evals,
                                 void *stream);

/* Measurement: copy `bytes` (a multiple of 16) from src to dst (DEVICE,
 * 16-byte aligned, not overlapping) with the library's streaming copy
 * kernel, to time the achievable HBM bandwidth against which the kernels'
 * bytes are reported.  Enqueues only; GSR_ERR_INVALID_ARG on a misaligned or
 * NULL pointer or a size that is not a multiple of 16.  Needs no context.   */
gsr_status gsr_copy_bytes(void *dst, const void *src, size_t bytes, void *stream);

/* Synchronise `stream`, then report GSR_ERR_CAPACITY if the last forward ran
 * out of record or pair capacity, else GSR_OK.  workspace = NULL reads the
 * no-alloc scratch of the context's GPU (after gsr_render_forward_noalloc).  */
gsr_status gsr_check(gsr_ctx *ctx, void *workspace, void *stream);

/* Synchronise `stream` and read the record and pair counts the last forward
 * needed (valid also after a capacity overflow), and the total tile count.
 * workspace = NULL: the no-alloc scratch, as for gsr_check.                 */
gsr_status gsr_required_capacity(gsr_ctx *ctx, void *workspace, int64_t *records, int64_t *pairs,
                                 int64_t *tiles, void *stream);

/* Stage timing.  While enabled, every render / loss / Adam call records HIP
 * events around each of its stages on its own stream, waits for them, and
 * accumulates the elapsed milliseconds per stage (so it synchronises: not
 * for use under graph capture).  gsr_profile_read copies the per-stage
 * totals and call counts into HOST arrays of GSR_N_STAGES entries, indexed
 * by gsr_stage, and optionally resets them.                               */
#define GSR_N_STAGES 9
typedef enum {
  GSR_STAGE_PREPROCESS = 0, /* projection, record compaction                 */
  GSR_STAGE_BINNING = 1,    /* pair emission, tile sort, list bounds, order  */
  GSR_STAGE_SORT = 2,       /* depth sort of the records (runs before binning) */
  GSR_STAGE_RASTER_FWD = 3, /* forward compositing                           */
  GSR_STAGE_LOSS = 4,       /* L1 loss and its gradient                      */
  GSR_STAGE_RASTER_BWD = 5, /* backward compositing                          */
  GSR_STAGE_REDUCE = 6,     /* per-record sum of the per-tile partials       */
  GSR_STAGE_PRE_BWD = 7,    /* per-Gaussian chain rule (with Adam if fused)  */
  GSR_STAGE_ADAM = 8        /* standalone Adam step                          */
} gsr_stage;
gsr_status gsr_profile(gsr_ctx *ctx, int32_t enable);
gsr_status gsr_profile_read(gsr_ctx *ctx, double *ms, int64_t *calls, int32_t reset);

/* Launch configuration of the compositing kernels.  Images do not depend on
 * it (the pixel boxes are exact, so the tile size only changes which lists
 * a Gaussian is binned into); gradients change only by the summation order
 * of the per-record reductions.
 *  tile_size  8, 16 or 32.
 *  long_list  16 px tiles: in the backward, tiles whose list has at least
 *             this many entries are walked by a workgroup of four waves (an
 *             8 x 8 quadrant each, one pixel per lane); shorter tiles take one
 *             wave each (four pixels per lane), four tiles per workgroup.
 *             0 sends every tile to the four-wave walk, 0xFFFFFFFF none.
 *  persistent 0: one workgroup per work item (a tile, or at 16 px a group
 *             of four short tiles), dispatched by the hardware in the
 *             longest-first order.  1: a persistent launch of as many
 *             workgroups as the device holds at once, each taking work items
 *             in that order from a queue of eight device counters (one per
 *             XCD) until none is left.  Results are identical.
 *  step_ms    (gsr_autotune output) measured forward + backward time.     */
typedef struct {
  int32_t tile_size;
  uint32_t long_list;
  int32_t persistent;
  float step_ms;
} gsr_tuning;

/* Set the tuning (HOST struct) used by the next gsr_plan, or read the
 * current one.  Defaults: tile size 16, long_list 1024, persistent 0.
 * Errors: INVALID_ARG for a tile size other than 8/16/32 or persistent
 * other than 0/1.                                                          */
gsr_status gsr_set_tuning(gsr_ctx *ctx, const gsr_tuning *t);
gsr_status gsr_get_tuning(gsr_ctx *ctx, gsr_tuning *t);

/* Rig parameterisation of the view poses (Sec. 3.1, Eq. 3, and Sec. 3.3,
 * "Optimization"): the cameras of the rig are rigidly linked, so view v --
 * camera c = view_camera[v] of the rig at frame f = view_frame[v] -- has the
 * extrinsics T_v = T_m^f T_{c->m}, the product (in the order the paper
 * writes it) of the central camera's pose at frame f and camera c's fixed
 * relative transform.  A pose is 12 floats: R row-major, then t, of the map
 * x -> R x + t from world to camera coordinates (the gsr_camera R, t).
 *
 * gsr_rig_plan: set the rig structure (HOST arrays of n_views indices,
 * copied; synchronises).  Errors: INVALID_ARG for an index outside
 * [0, n_frames) / [0, n_cams) or a negative size.                          */
gsr_status gsr_rig_plan(gsr_ctx *ctx, const int32_t *view_frame, const int32_t *view_camera, int32_t n_views,
                        int32_t n_frames, int32_t n_cams);

/* Write T_v into cams[v].R, cams[v].t for every view of the rig plan
 * (central [n_frames][12], relative [n_cams][12]; cams a DEVICE array of
 * gsr_camera whose intrinsics and sizes are left as they are).            */
gsr_status gsr_rig_compose(gsr_ctx *ctx, const float *central, const float *relative, gsr_camera *cams,
                           void *stream);

/* Carry the views' pose gradients view_grads [n_views][12] (gsr_grads.camera)
 * back through T_v = T_m^f T_{c->m}: d_central [n_frames][12] = dL/dT_m^f,
 * d_relative [n_cams][12] = dL/dT_{c->m} (written, summed over the views in
 * view order), and optionally (NULL: skipped) the same in the tangent of a
 * left perturbation T <- exp(xi^) T, xi = (rho, phi) with rho the
 * translation part: xi_central [n_frames][6], xi_relative [n_cams][6].
 * The paper fixes no update rule for the poses; these are what one needs.  */
gsr_status gsr_rig_gradients(gsr_ctx *ctx, const float *central, const float *relative, const float *view_grads,
                             float *d_central, float *d_relative, float *xi_central, float *xi_relative,
                             void *stream);

/* Frequency-based scheduling (Sec. 3.3, "Frequency-based Scheduling",
 * Eqs. 9-12).  The frequency significance of an RGB image is
 *   X(I) = sum over all frequency bins (i, j) of || DFT(I)(i, j) ||_2,
 * the unnormalised 2D DFT of each channel with the 2-norm taken over the
 * three channels' complex values at the bin.
 *
 * gsr_freq_plan: fix a batch of images (HOST arrays of n_images widths and
 * heights, copied; synchronises) and return the workspace size.  Each side
 * must be 1..2560 with no prime factor above 7.  Errors: UNSUPPORTED for
 * other sizes.                                                             */
gsr_status gsr_freq_plan(gsr_ctx *ctx, const int32_t *widths, const int32_t *heights, int32_t n_images,
                         size_t *workspace_bytes);

/* X of every planned image: images holds them planar [3][h][w], one after
 * the other in plan order (the layout of gsr_fwd_out.image); X [n_images].
 * workspace: DEVICE, 256-byte aligned, of the planned size (the half spectra
 * of the batch, 24 bytes per pixel and column pair).  Deterministic.      */
gsr_status gsr_freq_significance(gsr_ctx *ctx, const float *images, void *workspace, size_t workspace_bytes,
                                 float *X, void *stream);

/* I^n of the level-of-detail structure: the mean over n x n blocks of a
 * planar [3][height][width] image into dst [3][height/n][width/n] (rows and
 * columns beyond a multiple of n dropped).                                */
gsr_status gsr_downsample(gsr_ctx *ctx, const float *src, int32_t width, int32_t height, int32_t factor, float *dst,
                          void *stream);

/* One scheduling step over n_frames frames (all arrays DEVICE, float32):
 *  r[f]  = x_gt[f] / x_render[f]            (Eq. 9; x_gt = X of the full-
 *                                           resolution ground truth, x_render
 *                                           = X of the current render)
 *  r'[f] = x_gt_level[f] / x_render[f]      (Eq. 12; the ground truth at the
 *                                           frame's current downsampling)
 *  levels[f] -= 1 where r'[f] < tau_f and levels[f] > 0 (one level finer;
 *                                           level 0 = full resolution)
 *  picks[b] = the first frame whose inclusive prefix sum of the weights
 *             exceeds uniforms[b] * (their total), the weights being r capped
 *             at FLT_MAX / (2 n_frames), NaN taken as 0; uniform draws
 *             floor(u n_frames) if all weights are 0.  The paper samples the
 *             frames to optimise by r; the random numbers are the caller's.
 * r, r_prime, levels (with x_gt_level) and picks (with uniforms) may each be
 * NULL.  n_frames <= 16384.  The paper sets tau_f = 2 (Sec. 4).           */
gsr_status gsr_freq_schedule(gsr_ctx *ctx, const float *x_gt, const float *x_gt_level, const float *x_render,
                             int32_t n_frames, float tau_f, int32_t *levels, const float *uniforms, int32_t n_picks,
                             float *r, float *r_prime, int32_t *picks, void *stream);

/* LoG-based insertion of new Gaussians (Sec. 3.2, "Redundancy-free Gaussian
 * Sampling", Eqs. 4-6), over all planned views:
 *   P(I)  = min(|| LoG_sigma * I ||_2, 1) per pixel, the norm over the three
 *           channels' responses; LoG_sigma sampled at offsets -R..R,
 *           R = ceil(3 sigma), as h x g + g x h with g the Gaussian (sum 1)
 *           and h its second derivative (sum 0, second moment 2); image
 *           borders replicated.
 *   P_a   = max(P(I) - P(I~), 0); a pixel inserts a Gaussian when P_a > tau_a.
 *   S     = d / (2 sqrt(P(I)) fx), d = |x_c| for the pixel centre back-
 *           projected to the depth map's z: x_c = z ((u + 0.5 - cx) / fx,
 *           (v + 0.5 - cy) / fy, 1); centre x_w = R^T (x_c - t).
 * gt, render: flat planar images of all views (the gsr_fwd_out.image
 * layout); depth: [total_pixels] z-depth; p_gt [total_pixels] receives P(I),
 * p_render (optional) P(I~).  The inserting pixels are listed in ascending
 * flat pixel index: out->pix, out->scale, out->mean [capacity][3]; *count
 * (DEVICE) receives their number, which may exceed capacity (then only the
 * first capacity are written).  workspace: DEVICE, 256-byte aligned, of
 * gsr_insert_workspace bytes (about one byte per pixel).  The paper sets
 * tau_a = 0.2 (Sec. 4) and leaves sigma open (0 < sigma <= 5/3 here, so
 * R <= 5 and a tile with its halo fits the 64 KB of LDS of a workgroup).  */
typedef struct {
  float sigma;
  float tau_a;
} gsr_insert_config;

typedef struct {
  uint32_t *pix;
  float *scale;
  float *mean;
  uint32_t *count;
  int64_t capacity;
} gsr_insert_out;

gsr_status gsr_insert_workspace(gsr_ctx *ctx, size_t *bytes);
gsr_status gsr_log_insert(gsr_ctx *ctx, const gsr_camera *cams, const float *gt, const float *render,
                          const float *depth, const gsr_insert_config *cfg, float *p_gt, float *p_render,
                          const gsr_insert_out *out, void *workspace, size_t workspace_bytes, void *stream);

/* Per-camera merging (Sec. 3.2, Eqs. 7-8): before the samples of camera i
 * (gsr_log_insert's list; only those in view `view` are used) are added,
 * each existing Gaussian g (mean, log_scale and the degree-0 SH of `g`) is
 * reprojected into the view: x' = (fx x/z + cx, fy y/z + cy) of x_c = R mu + t,
 * d' = |x_c|.  If z > 0.2 and x' lies in [0, W) x [0, H), g corresponds to the
 * sampled pixel, among the four pixel centres around x', with the largest
 * positive bilinear weight (lowest pixel index on equal weights; the paper
 * matches x' and the sampled pixels by bilinear interpolation of P), provided
 * | d' - d | <= tau_d (d the sample centre's distance).  Each member of a
 * group (a sample and its corresponding Gaussians) is measured against the
 * view's scale where it sits: rho = s' / s_i(x'), s' = kappa S fx / d' (S =
 * exp of the mean log-scale; the paper prints kappa = 2, which disagrees with
 * Eqs. 6 and 8 by that factor), s_i(x') = 1 / (2 sqrt(P(x'))) with P(I)
 * (p_gt from gsr_log_insert) interpolated bilinearly at x', borders
 * replicated; a sample's own rho is 1.  Only the smallest rho survives
 * (existing Gaussians win ties, the lower index first); the survivor takes
 * the group's mean colour (the Gaussians' DC colour Y0 sh_0 + 1/2, the
 * sample's ground-truth pixel gt) and, re-aligning the depth (a reading: the
 * paper does not say how), is moved along the view's ray through it to the
 * group's mean distance.  The geometry is evaluated in double precision.
 * Outputs (DEVICE): keep [n] and colour [3][n] (RGB, planar) for the
 * Gaussians, keep_new and colour_new [capacity][3] for the view's samples
 * (entries of other views untouched); optionally (NULL to skip) mean [3][n],
 * the Gaussians' centres after the re-alignment (unchanged where not
 * moved), and mean_new [capacity][3], the samples' centres likewise.
 * Deterministic (integer atomics only).  A pixel must appear at most once in
 * the sample list, as gsr_log_insert writes it.
 * workspace: DEVICE, 256-byte aligned, gsr_merge_workspace(n) bytes (48
 * bytes per pixel of the largest view plus 4 per Gaussian).  tau_d is open
 * in the paper: a parameter.  Errors: GSR_ERR_INVALID_ARG for a NULL required
 * pointer, a view out of range, tau_d < 0, kappa <= 0, a short or unaligned
 * workspace; GSR_ERR_NOT_PLANNED before gsr_plan. */
typedef struct {
  float tau_d;
  float kappa;
} gsr_merge_config;

typedef struct {
  uint8_t *keep;
  float *colour;
  uint8_t *keep_new;
  float *colour_new;
  float *mean;     /* optional [3][n] */
  float *mean_new; /* optional [capacity][3] */
} gsr_merge_out;

gsr_status gsr_merge_workspace(gsr_ctx *ctx, int64_t n, size_t *bytes);
gsr_status gsr_merge(gsr_ctx *ctx, const gsr_gaussians *g, int32_t view, const gsr_camera *cams, const float *gt,
                     const float *p_gt, const gsr_insert_out *samples, const gsr_merge_config *cfg,
                     const gsr_merge_out *out, void *workspace, size_t workspace_bytes, void *stream);

/* Autotuner of the batched launch (the keyframe-window batches of Sec. 3.3
 * mix resolutions, so no one tile size suits all): times forward plus
 * backward on this batch for tile sizes 8, 16 and 32 and, at 16, for
 * long_list in {0, 256, 512, 1024, 0xFFFFFFFF}, each with the grid and the
 * persistent schedule (gsr_tuning), and keeps the fastest (median of
 * `repeats` >= 1 timed passes after one warm-up pass); candidates are tried
 * grid schedule first, 16 px with long_list 1024 first, and a later one is
 * kept only if at least 1% faster than the choice so far.
 * g: the Gaussians (DEVICE arrays); cams_host: HOST cameras; opt: capacities
 * and background as for gsr_plan (tile_size ignored; NULL = defaults).  With
 * cache_path (NULL = none) the choice is looked up first in that text file,
 * keyed by the device (architecture and compute units) and the batch shape
 * (n, SH degree, view sizes), and appended to it after a measurement.
 * On success *best (HOST) holds the choice, the context's tuning is set to
 * it and the context is left UNPLANNED: call gsr_plan again (tile size 0
 * takes the tuned one) and size the workspace from it.  Allocates and frees
 * its own device buffers (a few times the workspace of one plan) and
 * synchronises `stream`: not for graph capture.  The gradients it computes
 * are discarded.  No prior gsr_plan is needed.  Errors: INVALID_ARG (also
 * when the cache file cannot be written, or a cached line is malformed),
 * CAPACITY if the batch does not fit 32-bit pair indices, HIP for failed
 * allocations or launches.                                                  */
gsr_status gsr_autotune(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams_host, int32_t n_views,
                        const gsr_plan_options *opt, int32_t repeats, const char *cache_path, gsr_tuning *best,
                        void *stream);

/* Message of the context's last failure; with ctx NULL, that of this
 * thread's last failed call that takes no context (gsr_copy_bytes).  The
 * string is owned by the library and valid until the next call.            */
const char *gsr_last_error(const gsr_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */

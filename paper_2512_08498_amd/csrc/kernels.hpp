// Host-side launchers of the rasterizer kernels (one translation unit per
// stage; the runtime calls these in stream order).
#pragma once

#include "common.hpp"
#include "gsr.h"

namespace gsr {

struct GaussPtrs {
  const float *mean, *log_scale, *quat, *opacity_logit, *sh;
};

struct MutPtrs {
  float *mean, *log_scale, *quat, *opacity_logit, *sh;
};

// Rig structure: view v is camera cam[v] of the rig at frame frame[v]
// (DEVICE arrays, validated on the host).
struct RigIdx {
  const int32_t *frame, *cam;
  int32_t n_views, n_frames, n_cams;
};

// One image of a frequency-significance batch: planar RGB [3][h][w] at float
// offset pix_off; its half spectrum (w/2 + 1 columns of h bins per channel,
// column-major) at float2 offset inter_off; its rows and half-spectrum
// columns numbered from row_base and col_base across the batch.  fac_* are
// the radices of the row (w) and column (h) transforms, tw_* the offsets of
// their twiddle tables exp(-2 pi i t / n), t < n, in the batch's table.
struct FreqImg {
  int32_t w, h, nfac_w, nfac_h;
  uint8_t fac_w[16], fac_h[16];
  int64_t pix_off, inter_off, row_base, col_base, tw_w, tw_h;
};

// Taps of the sampled LoG: g (Gaussian, sum 1) and h (second derivative,
// sum 0, second moment 2) at offsets -R..R, R <= 5 (room for R <= 8).
struct LogTaps {
  float g[17], h[17];
  int32_t R;
};

// L1 loss fused into the forward compositing (NULL target: none): per
// pixel dl = sign(image - target) * inv_n and the sum of |image - target|
// per workgroup into part[workgroup].
struct LossArgs {
  const float *target;
  float *dl;
  float *part;
  float inv_n;
};

struct AdamArgs {
  MutPtrs p, m, v;
  float lr[6];
  float beta1, beta2, eps;
  int32_t *step;
  int32_t p_is_g;  // the parameters p are the rendered Gaussians' own arrays (values already loaded)
};

void launch_zero(uint32_t *p, uint64_t n_words, hipStream_t st);
void launch_preprocess(const GaussPtrs &gp, const Cam *cams, const ViewInfo *views, const Ws &ws,
                       const Sizes &sz, int sh_degree, uint32_t *zero, uint64_t n_zero, hipStream_t st);
void launch_depth_sort(const Ws &ws, const Sizes &sz, hipStream_t st);
void launch_binning(const ViewInfo *views, const Ws &ws, const Sizes &sz, hipStream_t st);
void launch_tile_csr(const Ws &ws, const Sizes &sz, uint32_t *csr, hipStream_t st);
void launch_raster_fwd(const ViewInfo *views, const Ws &ws, const Sizes &sz, float *image, float *t_final,
                       uint32_t *last_pos, uint32_t *n_contrib, const LossArgs &loss, hipStream_t st);
void launch_l1_sum(const float *partials, uint32_t nb, int64_t n, float *loss, hipStream_t st);
void launch_copy16(void *dst, const void *src, uint64_t n16, hipStream_t st);
uint32_t raster_fwd_grid(const Sizes &sz);
void launch_raster_bwd(const ViewInfo *views, const Ws &ws, const Sizes &sz, const float *t_final,
                       const uint32_t *last_pos, const float *dL_dimage, hipStream_t st);
void launch_reduce_pairs(const Ws &ws, const Sizes &sz, int32_t *step, hipStream_t st);
void launch_pre_bwd(const GaussPtrs &gp, const Cam *cams, const Ws &ws, const Sizes &sz, int sh_degree,
                    const MutPtrs *grads, int accumulate, const AdamArgs *adam, float4 *cam_rec, hipStream_t st);
uint32_t cam_chunks(uint32_t cap_rec);
void launch_freq_significance(const float *images, const FreqImg *imgs, int n_imgs, int64_t n_rows, int64_t n_cols,
                              int max_w, int max_h, const float2 *tw, float2 *inter, float *col_sum, float *X,
                              hipStream_t st);
uint32_t ins_tiles(const ViewInfo *views_host, int n_views);
uint32_t ins_blocks(int64_t n_pix);
size_t ins_lds_bytes(int R);
void launch_log_insert(const ViewInfo *views_d, int n_views, uint32_t n_tiles, int64_t n_pix, const Cam *cams,
                       const float *gt, const float *rd, const float *depth, const LogTaps &taps, float tau,
                       float *p_gt, float *p_rd, uint8_t *mask, uint32_t *counts, uint32_t *offsets,
                       uint32_t *total, uint32_t *out_pix, float *out_scale, float *out_mean, int64_t capacity,
                       hipStream_t st);
// Device scratch of gsr_render_forward_noalloc (scratch.hip): its size, and
// the address of a device's copy (looked up once per device).
constexpr size_t kScratchBytes = GSR_NOALLOC_SCRATCH_BYTES;
hipError_t scratch_address(int device, void **out);

// Per-pixel (of the view) and per-Gaussian scratch of the merge.
struct MergeBufs {
  int32_t *slot;
  uint32_t *cnt;
  unsigned long long *csum, *dsum, *win;
  int32_t *match;
};
void launch_merge(const GaussPtrs &gp, int64_t n, const Cam *cams, int view, const ViewInfo &vi, const float *gt,
                  const float *p_gt, const uint32_t *pix, const float *s_mean, const uint32_t *count,
                  int64_t capacity, float tau_d, float kappa, const MergeBufs &mb, uint8_t *keep, float *colour,
                  float *mean_out, uint8_t *keep_new, float *colour_new, float *mean_new, hipStream_t st);
void launch_downsample(const float *src, int W, int H, int n, float *dst, hipStream_t st);
void launch_freq_schedule(const float *x_gt, const float *x_gt_level, const float *x_render, int F, float tau_f,
                          int32_t *levels, const float *u, int n_picks, float *r, float *rp, int32_t *picks,
                          hipStream_t st);
void launch_cam_grads(const Ws &ws, const Sizes &sz, const float4 *cam_rec, float *cam_part, float *out,
                      int accumulate, hipStream_t st);
void launch_rig_compose(const float *central, const float *relative, const RigIdx &ri, Cam *cams, hipStream_t st);
void launch_rig_grads(const float *central, const float *relative, const float *view_grads, const RigIdx &ri,
                      float *d_central, float *d_relative, float *xi_central, float *xi_relative, hipStream_t st);
void launch_adam(const MutPtrs &grads, const AdamArgs &a, int64_t n, int sh_degree, hipStream_t st);
void launch_step_inc(int32_t *step, hipStream_t st);
void launch_l1(const float *img, const float *tgt, int64_t n, float *loss, float *dl, float *partials,
               hipStream_t st);
void launch_debug_binning(const ViewInfo *views, const Ws &ws, const Sizes &sz, uint64_t *keys,
                          uint32_t *vals, uint32_t *csr, hipStream_t st);
void launch_fill(float *p, uint64_t n, float value, hipStream_t st);
void launch_count_evals(const ViewInfo *views, const Ws &ws, const Sizes &sz, const uint32_t *last_pos,
                        uint64_t *evals, hipStream_t st);

// Grid of the per-tile raster kernels: T_tot rounded up to a multiple of 8
// (one contiguous run of tiles per XCD).
inline uint32_t tile_grid(uint32_t t_tot) { return (t_tot + 7u) / 8u * 8u; }

}  // namespace gsr

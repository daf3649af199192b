// Host runtime of the C ABI declared in include/gsr.h: planning, workspace
// layout, argument validation and the stream-ordered launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gsr.h"
#include "kernels.hpp"
#include "runtime.hpp"

using namespace gsr;

namespace {

struct Layout {
  size_t scalars, queues, tile_count, tile_start, zero_end;
  size_t block_sums, vis_mask, rec_start, payload, rec_g, rec_view, rec_pairoff, rec_rect, rec_zbits;
  size_t rec_tmp, tile_order, tile_tmp, radix_hist, scan_part, pairs_tmp, tile_recs, partials, g2d, cam_part, loss_part;
  size_t total;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct gsr_ctx {
  std::string err;
  bool planned = false;
  // device current at gsr_create, and its copy of the no-alloc scratch
  int device = 0;
  void *scratch = nullptr;
  int32_t n_views = 0;
  int64_t n = 0;
  int32_t sh_degree = 0;
  std::vector<ViewInfo> views;
  ViewInfo *views_d = nullptr;
  size_t views_d_count = 0;
  Sizes sz{};
  Layout lay{};
  float *loss_partials = nullptr;
  // rig structure (gsr_rig_plan): frame and camera of each view, on the device
  int32_t *rig_idx_d = nullptr;
  int32_t rig_views = 0, rig_frames = 0, rig_cams = 0;
  // frequency-significance batch (gsr_freq_plan)
  std::vector<FreqImg> freq;
  FreqImg *freq_d = nullptr;
  float2 *freq_tw_d = nullptr;
  int64_t freq_rows = 0, freq_cols = 0, freq_inter = 0;
  int32_t freq_max_w = 0, freq_max_h = 0;
  size_t freq_ws = 0;
  // tuning applied at the next gsr_plan
  int32_t tuned_ts = 16;
  uint32_t long_list = 1024;
  int32_t persistent = 0;
  // stage timing
  bool prof = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double prof_ms[GSR_N_STAGES] = {};
  int64_t prof_calls[GSR_N_STAGES] = {};
};

namespace {

gsr_status fail(gsr_ctx *c, gsr_status s, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define GSR_HIP(ctx, call)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(ctx, GSR_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Brackets one stage with HIP events when stage timing is on.
struct StageTimer {
  gsr_ctx *c;
  int stage;
  hipStream_t s;
  StageTimer(gsr_ctx *c_, int stage_, hipStream_t s_) : c(c_), stage(stage_), s(s_) {
    if (c->prof) (void)hipEventRecord(c->ev0, s);
  }
  ~StageTimer() {
    if (!c->prof) return;
    float ms = 0.0f;
    if (hipEventRecord(c->ev1, s) == hipSuccess && hipEventSynchronize(c->ev1) == hipSuccess &&
        hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) {
      c->prof_ms[stage] += ms;
      c->prof_calls[stage] += 1;
    }
  }
};

Ws make_ws(const gsr_ctx *c, void *base) {
  char *b = static_cast<char *>(base);
  const Layout &L = c->lay;
  Ws w;
  w.scalars = reinterpret_cast<uint32_t *>(b + L.scalars);
  w.queues = reinterpret_cast<uint32_t *>(b + L.queues);
  w.block_sums = reinterpret_cast<uint2 *>(b + L.block_sums);
  w.vis_mask = reinterpret_cast<uint64_t *>(b + L.vis_mask);
  w.rec_start = reinterpret_cast<uint32_t *>(b + L.rec_start);
  w.rec_payload = reinterpret_cast<float4 *>(b + L.payload);
  w.rec_g = reinterpret_cast<uint32_t *>(b + L.rec_g);
  w.rec_view = reinterpret_cast<uint32_t *>(b + L.rec_view);
  w.rec_pairoff = reinterpret_cast<uint32_t *>(b + L.rec_pairoff);
  w.rec_rect = reinterpret_cast<uint4 *>(b + L.rec_rect);
  w.rec_zbits = reinterpret_cast<uint32_t *>(b + L.rec_zbits);
  w.tile_count = reinterpret_cast<uint32_t *>(b + L.tile_count);
  w.tile_start = reinterpret_cast<uint32_t *>(b + L.tile_start);
  w.tile_order = reinterpret_cast<uint32_t *>(b + L.tile_order);
  w.rec_tmp = reinterpret_cast<uint32_t *>(b + L.rec_tmp);
  w.tile_tmp = reinterpret_cast<uint32_t *>(b + L.tile_tmp);
  w.radix_hist = reinterpret_cast<uint32_t *>(b + L.radix_hist);
  w.scan_part = reinterpret_cast<uint32_t *>(b + L.scan_part);
  w.pairs_tmp = reinterpret_cast<uint32_t *>(b + L.pairs_tmp);
  w.tile_recs = reinterpret_cast<uint32_t *>(b + L.tile_recs);
  w.partials = reinterpret_cast<float *>(b + L.partials);
  w.g2d = reinterpret_cast<float4 *>(b + L.g2d);
  w.loss_partials = c->loss_partials;
  return w;
}

Layout make_layout(const Sizes &s) {
  Layout L{};
  size_t o = 0;
  auto put = [&](size_t &field, size_t bytes) {
    field = o;
    o = align_up(o + bytes);
  };
  // counting passes of the binning: at least 2048 items per block, 256
  // digits; the device-wide scans take 4096 words per chunk
  const size_t items = std::max<size_t>(std::max<size_t>(s.cap_pairs, s.cap_rec), s.t_tot);
  const size_t radix_blocks = std::max<size_t>((items + 2047) / 2048, 1);
  const size_t scan_words = std::max<size_t>(std::max<size_t>(1024 * radix_blocks, s.cap_rec), (size_t)s.t_tot + 1);
  put(L.scalars, kNumScalars * 4);
  put(L.queues, 2 * kQueueLanes * kQueueStride * 4);
  put(L.tile_count, (size_t)s.t_tot * 4);
  put(L.tile_start, (size_t)s.t_tot * 4);
  L.zero_end = o;
  put(L.block_sums, (size_t)s.n_blocks * 8);
  put(L.vis_mask, (size_t)s.vis_words * (size_t)s.n * 8);
  put(L.rec_start, (size_t)(s.n + 1) * 4);
  put(L.payload, (size_t)s.cap_rec * 64);
  put(L.rec_g, (size_t)s.cap_rec * 4);
  put(L.rec_view, (size_t)s.cap_rec * 4);
  put(L.rec_pairoff, (size_t)s.cap_rec * 4);
  put(L.rec_rect, (size_t)s.cap_rec * 16);
  put(L.rec_zbits, (size_t)s.cap_rec * 4);
  put(L.rec_tmp, (size_t)s.cap_rec * 20);
  put(L.tile_order, (size_t)s.t_tot * 4);
  put(L.tile_tmp, (size_t)s.t_tot * 16);
  put(L.radix_hist, 1024 * radix_blocks * 4);
  put(L.scan_part, (scan_words + 4095) / 4096 * 4);
  put(L.pairs_tmp, (size_t)s.cap_pairs * 8);
  put(L.tile_recs, (size_t)s.cap_pairs * 4);
  // per-pair partials (36 bytes); the pose gradients reuse them afterwards
  // as 48 bytes per record
  put(L.partials, std::max((size_t)s.cap_pairs * 36, (size_t)s.cap_rec * 48));
  put(L.g2d, (size_t)s.cap_rec * 48);
  put(L.cam_part, (size_t)cam_chunks(s.cap_rec) * (size_t)s.n_views * 48);
  put(L.loss_part, (size_t)raster_fwd_grid(s) * 4);
  L.total = o;
  return L;
}

gsr_status check_gauss(gsr_ctx *c, const gsr_gaussians *g) {
  if (!g) return fail(c, GSR_ERR_INVALID_ARG, "gaussians is NULL");
  if (g->n != c->n || g->sh_degree != c->sh_degree)
    return fail(c, GSR_ERR_NOT_PLANNED, "gaussians (n=%lld, degree %d) differ from the plan (n=%lld, degree %d)",
                (long long)g->n, g->sh_degree, (long long)c->n, c->sh_degree);
  if (g->n > 0 && (!g->mean || !g->log_scale || !g->quat || !g->opacity_logit || !g->sh))
    return fail(c, GSR_ERR_INVALID_ARG, "a Gaussian parameter pointer is NULL");
  return GSR_OK;
}

gsr_status check_common(gsr_ctx *c, const gsr_camera *cams, int32_t n_views, void *ws, size_t ws_bytes) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  if (n_views != c->n_views)
    return fail(c, GSR_ERR_NOT_PLANNED, "n_views %d differs from the plan (%d)", n_views, c->n_views);
  if (!cams) return fail(c, GSR_ERR_INVALID_ARG, "cams is NULL");
  if (!ws) return fail(c, GSR_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(c, GSR_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < c->lay.total)
    return fail(c, GSR_ERR_INVALID_ARG, "workspace of %zu bytes < %zu needed", ws_bytes, c->lay.total);
  return GSR_OK;
}

GaussPtrs gauss_ptrs(const gsr_gaussians *g) {
  return GaussPtrs{g->mean, g->log_scale, g->quat, g->opacity_logit, g->sh};
}

MutPtrs mut_ptrs(const gsr_grads *g) {
  return MutPtrs{g->mean, g->log_scale, g->quat, g->opacity_logit, g->sh};
}

MutPtrs mut_ptrs(const gsr_adam_moments *g) {
  return MutPtrs{g->mean, g->log_scale, g->quat, g->opacity_logit, g->sh};
}

bool any_null(const MutPtrs &p) { return !p.mean || !p.log_scale || !p.quat || !p.opacity_logit || !p.sh; }

// Pixels of all planned views.
int64_t total_px(const gsr_ctx *c) {
  if (c->views.empty()) return 0;
  const ViewInfo &v = c->views.back();
  return (int64_t)v.pix_off + (int64_t)v.w * v.h;
}

float *cam_part(const gsr_ctx *c, void *base) { return reinterpret_cast<float *>(static_cast<char *>(base) + c->lay.cam_part); }

// Stage radices of an FFT of length n: the fewest stages over the radices
// the kernels implement (composites 27, 25, 20, 16, 15, 9, 8 and primes 7,
// 5, 3, 2; ties to the larger first radix); false if n has a prime factor
// above 7 or needs more than 16 stages.
bool fft_radices(int n, uint8_t *fac, int32_t &nfac) {
  static const int kRadices[] = {27, 25, 20, 16, 15, 9, 8, 7, 5, 4, 3, 2};
  if (n < 1) return false;
  std::vector<int> best(n + 1, 1 << 20), first(n + 1, 0);
  best[1] = 0;
  for (int m = 2; m <= n; ++m) {
    if (n % m != 0) continue;
    for (int p : kRadices)
      if (m % p == 0 && best[m / p] + 1 < best[m]) {
        best[m] = best[m / p] + 1;
        first[m] = p;
      }
  }
  if (best[n] > 16) return false;
  nfac = 0;
  for (int m = n; m > 1; m /= first[m]) fac[nfac++] = (uint8_t)first[m];
  return true;
}

constexpr int kFreqMaxN = 2560;      // longest row or column transform (three LDS buffers of it)
constexpr int kFreqMaxFrames = 16384;  // frames of one scheduling step (LDS prefix sums)

RigIdx rig_idx(const gsr_ctx *c) {
  return RigIdx{c->rig_idx_d, c->rig_idx_d + c->rig_views, c->rig_views, c->rig_frames, c->rig_cams};
}

}  // namespace

extern "C" {

gsr_status gsr_create(gsr_ctx **out) {
  if (!out) return GSR_ERR_INVALID_ARG;
  *out = nullptr;
  gsr_ctx *c = new gsr_ctx();
  if (hipGetDevice(&c->device) != hipSuccess || scratch_address(c->device, &c->scratch) != hipSuccess ||
      hipMalloc(&c->loss_partials, kLossBlocks * sizeof(float)) != hipSuccess) {
    gsr_destroy(c);
    return GSR_ERR_HIP;
  }
  *out = c;
  return GSR_OK;
}

void gsr_destroy(gsr_ctx *c) {
  if (!c) return;
  if (c->views_d) (void)hipFree(c->views_d);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->loss_partials) (void)hipFree(c->loss_partials);
  if (c->rig_idx_d) (void)hipFree(c->rig_idx_d);
  if (c->freq_d) (void)hipFree(c->freq_d);
  if (c->freq_tw_d) (void)hipFree(c->freq_tw_d);
  delete c;
}

gsr_status gsr_plan(gsr_ctx *c, const gsr_camera *cams, int32_t n_views, int64_t n, int32_t sh_degree,
                    const gsr_plan_options *opt, size_t *ws_bytes, int64_t *pix_off) {
  if (!c) return GSR_ERR_INVALID_ARG;
  c->planned = false;
  if (!cams || !ws_bytes || !pix_off) return fail(c, GSR_ERR_INVALID_ARG, "NULL argument to gsr_plan");
  if (n_views < 1) return fail(c, GSR_ERR_INVALID_ARG, "n_views must be >= 1 (got %d)", n_views);
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(c, GSR_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (sh_degree < 0 || sh_degree > 3) return fail(c, GSR_ERR_UNSUPPORTED, "SH degree %d not in 0..3", sh_degree);
  int32_t ts = opt ? opt->tile_size : 0;
  if (ts == 0) ts = c->tuned_ts;
  if (ts != 8 && ts != 16 && ts != 32) return fail(c, GSR_ERR_INVALID_ARG, "tile size %d not in {8, 16, 32}", ts);
  std::vector<ViewInfo> views(n_views);
  uint64_t tiles = 0, pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const int w = cams[v].width, h = cams[v].height;
    if (w <= 0 || h <= 0 || w > 65535 || h > 65535)
      return fail(c, GSR_ERR_INVALID_ARG, "view %d has image size %dx%d", v, w, h);
    ViewInfo &vi = views[v];
    vi.w = w;
    vi.h = h;
    vi.tiles_x = (w + ts - 1) / ts;
    vi.tiles_y = (h + ts - 1) / ts;
    vi.tile_base = (uint32_t)tiles;
    vi.pix_off = (uint32_t)pix;
    vi.pad[0] = vi.pad[1] = 0;
    pix_off[v] = (int64_t)pix;
    tiles += (uint64_t)vi.tiles_x * vi.tiles_y;
    pix += (uint64_t)w * h;
  }
  pix_off[n_views] = (int64_t)pix;
  if (tiles >= (1ull << 31) || pix * 3 >= (1ull << 32))
    return fail(c, GSR_ERR_INVALID_ARG, "batch too large for 32-bit tile/pixel indices");
  uint64_t cap_rec = opt && opt->capacity_records > 0 ? (uint64_t)opt->capacity_records : (uint64_t)n_views * n;
  uint64_t cap_pairs = opt && opt->capacity_pairs > 0 ? (uint64_t)opt->capacity_pairs : 8ull * n_views * n;
  cap_rec = std::min<uint64_t>(std::max<uint64_t>(cap_rec, 1), 0xFFFFFFF0ull);
  cap_pairs = std::min<uint64_t>(std::max<uint64_t>(cap_pairs, 1), 0xFFFFFFF0ull);

  if (c->views_d_count < (size_t)n_views) {
    if (c->views_d) (void)hipFree(c->views_d);
    c->views_d = nullptr;
    c->views_d_count = 0;
    GSR_HIP(c, hipMalloc(&c->views_d, sizeof(ViewInfo) * n_views));
    c->views_d_count = n_views;
  }
  GSR_HIP(c, hipMemcpy(c->views_d, views.data(), sizeof(ViewInfo) * n_views, hipMemcpyHostToDevice));

  Sizes s{};
  s.n = n;
  s.n_views = n_views;
  s.sh_k = (sh_degree + 1) * (sh_degree + 1);
  s.ts = ts;
  s.t_tot = (uint32_t)tiles;
  s.cap_rec = (uint32_t)cap_rec;
  s.cap_pairs = (uint32_t)cap_pairs;
  s.n_blocks = (uint32_t)((n + kPreBlock - 1) / kPreBlock);
  s.long_list = c->long_list;
  s.persistent = (uint32_t)c->persistent;
  s.vis_words = (uint32_t)((n_views + 63) / 64);
  for (int k = 0; k < 3; ++k) s.bg[k] = opt ? opt->bg[k] : 0.0f;
  c->views = views;
  c->sz = s;
  c->n_views = n_views;
  c->n = n;
  c->sh_degree = sh_degree;
  c->lay = make_layout(s);
  *ws_bytes = c->lay.total;
  c->planned = true;
  return GSR_OK;
}

static gsr_status forward_common(gsr_ctx *c, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                 void *ws_base, size_t ws_bytes, const gsr_fwd_out *out, const LossArgs &la,
                                 void *stream) {
  gsr_status st = check_common(c, cams, n_views, ws_base, ws_bytes);
  if (st != GSR_OK) return st;
  if ((st = check_gauss(c, g)) != GSR_OK) return st;
  if (!out || !out->image || !out->t_final || !out->last_pos || !out->n_contrib)
    return fail(c, GSR_ERR_INVALID_ARG, "forward output pointer is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws ws = make_ws(c, ws_base);
  const Cam *cm = reinterpret_cast<const Cam *>(cams);
  {
    StageTimer tm(c, GSR_STAGE_PREPROCESS, s);
    launch_preprocess(gauss_ptrs(g), cm, c->views_d, ws, c->sz, c->sh_degree, ws.scalars,
                      (c->lay.zero_end - c->lay.scalars) / 4, s);
  }
  {
    StageTimer tm(c, GSR_STAGE_SORT, s);
    launch_depth_sort(ws, c->sz, s);
  }
  {
    StageTimer tm(c, GSR_STAGE_BINNING, s);
    launch_binning(c->views_d, ws, c->sz, s);
  }
  {
    StageTimer tm(c, GSR_STAGE_RASTER_FWD, s);
    launch_raster_fwd(c->views_d, ws, c->sz, out->image, out->t_final, out->last_pos, out->n_contrib, la, s);
  }
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

gsr_status gsr_render_forward(gsr_ctx *c, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                              void *ws_base, size_t ws_bytes, const gsr_fwd_out *out, void *stream) {
  return forward_common(c, g, cams, n_views, ws_base, ws_bytes, out, LossArgs{nullptr, nullptr, nullptr, 0.0f},
                        stream);
}

gsr_status gsr_render_forward_noalloc(gsr_ctx *c, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                      const gsr_fwd_out *out, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  if (c->lay.total > kScratchBytes)
    return fail(c, GSR_ERR_CAPACITY, "the plan needs a workspace of %zu bytes, above the %zu bytes of the library's "
                "no-alloc scratch; use gsr_render_forward with a caller workspace", c->lay.total, kScratchBytes);
  int dev = -1;
  GSR_HIP(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, GSR_ERR_INVALID_ARG, "current device %d is not the context's device %d", dev, c->device);
  // the forward's first kernel clears the counters and tile counts it needs
  // at zero, so what an earlier call left in the scratch does not matter
  return forward_common(c, g, cams, n_views, c->scratch, kScratchBytes, out, LossArgs{nullptr, nullptr, nullptr, 0.0f},
                        stream);
}

gsr_status gsr_render_forward_l1(gsr_ctx *c, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                 void *ws_base, size_t ws_bytes, const gsr_fwd_out *out, const float *target,
                                 float *loss_out, float *dL_dimage, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!target || !loss_out || !dL_dimage) return fail(c, GSR_ERR_INVALID_ARG, "target, loss or dL_dimage is NULL");
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  const int64_t n = 3 * total_px(c);
  float *part = reinterpret_cast<float *>(static_cast<char *>(ws_base) + c->lay.loss_part);
  const LossArgs la{target, dL_dimage, part, (float)(1.0 / (double)n)};
  gsr_status st = forward_common(c, g, cams, n_views, ws_base, ws_bytes, out, la, stream);
  if (st != GSR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    StageTimer tm(c, GSR_STAGE_LOSS, s);
    launch_l1_sum(part, raster_fwd_grid(c->sz), n, loss_out, s);
  }
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

gsr_status gsr_l1_loss(gsr_ctx *c, const float *image, const float *target, int64_t n_elems, float *loss_out,
                       float *dL_dimage, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!image || !target || !loss_out || !dL_dimage) return fail(c, GSR_ERR_INVALID_ARG, "NULL argument to gsr_l1_loss");
  if (n_elems <= 0) return fail(c, GSR_ERR_INVALID_ARG, "n_elems must be positive");
  {
    StageTimer tm(c, GSR_STAGE_LOSS, static_cast<hipStream_t>(stream));
    launch_l1(image, target, n_elems, loss_out, dL_dimage, c->loss_partials, static_cast<hipStream_t>(stream));
  }
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

static gsr_status backward_common(gsr_ctx *c, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                  void *ws_base, size_t ws_bytes, const gsr_fwd_out *fwd, const float *dL) {
  gsr_status st = check_common(c, cams, n_views, ws_base, ws_bytes);
  if (st != GSR_OK) return st;
  if ((st = check_gauss(c, g)) != GSR_OK) return st;
  if (!fwd || !fwd->t_final || !fwd->last_pos) return fail(c, GSR_ERR_INVALID_ARG, "forward state pointer is NULL");
  if (!dL) return fail(c, GSR_ERR_INVALID_ARG, "dL_dimage is NULL");
  return GSR_OK;
}

gsr_status gsr_render_backward(gsr_ctx *c, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                               void *ws_base, size_t ws_bytes, const gsr_fwd_out *fwd, const float *dL_dimage,
                               const gsr_grads *grads, int32_t accumulate, void *stream) {
  gsr_status st = backward_common(c, g, cams, n_views, ws_base, ws_bytes, fwd, dL_dimage);
  if (st != GSR_OK) return st;
  if (!grads) return fail(c, GSR_ERR_INVALID_ARG, "grads is NULL");
  const MutPtrs gr = mut_ptrs(grads);
  if (c->n > 0 && any_null(gr)) return fail(c, GSR_ERR_INVALID_ARG, "a gradient pointer is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws ws = make_ws(c, ws_base);
  float4 *cam_rec = grads->camera ? reinterpret_cast<float4 *>(ws.partials) : nullptr;
  {
    StageTimer tm(c, GSR_STAGE_RASTER_BWD, s);
    launch_raster_bwd(c->views_d, ws, c->sz, fwd->t_final, fwd->last_pos, dL_dimage, s);
  }
  {
    StageTimer tm(c, GSR_STAGE_REDUCE, s);
    launch_reduce_pairs(ws, c->sz, nullptr, s);
  }
  {
    StageTimer tm(c, GSR_STAGE_PRE_BWD, s);
    launch_pre_bwd(gauss_ptrs(g), reinterpret_cast<const Cam *>(cams), ws, c->sz, c->sh_degree, &gr,
                   accumulate ? 1 : 0, nullptr, cam_rec, s);
    if (cam_rec) launch_cam_grads(ws, c->sz, cam_rec, cam_part(c, ws_base), grads->camera, accumulate ? 1 : 0, s);
  }
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

static gsr_status adam_args(gsr_ctx *c, const gsr_grads *params, const gsr_adam_moments *m,
                            const gsr_adam_moments *v, const gsr_adam_config *cfg, int32_t *step, AdamArgs &a) {
  if (!params || !m || !v || !cfg || !step) return fail(c, GSR_ERR_INVALID_ARG, "NULL Adam argument");
  a.p = mut_ptrs(params);
  a.m = mut_ptrs(m);
  a.v = mut_ptrs(v);
  if (c->n > 0 && (any_null(a.p) || any_null(a.m) || any_null(a.v)))
    return fail(c, GSR_ERR_INVALID_ARG, "a parameter or moment pointer is NULL");
  for (int k = 0; k < 6; ++k) a.lr[k] = cfg->lr[k];
  a.beta1 = cfg->beta1;
  a.beta2 = cfg->beta2;
  a.eps = cfg->eps;
  a.step = step;
  if (!(cfg->beta1 >= 0.f && cfg->beta1 < 1.f && cfg->beta2 >= 0.f && cfg->beta2 < 1.f && cfg->eps >= 0.f))
    return fail(c, GSR_ERR_INVALID_ARG, "Adam betas must lie in [0, 1) and eps >= 0");
  return GSR_OK;
}

gsr_status gsr_adam_step(gsr_ctx *c, const gsr_grads *params, const gsr_grads *grads, const gsr_adam_moments *m,
                         const gsr_adam_moments *v, const gsr_adam_config *cfg, int32_t *step_dev, int64_t n,
                         int32_t sh_degree, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (n < 0) return fail(c, GSR_ERR_INVALID_ARG, "n < 0");
  if (sh_degree < 0 || sh_degree > 3) return fail(c, GSR_ERR_UNSUPPORTED, "SH degree %d not in 0..3", sh_degree);
  if (!grads) return fail(c, GSR_ERR_INVALID_ARG, "grads is NULL");
  const int64_t keep_n = c->n;
  c->n = n;  // pointer checks below use the step's own n
  AdamArgs a{};
  gsr_status st = adam_args(c, params, m, v, cfg, step_dev, a);
  const MutPtrs gr = mut_ptrs(grads);
  if (st == GSR_OK && n > 0 && any_null(gr)) st = fail(c, GSR_ERR_INVALID_ARG, "a gradient pointer is NULL");
  c->n = keep_n;
  if (st != GSR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    StageTimer tm(c, GSR_STAGE_ADAM, s);
    launch_step_inc(step_dev, s);
    launch_adam(gr, a, n, sh_degree, s);
  }
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

gsr_status gsr_render_backward_adam(gsr_ctx *c, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                    void *ws_base, size_t ws_bytes, const gsr_fwd_out *fwd, const float *dL_dimage,
                                    const gsr_grads *params, const gsr_adam_moments *m, const gsr_adam_moments *v,
                                    const gsr_adam_config *cfg, int32_t *step_dev, const gsr_grads *grads_out,
                                    void *stream) {
  gsr_status st = backward_common(c, g, cams, n_views, ws_base, ws_bytes, fwd, dL_dimage);
  if (st != GSR_OK) return st;
  AdamArgs a{};
  if ((st = adam_args(c, params, m, v, cfg, step_dev, a)) != GSR_OK) return st;
  a.p_is_g = a.p.mean == g->mean && a.p.log_scale == g->log_scale && a.p.quat == g->quat &&
             a.p.opacity_logit == g->opacity_logit && a.p.sh == g->sh;
  MutPtrs gr{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (grads_out) {
    gr = mut_ptrs(grads_out);
    const bool none = !gr.mean && !gr.log_scale && !gr.quat && !gr.opacity_logit && !gr.sh;
    if (c->n > 0 && any_null(gr) && !none)
      return fail(c, GSR_ERR_INVALID_ARG, "the Gaussian gradient outputs must be all set or all NULL");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws ws = make_ws(c, ws_base);
  float4 *cam_rec = grads_out && grads_out->camera ? reinterpret_cast<float4 *>(ws.partials) : nullptr;
  {
    StageTimer tm(c, GSR_STAGE_RASTER_BWD, s);
    launch_raster_bwd(c->views_d, ws, c->sz, fwd->t_final, fwd->last_pos, dL_dimage, s);
  }
  {
    StageTimer tm(c, GSR_STAGE_REDUCE, s);
    launch_reduce_pairs(ws, c->sz, step_dev, s);  // also advances the Adam step
  }
  {
    StageTimer tm(c, GSR_STAGE_PRE_BWD, s);
    launch_pre_bwd(gauss_ptrs(g), reinterpret_cast<const Cam *>(cams), ws, c->sz, c->sh_degree, &gr, 0, &a,
                   cam_rec, s);
    if (cam_rec) launch_cam_grads(ws, c->sz, cam_rec, cam_part(c, ws_base), grads_out->camera, 0, s);
  }
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

gsr_status gsr_debug_binning(gsr_ctx *c, void *ws_base, uint64_t *keys, uint32_t *vals, uint32_t *tile_csr,
                             void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  if (!ws_base || !keys || !vals || !tile_csr) return fail(c, GSR_ERR_INVALID_ARG, "NULL argument to gsr_debug_binning");
  launch_debug_binning(c->views_d, make_ws(c, ws_base), c->sz, keys, vals, tile_csr, static_cast<hipStream_t>(stream));
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

gsr_status gsr_count_evaluations(gsr_ctx *c, void *ws_base, const gsr_fwd_out *fwd, uint64_t *evals,
                                 void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  if (!ws_base || !fwd || !fwd->last_pos || !evals)
    return fail(c, GSR_ERR_INVALID_ARG, "NULL argument to gsr_count_evaluations");
  launch_count_evals(c->views_d, make_ws(c, ws_base), c->sz, fwd->last_pos, evals,
                     static_cast<hipStream_t>(stream));
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

// Message of the last failed call that has no context (gsr_copy_bytes).
static thread_local std::string g_err_no_ctx = "NULL context";

gsr_status gsr_copy_bytes(void *dst, const void *src, size_t bytes, void *stream) {
  if (!dst || !src || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16 != 0 ||
      bytes / 16 > (uint64_t(1) << 40)) {
    g_err_no_ctx = "gsr_copy_bytes: pointers must be non-NULL and 16-byte aligned, the size a multiple of 16 (< 16 TiB)";
    return GSR_ERR_INVALID_ARG;
  }
  launch_copy16(dst, src, bytes / 16, static_cast<hipStream_t>(stream));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_err_no_ctx = std::string("gsr_copy_bytes: ") + hipGetErrorString(e);
    return GSR_ERR_HIP;
  }
  return GSR_OK;
}

static gsr_status read_scalars(gsr_ctx *c, void *ws_base, void *stream, uint32_t out[kNumScalars]) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  if (!ws_base) {  // the no-alloc forward's scratch
    if (c->lay.total > kScratchBytes) return fail(c, GSR_ERR_INVALID_ARG, "workspace is NULL");
    ws_base = c->scratch;
  }
  GSR_HIP(c, hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  GSR_HIP(c, hipMemcpy(out, static_cast<char *>(ws_base) + c->lay.scalars, kNumScalars * 4, hipMemcpyDeviceToHost));
  return GSR_OK;
}

gsr_status gsr_check(gsr_ctx *c, void *ws_base, void *stream) {
  uint32_t sc[kNumScalars];
  gsr_status st = read_scalars(c, ws_base, stream, sc);
  if (st != GSR_OK) return st;
  if (sc[kOverflow] == 1u)
    return fail(c, GSR_ERR_CAPACITY, "capacity exceeded: %u records (capacity %u), %u pairs (capacity %u)",
                sc[kNumRecords], c->sz.cap_rec, sc[kNumPairs], c->sz.cap_pairs);
  if (sc[kOverflow] != 0u) return fail(c, GSR_ERR_HIP, "internal binning inconsistency (code %u)", sc[kOverflow]);
  return GSR_OK;
}

gsr_status gsr_required_capacity(gsr_ctx *c, void *ws_base, int64_t *records, int64_t *pairs, int64_t *tiles,
                                 void *stream) {
  uint32_t sc[kNumScalars];
  gsr_status st = read_scalars(c, ws_base, stream, sc);
  if (st != GSR_OK) return st;
  if (records) *records = sc[kNumRecords];
  if (pairs) *pairs = sc[kNumPairs];
  if (tiles) *tiles = c->sz.t_tot;
  return GSR_OK;
}

gsr_status gsr_set_tuning(gsr_ctx *c, const gsr_tuning *t) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!t) return fail(c, GSR_ERR_INVALID_ARG, "tuning is NULL");
  if (t->tile_size != 8 && t->tile_size != 16 && t->tile_size != 32)
    return fail(c, GSR_ERR_INVALID_ARG, "tile size %d not in {8, 16, 32}", t->tile_size);
  if (t->persistent != 0 && t->persistent != 1)
    return fail(c, GSR_ERR_INVALID_ARG, "persistent %d not in {0, 1}", t->persistent);
  c->tuned_ts = t->tile_size;
  c->long_list = t->long_list;
  c->persistent = t->persistent;
  return GSR_OK;
}

gsr_status gsr_get_tuning(gsr_ctx *c, gsr_tuning *t) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!t) return fail(c, GSR_ERR_INVALID_ARG, "tuning is NULL");
  t->tile_size = c->tuned_ts;
  t->long_list = c->long_list;
  t->persistent = c->persistent;
  t->step_ms = 0.0f;
  return GSR_OK;
}

gsr_status gsr_profile(gsr_ctx *c, int32_t enable) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (enable && !c->ev0) {
    GSR_HIP(c, hipEventCreate(&c->ev0));
    GSR_HIP(c, hipEventCreate(&c->ev1));
  }
  c->prof = enable != 0;
  return GSR_OK;
}

gsr_status gsr_profile_read(gsr_ctx *c, double *ms, int64_t *calls, int32_t reset) {
  if (!c) return GSR_ERR_INVALID_ARG;
  for (int k = 0; k < GSR_N_STAGES; ++k) {
    if (ms) ms[k] = c->prof_ms[k];
    if (calls) calls[k] = c->prof_calls[k];
    if (reset) {
      c->prof_ms[k] = 0.0;
      c->prof_calls[k] = 0;
    }
  }
  return GSR_OK;
}

const char *gsr_last_error(const gsr_ctx *c) { return c ? c->err.c_str() : g_err_no_ctx.c_str(); }

gsr_status gsr_freq_plan(gsr_ctx *c, const int32_t *widths, const int32_t *heights, int32_t n_images,
                         size_t *workspace_bytes) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (n_images < 0) return fail(c, GSR_ERR_INVALID_ARG, "n_images < 0");
  if (n_images > 0 && (!widths || !heights)) return fail(c, GSR_ERR_INVALID_ARG, "size array is NULL");
  std::vector<FreqImg> imgs((size_t)n_images);
  int64_t pix = 0, inter = 0, rows = 0, cols = 0;
  int32_t max_w = 1, max_h = 1;
  // one twiddle table exp(-2 pi i t / n) per distinct transform length,
  // computed in double precision
  std::vector<float2> tw;
  std::vector<std::pair<int, int64_t>> tables;
  auto table = [&](int n) -> int64_t {
    for (const auto &t : tables)
      if (t.first == n) return t.second;
    const int64_t off = (int64_t)tw.size();
    for (int t = 0; t < n; ++t) {
      const double a = -2.0 * 3.14159265358979323846 * (double)t / (double)n;
      tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
    }
    tables.emplace_back(n, off);
    return off;
  };
  for (int32_t i = 0; i < n_images; ++i) {
    FreqImg &f = imgs[(size_t)i];
    f = FreqImg{};
    f.w = widths[i];
    f.h = heights[i];
    if (f.w < 1 || f.h < 1 || f.w > kFreqMaxN || f.h > kFreqMaxN)
      return fail(c, GSR_ERR_UNSUPPORTED, "image %d: %d x %d outside 1..%d", i, f.w, f.h, kFreqMaxN);
    if (!fft_radices(f.w, f.fac_w, f.nfac_w) || !fft_radices(f.h, f.fac_h, f.nfac_h))
      return fail(c, GSR_ERR_UNSUPPORTED, "image %d: %d x %d has a prime factor above 7", i, f.w, f.h);
    const int64_t half = f.w / 2 + 1;
    f.pix_off = pix;
    f.inter_off = inter;
    f.row_base = rows;
    f.col_base = cols;
    f.tw_w = table(f.w);
    f.tw_h = table(f.h);
    pix += 3ll * f.w * f.h;
    inter += 3 * half * f.h;
    rows += f.h;
    cols += half;
    max_w = std::max(max_w, f.w);
    max_h = std::max(max_h, f.h);
  }
  if (c->freq_d) {
    GSR_HIP(c, hipFree(c->freq_d));
    c->freq_d = nullptr;
  }
  if (c->freq_tw_d) {
    GSR_HIP(c, hipFree(c->freq_tw_d));
    c->freq_tw_d = nullptr;
  }
  c->freq.clear();
  c->freq_rows = c->freq_cols = c->freq_inter = 0;
  c->freq_ws = 0;
  if (n_images > 0) {
    GSR_HIP(c, hipMalloc(&c->freq_d, imgs.size() * sizeof(FreqImg)));
    GSR_HIP(c, hipMemcpy(c->freq_d, imgs.data(), imgs.size() * sizeof(FreqImg), hipMemcpyHostToDevice));
    GSR_HIP(c, hipMalloc(&c->freq_tw_d, tw.size() * sizeof(float2)));
    GSR_HIP(c, hipMemcpy(c->freq_tw_d, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
  }
  c->freq = imgs;
  c->freq_rows = rows;
  c->freq_cols = cols;
  c->freq_inter = inter;
  c->freq_max_w = max_w;
  c->freq_max_h = max_h;
  c->freq_ws = align_up((size_t)inter * 8) + align_up((size_t)cols * 4);
  if (workspace_bytes) *workspace_bytes = c->freq_ws;
  return GSR_OK;
}

gsr_status gsr_freq_significance(gsr_ctx *c, const float *images, void *ws, size_t ws_bytes, float *X, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (c->freq.empty()) return GSR_OK;
  if (!images || !X || !ws) return fail(c, GSR_ERR_INVALID_ARG, "an image, output or workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(c, GSR_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < c->freq_ws)
    return fail(c, GSR_ERR_INVALID_ARG, "workspace of %zu bytes < %zu needed", ws_bytes, c->freq_ws);
  char *b = static_cast<char *>(ws);
  float2 *inter = reinterpret_cast<float2 *>(b);
  float *col_sum = reinterpret_cast<float *>(b + align_up((size_t)c->freq_inter * 8));
  launch_freq_significance(images, c->freq_d, (int)c->freq.size(), c->freq_rows, c->freq_cols, c->freq_max_w,
                           c->freq_max_h, c->freq_tw_d, inter, col_sum, X, static_cast<hipStream_t>(stream));
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

gsr_status gsr_downsample(gsr_ctx *c, const float *src, int32_t width, int32_t height, int32_t factor, float *dst,
                          void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (width < 0 || height < 0 || factor < 1)
    return fail(c, GSR_ERR_INVALID_ARG, "bad size %d x %d or factor %d", width, height, factor);
  if ((width / factor) * (height / factor) > 0 && (!src || !dst))
    return fail(c, GSR_ERR_INVALID_ARG, "image pointer is NULL");
  launch_downsample(src, width, height, factor, dst, static_cast<hipStream_t>(stream));
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

gsr_status gsr_freq_schedule(gsr_ctx *c, const float *x_gt, const float *x_gt_level, const float *x_render,
                             int32_t n_frames, float tau_f, int32_t *levels, const float *uniforms, int32_t n_picks,
                             float *r, float *r_prime, int32_t *picks, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (n_frames < 0 || n_frames > kFreqMaxFrames || n_picks < 0)
    return fail(c, GSR_ERR_INVALID_ARG, "n_frames %d outside 0..%d or n_picks < 0", n_frames, kFreqMaxFrames);
  if (n_frames == 0) {
    if (n_picks > 0) return fail(c, GSR_ERR_INVALID_ARG, "picks requested from zero frames");
    return GSR_OK;
  }
  if (!x_gt || !x_render) return fail(c, GSR_ERR_INVALID_ARG, "x_gt or x_render is NULL");
  if (levels && !x_gt_level) return fail(c, GSR_ERR_INVALID_ARG, "level updates need x_gt_level");
  if (n_picks > 0 && (!uniforms || !picks)) return fail(c, GSR_ERR_INVALID_ARG, "uniforms or picks is NULL");
  launch_freq_schedule(x_gt, x_gt_level, x_render, n_frames, tau_f, levels, uniforms, n_picks, r, r_prime,
                       n_picks > 0 ? picks : nullptr, static_cast<hipStream_t>(stream));
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

// Workspace of gsr_log_insert: the byte mask, then the per-block counts and
// offsets of the compaction, then the total.
struct InsLayout {
  size_t mask, counts, offsets, total, bytes;
};

InsLayout ins_layout(const gsr_ctx *c) {
  InsLayout L{};
  const int64_t px = total_px(c);
  const size_t nb = ins_blocks(px);
  L.mask = 0;
  L.counts = align_up((size_t)px);
  L.offsets = L.counts + align_up(nb * 4);
  L.total = L.offsets + align_up(nb * 4);
  L.bytes = L.total + 256;
  return L;
}

gsr_status gsr_insert_workspace(gsr_ctx *c, size_t *bytes) {
  if (!c || !bytes) return GSR_ERR_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  *bytes = ins_layout(c).bytes;
  return GSR_OK;
}

gsr_status gsr_log_insert(gsr_ctx *c, const gsr_camera *cams, const float *gt, const float *render, const float *depth,
                          const gsr_insert_config *cfg, float *p_gt, float *p_render, const gsr_insert_out *out,
                          void *ws, size_t ws_bytes, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  if (!cams || !gt || !render || !depth || !cfg || !p_gt || !out || !ws)
    return fail(c, GSR_ERR_INVALID_ARG, "a required pointer is NULL");
  if (!(cfg->sigma > 0.0f && cfg->sigma <= 5.0f / 3.0f))
    return fail(c, GSR_ERR_INVALID_ARG, "sigma %g outside (0, 5/3]", (double)cfg->sigma);
  if (out->capacity < 0 || !out->count || (out->capacity > 0 && (!out->pix || !out->scale || !out->mean)))
    return fail(c, GSR_ERR_INVALID_ARG, "insertion output arrays missing");
  const InsLayout L = ins_layout(c);
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(c, GSR_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < L.bytes) return fail(c, GSR_ERR_INVALID_ARG, "workspace of %zu bytes < %zu needed", ws_bytes, L.bytes);
  // taps in double precision, rounded once
  LogTaps taps{};
  const double sg = cfg->sigma;
  const int R = (int)std::ceil(3.0 * sg);
  double g[17], h[17], gs = 0.0, hs = 0.0, hm = 0.0;
  for (int k = 0; k <= 2 * R; ++k) {
    const double x = k - R;
    g[k] = std::exp(-x * x / (2.0 * sg * sg));
    gs += g[k];
  }
  for (int k = 0; k <= 2 * R; ++k) {
    const double x = k - R;
    g[k] /= gs;
    h[k] = (x * x - sg * sg) / (sg * sg * sg * sg) * g[k];
    hs += h[k];
  }
  for (int k = 0; k <= 2 * R; ++k) {
    const double x = k - R;
    h[k] -= hs / (2 * R + 1);
    hm += x * x * h[k];
  }
  for (int k = 0; k <= 2 * R; ++k) {
    taps.g[k] = (float)g[k];
    taps.h[k] = (float)(h[k] * 2.0 / hm);
  }
  taps.R = R;
  const int64_t px = total_px(c);
  char *b = static_cast<char *>(ws);
  launch_log_insert(c->views_d, c->n_views, ins_tiles(c->views.data(), c->n_views), px,
                    reinterpret_cast<const Cam *>(cams), gt, render, depth, taps, cfg->tau_a, p_gt, p_render,
                    reinterpret_cast<uint8_t *>(b + L.mask), reinterpret_cast<uint32_t *>(b + L.counts),
                    reinterpret_cast<uint32_t *>(b + L.offsets), out->count, out->pix, out->scale, out->mean,
                    out->capacity, static_cast<hipStream_t>(stream));
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

// Workspace of gsr_merge: per pixel of the largest view the slot, the group
// count, colour sums (3 x 64 bit), the distance sum and the 64-bit winner
// key; per Gaussian the matched pixel.
struct MergeLayout {
  size_t slot, cnt, csum, dsum, win, match, bytes;
};

MergeLayout merge_layout(const gsr_ctx *c, int64_t n) {
  MergeLayout L{};
  size_t px = 0;
  for (const ViewInfo &v : c->views) px = std::max(px, (size_t)v.w * (size_t)v.h);
  L.slot = 0;
  L.cnt = align_up(px * 4);
  L.csum = L.cnt + align_up(px * 4);
  L.dsum = L.csum + align_up(px * 24);
  L.win = L.dsum + align_up(px * 8);
  L.match = L.win + align_up(px * 8);
  L.bytes = L.match + align_up((size_t)std::max<int64_t>(n, 1) * 4);
  return L;
}

gsr_status gsr_merge_workspace(gsr_ctx *c, int64_t n, size_t *bytes) {
  if (!c || !bytes || n < 0) return GSR_ERR_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  *bytes = merge_layout(c, n).bytes;
  return GSR_OK;
}

gsr_status gsr_merge(gsr_ctx *c, const gsr_gaussians *g, int32_t view, const gsr_camera *cams, const float *gt,
                     const float *p_gt, const gsr_insert_out *samples, const gsr_merge_config *cfg,
                     const gsr_merge_out *out, void *ws, size_t ws_bytes, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_ERR_NOT_PLANNED, "gsr_plan has not been called");
  if (!g || !cams || !gt || !p_gt || !samples || !cfg || !out || !ws)
    return fail(c, GSR_ERR_INVALID_ARG, "a required pointer is NULL");
  if (view < 0 || view >= c->n_views) return fail(c, GSR_ERR_INVALID_ARG, "view %d outside [0, %d)", view, c->n_views);
  if (g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3) return fail(c, GSR_ERR_INVALID_ARG, "bad Gaussian set");
  if (g->n > 0 && (!g->mean || !g->log_scale || !g->sh || !out->keep || !out->colour))
    return fail(c, GSR_ERR_INVALID_ARG, "a Gaussian or output pointer is NULL");
  if (g->n >= (int64_t)0xFFFFFFFFll) return fail(c, GSR_ERR_UNSUPPORTED, "more than 2^32 - 1 Gaussians");
  if (samples->capacity < 0 || !samples->count ||
      (samples->capacity > 0 && (!samples->pix || !samples->mean || !out->keep_new || !out->colour_new)))
    return fail(c, GSR_ERR_INVALID_ARG, "sample arrays missing");
  if (!(cfg->tau_d >= 0.0f) || !(cfg->kappa > 0.0f))
    return fail(c, GSR_ERR_INVALID_ARG, "tau_d must be >= 0 and kappa > 0");
  const MergeLayout L = merge_layout(c, g->n);
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(c, GSR_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < L.bytes) return fail(c, GSR_ERR_INVALID_ARG, "workspace of %zu bytes < %zu needed", ws_bytes, L.bytes);
  char *b = static_cast<char *>(ws);
  const MergeBufs mb{reinterpret_cast<int32_t *>(b + L.slot), reinterpret_cast<uint32_t *>(b + L.cnt),
                     reinterpret_cast<unsigned long long *>(b + L.csum),
                     reinterpret_cast<unsigned long long *>(b + L.dsum),
                     reinterpret_cast<unsigned long long *>(b + L.win), reinterpret_cast<int32_t *>(b + L.match)};
  launch_merge(gauss_ptrs(g), g->n, reinterpret_cast<const Cam *>(cams), view, c->views[(size_t)view], gt, p_gt,
               samples->pix, samples->mean, samples->count, samples->capacity, cfg->tau_d, cfg->kappa, mb, out->keep,
               out->colour, out->mean, out->keep_new, out->colour_new, out->mean_new,
               static_cast<hipStream_t>(stream));
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

gsr_status gsr_rig_plan(gsr_ctx *c, const int32_t *view_frame, const int32_t *view_camera, int32_t n_views,
                        int32_t n_frames, int32_t n_cams) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (n_views < 0 || n_frames < 0 || n_cams < 0)
    return fail(c, GSR_ERR_INVALID_ARG, "negative rig size (views %d, frames %d, cameras %d)", n_views, n_frames,
                n_cams);
  if (n_views > 0 && (!view_frame || !view_camera)) return fail(c, GSR_ERR_INVALID_ARG, "rig index array is NULL");
  for (int32_t v = 0; v < n_views; ++v) {
    if (view_frame[v] < 0 || view_frame[v] >= n_frames)
      return fail(c, GSR_ERR_INVALID_ARG, "view %d: frame %d outside [0, %d)", v, view_frame[v], n_frames);
    if (view_camera[v] < 0 || view_camera[v] >= n_cams)
      return fail(c, GSR_ERR_INVALID_ARG, "view %d: camera %d outside [0, %d)", v, view_camera[v], n_cams);
  }
  std::vector<int32_t> idx(2 * (size_t)n_views);
  std::copy(view_frame, view_frame + n_views, idx.begin());
  std::copy(view_camera, view_camera + n_views, idx.begin() + n_views);
  if (c->rig_idx_d) {
    GSR_HIP(c, hipFree(c->rig_idx_d));
    c->rig_idx_d = nullptr;
  }
  c->rig_views = c->rig_frames = c->rig_cams = 0;
  if (n_views > 0) {
    GSR_HIP(c, hipMalloc(&c->rig_idx_d, idx.size() * sizeof(int32_t)));
    GSR_HIP(c, hipMemcpy(c->rig_idx_d, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  c->rig_views = n_views;
  c->rig_frames = n_frames;
  c->rig_cams = n_cams;
  return GSR_OK;
}

gsr_status gsr_rig_compose(gsr_ctx *c, const float *central, const float *relative, gsr_camera *cams, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (c->rig_views > 0 && (!central || !relative || !cams))
    return fail(c, GSR_ERR_INVALID_ARG, "a rig pose or camera pointer is NULL");
  launch_rig_compose(central, relative, rig_idx(c), reinterpret_cast<Cam *>(cams), static_cast<hipStream_t>(stream));
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

gsr_status gsr_rig_gradients(gsr_ctx *c, const float *central, const float *relative, const float *view_grads,
                             float *d_central, float *d_relative, float *xi_central, float *xi_relative,
                             void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if ((c->rig_frames > 0 && (!central || !d_central)) || (c->rig_cams > 0 && (!relative || !d_relative)) ||
      (c->rig_views > 0 && !view_grads))
    return fail(c, GSR_ERR_INVALID_ARG, "a rig pose, view gradient or output pointer is NULL");
  launch_rig_grads(central, relative, view_grads, rig_idx(c), d_central, d_relative, xi_central, xi_relative,
                   static_cast<hipStream_t>(stream));
  GSR_HIP(c, hipGetLastError());
  return GSR_OK;
}

}  // extern "C"

gsr_status gsr::ctx_error(gsr_ctx *c, gsr_status s, const char *msg) { return fail(c, s, "%s", msg); }

void gsr::ctx_unplan(gsr_ctx *c) {
  if (c) c->planned = false;
}

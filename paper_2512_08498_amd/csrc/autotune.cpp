// Autotuner of the batched launch: measures forward + backward on the
// caller's batch for each candidate launch configuration (tile size, at
// 16 px the long-list split, and the grid or persistent schedule) and keeps
// the fastest.  Built on the
// public entry points; its device buffers live only for the measurement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gsr.h"
#include "kernels.hpp"
#include "runtime.hpp"

using namespace gsr;

namespace {

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
  hipError_t alloc(size_t bytes) {
    reset();
    return hipMalloc(&p, std::max<size_t>(bytes, 256));
  }
  template <class T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Device and batch-shape key of a cache line (no spaces).
std::string cache_key(const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views, const gsr_plan_options *opt) {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  arch = arch.substr(0, arch.find(':'));
  char buf[128];
  snprintf(buf, sizeof buf, "%s/%dcu/n=%lld/deg=%d/cap=%lld,%lld/views=", arch.c_str(), cus, (long long)g->n,
           g->sh_degree, opt ? (long long)opt->capacity_records : 0LL, opt ? (long long)opt->capacity_pairs : 0LL);
  std::string key = buf;
  for (int v = 0; v < n_views; ++v) {
    snprintf(buf, sizeof buf, "%s%dx%d", v ? "," : "", cams[v].width, cams[v].height);
    key += buf;
  }
  return key;
}

// Last line of the cache file whose first field is `key`.
bool cache_lookup(const char *path, const std::string &key, gsr_tuning *t, bool *malformed) {
  *malformed = false;
  FILE *f = fopen(path, "r");
  if (!f) return false;
  bool found = false;
  std::string line;
  char chunk[512];
  while (fgets(chunk, sizeof chunk, f)) {
    line += chunk;
    if (line.empty() || line.back() != '\n') {
      if (!feof(f)) continue;
    }
    const size_t sp = line.find(' ');
    if (sp != std::string::npos && line.compare(0, sp, key) == 0 && sp == key.size()) {
      gsr_tuning u{};
      if (sscanf(line.c_str() + sp, " tile_size=%d long_list=%u persistent=%d step_ms=%f", &u.tile_size,
                 &u.long_list, &u.persistent, &u.step_ms) == 4 &&
          (u.tile_size == 8 || u.tile_size == 16 || u.tile_size == 32) && (u.persistent == 0 || u.persistent == 1)) {
        *t = u;
        found = true;
        *malformed = false;
      } else {
        *malformed = true;
      }
    }
    line.clear();
  }
  fclose(f);
  return found;
}

}  // namespace

extern "C" gsr_status gsr_autotune(gsr_ctx *c, const gsr_gaussians *g, const gsr_camera *cams_host, int32_t n_views,
                                   const gsr_plan_options *opt, int32_t repeats, const char *cache_path,
                                   gsr_tuning *best, void *stream) {
  if (!c) return GSR_ERR_INVALID_ARG;
  if (!g || !cams_host || !best) return ctx_error(c, GSR_ERR_INVALID_ARG, "NULL argument to gsr_autotune");
  if (n_views < 1) return ctx_error(c, GSR_ERR_INVALID_ARG, "n_views must be >= 1");
  if (repeats < 1) return ctx_error(c, GSR_ERR_INVALID_ARG, "repeats must be >= 1");
  if (g->n > 0 && (!g->mean || !g->log_scale || !g->quat || !g->opacity_logit || !g->sh))
    return ctx_error(c, GSR_ERR_INVALID_ARG, "a Gaussian parameter pointer is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);

  const std::string key = cache_key(g, cams_host, n_views, opt);
  if (cache_path) {
    bool malformed = false;
    gsr_tuning t{};
    if (cache_lookup(cache_path, key, &t, &malformed)) {
      gsr_status st = gsr_set_tuning(c, &t);
      if (st != GSR_OK) return st;
      ctx_unplan(c);
      *best = t;
      return GSR_OK;
    }
    if (malformed) return ctx_error(c, GSR_ERR_INVALID_ARG, "malformed autotune cache line for this batch");
  }

  std::vector<gsr_tuning> candidates;
  for (int pers = 0; pers < 2; ++pers) {
    for (uint32_t ll : {1024u, 512u, 256u, 0u, 0xFFFFFFFFu}) candidates.push_back({16, ll, pers, 0.f});
    candidates.push_back({8, 512u, pers, 0.f});
    candidates.push_back({32, 512u, pers, 0.f});
  }
  gsr_tuning keep{};
  gsr_status st = gsr_get_tuning(c, &keep);
  if (st != GSR_OK) return st;

  // buffers that do not depend on the candidate
  const int64_t n = g->n, k = (int64_t)(g->sh_degree + 1) * (g->sh_degree + 1);
  std::vector<int64_t> pix_off(n_views + 1);
  gsr_plan_options po{};
  if (opt) po = *opt;
  po.tile_size = 16;
  size_t ws_bytes = 0;
  st = gsr_plan(c, cams_host, n_views, n, g->sh_degree, &po, &ws_bytes, pix_off.data());
  if (st != GSR_OK) return st;
  const uint64_t px = (uint64_t)pix_off[n_views];
  DevBuf cams_d, img, tfin, last, cnt, dl, grads, ws;
  Events ev;
  const int64_t per_g = 3 + 3 + 4 + 1 + 3 * k;
#define TUNE_HIP(call)                                                                \
  do {                                                                                \
    if ((call) != hipSuccess) {                                                       \
      (void)gsr_set_tuning(c, &keep);                                                 \
      ctx_unplan(c);                                                                  \
      return ctx_error(c, GSR_ERR_HIP, "gsr_autotune: " #call " failed");             \
    }                                                                                 \
  } while (0)
  TUNE_HIP(cams_d.alloc(sizeof(gsr_camera) * n_views));
  TUNE_HIP(hipMemcpy(cams_d.p, cams_host, sizeof(gsr_camera) * n_views, hipMemcpyHostToDevice));
  TUNE_HIP(img.alloc(12 * px));
  TUNE_HIP(tfin.alloc(4 * px));
  TUNE_HIP(last.alloc(4 * px));
  TUNE_HIP(cnt.alloc(4 * px));
  TUNE_HIP(dl.alloc(12 * px));
  TUNE_HIP(grads.alloc(sizeof(float) * (size_t)(per_g * n)));
  TUNE_HIP(hipEventCreate(&ev.a));
  TUNE_HIP(hipEventCreate(&ev.b));
  // any non-zero cotangent gives the backward its full work
  launch_fill(dl.as<float>(), 3 * px, 1.0f / (float)std::max<uint64_t>(3 * px, 1), s);

  const gsr_camera *cams_dev = cams_d.as<gsr_camera>();
  const gsr_fwd_out fo{img.as<float>(), tfin.as<float>(), last.as<uint32_t>(), cnt.as<uint32_t>()};
  float *gp = grads.as<float>();
  const gsr_grads gr{gp, gp + 3 * n, gp + 6 * n, gp + 10 * n, gp + 11 * n};

  float best_ms = 0.0f;
  gsr_tuning chosen{};
  int64_t known_rec = 0, known_pairs16 = 0;
  std::vector<float> times(repeats);
  for (const gsr_tuning &cand : candidates) {
    if ((st = gsr_set_tuning(c, &cand)) != GSR_OK) break;
    gsr_plan_options pc = po;
    pc.tile_size = cand.tile_size;
    // capacities from the first measurement: records do not depend on the
    // tiling; a footprint covers at most 4x the tiles at 8 px than at 16 px
    // and at most as many at 32 px
    if (pc.capacity_records <= 0 && known_rec > 0) pc.capacity_records = known_rec + known_rec / 8 + 4096;
    if (pc.capacity_pairs <= 0 && known_pairs16 > 0) {
      const int64_t est = cand.tile_size == 8 ? 4 * known_pairs16 : known_pairs16 + known_pairs16 / 8;
      pc.capacity_pairs = std::min<int64_t>(est + 65536, (int64_t)0xFFFFFFF0);
    }
    // plan, render once, and re-plan to the measured sizes if they overflowed
    for (int attempt = 0; attempt < 2; ++attempt) {
      if ((st = gsr_plan(c, cams_host, n_views, n, g->sh_degree, &pc, &ws_bytes, pix_off.data())) != GSR_OK) break;
      TUNE_HIP(ws.alloc(ws_bytes));
      if ((st = gsr_render_forward(c, g, cams_dev, n_views, ws.p, ws_bytes, &fo, s)) != GSR_OK) break;
      st = gsr_check(c, ws.p, s);
      if (st != GSR_ERR_CAPACITY) break;
      int64_t rec = 0, pairs = 0, tiles = 0;
      if ((st = gsr_required_capacity(c, ws.p, &rec, &pairs, &tiles, s)) != GSR_OK) break;
      if (pairs + pairs / 8 + 65536 > (int64_t)0xFFFFFFF0) {
        st = ctx_error(c, GSR_ERR_CAPACITY, "gsr_autotune: the batch exceeds 32-bit pair indices");
        break;
      }
      pc.capacity_records = rec + rec / 8 + 4096;
      pc.capacity_pairs = pairs + pairs / 8 + 65536;
      st = GSR_ERR_CAPACITY;
    }
    if (st != GSR_OK) break;
    {
      int64_t rec = 0, pairs = 0, tiles = 0;
      if ((st = gsr_required_capacity(c, ws.p, &rec, &pairs, &tiles, s)) != GSR_OK) break;
      known_rec = rec;
      if (cand.tile_size == 16) known_pairs16 = pairs;
    }
    // warm-up, then the timed passes
    if ((st = gsr_render_backward(c, g, cams_dev, n_views, ws.p, ws_bytes, &fo, dl.as<float>(), &gr, 0, s)) != GSR_OK)
      break;
    for (int r = 0; r < repeats && st == GSR_OK; ++r) {
      TUNE_HIP(hipEventRecord(ev.a, s));
      if ((st = gsr_render_forward(c, g, cams_dev, n_views, ws.p, ws_bytes, &fo, s)) != GSR_OK) break;
      if ((st = gsr_render_backward(c, g, cams_dev, n_views, ws.p, ws_bytes, &fo, dl.as<float>(), &gr, 0, s)) !=
          GSR_OK)
        break;
      TUNE_HIP(hipEventRecord(ev.b, s));
      TUNE_HIP(hipEventSynchronize(ev.b));
      TUNE_HIP(hipEventElapsedTime(&times[r], ev.a, ev.b));
    }
    if (st != GSR_OK) break;
    if ((st = gsr_check(c, ws.p, s)) != GSR_OK) break;
    std::sort(times.begin(), times.end());
    // candidates are listed in order of preference (the grid schedule
    // first); a later one must be at least 1% faster to replace the choice,
    // so timing noise between near-equal configurations does not decide
    const float med = times[repeats / 2];
    if (best_ms == 0.0f || med < 0.99f * best_ms) {
      best_ms = med;
      chosen = cand;
      chosen.step_ms = med;
    }
    ws.reset();
  }
#undef TUNE_HIP
  ws.reset();
  ctx_unplan(c);
  if (st != GSR_OK) {
    (void)gsr_set_tuning(c, &keep);
    return st;
  }
  if ((st = gsr_set_tuning(c, &chosen)) != GSR_OK) return st;
  *best = chosen;
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (!f) return ctx_error(c, GSR_ERR_INVALID_ARG, "gsr_autotune: cannot append to the cache file");
    fprintf(f, "%s tile_size=%d long_list=%u persistent=%d step_ms=%.4f\n", key.c_str(), chosen.tile_size,
            chosen.long_list, chosen.persistent, chosen.step_ms);
    fclose(f);
  }
  return GSR_OK;
}

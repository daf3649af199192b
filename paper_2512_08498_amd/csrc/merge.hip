// Per-camera merging of existing Gaussians with the samples of camera i
// (Sec. 3.2, "Redundancy-free Gaussian Sampling", Eqs. 7-8).
//
// Each existing Gaussian is reprojected into camera i (x', distance d').  Of
// the four pixel centres around x', the sampled one with the largest
// positive bilinear weight is its correspondence (the lowest pixel index on
// equal weights), if it lies in front of the near plane and d' is within
// tau_d of the sample's distance.  Each member of a group (a sample and the
// Gaussians that correspond to it) is measured against the new camera's
// scale where it sits: rho = s' / s_i(x') with s' = kappa S fx / d' (S the
// geometric mean of its scales) and s_i(x') = 1 / (2 sqrt(P(x'))), P
// interpolated bilinearly (borders replicated); the sample's own rho is 1.
// Only the smallest rho survives (existing Gaussians win ties, the lower
// index first); it takes the mean colour of the group and is moved along
// camera i's ray to the group's mean distance.
//
// The geometry (projection, weights, interpolation, ratio, distances) is
// evaluated in double precision, so a decision differs from the exact one
// only within a relative 1e-5 or so of its threshold.
//
// Deterministic without sorting: the groups are accumulated with integer
// atomics only -- the member count, the colour and distance sums in 2^-32
// fixed point (exact, so the order of the additions does not matter), and
// the 64-bit minimum of (ratio bits, index), which orders positive floats
// correctly.
//   k_merge_slots     slot map pixel -> sample of the view, grid-stride (entries
//                     of other pixels are stale, rejected by the match), group init
//   k_merge_match     one thread per Gaussian: projection, correspondence,
//                     group accumulation
//   k_merge_samples   the samples of the view (grid-stride): keep / colour / centre
//   k_merge_gaussians one thread per Gaussian: keep / colour / centre
#include <algorithm>

#include "kernels.hpp"

namespace gsr {

namespace {

constexpr double kFix = 4294967296.0;  // 2^32
constexpr double kY0 = 0.28209479177387814;
constexpr int64_t kSampleBlocks = 1024;  // grid of the per-sample kernels (4 workgroups per CU)

typedef unsigned long long u64;

__device__ __forceinline__ u64 to_fix(double c) { return (u64)llrint(c * kFix); }

// Camera-space point of world point (x, y, z) and its distance to the camera.
__device__ __forceinline__ double view_dist(const Cam &c, double x, double y, double z, double &xc, double &yc,
                                            double &zc) {
  xc = ((double)c.R[0] * x + (double)c.R[1] * y) + (double)c.R[2] * z + (double)c.t[0];
  yc = ((double)c.R[3] * x + (double)c.R[4] * y) + (double)c.R[5] * z + (double)c.t[1];
  zc = ((double)c.R[6] * x + (double)c.R[7] * y) + (double)c.R[8] * z + (double)c.t[2];
  return sqrt(xc * xc + yc * yc + zc * zc);
}

__device__ __forceinline__ double sample_dist(const Cam &c, const float *s_mean, int64_t k) {
  double a, b, e;
  return view_dist(c, s_mean[3 * k], s_mean[3 * k + 1], s_mean[3 * k + 2], a, b, e);
}

// p moved along the ray from the camera centre C = -R^T t through it, its
// distance d scaled to dbar, written as float to out[0], out[stride], out[2 stride].
__device__ __forceinline__ void realign(const Cam &c, const double p[3], double d, double dbar, float *out,
                                        int64_t stride) {
  double C[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    C[a] = -((double)c.R[a] * c.t[0] + (double)c.R[3 + a] * c.t[1] + (double)c.R[6 + a] * c.t[2]);
  const double f = dbar / d;
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a * stride] = (float)(C[a] + (p[a] - C[a]) * f);
}

__global__ __launch_bounds__(256) void k_merge_slots(const uint32_t *__restrict__ pix, const uint32_t *__restrict__ count,
                                                     int64_t capacity, uint32_t off, uint32_t npx,
                                                     int32_t *__restrict__ slot, uint32_t *__restrict__ cnt,
                                                     u64 *__restrict__ csum, u64 *__restrict__ dsum,
                                                     u64 *__restrict__ win) {
  const int64_t n = min((int64_t)*count, capacity);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = pix[k] - off;
    if (pix[k] < off || p >= npx) continue;
    slot[p] = (int32_t)k;
    cnt[p] = 0u;
    csum[3 * (size_t)p + 0] = csum[3 * (size_t)p + 1] = csum[3 * (size_t)p + 2] = 0ull;
    dsum[p] = 0ull;
    win[p] = ~0ull;
  }
}

__global__ __launch_bounds__(256) void k_merge_match(GaussPtrs gp, int64_t n, const Cam *__restrict__ cams, int view,
                                                     ViewInfo vi, const int32_t *__restrict__ slot,
                                                     const uint32_t *__restrict__ pix, const uint32_t *__restrict__ count,
                                                     int64_t capacity, const float *__restrict__ s_mean,
                                                     const float *__restrict__ p_gt, float tau_d, float kappa,
                                                     int32_t *__restrict__ match, uint32_t *__restrict__ cnt,
                                                     u64 *__restrict__ csum, u64 *__restrict__ dsum,
                                                     u64 *__restrict__ win) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const Cam c = cams[view];
  double xc, yc, zc;
  const double dg = view_dist(c, gp.mean[g], gp.mean[n + g], gp.mean[2 * n + g], xc, yc, zc);
  int32_t m = -1;
  const int W = vi.w, H = vi.h;
  if (zc > (double)kNearZ) {
    const double u = (double)c.fx * (xc / zc) + (double)c.cx, v = (double)c.fy * (yc / zc) + (double)c.cy;
    if (u >= 0.0 && u < (double)W && v >= 0.0 && v < (double)H) {
      const double a = u - 0.5, b = v - 0.5;
      const double fi = floor(a), fj = floor(b);
      const double al = a - fi, be = b - fj;
      const int i0 = (int)fi, j0 = (int)fj;
      const int64_t nk = min((int64_t)*count, capacity);
      // the four neighbours in ascending pixel index; P replicated at the borders
      double pv[4], best_w = 0.0;
      int32_t best_p = -1, best_k = -1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + (q & 1), j = j0 + (q >> 1);
        const double w = ((q & 1) ? al : 1.0 - al) * ((q >> 1) ? be : 1.0 - be);
        const int ic = min(max(i, 0), W - 1), jc = min(max(j, 0), H - 1);
        pv[q] = (double)p_gt[vi.pix_off + (uint32_t)(jc * W + ic)];
        if (i >= 0 && i < W && j >= 0 && j < H && w > best_w) {
          // the slot map is not cleared between calls: an entry counts only
          // if it names a live sample whose pixel is this one (each pixel is
          // sampled once)
          const int32_t p = j * W + i;
          const int32_t k = slot[p];
          if (k >= 0 && k < nk && pix[k] == vi.pix_off + (uint32_t)p) {
            best_w = w;
            best_p = p;
            best_k = k;
          }
        }
      }
      if (best_k >= 0 && fabs(dg - sample_dist(c, s_mean, best_k)) <= (double)tau_d) {
        m = best_p;
        const double p_at = (1.0 - be) * ((1.0 - al) * pv[0] + al * pv[1]) + be * ((1.0 - al) * pv[2] + al * pv[3]);
        const double ls = ((double)gp.log_scale[g] + (double)gp.log_scale[n + g] + (double)gp.log_scale[2 * n + g]) / 3.0;
        const double rho = (double)kappa * exp(ls) * (double)c.fx / dg * 2.0 * sqrt(p_at);
        atomicAdd(&cnt[best_p], 1u);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
          atomicAdd(&csum[3 * (size_t)best_p + ch], to_fix(kY0 * (double)gp.sh[ch * n + g] + 0.5));
        atomicAdd(&dsum[best_p], to_fix(dg));
        atomicMin(&win[best_p], ((u64)__float_as_uint((float)rho) << 32) | (u64)(uint32_t)g);
      }
    }
  }
  match[g] = m;
}

// Group mean colour channel ch of pixel p with sample colour cs, and the
// group's mean distance with sample distance ds.
__device__ __forceinline__ float group_mean(const u64 *csum, const uint32_t *cnt, uint32_t p, int ch, float cs) {
  const long long tot = (long long)csum[3 * (size_t)p + ch] + (long long)to_fix(cs);
  return (float)((double)tot / kFix / (double)(cnt[p] + 1u));
}

__device__ __forceinline__ double group_dist(const u64 *dsum, const uint32_t *cnt, uint32_t p, double ds) {
  return (double)(long long)(dsum[p] + to_fix(ds)) / kFix / (double)(cnt[p] + 1u);
}

__device__ __forceinline__ bool existing_wins(const u64 *win, uint32_t p) {
  return __uint_as_float((uint32_t)(win[p] >> 32)) <= 1.0f;
}

__global__ __launch_bounds__(256) void k_merge_samples(const Cam *__restrict__ cams, int view,
                                                       const uint32_t *__restrict__ pix,
                                                       const uint32_t *__restrict__ count, int64_t capacity,
                                                       uint32_t off, uint32_t npx, const float *__restrict__ gt,
                                                       const float *__restrict__ s_mean,
                                                       const uint32_t *__restrict__ cnt, const u64 *__restrict__ csum,
                                                       const u64 *__restrict__ dsum, const u64 *__restrict__ win,
                                                       uint8_t *__restrict__ keep_new, float *__restrict__ colour_new,
                                                       float *__restrict__ mean_new) {
  const int64_t nk = min((int64_t)*count, capacity);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nk; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t gpix = pix[k], p = gpix - off;
    if (gpix < off || p >= npx) continue;
    float cs[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) cs[ch] = gt[3 * (size_t)off + (size_t)ch * npx + p];
    const bool group = cnt[p] > 0u;
    const bool lost = group && existing_wins(win, p);
    const bool merged = group && !lost;
    keep_new[k] = lost ? 0 : 1;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) colour_new[3 * (size_t)k + ch] = merged ? group_mean(csum, cnt, p, ch, cs[ch]) : cs[ch];
    if (mean_new) {
      const double c3[3] = {s_mean[3 * k], s_mean[3 * k + 1], s_mean[3 * k + 2]};
      if (merged) {
        const Cam c = cams[view];
        const double ds = sample_dist(c, s_mean, k);
        realign(c, c3, ds, group_dist(dsum, cnt, p, ds), mean_new + 3 * k, 1);
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) mean_new[3 * k + a] = (float)c3[a];
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_merge_gaussians(GaussPtrs gp, int64_t n, const Cam *__restrict__ cams,
                                                         int view, uint32_t off, uint32_t npx,
                                                         const int32_t *__restrict__ match,
                                                         const int32_t *__restrict__ slot,
                                                         const float *__restrict__ gt, const float *__restrict__ s_mean,
                                                         const uint32_t *__restrict__ cnt,
                                                         const u64 *__restrict__ csum, const u64 *__restrict__ dsum,
                                                         const u64 *__restrict__ win, uint8_t *__restrict__ keep,
                                                         float *__restrict__ colour, float *__restrict__ mean_out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float own[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) own[ch] = (float)(kY0 * (double)gp.sh[ch * n + g] + 0.5);
  const int32_t p = match[g];
  bool k = true, winner = false;
  if (p >= 0) {
    winner = (uint32_t)(win[p] & 0xFFFFFFFFull) == (uint32_t)g && existing_wins(win, (uint32_t)p);
    k = winner;
  }
  keep[g] = k ? 1 : 0;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float c = own[ch];
    if (winner) c = group_mean(csum, cnt, (uint32_t)p, ch, gt[3 * (size_t)off + (size_t)ch * npx + (uint32_t)p]);
    colour[ch * n + g] = c;
  }
  if (mean_out) {
    const double m3[3] = {gp.mean[g], gp.mean[n + g], gp.mean[2 * n + g]};
    if (winner) {
      const Cam c = cams[view];
      double xc, yc, zc;
      const double dg = view_dist(c, m3[0], m3[1], m3[2], xc, yc, zc);
      const double ds = sample_dist(c, s_mean, slot[p]);
      realign(c, m3, dg, group_dist(dsum, cnt, (uint32_t)p, ds), mean_out + g, n);
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) mean_out[a * n + g] = (float)m3[a];
    }
  }
}

}  // namespace

void launch_merge(const GaussPtrs &gp, int64_t n, const Cam *cams, int view, const ViewInfo &vi, const float *gt,
                  const float *p_gt, const uint32_t *pix, const float *s_mean, const uint32_t *count,
                  int64_t capacity, float tau_d, float kappa, const MergeBufs &mb, uint8_t *keep, float *colour,
                  float *mean_out, uint8_t *keep_new, float *colour_new, float *mean_new, hipStream_t st) {
  const uint32_t npx = (uint32_t)vi.w * (uint32_t)vi.h;
  // the sample kernels stride over the live count, which only the device
  // knows; a capacity-sized grid would be mostly empty workgroups
  const unsigned sgrid = (unsigned)std::min<int64_t>((capacity + 255) / 256, kSampleBlocks);
  if (capacity > 0)
    k_merge_slots<<<sgrid, 256, 0, st>>>(pix, count, capacity, vi.pix_off, npx, mb.slot, mb.cnt, mb.csum, mb.dsum,
                                         mb.win);
  if (n > 0)
    k_merge_match<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(gp, n, cams, view, vi, mb.slot, pix, count, capacity,
                                                               s_mean, p_gt, tau_d, kappa, mb.match, mb.cnt, mb.csum,
                                                               mb.dsum, mb.win);
  if (capacity > 0)
    k_merge_samples<<<sgrid, 256, 0, st>>>(cams, view, pix, count, capacity, vi.pix_off, npx, gt, s_mean, mb.cnt,
                                           mb.csum, mb.dsum, mb.win, keep_new, colour_new, mean_new);
  if (n > 0)
    k_merge_gaussians<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(gp, n, cams, view, vi.pix_off, npx, mb.match,
                                                                   mb.slot, gt, s_mean, mb.cnt, mb.csum, mb.dsum,
                                                                   mb.win, keep, colour, mean_out);
}

}  // namespace gsr

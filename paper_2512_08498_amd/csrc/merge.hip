// Per-camera merging of existing Gaussians with the samples of camera i
// (Sec. 3.2, "Redundancy-free Gaussian Sampling", Eqs. 7-8).
//
// A Gaussian corresponds to the sample whose pixel contains its projection
// into camera i, when it lies in front of the near plane and its distance to
// the camera is within tau_d of the sample's.  In each group (a sample and
// the Gaussians that correspond to it) only the primitive with the smallest
// image-space scale survives -- s' = kappa S fx / d' for a Gaussian (S the
// geometric mean of its scales), s = 1 / (2 sqrt(P)) for the sample -- and it
// takes the mean colour of the group.  Existing Gaussians win ties, the lower
// index first.
//
// Deterministic without sorting: the groups are accumulated with integer
// atomics only -- the member count, the colour sums in 2^-32 fixed point
// (exact, so the order of the additions does not matter), and the 64-bit
// minimum of (scale bits, index), which orders positive floats correctly.
//   k_merge_slots     slot map pixel -> sample of the view, grid-stride (entries
//                     of other pixels are stale, rejected by the match), group init
//   k_merge_match     one thread per Gaussian: projection, correspondence,
//                     group accumulation
//   k_merge_samples   the samples of the view (grid-stride): keep / colour
//   k_merge_gaussians one thread per Gaussian: keep / colour
#include <algorithm>

#include "kernels.hpp"

namespace gsr {

namespace {

constexpr double kFix = 4294967296.0;  // 2^32
constexpr float kY0 = 0.28209479177387814f;
constexpr int64_t kSampleBlocks = 1024;  // grid of the per-sample kernels (4 workgroups per CU)

__device__ __forceinline__ unsigned long long to_fix(float c) {
  return (unsigned long long)llrint((double)c * kFix);
}

__device__ __forceinline__ float view_dist(const Cam &c, float x, float y, float z, float &xc, float &yc, float &zc) {
  xc = (c.R[0] * x + c.R[1] * y) + c.R[2] * z + c.t[0];
  yc = (c.R[3] * x + c.R[4] * y) + c.R[5] * z + c.t[1];
  zc = (c.R[6] * x + c.R[7] * y) + c.R[8] * z + c.t[2];
  return sqrtf(xc * xc + yc * yc + zc * zc);
}

__global__ __launch_bounds__(256) void k_merge_slots(const uint32_t *__restrict__ pix, const uint32_t *__restrict__ count,
                                                     int64_t capacity, uint32_t off, uint32_t npx,
                                                     int32_t *__restrict__ slot, uint32_t *__restrict__ cnt,
                                                     unsigned long long *__restrict__ csum,
                                                     unsigned long long *__restrict__ win) {
  const int64_t n = min((int64_t)*count, capacity);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = pix[k] - off;
    if (pix[k] < off || p >= npx) continue;
    slot[p] = (int32_t)k;
    cnt[p] = 0u;
    csum[3 * (size_t)p + 0] = csum[3 * (size_t)p + 1] = csum[3 * (size_t)p + 2] = 0ull;
    win[p] = ~0ull;
  }
}

__global__ __launch_bounds__(256) void k_merge_match(GaussPtrs gp, int64_t n, const Cam *__restrict__ cams, int view,
                                                     ViewInfo vi, const int32_t *__restrict__ slot,
                                                     const uint32_t *__restrict__ pix, const uint32_t *__restrict__ count,
                                                     int64_t capacity,
                                                     const float *__restrict__ s_mean, float tau_d, float kappa,
                                                     int32_t *__restrict__ match, uint32_t *__restrict__ cnt,
                                                     unsigned long long *__restrict__ csum,
                                                     unsigned long long *__restrict__ win) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const Cam c = cams[view];
  float xc, yc, zc;
  const float dg = view_dist(c, gp.mean[g], gp.mean[n + g], gp.mean[2 * n + g], xc, yc, zc);
  int32_t m = -1;
  if (zc > kNearZ) {
    const float u = c.fx * (xc / zc) + c.cx, v = c.fy * (yc / zc) + c.cy;
    const float fu = floorf(u), fv = floorf(v);
    if (fu >= 0.0f && fu < (float)vi.w && fv >= 0.0f && fv < (float)vi.h) {
      const int32_t p = (int32_t)fv * vi.w + (int32_t)fu;
      // the slot map is not cleared between calls: an entry counts only if it
      // names a live sample whose pixel is p (each pixel is sampled once)
      const int32_t k = slot[p];
      const int64_t nk = min((int64_t)*count, capacity);
      if (k >= 0 && k < nk && pix[k] == vi.pix_off + (uint32_t)p) {
        float a, b, e;
        const float *sm = s_mean + 3 * (size_t)k;
        const float dn = view_dist(c, sm[0], sm[1], sm[2], a, b, e);
        if (fabsf(dg - dn) <= tau_d) {
          m = p;
          const float ls = (gp.log_scale[g] + gp.log_scale[n + g] + gp.log_scale[2 * n + g]) / 3.0f;
          const float s = kappa * expf(ls) * c.fx / dg;
          atomicAdd(&cnt[p], 1u);
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) atomicAdd(&csum[3 * (size_t)p + ch], to_fix(kY0 * gp.sh[ch * n + g] + 0.5f));
          atomicMin(&win[p], ((unsigned long long)__float_as_uint(s) << 32) | (unsigned long long)(uint32_t)g);
        }
      }
    }
  }
  match[g] = m;
}

// Group mean colour channel ch of pixel p with sample colour cs.
__device__ __forceinline__ float group_mean(const unsigned long long *csum, const uint32_t *cnt, uint32_t p, int ch,
                                            float cs) {
  const long long tot = (long long)csum[3 * (size_t)p + ch] + (long long)to_fix(cs);
  return (float)((double)tot / kFix / (double)(cnt[p] + 1u));
}

__global__ __launch_bounds__(256) void k_merge_samples(const uint32_t *__restrict__ pix,
                                                       const uint32_t *__restrict__ count, int64_t capacity,
                                                       uint32_t off, uint32_t npx, const float *__restrict__ gt,
                                                       const float *__restrict__ p_gt, const uint32_t *__restrict__ cnt,
                                                       const unsigned long long *__restrict__ csum,
                                                       const unsigned long long *__restrict__ win,
                                                       uint8_t *__restrict__ keep_new, float *__restrict__ colour_new) {
  const int64_t nk = min((int64_t)*count, capacity);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nk; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t gpix = pix[k], p = gpix - off;
    if (gpix < off || p >= npx) continue;
    float cs[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) cs[ch] = gt[3 * (size_t)off + (size_t)ch * npx + p];
    const float s_new = 1.0f / (2.0f * sqrtf(p_gt[gpix]));
    const bool group = cnt[p] > 0u;
    const bool existing_wins = group && __uint_as_float((uint32_t)(win[p] >> 32)) <= s_new;
    keep_new[k] = existing_wins ? 0 : 1;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
      colour_new[3 * (size_t)k + ch] = (group && !existing_wins) ? group_mean(csum, cnt, p, ch, cs[ch]) : cs[ch];
  }
}

__global__ __launch_bounds__(256) void k_merge_gaussians(GaussPtrs gp, int64_t n, uint32_t off, uint32_t npx,
                                                         const int32_t *__restrict__ match,
                                                         const float *__restrict__ gt, const float *__restrict__ p_gt,
                                                         const uint32_t *__restrict__ cnt,
                                                         const unsigned long long *__restrict__ csum,
                                                         const unsigned long long *__restrict__ win,
                                                         uint8_t *__restrict__ keep, float *__restrict__ colour) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float own[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) own[ch] = kY0 * gp.sh[ch * n + g] + 0.5f;
  const int32_t p = match[g];
  bool k = true, winner = false;
  if (p >= 0) {
    const unsigned long long w = win[p];
    const float s_new = 1.0f / (2.0f * sqrtf(p_gt[off + (uint32_t)p]));
    winner = (uint32_t)(w & 0xFFFFFFFFull) == (uint32_t)g && __uint_as_float((uint32_t)(w >> 32)) <= s_new;
    k = winner;
  }
  keep[g] = k ? 1 : 0;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float c = own[ch];
    if (winner) c = group_mean(csum, cnt, (uint32_t)p, ch, gt[3 * (size_t)off + (size_t)ch * npx + (uint32_t)p]);
    colour[ch * n + g] = c;
  }
}

}  // namespace

void launch_merge(const GaussPtrs &gp, int64_t n, const Cam *cams, int view, const ViewInfo &vi, const float *gt,
                  const float *p_gt, const uint32_t *pix, const float *s_mean, const uint32_t *count,
                  int64_t capacity, float tau_d, float kappa, int32_t *slot, uint32_t *cnt, unsigned long long *csum,
                  unsigned long long *win, int32_t *match, uint8_t *keep, float *colour, uint8_t *keep_new,
                  float *colour_new, hipStream_t st) {
  const uint32_t npx = (uint32_t)vi.w * (uint32_t)vi.h;
  // the sample kernels stride over the live count, which only the device
  // knows; a capacity-sized grid would be mostly empty workgroups
  const unsigned sgrid = (unsigned)std::min<int64_t>((capacity + 255) / 256, kSampleBlocks);
  if (capacity > 0)
    k_merge_slots<<<sgrid, 256, 0, st>>>(pix, count, capacity, vi.pix_off, npx, slot, cnt,
                                                                      csum, win);
  if (n > 0)
    k_merge_match<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(gp, n, cams, view, vi, slot, pix, count, capacity,
                                                               s_mean, tau_d, kappa, match, cnt, csum, win);
  if (capacity > 0)
    k_merge_samples<<<sgrid, 256, 0, st>>>(pix, count, capacity, vi.pix_off, npx, gt,
                                                                        p_gt, cnt, csum, win, keep_new, colour_new);
  if (n > 0)
    k_merge_gaussians<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(gp, n, vi.pix_off, npx, match, gt, p_gt, cnt, csum,
                                                                   win, keep, colour);
}

}  // namespace gsr

// LoG-based insertion of new Gaussians (Sec. 3.2, "Redundancy-free Gaussian
// Sampling", Eqs. 4-6) over all views of the plan:
//   P(I) = min(|| LoG_sigma * I ||, 1) per pixel (norm over the channels),
//   P_a  = max(P(I) - P(I~), 0), a Gaussian is inserted where P_a > tau_a,
//   S    = d / (2 sqrt(P(I)) f) for the inserted pixel, d the distance from
//          the back-projected centre (z from the depth map) to the camera.
//
// k_log_prob: one workgroup per 64 x 16 pixel tile of a view.  For each of
// the two images a horizontal pass convolves the tile's rows and a halo of
// R = ceil(3 sigma) rows (border pixels replicated) with the 1D Gaussian g
// and its second derivative h, reading each item's window straight into
// registers and leaving the results in LDS; a vertical pass finishes
// L = (h x g + g x h) * I.  Each thread produces four pixels of one column,
// sharing the 2R + 4 rows of the vertical window.  Writes P(I),
// optionally P(I~), and a byte mask of the inserting pixels.
// k_ins_count / k_ins_scan / k_ins_write: stream compaction of the mask in
// ascending pixel order (counts per 4096 pixels, one scan, then each
// workgroup writes its pixels in order) with the new Gaussians' scale and
// world centre.
#include "kernels.hpp"
#include "util.hpp"

namespace gsr {

namespace {

constexpr int kTW = 64, kTH = 16;
constexpr int kInsBlock = 4096;  // pixels per compaction workgroup (256 threads x 16)

__device__ __forceinline__ int view_of_ins_tile(const ViewInfo *__restrict__ views, int n_views, int tile, int &base) {
  base = 0;
  for (int v = 0; v < n_views; ++v) {
    const int nt = ((views[v].w + kTW - 1) / kTW) * ((views[v].h + kTH - 1) / kTH);
    if (tile < base + nt) return v;
    base += nt;
  }
  return -1;
}

// R is a template parameter so that the tap loops unroll and the taps are
// read at compile-time indices.
template <int R>
__global__ __launch_bounds__(256) void k_log_prob(const ViewInfo *__restrict__ views, int n_views,
                                                  const float *__restrict__ gt, const float *__restrict__ rd,
                                                  LogTaps taps, float tau, float *__restrict__ p_gt,
                                                  float *__restrict__ p_rd, uint8_t *__restrict__ mask) {
  extern __shared__ float lds[];
  int base;
  const int v = view_of_ins_tile(views, n_views, blockIdx.x, base);
  if (v < 0) return;
  const ViewInfo vi = views[v];
  const int W = vi.w, H = vi.h;
  const int txs = (W + kTW - 1) / kTW;
  const int t = blockIdx.x - base;
  const int x0 = (t % txs) * kTW, y0 = (t / txs) * kTH;
  constexpr int rows = kTH + 2 * R;
  constexpr int RA = (R + 3) / 4 * 4;  // the filter radius rounded up to whole float4s
  float *A = lds;                    // [3][rows][kTW]: rows * g
  float *B = A + 3 * rows * kTW;     // [3][rows][kTW]: rows * h
  const int x = threadIdx.x & 63, yb = (threadIdx.x >> 6) * 4;
  float P[2][4];
  for (int img = 0; img < 2; ++img) {
    const float *src = (img == 0 ? gt : rd) + 3 * vi.pix_off;
    // horizontal pass straight from global memory: item = (row, group of
    // four columns); its 4 + 2R inputs per channel (border replicated) are
    // loaded into registers and give four a and four b values per channel.
    // With 16-byte aligned rows an interior item reads whole float4s.
    const bool vec = ((reinterpret_cast<uintptr_t>(src) | (uintptr_t)W * 4u) & 15u) == 0;
    for (int e = threadIdx.x; e < rows * (kTW / 4); e += 256) {
      const int r = e >> 4, c0 = (e & 15) * 4;
      const int gy = min(max(y0 + r - R, 0), H - 1);
      const bool interior = vec && x0 + c0 - RA >= 0 && x0 + c0 + 4 + RA <= W;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float *row = src + ((int64_t)ch * H + gy) * W;
        float in[4 + 2 * R];
        if (interior) {
          const float4 *rv = reinterpret_cast<const float4 *>(row + x0 + c0 - RA);
          float buf[4 + 2 * RA];
#pragma unroll
          for (int k = 0; k < (4 + 2 * RA) / 4; ++k) {
            const float4 t = rv[k];
            buf[4 * k] = t.x;
            buf[4 * k + 1] = t.y;
            buf[4 * k + 2] = t.z;
            buf[4 * k + 3] = t.w;
          }
#pragma unroll
          for (int q = 0; q < 4 + 2 * R; ++q) in[q] = buf[q + RA - R];
        } else {
#pragma unroll
          for (int q = 0; q < 4 + 2 * R; ++q) in[q] = row[min(max(x0 + c0 + q - R, 0), W - 1)];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float a = 0.0f, b = 0.0f;
#pragma unroll
          for (int k = 0; k <= 2 * R; ++k) {
            a += taps.g[k] * in[j + k];
            b += taps.h[k] * in[j + k];
          }
          A[(ch * rows + r) * kTW + c0 + j] = a;
          B[(ch * rows + r) * kTW + c0 + j] = b;
        }
      }
    }
    __syncthreads();
    float L2[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float l[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 2 * R + 4; ++k) {
        const float a = A[(ch * rows + yb + k) * kTW + x], b = B[(ch * rows + yb + k) * kTW + x];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int kk = k - j;  // tap index of this row for output row yb + j
          if (kk >= 0 && kk <= 2 * R) l[j] += taps.g[kk] * b + taps.h[kk] * a;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) L2[j] += l[j] * l[j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) P[img][j] = fminf(sqrtf(L2[j]), 1.0f);
    __syncthreads();
  }
  const int gx = x0 + x;
  if (gx >= W) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int gy = y0 + yb + j;
    if (gy >= H) break;
    const int64_t pix = vi.pix_off + (int64_t)gy * W + gx;
    p_gt[pix] = P[0][j];
    if (p_rd) p_rd[pix] = P[1][j];
    const float pa = fmaxf(P[0][j] - P[1][j], 0.0f);
    mask[pix] = pa > tau ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void k_ins_count(const uint8_t *__restrict__ mask, int64_t n_pix,
                                                   uint32_t *__restrict__ counts) {
  __shared__ uint32_t red[4];
  const int64_t p0 = (int64_t)blockIdx.x * kInsBlock + (int64_t)threadIdx.x * 16;
  uint32_t c = 0;
  if (p0 + 16 <= n_pix) {  // mask bytes are 0 or 1: the popcount of the 16 bytes is their sum
    const uint4 m = *reinterpret_cast<const uint4 *>(mask + p0);
    c = __popc(m.x) + __popc(m.y) + __popc(m.z) + __popc(m.w);
  } else {
    for (int i = 0; i < 16; ++i) c += (p0 + i < n_pix) ? mask[p0 + i] : 0u;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Exclusive offsets of the blocks' counts and the total (one workgroup).
__global__ __launch_bounds__(1024) void k_ins_scan(const uint32_t *__restrict__ counts, uint32_t nb,
                                                   uint32_t *__restrict__ offsets, uint32_t *__restrict__ total) {
  __shared__ uint32_t wsum[16];
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t b0 = threadIdx.x * per, b1 = min(b0 + per, nb);
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t s = 0;
  for (uint32_t b = b0; b < b1; ++b) s += counts[b];
  // inclusive scan of the threads' sums: within each wave by shuffles, then
  // over the 16 wave totals in the first wave
  uint32_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (w == 0) {
    uint32_t t = lane < 16 ? wsum[lane] : 0u;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      const uint32_t y = __shfl_up(t, d);
      if (lane >= (uint32_t)d) t += y;
    }
    if (lane < 16) wsum[lane] = t;
  }
  __syncthreads();
  if (threadIdx.x == 1023) *total = wsum[15];
  uint32_t acc = x - s + (w > 0 ? wsum[w - 1] : 0u);
  for (uint32_t b = b0; b < b1; ++b) {
    offsets[b] = acc;
    acc += counts[b];
  }
}

__global__ __launch_bounds__(256) void k_ins_write(const ViewInfo *__restrict__ views, int n_views,
                                                   const Cam *__restrict__ cams, const uint8_t *__restrict__ mask,
                                                   int64_t n_pix, const uint32_t *__restrict__ offsets,
                                                   const float *__restrict__ p_gt, const float *__restrict__ depth,
                                                   uint32_t *__restrict__ out_pix, float *__restrict__ out_scale,
                                                   float *__restrict__ out_mean, int64_t capacity) {
  __shared__ uint32_t scan_tmp[4];
  constexpr int kPer = kInsBlock / 256;
  const int64_t p0 = (int64_t)blockIdx.x * kInsBlock + (int64_t)threadIdx.x * kPer;
  uint32_t bits = 0;
  if (p0 + kPer <= n_pix) {
    const uint4 m = *reinterpret_cast<const uint4 *>(mask + p0);
    const uint32_t w[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
    for (int i = 0; i < kPer; ++i) bits |= ((w[i >> 2] >> (8 * (i & 3))) & 1u) << i;
  } else {
    for (int i = 0; i < kPer; ++i)
      if (p0 + i < n_pix && mask[p0 + i]) bits |= 1u << i;
  }
  const uint32_t mine = __popc(bits);
  uint32_t block_total;
  const uint32_t before = block_excl_scan<256>(mine, scan_tmp, block_total);
  uint32_t k = offsets[blockIdx.x] + before;
  if (bits == 0) return;
  // view of the thread's first pixel (binary search), then forward at the
  // (rare) view boundary inside its 16 pixels
  int v = 0;
  for (int hi = n_views - 1; v < hi;) {
    const int mid = (v + hi + 1) >> 1;
    if ((int64_t)views[mid].pix_off <= p0) v = mid;
    else hi = mid - 1;
  }
  int64_t next = v + 1 < n_views ? (int64_t)views[v + 1].pix_off : INT64_MAX;
  ViewInfo vi = views[v];
  Cam c = cams[v];
  for (int i = 0; i < kPer; ++i) {
    if (!(bits >> i & 1u)) continue;
    const int64_t p = p0 + i;
    while (p >= next) {
      ++v;
      vi = views[v];
      c = cams[v];
      next = v + 1 < n_views ? (int64_t)views[v + 1].pix_off : INT64_MAX;
    }
    if ((int64_t)k < capacity) {
      const uint32_t local = (uint32_t)(p - vi.pix_off);  // a view's pixels fit 32 bits
      const int row = (int)(local / (uint32_t)vi.w), u = (int)(local - (uint32_t)row * (uint32_t)vi.w);
      const float z = depth[p];
      const float xc = z * (((float)u + 0.5f - c.cx) / c.fx);
      const float yc = z * (((float)row + 0.5f - c.cy) / c.fy);
      const float d = sqrtf(xc * xc + yc * yc + z * z);
      out_pix[k] = (uint32_t)p;
      out_scale[k] = d / (2.0f * sqrtf(p_gt[p]) * c.fx);
      // x_w = R^T (x_c - t)
      const float ex = xc - c.t[0], ey = yc - c.t[1], ez = z - c.t[2];
      out_mean[3 * k + 0] = c.R[0] * ex + c.R[3] * ey + c.R[6] * ez;
      out_mean[3 * k + 1] = c.R[1] * ex + c.R[4] * ey + c.R[7] * ez;
      out_mean[3 * k + 2] = c.R[2] * ex + c.R[5] * ey + c.R[8] * ez;
    }
    ++k;
  }
}

}  // namespace

uint32_t ins_tiles(const ViewInfo *views_host, int n_views) {
  uint32_t n = 0;
  for (int v = 0; v < n_views; ++v)
    n += (uint32_t)(((views_host[v].w + kTW - 1) / kTW) * ((views_host[v].h + kTH - 1) / kTH));
  return n;
}

uint32_t ins_blocks(int64_t n_pix) { return (uint32_t)((n_pix + kInsBlock - 1) / kInsBlock); }

size_t ins_lds_bytes(int R) {
  const int rows = kTH + 2 * R;
  return (size_t)(2 * 3 * rows * kTW) * sizeof(float);
}

void launch_log_insert(const ViewInfo *views_d, int n_views, uint32_t n_tiles, int64_t n_pix, const Cam *cams,
                       const float *gt, const float *rd, const float *depth, const LogTaps &taps, float tau,
                       float *p_gt, float *p_rd, uint8_t *mask, uint32_t *counts, uint32_t *offsets,
                       uint32_t *total, uint32_t *out_pix, float *out_scale, float *out_mean, int64_t capacity,
                       hipStream_t st) {
  if (n_tiles == 0) return;
#define GSR_LOG_PROB(RR)                                                                                    \
  case RR:                                                                                                  \
    k_log_prob<RR><<<n_tiles, 256, ins_lds_bytes(RR), st>>>(views_d, n_views, gt, rd, taps, tau, p_gt, p_rd, \
                                                            mask);                                          \
    break;
  switch (taps.R) {
    GSR_LOG_PROB(1)
    GSR_LOG_PROB(2)
    GSR_LOG_PROB(3)
    GSR_LOG_PROB(4)
    default: GSR_LOG_PROB(5)
  }
#undef GSR_LOG_PROB
  const uint32_t nb = ins_blocks(n_pix);
  k_ins_count<<<nb, 256, 0, st>>>(mask, n_pix, counts);
  k_ins_scan<<<1, 1024, 0, st>>>(counts, nb, offsets, total);
  k_ins_write<<<nb, 256, 0, st>>>(views_d, n_views, cams, mask, n_pix, offsets, p_gt, depth, out_pix, out_scale,
                                  out_mean, capacity);
}

}  // namespace gsr

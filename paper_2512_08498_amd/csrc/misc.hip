// L1 photometric loss with its gradient, the binning export used by the
// parity checks, and the compositing work counter.
#include <algorithm>

#include "kernels.hpp"
#include "util.hpp"

namespace gsr {

// loss = sum |img - tgt| / n, dL/dimg = sign(img - tgt) / n.  Per-block
// partial sums, then one workgroup adds the partials in block order, so the
// value is deterministic.  (A last-block ticket would need a device-scope
// release per block, which on a multi-XCD part writes back the L2.)  float4
// accesses when all three arrays are 16-byte aligned.
__global__ __launch_bounds__(256) void k_l1(const float *__restrict__ img, const float *__restrict__ tgt, int64_t n,
                                            float *__restrict__ dl, float *__restrict__ partials, int vec) {
  __shared__ float s_red[4];
  const float inv_n = (float)(1.0 / (double)n);
  float acc = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  auto sgn = [&](float d) { return d > 0.0f ? inv_n : (d < 0.0f ? -inv_n : 0.0f); };
  int64_t tail0 = 0;
  if (vec) {
    const int64_t n4 = n / 4;
    const float4 *a4 = reinterpret_cast<const float4 *>(img);
    const float4 *b4 = reinterpret_cast<const float4 *>(tgt);
    float4 *d4 = reinterpret_cast<float4 *>(dl);
    for (int64_t i = gid; i < n4; i += stride) {
      const float4 a = a4[i], b = b4[i];
      const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, dw = a.w - b.w;
      acc += (fabsf(dx) + fabsf(dy)) + (fabsf(dz) + fabsf(dw));
      d4[i] = make_float4(sgn(dx), sgn(dy), sgn(dz), sgn(dw));
    }
    tail0 = n4 * 4;
  }
  for (int64_t i = tail0 + gid; i < n; i += stride) {
    const float d = img[i] - tgt[i];
    acc += fabsf(d);
    dl[i] = sgn(d);
  }
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (lane_id() == 0) s_red[wave_id()] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// The mean from many partials: 1024 threads, thread t adding partials
// t, t + 1024, ... in order (in double), then the 16 waves' sums in order.
__global__ __launch_bounds__(1024) void k_l1_sum(const float *__restrict__ partials, uint32_t nb, int64_t n,
                                                 float *__restrict__ loss) {
  __shared__ double s_d[16];
  double s = 0.0;
#pragma unroll 4
  for (uint32_t b = threadIdx.x; b < nb; b += 1024u) s += (double)partials[b];
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, kWave);
  if (lane_id() == 0) s_d[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = s_d[0];
    for (int w = 1; w < 16; ++w) t += s_d[w];
    *loss = (float)(t / (double)n);
  }
}

void launch_l1_sum(const float *partials, uint32_t nb, int64_t n, float *loss, hipStream_t st) {
  k_l1_sum<<<1, 1024, 0, st>>>(partials, nb, n, loss);
}

void launch_l1(const float *img, const float *tgt, int64_t n, float *loss, float *dl, float *partials,
               hipStream_t st) {
  const bool vec = ((reinterpret_cast<uintptr_t>(img) | reinterpret_cast<uintptr_t>(tgt) |
                     reinterpret_cast<uintptr_t>(dl)) & 15u) == 0;
  const int64_t work = vec ? (n + 3) / 4 : n;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, kLossBlocks));
  k_l1<<<(unsigned)blocks, 256, 0, st>>>(img, tgt, n, dl, partials, vec ? 1 : 0);
  launch_l1_sum(partials, (uint32_t)blocks, n, loss, st);
}

// Streaming copy for the bandwidth measurement: each workgroup moves one
// contiguous 16 KB chunk, each thread four 16-byte words (all loads issued
// before the stores), with non-temporal accesses so the copy does not
// occupy the caches.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr uint64_t kCopyChunk = 256 * 4;  // 16-byte words per workgroup

__global__ __launch_bounds__(256) void k_copy16(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src, uint64_t n) {
  const uint64_t base = (uint64_t)blockIdx.x * kCopyChunk + threadIdx.x;
  u32x4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t i = base + 256u * k;
    if (i < n) v[k] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t i = base + 256u * k;
    if (i < n) __builtin_nontemporal_store(v[k], dst + i);
  }
}

void launch_copy16(void *dst, const void *src, uint64_t n16, hipStream_t st) {
  if (n16 == 0) return;
  const uint64_t blocks = (n16 + kCopyChunk - 1) / kCopyChunk;
  k_copy16<<<(unsigned)blocks, 256, 0, st>>>(static_cast<u32x4 *>(dst), static_cast<const u32x4 *>(src), n16);
}

// One workgroup per tile: keys = tile << 32 | depth bits, values = Gaussian;
// the CSR offsets are the exclusive scan of the list lengths.
__global__ __launch_bounds__(256) void k_debug_binning(Ws ws, Sizes sz, uint64_t *__restrict__ keys,
                                                       uint32_t *__restrict__ vals) {
  const uint32_t tile = blockIdx.x;
  const uint32_t start = ws.tile_start[tile], n = ws.tile_count[tile];
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t rec = ws.tile_recs[start + i];
    keys[start + i] = ((uint64_t)tile << 32) | ws.rec_zbits[rec];
    vals[start + i] = ws.rec_g[rec];
  }
}

void launch_debug_binning(const ViewInfo *views, const Ws &ws, const Sizes &sz, uint64_t *keys, uint32_t *vals,
                          uint32_t *csr, hipStream_t st) {
  (void)views;
  if (sz.t_tot == 0) return;
  k_debug_binning<<<sz.t_tot, 256, 0, st>>>(ws, sz, keys, vals);
  launch_tile_csr(ws, sz, csr, st);
}

// Compositing work of the last forward: for every pixel, the entries of its
// tile's list in front of its stop position (last_pos) whose binning box
// contains the pixel -- the (pixel, Gaussian) evaluations of the method's
// definition.  The compositing kernels skip the pixels outside a record's
// opacity-narrowed box, where alpha < 1/255, so they perform fewer.  One workgroup per tile, boxes staged in
// LDS; a per-workgroup integer sum is added to *evals.
__global__ __launch_bounds__(256) void k_count_evals(const ViewInfo *__restrict__ views, Ws ws, Sizes sz,
                                                     const uint32_t *__restrict__ last_pos,
                                                     unsigned long long *__restrict__ evals) {
  __shared__ float4 s_box[256];
  __shared__ unsigned long long s_sum[4];
  if (ws.scalars[kOverflow]) return;
  const uint32_t tile = blockIdx.x;
  const int v = view_of_tile(views, sz.n_views, tile);
  const ViewInfo vi = views[v];
  const uint32_t lt = tile - vi.tile_base;
  const int tx = (int)(lt % (uint32_t)vi.tiles_x), ty = (int)(lt / (uint32_t)vi.tiles_x);
  const uint32_t start = ws.tile_start[tile], n = ws.tile_count[tile];
  const uint32_t nrec = ws.scalars[kNumRecords];
  const int ts = sz.ts, npix = ts * ts;
  constexpr int kMaxPix = 4;  // 32 x 32 tiles over 256 threads
  float fx[kMaxPix], fy[kMaxPix];
  uint32_t last[kMaxPix];
  for (int p = 0; p < kMaxPix; ++p) {
    const int q = (int)threadIdx.x + p * 256;
    const int px = tx * ts + q % ts, py = ty * ts + q / ts;
    fx[p] = (float)px;
    fy[p] = (float)py;
    last[p] = 0;
    if (q < npix && px < vi.w && py < vi.h)
      last[p] = min(n, last_pos[vi.pix_off + (uint32_t)py * (uint32_t)vi.w + (uint32_t)px]);
  }
  unsigned long long cnt = 0;
  for (uint32_t b0 = 0; b0 < n; b0 += 256) {
    const uint32_t m = min(256u, n - b0);
    __syncthreads();
    if (threadIdx.x < m) {
      uint32_t rec = ws.tile_recs[start + b0 + threadIdx.x];
      if (rec >= nrec) rec = 0;
      // the binning box (p3, packed): evaluations are counted against it
      const float4 p3 = ws.rec_payload[(size_t)rec * 4 + 3];
      const uint32_t bx = __float_as_uint(p3.y), by = __float_as_uint(p3.z);
      s_box[threadIdx.x] = make_float4((float)(bx & 0xFFFFu), (float)(bx >> 16), (float)(by & 0xFFFFu),
                                       (float)(by >> 16));
    }
    __syncthreads();
    for (uint32_t j = 0; j < m; ++j) {
      const float4 box = s_box[j];
      for (int p = 0; p < kMaxPix; ++p)
        cnt += (b0 + j < last[p] && fx[p] >= box.x && fx[p] <= box.y && fy[p] >= box.z && fy[p] <= box.w) ? 1 : 0;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, kWave);
  if (lane_id() == 0) s_sum[wave_id()] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(evals, (s_sum[0] + s_sum[1]) + (s_sum[2] + s_sum[3]));
}

__global__ void k_fill(float *__restrict__ p, uint64_t n, float value) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

void launch_fill(float *p, uint64_t n, float value, hipStream_t st) {
  if (n == 0) return;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 8192);
  k_fill<<<(unsigned)blocks, 256, 0, st>>>(p, n, value);
}

void launch_count_evals(const ViewInfo *views, const Ws &ws, const Sizes &sz, const uint32_t *last_pos,
                        uint64_t *evals, hipStream_t st) {
  launch_zero(reinterpret_cast<uint32_t *>(evals), 2, st);
  if (sz.t_tot == 0) return;
  k_count_evals<<<sz.t_tot, 256, 0, st>>>(views, ws, sz, last_pos, reinterpret_cast<unsigned long long *>(evals));
}

}  // namespace gsr

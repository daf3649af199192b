// Preprocess: project every (view, Gaussian) pair, compact the visible ones
// into records (Gaussian-major) with their raster payload and tile
// rectangles.
//
// Two passes over the Gaussians with a scan between them (reduce, then
// scan, then write), so record indices are deterministic and increase with
// the Gaussian index within each view -- the tie-break order of the sort.
// Each thread owns one Gaussian: the counting pass projects it into every
// view and keeps a bit mask of the views that see it; the writing pass
// projects it again only into those views.
#include <algorithm>

#include "kernels.hpp"
#include "sh.hpp"
#include "spec.hpp"
#include "util.hpp"

namespace gsr {

__global__ void k_zero_words(uint32_t *__restrict__ p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

__device__ __forceinline__ uint32_t rect_area(const Proj &P, int ts_shift) {
  const uint32_t w = (uint32_t)((P.i1 >> ts_shift) - (P.i0 >> ts_shift) + 1);
  const uint32_t h = (uint32_t)((P.j1 >> ts_shift) - (P.j0 >> ts_shift) + 1);
  return w * h;
}

// Screen for the counting pass: false only if (view c, Gaussian) is certainly
// invisible under the binning rules of spec.hpp.  The camera-space depth is
// computed exactly as there (the same operations in the same order), so
// the near-plane test is the same decision.
// The pixel box is bounded from above with fast reciprocals: the half
// extent hx = sqrt(K (|t0 M|^2 + 0.3)) with |t0 M| <= |t0| s_max and
// |t0| <= |j00| |R_0| + |j02| |R_2| (rows of the view rotation, bounded by
// their L1 norms), so hx_b >= hx after a 1e-4 relative inflation that covers
// every rounding involved (hardware reciprocal and square root included);
// the box misses the image only if u + hx < 0.5 or u - hx > w - 0.5, tested
// with a margin of 1 px plus 2e-5 of the magnitudes for the rounding of u.
// s2 is the square of the largest scale, inflated the same way.  NaN keeps
// the pair.
__device__ __forceinline__ bool may_be_visible(const float m3[3], float s2, const Cam &c) {
  float xc, yc, zc;
  {
#pragma clang fp contract(off)
    xc = ((c.R[0] * m3[0] + c.R[1] * m3[1]) + c.R[2] * m3[2]) + c.t[0];
    yc = ((c.R[3] * m3[0] + c.R[4] * m3[1]) + c.R[5] * m3[2]) + c.t[1];
    zc = ((c.R[6] * m3[0] + c.R[7] * m3[1]) + c.R[8] * m3[2]) + c.t[2];
  }
  if (!(zc > kNearZ)) return false;
  const float rz = __builtin_amdgcn_rcpf(zc);
  const float xz = xc * rz, yz = yc * rz;
  const float u = fmaf(c.fx, xz, c.cx), v = fmaf(c.fy, yz, c.cy);
  const float wf = (float)c.w, hf = (float)c.h;
  // |xt| of the guard clamp: min(|x/z|, lim) for lim >= 0, |lim| otherwise
  const float lim_x = kClampFov * fmaxf(c.cx, wf - c.cx) * __builtin_amdgcn_rcpf(c.fx);
  const float lim_y = kClampFov * fmaxf(c.cy, hf - c.cy) * __builtin_amdgcn_rcpf(c.fy);
  const float axt = lim_x >= 0.0f ? fminf(fabsf(xz), lim_x) : -lim_x;
  const float ayt = lim_y >= 0.0f ? fminf(fabsf(yz), lim_y) : -lim_y;
  // row norms of the view rotation, bounded by their L1 norms
  const float n0 = (fabsf(c.R[0]) + fabsf(c.R[1])) + fabsf(c.R[2]);
  const float n1 = (fabsf(c.R[3]) + fabsf(c.R[4])) + fabsf(c.R[5]);
  const float n2 = (fabsf(c.R[6]) + fabsf(c.R[7])) + fabsf(c.R[8]);
  const float tx = fabsf(c.fx) * rz * fmaf(axt, n2, n0);
  const float ty = fabsf(c.fy) * rz * fmaf(ayt, n2, n1);
  const float hx = 1.0001f * __builtin_amdgcn_sqrtf(kSupportK * fmaf(tx * tx, s2, kDilation));
  const float hy = 1.0001f * __builtin_amdgcn_sqrtf(kSupportK * fmaf(ty * ty, s2, kDilation));
  const float ex = fmaf(2e-5f, (fabsf(c.fx * xz) + fabsf(c.cx)) + hx, 1.0f);
  const float ey = fmaf(2e-5f, (fabsf(c.fy * yz) + fabsf(c.cy)) + hy, 1.0f);
  const bool out = (u + hx < 0.5f - ex) || (u - hx > wf - 0.5f + ex) || (v + hy < 0.5f - ey) ||
                   (v - hy > hf - 0.5f + ey);
  return !out;
}

constexpr int kScreenViews = 16;  // views screened per round of the counting pass

// Counting pass: per Gaussian, its visible views (a bit mask), record count
// and (record, tile) pair count, block-scanned.  Each wave screens its 64
// Gaussians against 16 views at a time, queues the (Gaussian, view) pairs
// that may be visible in LDS and runs the exact binning rules on the queue
// 64 at a time, so the rules' cost follows the visible pairs rather than
// every lane's every view.  The results are integer LDS atomics on the
// owning Gaussian's counters, the same whatever the order.
// Also clears the n_zero words at `zero` (the forward's counters and tile
// ranges, which no kernel before the scan reads), saving a launch.
__global__ __launch_bounds__(kPreBlock) void k_pre_count(GaussPtrs gp, const Cam *__restrict__ cams,
                                                         Ws ws, Sizes sz, int ts_shift, uint32_t *__restrict__ zero,
                                                         uint64_t n_zero) {
  constexpr int NW = kPreBlock / kWave;
  __shared__ uint32_t s_scan[NW * 2];
  __shared__ float s_par[10][kPreBlock];                   // mean, log-scale, quaternion of each Gaussian
  __shared__ uint32_t s_cnt[3][kPreBlock];                 // records, pairs, visible-view bits of the round
  __shared__ uint16_t s_q[NW][kWave * kScreenViews];       // queued (lane, view) pairs of each wave
  const int t = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int64_t g = (int64_t)blockIdx.x * kPreBlock + t;
  for (uint64_t i = (uint64_t)g; i < n_zero; i += (uint64_t)gridDim.x * kPreBlock) zero[i] = 0u;
  const bool live = g < sz.n;
  float m3[3] = {0.f, 0.f, 0.f}, l3[3] = {0.f, 0.f, 0.f}, q4[4] = {0.f, 0.f, 0.f, 0.f};
  if (live) load_gaussian(gp.mean, gp.log_scale, gp.quat, sz.n, g, m3, l3, q4);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s_par[k][t] = m3[k];
    s_par[3 + k][t] = l3[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) s_par[6 + k][t] = q4[k];
  s_cnt[0][t] = s_cnt[1][t] = s_cnt[2][t] = 0u;
  const float smax = expf(fmaxf(fmaxf(l3[0], l3[1]), l3[2]));
  const float s2 = 1.0001f * (smax * smax);
  uint64_t word = 0;
  for (int v0 = 0; v0 < sz.n_views; v0 += kScreenViews) {
    const int nv = min(kScreenViews, sz.n_views - v0);
    uint32_t m = 0;
    if (live)
      for (int j = 0; j < nv; ++j)
        if (may_be_visible(m3, s2, load_cam(cams, v0 + j))) m |= 1u << j;
    // queue this lane's candidate views after those of the lanes below it
    const uint32_t c = (uint32_t)__popc(m);
    const uint32_t incl = wave_incl_scan(c);
    const uint32_t total = (uint32_t)__shfl(incl, kWave - 1, kWave);
    uint32_t pos = incl - c;
    for (uint32_t mm = m; mm; mm &= mm - 1) s_q[wv][pos++] = (uint16_t)((lane << 4) | (__ffs(mm) - 1));
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the wave's queue is written
    __builtin_amdgcn_wave_barrier();
    for (uint32_t base = 0; base < total; base += kWave) {
      const uint32_t e = base + (uint32_t)lane;
      if (e < total) {
        const uint32_t q = s_q[wv][e];
        const int o = wv * kWave + (int)(q >> 4), j = (int)(q & 15u);
        float pm[3], pl[3], pq[4];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          pm[k] = s_par[k][o];
          pl[k] = s_par[3 + k][o];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) pq[k] = s_par[6 + k][o];
        Proj P;
        project_spec(pm, pl, pq, load_cam(cams, v0 + j), P);
        if (P.visible) {
          atomicAdd(&s_cnt[0][o], 1u);
          atomicAdd(&s_cnt[1][o], rect_area(P, ts_shift));
          atomicOr(&s_cnt[2][o], 1u << j);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // the wave's counter updates are done
    __builtin_amdgcn_wave_barrier();
    word |= (uint64_t)s_cnt[2][t] << (v0 & 63);
    s_cnt[2][t] = 0u;
    const int v_end = v0 + nv;
    if ((v_end & 63) == 0 || v_end == sz.n_views) {
      if (live) ws.vis_mask[(int64_t)(v0 >> 6) * sz.n + g] = word;
      word = 0;
    }
  }
  const uint32_t recs = s_cnt[0][t], pairs = s_cnt[1][t];
  uint32_t tr, tp;
  block_excl_scan<kPreBlock>(recs, s_scan, tr);
  block_excl_scan<kPreBlock>(pairs, s_scan + NW, tp);
  if (threadIdx.x == 0) ws.block_sums[blockIdx.x] = make_uint2(tr, tp);
}

// One workgroup: exclusive scan of the per-block (records, pairs) totals.
__global__ __launch_bounds__(1024) void k_scan_blocks(Ws ws, Sizes sz) {
  __shared__ uint64_t s_a[16], s_b[16];
  const uint32_t nb = sz.n_blocks;
  const uint32_t per = (nb + 1023u) / 1024u;
  const uint32_t lo = min(nb, threadIdx.x * per), hi = min(nb, lo + per);
  uint64_t sr = 0, sp = 0;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint2 b = ws.block_sums[i];
    sr += b.x;
    sp += b.y;
  }
  uint64_t tr, tp;
  uint64_t er = block_excl_scan<1024>(sr, s_a, tr);
  uint64_t ep = block_excl_scan<1024>(sp, s_b, tp);
  const bool over = tr > sz.cap_rec || tp > sz.cap_pairs;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint2 b = ws.block_sums[i];
    ws.block_sums[i] = make_uint2((uint32_t)er, (uint32_t)ep);
    er += b.x;
    ep += b.y;
  }
  if (threadIdx.x == 0) {
    ws.scalars[kNumRecords] = (uint32_t)min<uint64_t>(tr, 0xFFFFFFFFull);
    ws.scalars[kNumPairs] = (uint32_t)min<uint64_t>(tp, 0xFFFFFFFFull);
    ws.scalars[kOverflow] = over ? 1u : 0u;
  }
}

template <int DEG>
__global__ __launch_bounds__(kPreBlock) void k_pre_write(GaussPtrs gp, const Cam *__restrict__ cams,
                                                         const ViewInfo *__restrict__ views, Ws ws,
                                                         Sizes sz, int ts_shift) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ uint32_t s_scan[kPreBlock / kWave * 2];
  if (ws.scalars[kOverflow]) return;
  const int64_t g = (int64_t)blockIdx.x * kPreBlock + threadIdx.x;
  const bool live = g < sz.n;
  // the visible views from the counting pass: only those are projected again
  uint32_t recs = 0;
  if (live)
    for (uint32_t w = 0; w < sz.vis_words; ++w) recs += (uint32_t)__popcll(ws.vis_mask[(int64_t)w * sz.n + g]);
  uint32_t tr;
  const uint2 base = ws.block_sums[blockIdx.x];
  uint32_t rec = base.x + block_excl_scan<kPreBlock>(recs, s_scan, tr);
  const uint32_t rec0 = rec;
  uint32_t pairs = 0;
  if (live) {
    ws.rec_start[g] = rec;
    if (g == sz.n - 1) ws.rec_start[sz.n] = rec + recs;
  }
  if (live && recs > 0) {
    float sh[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) sh[k][ch] = gp.sh[((int64_t)k * 3 + ch) * sz.n + g];
    const float op = 1.0f / (1.0f + expf(-gp.opacity_logit[g]));

    float m3[3], l3[3], q4[4];
    load_gaussian(gp.mean, gp.log_scale, gp.quat, sz.n, g, m3, l3, q4);
    for (uint32_t wd = 0; wd < sz.vis_words; ++wd)
      for (uint64_t bits = ws.vis_mask[(int64_t)wd * sz.n + g]; bits; bits &= bits - 1) {
      const int v = (int)(wd * 64u) + __ffsll((unsigned long long)bits) - 1;
      const Cam c = load_cam(cams, v);
      Proj P;
      project_spec(m3, l3, q4, c, P);
      // 2D mean in float64 (the pixel grid is ~2^11 wide, so a float32
      // projection would be off by up to ~1e-4 px); stored as the offset from
      // the box corner, which float32 represents to ~1e-7 px.
      const double xd = ((double)c.R[0] * m3[0] + (double)c.R[1] * m3[1]) + (double)c.R[2] * m3[2] + c.t[0];
      const double yd = ((double)c.R[3] * m3[0] + (double)c.R[4] * m3[1]) + (double)c.R[5] * m3[2] + c.t[1];
      const double zd = ((double)c.R[6] * m3[0] + (double)c.R[7] * m3[1]) + (double)c.R[8] * m3[2] + c.t[2];
      const double mux = (double)c.fx * (xd / zd) + (double)c.cx, muy = (double)c.fy * (yd / zd) + (double)c.cy;
      // The compositing kernels test the box of d^2 <= 2 ln(255 opacity)
      // instead of the binning box: outside it alpha < 1/255 (for a pixel
      // centre dx from the mean, d^2 >= dx^2 / S_xx), so the same entries are
      // composited.  The 0.01 margin in d^2 covers the rounding of the kernels'
      // d^2 and of this box.  The binning (tile lists) keeps the full box.
      float bi0 = (float)P.i0, bi1 = (float)P.i1, bj0 = (float)P.j0, bj1 = (float)P.j1;
      const float keff = 2.0f * logf(255.0f * op) + 0.01f;
      if (keff < kSupportK) {
        if (!(keff > 0.0f)) {  // opacity below 1/255: nothing can composite
          bi0 = bj0 = 1.0f;
          bi1 = bj1 = 0.0f;
        } else {
          const float hxt = sqrtf(keff * (P.p0 + kDilation)), hyt = sqrtf(keff * (P.p1 + kDilation));
          bi0 = fmaxf(bi0, ceilf((float)mux - hxt - 0.5f));
          bi1 = fminf(bi1, floorf((float)mux + hxt - 0.5f));
          bj0 = fmaxf(bj0, ceilf((float)muy - hyt - 0.5f));
          bj1 = fminf(bj1, floorf((float)muy + hyt - 0.5f));
        }
      }
      const float offx = (float)(mux - (double)bi0 - 0.5);
      const float offy = (float)(muy - (double)bj0 - 0.5);
      // Conic in Cholesky form.  With S = A A^T + 0.3 I:
      //   d^T S^-1 d = (dx + qb dy)^2 * S_yy / det + dy^2 / S_yy,  qb = -S_xy / S_yy
      // and det = |a0 x a1|^2 + 0.3 (|a0|^2 + |a1|^2) + 0.09 has no cancellation.
      const float sxx = P.p0 + kDilation, syy = P.p1 + kDilation;
      const float sxy = (P.a0[0] * P.a1[0] + P.a0[1] * P.a1[1]) + P.a0[2] * P.a1[2];
      const float cx_ = P.a0[1] * P.a1[2] - P.a0[2] * P.a1[1];
      const float cy_ = P.a0[2] * P.a1[0] - P.a0[0] * P.a1[2];
      const float cz_ = P.a0[0] * P.a1[1] - P.a0[1] * P.a1[0];
      const float det = (cx_ * cx_ + cy_ * cy_ + cz_ * cz_) + kDilation * (P.p0 + P.p1) + kDilation * kDilation;
      (void)sxx;
      const float qa = -kHalfLog2e * (syy / det);
      const float qb = -sxy / syy;
      const float qc = -kHalfLog2e / syy;
      // view-dependent colour
      const float cxw = -(c.R[0] * c.t[0] + c.R[3] * c.t[1] + c.R[6] * c.t[2]);
      const float cyw = -(c.R[1] * c.t[0] + c.R[4] * c.t[1] + c.R[7] * c.t[2]);
      const float czw = -(c.R[2] * c.t[0] + c.R[5] * c.t[1] + c.R[8] * c.t[2]);
      const float dx = m3[0] - cxw, dy = m3[1] - cyw, dz = m3[2] - czw;
      const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
      float Y[16];
      sh_basis(dx * inv, dy * inv, dz * inv, DEG, Y);
      float rgb[3];
      uint32_t pass = 0;  // bit ch: colour channel ch not clamped (gradient passes)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float s = 0.5f;
#pragma unroll
        for (int k = 0; k < K; ++k) s += sh[k][ch] * Y[k];
        rgb[ch] = fmaxf(s, 0.0f);
        pass |= (s >= 0.0f ? 1u : 0u) << ch;
      }
      ws.rec_payload[(size_t)rec * 4 + 0] = make_float4(bi0, bi1, bj0, bj1);
      ws.rec_payload[(size_t)rec * 4 + 1] = make_float4(offx, offy, qa, qb);
      ws.rec_payload[(size_t)rec * 4 + 2] = make_float4(qc, op, rgb[0], rgb[1]);
      ws.rec_payload[(size_t)rec * 4 + 3] =
          make_float4(rgb[2], __uint_as_float((uint32_t)P.i0 | ((uint32_t)P.i1 << 16)),
                      __uint_as_float((uint32_t)P.j0 | ((uint32_t)P.j1 << 16)), __uint_as_float(pass));
      const int tx0 = P.i0 >> ts_shift, tx1 = P.i1 >> ts_shift;
      const int ty0 = P.j0 >> ts_shift, ty1 = P.j1 >> ts_shift;
      ws.rec_g[rec] = (uint32_t)g;
      ws.rec_view[rec] = (uint32_t)v;
      const ViewInfo vi = views[v];
      ws.rec_rect[rec] = make_uint4((uint32_t)tx0 | ((uint32_t)tx1 << 16), (uint32_t)ty0 | ((uint32_t)ty1 << 16),
                                    vi.tile_base + (uint32_t)ty0 * (uint32_t)vi.tiles_x + (uint32_t)tx0,
                                    (uint32_t)vi.tiles_x);
      ws.rec_zbits[rec] = P.zbits;
      pairs += (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
      rec += 1;
    }
  }
  // First (record, tile) slot of each record in record order: the gradient
  // partials of a record's tiles are contiguous and consecutive records'
  // slots follow each other, so the per-record reduction streams them.
  uint32_t tp;
  uint32_t slot = base.y + block_excl_scan<kPreBlock>(pairs, s_scan + kPreBlock / kWave, tp);
  if (live)
    for (uint32_t r = rec0; r < rec0 + recs; ++r) {
      const uint4 rc = ws.rec_rect[r];
      ws.rec_pairoff[r] = slot;
      slot += ((rc.x >> 16) - (rc.x & 0xFFFFu) + 1) * ((rc.y >> 16) - (rc.y & 0xFFFFu) + 1);
    }
}

void launch_zero(uint32_t *p, uint64_t n_words, hipStream_t st);

void launch_preprocess(const GaussPtrs &gp, const Cam *cams, const ViewInfo *views, const Ws &ws,
                       const Sizes &sz, int sh_degree, uint32_t *zero, uint64_t n_zero, hipStream_t st) {
    const int ts_shift = sz.ts == 8 ? 3 : (sz.ts == 16 ? 4 : 5);
  if (sz.n_blocks == 0) {
    launch_zero(zero, n_zero, st);
    return;
  }
  k_pre_count<<<sz.n_blocks, kPreBlock, 0, st>>>(gp, cams, ws, sz, ts_shift, zero, n_zero);
  k_scan_blocks<<<1, 1024, 0, st>>>(ws, sz);
  switch (sh_degree) {
    case 0: k_pre_write<0><<<sz.n_blocks, kPreBlock, 0, st>>>(gp, cams, views, ws, sz, ts_shift); break;
    case 1: k_pre_write<1><<<sz.n_blocks, kPreBlock, 0, st>>>(gp, cams, views, ws, sz, ts_shift); break;
    case 2: k_pre_write<2><<<sz.n_blocks, kPreBlock, 0, st>>>(gp, cams, views, ws, sz, ts_shift); break;
    default: k_pre_write<3><<<sz.n_blocks, kPreBlock, 0, st>>>(gp, cams, views, ws, sz, ts_shift); break;
  }
}

void launch_zero(uint32_t *p, uint64_t n_words, hipStream_t st) {
  if (n_words == 0) return;
  const uint64_t blocks = std::min<uint64_t>((n_words + 255) / 256, 4096);
  k_zero_words<<<(unsigned)blocks, 256, 0, st>>>(p, n_words);
}

}  // namespace gsr

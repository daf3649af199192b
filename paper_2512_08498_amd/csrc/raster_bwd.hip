// Backward compositing: the adjoint of the forward blend, walking each
// tile's list back to front.
//
// Per pixel the walk starts at the stored end position with T = T_final and
// the suffix colour Rb = bg.  For every entry it recomputes alpha exactly as
// the forward did, recovers the transmittance in front of it by division,
// T_i = T_{i+1} / (1 - alpha_i), and accumulates
//   dL/drgb   += g alpha T_i
//   dL/dalpha  = T_i sum_ch g_ch (rgb_ch - Rb_ch),  Rb <- alpha rgb + (1 - alpha) Rb
// and, unless alpha hit the 0.99 cap, dL/dopacity and dL/dq through
// alpha = opacity 2^q, then dL/d(qa, qb, qc, offx, offy) through q.
//
// The 9 per-entry gradients are summed over each wave by DPP row reductions
// (skipped when no lane of the wave touched the entry), combined over the
// waves in LDS, and written once per (record, tile) into that pair's slot --
// no floating-point atomics, so the result is deterministic.  The
// transmittance is recovered with the hardware reciprocal (1 ulp), which
// keeps the accumulated relative error of T near 1e-6 over a few hundred
// entries.
#include <algorithm>

#include "kernels.hpp"
#include "raster.hpp"
#include "util.hpp"

namespace gsr {

constexpr float kLn2 = 0x1.62e43p-1f;

template <int TS>
__global__ __launch_bounds__(TileCfg<TS>::NT) void k_raster_bwd(const ViewInfo *__restrict__ views, Ws ws,
                                                                Sizes sz, const float *__restrict__ t_final,
                                                                const uint32_t *__restrict__ last_pos,
                                                                const float *__restrict__ dL_dimage) {
  constexpr int NT = TileCfg<TS>::NT, PPT = TileCfg<TS>::PPT, NW = TileCfg<TS>::NW;
  constexpr int B = NT >= 128 ? 128 : NT;
  __shared__ float4 s_p0[B], s_p1[B], s_p2[B], s_p3[B];
  __shared__ uint32_t s_out[B];
  __shared__ float s_g[B * NW * 9];
  __shared__ uint32_t s_red[NW];
  if (ws.scalars[kOverflow]) return;
  if (blockIdx.x >= sz.t_tot) return;
  const uint32_t tile = ws.tile_order[blockIdx.x];  // longest lists first
  const int t = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int v = view_of_tile(views, sz.n_views, tile);
  const ViewInfo vi = views[v];
  const uint32_t lt = tile - vi.tile_base;
  const uint32_t tx = lt % (uint32_t)vi.tiles_x, ty = lt / (uint32_t)vi.tiles_x;
  const uint32_t start = ws.tile_start[tile], n = ws.tile_count[tile];
  const uint32_t nrec = ws.scalars[kNumRecords];
  if (n == 0) return;

  float fx[PPT], fy[PPT], T[PPT], g0[PPT], g1[PPT], g2[PPT], R0[PPT], R1[PPT], R2[PPT];
  uint32_t last[PPT];
  uint32_t my_max = 0;
  const uint32_t hw = (uint32_t)vi.w * (uint32_t)vi.h;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    int x, y;
    pixel_of<TS>(t, p, x, y);
    const int px = (int)tx * TS + x, py = (int)ty * TS + y;
    fx[p] = (float)px;
    fy[p] = (float)py;
    R0[p] = sz.bg[0];
    R1[p] = sz.bg[1];
    R2[p] = sz.bg[2];
    if (px < vi.w && py < vi.h) {
      const uint32_t pix = (uint32_t)py * (uint32_t)vi.w + (uint32_t)px;
      T[p] = t_final[vi.pix_off + pix];
      last[p] = last_pos[vi.pix_off + pix];
      const float *gi = dL_dimage + (size_t)3 * vi.pix_off;
      g0[p] = gi[pix];
      g1[p] = gi[hw + pix];
      g2[p] = gi[2 * hw + pix];
    } else {
      T[p] = 1.0f;
      last[p] = 0;
      g0[p] = g1[p] = g2[p] = 0.0f;
    }
    my_max = max(my_max, last[p]);
  }
  my_max = wave_reduce_max(my_max);
  if (lane == 0) s_red[wv] = my_max;
  __syncthreads();
  uint32_t max_last = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) max_last = max(max_last, s_red[w]);

  // slot of this tile's pair in the record-major partials array
  auto pair_slot = [&](uint32_t rec) {
    if (rec >= nrec) {  // corrupt list: flag it, stay in bounds
      ws.scalars[kOverflow] = 4u;
      rec = 0;
    }
    const uint2 rc = ws.rec_rect[rec];
    const uint32_t tx0 = rc.x & 0xFFFFu, tx1 = rc.x >> 16, ty0 = rc.y & 0xFFFFu;
    return ws.rec_pairoff[rec] + (ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0);
  };
  const float4 zero4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  // entries no pixel reaches get zero gradients
  for (uint32_t i = max_last + t; i < n; i += NT) {
    const uint32_t slot = pair_slot(ws.tile_recs[start + i]);
    ws.partials[(size_t)slot * 3 + 0] = zero4;
    ws.partials[(size_t)slot * 3 + 1] = zero4;
    ws.partials[(size_t)slot * 3 + 2] = zero4;
  }

  // batches walk the list backwards; the next (earlier) batch is fetched
  // into registers while the current one is processed
  float4 f0, f1, f2, f3;
  uint32_t fslot = 0;
  auto fetch = [&](uint32_t lo) {
    if ((uint32_t)t < B) {
      uint32_t rec = ws.tile_recs[start + lo + t];
      fslot = pair_slot(rec);
      if (rec >= nrec) rec = 0;
      const float4 *src = ws.rec_payload + (size_t)rec * 4;
      f0 = src[0];
      f1 = src[1];
      f2 = src[2];
      f3 = src[3];
    }
  };
  auto batch_lo = [&](uint32_t hi) { return hi > (uint32_t)B ? hi - B : 0u; };
  if (max_last > 0) {
    const uint32_t lo0 = batch_lo(max_last);
    if ((uint32_t)t < max_last - lo0) fetch(lo0);
  }
  for (uint32_t hi = max_last; hi > 0;) {
    const uint32_t lo = batch_lo(hi);
    const uint32_t m = hi - lo;
    __syncthreads();
    if ((uint32_t)t < m) {
      s_p0[t] = f0;
      s_p1[t] = f1;
      s_p2[t] = f2;
      s_p3[t] = f3;
      s_out[t] = fslot;
    }
    if (lo > 0) {
      const uint32_t lo2 = batch_lo(lo);
      if ((uint32_t)t < lo - lo2) fetch(lo2);
    }
    for (int k = t; k < B * NW * 9; k += NT) s_g[k] = 0.0f;
    __syncthreads();
    for (int jj = (int)m - 1; jj >= 0; --jj) {
      const uint32_t pos = lo + (uint32_t)jj;
      const float4 box = s_p0[jj];
      bool in[PPT];
      bool any_in = false;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        in[p] = pos < last[p] && fx[p] >= box.x && fx[p] <= box.y && fy[p] >= box.z && fy[p] <= box.w;
        any_in |= in[p];
      }
      // q-gradients are accumulated without the ln 2 of d alpha / dq,
      // applied once to the wave sums below
      float a_offx = 0.f, a_offy = 0.f, a_qa = 0.f, a_qb = 0.f, a_qc = 0.f, a_o = 0.f, a_r = 0.f, a_g = 0.f,
            a_b = 0.f;
      bool any = false;
      if (any_in) {
        const float4 q1 = s_p1[jj], q2 = s_p2[jj];
        const float cb = s_p3[jj].x;
        const float two_qa = 2.0f * q1.z, two_qc = 2.0f * q2.x;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          if (in[p]) {
            const float dx = (fx[p] - box.x) - q1.x;
            const float dy = (fy[p] - box.z) - q1.y;
            const float u = fmaf(q1.w, dy, dx);
            const float u2 = u * u, dy2 = dy * dy;
            const float q = fmaf(q1.z, u2, q2.x * dy2);
            const float e = __builtin_amdgcn_exp2f(q);
            const float oe = q2.y * e;
            const float alpha = fminf(kAlphaMax, oe);
            if (alpha >= kAlphaMin) {
              any = true;
              const float ti = T[p] * __builtin_amdgcn_rcpf(1.0f - alpha);
              const float w = alpha * ti;
              a_r = fmaf(g0[p], w, a_r);
              a_g = fmaf(g1[p], w, a_g);
              a_b = fmaf(g2[p], w, a_b);
              const float d0 = q2.z - R0[p], d1 = q2.w - R1[p], d2 = cb - R2[p];
              const float dla = ti * fmaf(g0[p], d0, fmaf(g1[p], d1, g2[p] * d2));
              R0[p] = fmaf(alpha, d0, R0[p]);
              R1[p] = fmaf(alpha, d1, R1[p]);
              R2[p] = fmaf(alpha, d2, R2[p]);
              T[p] = ti;
              if (oe <= kAlphaMax) {
                a_o = fmaf(e, dla, a_o);
                const float dq = dla * alpha;
                const float t1 = dq * (two_qa * u);
                a_qa = fmaf(dq, u2, a_qa);
                a_qc = fmaf(dq, dy2, a_qc);
                a_qb = fmaf(t1, dy, a_qb);
                a_offx -= t1;
                a_offy -= fmaf(t1, q1.w, dq * two_qc * dy);
              }
            }
          }
        }
      }
      if (__ballot(any)) {
        const float r0 = wave_sum_to_lane63(a_offx), r1 = wave_sum_to_lane63(a_offy);
        const float r2 = wave_sum_to_lane63(a_qa), r3 = wave_sum_to_lane63(a_qb);
        const float r4 = wave_sum_to_lane63(a_qc), r5 = wave_sum_to_lane63(a_o);
        const float r6 = wave_sum_to_lane63(a_r), r7 = wave_sum_to_lane63(a_g);
        const float r8 = wave_sum_to_lane63(a_b);
        if (lane == kWave - 1) {
          float *dst = s_g + ((size_t)jj * NW + wv) * 9;
          dst[0] = r0 * kLn2; dst[1] = r1 * kLn2; dst[2] = r2 * kLn2; dst[3] = r3 * kLn2;
          dst[4] = r4 * kLn2; dst[5] = r5; dst[6] = r6; dst[7] = r7; dst[8] = r8;
        }
      }
    }
    __syncthreads();
    for (uint32_t e = t; e < m; e += NT) {
      float s9[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) s9[c] = 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w)
#pragma unroll
        for (int c = 0; c < 9; ++c) s9[c] += s_g[((size_t)e * NW + w) * 9 + c];
      const uint32_t slot = s_out[e];
      ws.partials[(size_t)slot * 3 + 0] = make_float4(s9[0], s9[1], s9[2], s9[3]);
      ws.partials[(size_t)slot * 3 + 1] = make_float4(s9[4], s9[5], s9[6], s9[7]);
      ws.partials[(size_t)slot * 3 + 2] = make_float4(s9[8], 0.0f, 0.0f, 0.0f);
    }
    hi = lo;
  }
}

// Sum each record's per-tile partials (contiguous, record-major) into its
// reduced gradient.  Each wave takes 64 consecutive records: a lane sums a
// record of at most kBig pairs alone; larger footprints are summed by the
// whole wave (lane l takes pairs l, l + 64, ...) and reduced with DPP, so a
// record covering thousands of tiles does not stall its wave.
constexpr uint32_t kBig = 64;

__global__ __launch_bounds__(256) void k_reduce_pairs(Ws ws) {
  if (ws.scalars[kOverflow]) return;
  const uint32_t nrec = ws.scalars[kNumRecords];
  const int lane = lane_id();
  const uint32_t wave_stride = gridDim.x * (blockDim.x / kWave) * kWave;
  for (uint32_t wbase = (blockIdx.x * (blockDim.x / kWave) + wave_id()) * kWave; wbase < nrec;
       wbase += wave_stride) {
    const uint32_t r = wbase + lane;
    uint32_t cnt = 0, p0 = 0;
    if (r < nrec) {
      const uint2 rc = ws.rec_rect[r];
      cnt = ((rc.x >> 16) - (rc.x & 0xFFFFu) + 1) * ((rc.y >> 16) - (rc.y & 0xFFFFu) + 1);
      p0 = ws.rec_pairoff[r];
    }
    if (r < nrec && cnt <= kBig) {
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a;
      for (uint32_t k = 0; k < cnt; ++k) {
        const float4 *src = ws.partials + (size_t)(p0 + k) * 3;
        const float4 x = src[0], y = src[1], z = src[2];
        a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
        b.x += y.x; b.y += y.y; b.z += y.z; b.w += y.w;
        c.x += z.x;
      }
      ws.g2d[(size_t)r * 3 + 0] = a;
      ws.g2d[(size_t)r * 3 + 1] = b;
      ws.g2d[(size_t)r * 3 + 2] = c;
    }
    uint64_t big = __ballot(r < nrec && cnt > kBig);
    while (big) {
      const int l = __ffsll((unsigned long long)big) - 1;
      big &= big - 1;
      const uint32_t bc = __shfl(cnt, l, kWave), bp = __shfl(p0, l, kWave);
      float v[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = 0.0f;
      for (uint32_t k = lane; k < bc; k += kWave) {
        const float4 *src = ws.partials + (size_t)(bp + k) * 3;
        const float4 x = src[0], y = src[1], z = src[2];
        v[0] += x.x; v[1] += x.y; v[2] += x.z; v[3] += x.w;
        v[4] += y.x; v[5] += y.y; v[6] += y.z; v[7] += y.w;
        v[8] += z.x;
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = wave_sum_to_lane63(v[k]);
      if (lane == kWave - 1) {
        const size_t rr = (size_t)(wbase + l) * 3;
        ws.g2d[rr + 0] = make_float4(v[0], v[1], v[2], v[3]);
        ws.g2d[rr + 1] = make_float4(v[4], v[5], v[6], v[7]);
        ws.g2d[rr + 2] = make_float4(v[8], 0.0f, 0.0f, 0.0f);
      }
    }
  }
}

void launch_raster_bwd(const ViewInfo *views, const Ws &ws, const Sizes &sz, const float *t_final,
                       const uint32_t *last_pos, const float *dL_dimage, hipStream_t st) {
  const uint32_t grid = tile_grid(sz.t_tot);
  if (grid > 0) {
    switch (sz.ts) {
      case 8:
        k_raster_bwd<8><<<grid, TileCfg<8>::NT, 0, st>>>(views, ws, sz, t_final, last_pos, dL_dimage);
        break;
      case 32:
        k_raster_bwd<32><<<grid, TileCfg<32>::NT, 0, st>>>(views, ws, sz, t_final, last_pos, dL_dimage);
        break;
      default:
        k_raster_bwd<16><<<grid, TileCfg<16>::NT, 0, st>>>(views, ws, sz, t_final, last_pos, dL_dimage);
        break;
    }
  }
}

void launch_reduce_pairs(const Ws &ws, const Sizes &sz, hipStream_t st) {
  const uint32_t blocks = std::min<uint32_t>((sz.cap_rec + 255) / 256, 4096u);
  k_reduce_pairs<<<std::max(blocks, 1u), 256, 0, st>>>(ws);
}

}  // namespace gsr

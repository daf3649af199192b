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
// Each batch is compacted to the records whose alpha >= 1/255 ellipse
// reaches the tile (the others get zero partials at once).
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

// A pair's nine partial gradients, packed at slot * 9 (36 bytes, so only
// 4-byte aligned).
__device__ __forceinline__ void store_partial(const Ws &ws, uint32_t slot, const float (&v)[9]) {
  float *dst = ws.partials + (size_t)slot * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[k] = v[k];
}

__device__ __forceinline__ void store_zero_partial(const Ws &ws, uint32_t slot) {
  const float z[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  store_partial(ws, slot, z);
}

// Barrier over the threads that share one tile's LDS: the workgroup, or a
// single wave (whose LDS accesses are performed in order).
template <bool WG>
__device__ __forceinline__ void group_sync() {
  if (WG) {
    __syncthreads();
  } else {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
  }
}

template <bool WG>
__device__ __forceinline__ uint32_t group_max(uint32_t x, uint32_t *red) {
  x = wave_reduce_max(x);
  if (!WG) return __builtin_amdgcn_readfirstlane(x);
  if (lane_id() == 0) red[wave_id()] = x;
  __syncthreads();
  uint32_t m = 0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) m = max(m, red[w]);
  return m;
}

// LDS of one tile walk: a batch of B records' payloads, their partials
// slots and the per-wave gradient sums.
template <int B, int NW>
struct BwdLds {
  float4 p0[B], p1[B], p2[B], p3[B];
  uint32_t out[B], pos[B];
  float g[B * NW * 9];
  uint32_t red[4], wc[4];
};

// The adjoint walk over one tile's list by a group of NT threads (a
// workgroup when WG, else one wave), each thread holding PPT pixels given by
// `pix(t, p, x, y)` relative to the tile origin.
template <int TS, int NT, int PPT, bool WG, int B, class Pix>
__device__ __forceinline__ void bwd_walk(const ViewInfo *__restrict__ views, const Ws &ws, const Sizes &sz,
                                         uint32_t tile, int t, BwdLds<B, NT / kWave> &L,
                                         const float *__restrict__ t_final, const uint32_t *__restrict__ last_pos,
                                         const float *__restrict__ dL_dimage, Pix pix) {
  constexpr int NW = NT / kWave;
  const int lane = lane_id(), wv = t / kWave;
  const int v = view_of_tile(views, sz.n_views, tile);
  const ViewInfo vi = views[v];
  const uint32_t lt = tile - vi.tile_base;
  const uint32_t tx = lt % (uint32_t)vi.tiles_x, ty = lt / (uint32_t)vi.tiles_x;
  const uint32_t start = ws.tile_start[tile], n = ws.tile_count[tile];
  const uint32_t nrec = ws.scalars[kNumRecords];
  const float ox = (float)(tx * TS), oy = (float)(ty * TS);
  if (n == 0) return;

  float fx[PPT], fy[PPT], T[PPT], g0[PPT], g1[PPT], g2[PPT], R0[PPT], R1[PPT], R2[PPT];
  uint32_t last[PPT];
  uint32_t my_max = 0;
  const uint32_t hw = (uint32_t)vi.w * (uint32_t)vi.h;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    int x, y;
    pix(t, p, x, y);
    const int px = (int)tx * TS + x, py = (int)ty * TS + y;
    fx[p] = (float)px;
    fy[p] = (float)py;
    R0[p] = sz.bg[0];
    R1[p] = sz.bg[1];
    R2[p] = sz.bg[2];
    if (px < vi.w && py < vi.h) {
      const uint32_t pixi = (uint32_t)py * (uint32_t)vi.w + (uint32_t)px;
      T[p] = t_final[vi.pix_off + pixi];
      last[p] = last_pos[vi.pix_off + pixi];
      const float *gi = dL_dimage + (size_t)3 * vi.pix_off;
      g0[p] = gi[pixi];
      g1[p] = gi[hw + pixi];
      g2[p] = gi[2 * hw + pixi];
    } else {
      T[p] = 1.0f;
      last[p] = 0;
      g0[p] = g1[p] = g2[p] = 0.0f;
    }
    my_max = max(my_max, last[p]);
  }
  const uint32_t max_last = group_max<WG>(my_max, L.red);

  // slot of this tile's pair in the record-major partials array
  auto pair_slot = [&](uint32_t rec) {
    if (rec >= nrec) {  // corrupt list: flag it, stay in bounds
      ws.scalars[kOverflow] = 4u;
      rec = 0;
    }
    const uint4 rc = ws.rec_rect[rec];
    const uint32_t tx0 = rc.x & 0xFFFFu, tx1 = rc.x >> 16, ty0 = rc.y & 0xFFFFu, ty1 = rc.y >> 16;
    if (tx < tx0 || tx > tx1 || ty < ty0 || ty > ty1) {  // not this record's tile: corrupt list
      ws.scalars[kOverflow] = 4u;
      return ws.rec_pairoff[rec];
    }
    return ws.rec_pairoff[rec] + (ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0);
  };
  // entries no pixel reaches get zero gradients
  for (uint32_t i = max_last + t; i < n; i += NT) store_zero_partial(ws, pair_slot(ws.tile_recs[start + i]));

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
  auto batch_lo = [](uint32_t hi) { return hi > (uint32_t)B ? hi - B : 0u; };
  if (max_last > 0) {
    const uint32_t lo0 = batch_lo(max_last);
    if ((uint32_t)t < max_last - lo0) fetch(lo0);
  }
  for (uint32_t hi = max_last; hi > 0;) {
    const uint32_t lo = batch_lo(hi);
    const uint32_t m = hi - lo;
    group_sync<WG>();
    // compact the batch to the records that can composite in this tile; the
    // others get zero gradients here
    const bool keep = (uint32_t)t < m && tile_reaches(f0, f1, f2, ox, oy, (float)TS);
    uint32_t mc;
    const uint32_t cs = compact_slot<WG, NW>(keep, L.wc, mc);
    if (keep) {
      L.p0[cs] = f0;
      L.p1[cs] = f1;
      L.p2[cs] = f2;
      L.p3[cs] = f3;
      L.out[cs] = fslot;
      L.pos[cs] = lo + (uint32_t)t;
    } else if ((uint32_t)t < m) {
      store_zero_partial(ws, fslot);
    }
    if (lo > 0) {
      const uint32_t lo2 = batch_lo(lo);
      if ((uint32_t)t < lo - lo2) fetch(lo2);
    }
    for (uint32_t k = t; k < mc * NW * 9; k += NT) L.g[k] = 0.0f;
    group_sync<WG>();
    // records by 8 x 8 pixel block (wave-uniform bit masks), walked back to
    // front: a wave visits only the records that can composite in one of its
    // blocks, and there only the pixels in front of their stored end
    constexpr int NC = (B + kWave - 1) / kWave;
    uint64_t mk[PPT][NC];
    block_masks<PPT, NC, false>(L.p0, L.p1, L.p2, mc, t, ox, oy, pix, mk);
#pragma unroll
    for (int c = NC - 1; c >= 0; --c) {
      uint64_t rem = 0;
#pragma unroll
      for (int p = 0; p < PPT; ++p) rem |= mk[p][c];
      while (rem) {
        const int jb = 63 - __builtin_clzll(rem);
        rem &= ~(uint64_t(1) << jb);
        const int jj = c * kWave + jb;
        const uint32_t pos = L.pos[jj];
        const float4 box = L.p0[jj];
        // per 8 x 8 block: skipped (wave-uniform) unless one of its pixels
        // is in front of its stored end and reaches alpha >= 1/255; then
        // branch-free: lanes that do not composite take alpha = 0, which
        // leaves T (rcp(1) = 1), the suffix colours and every sum unchanged
        // bit for bit.  With dq = dL/dalpha alpha (dL/dq without the ln 2 of
        // d alpha / dq) each pixel adds dq u, dq dy, dq u^2, dq u dy and
        // dq dy^2; the record's constants qa, qb, qc and ln 2 turn the sums
        // into the payload gradients once, in the epilogue.  The empty asm
        // keeps the zeros opaque, so the compiler does not re-materialise
        // them on every path.
        float a_u = 0.f, a_dy = 0.f, a_qa = 0.f, a_udy = 0.f, a_qc = 0.f, a_o = 0.f, a_r = 0.f, a_g = 0.f,
              a_b = 0.f;
        asm volatile("" : "+v"(a_u), "+v"(a_dy), "+v"(a_qa), "+v"(a_udy), "+v"(a_qc), "+v"(a_o), "+v"(a_r),
                     "+v"(a_g), "+v"(a_b));
        bool any = false;
        const float4 q1 = L.p1[jj], q2 = L.p2[jj];
        const float cb = L.p3[jj].x;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          if (!((mk[p][c] >> jb) & 1u)) continue;  // uniform
          const bool in = pos < last[p];
          if (__ballot(in) == 0) continue;  // uniform
          const float dx = (fx[p] - box.x) - q1.x;
          const float dy = (fy[p] - box.z) - q1.y;
          const float u = fmaf(q1.w, dy, dx);
          const float u2 = u * u, dy2 = dy * dy;
          const float q = fmaf(q1.z, u2, q2.x * dy2);
          const float e = __builtin_amdgcn_exp2f(q);
          const float oe = q2.y * e;
          const float alpha = fminf(kAlphaMax, oe);
          const bool comp = in & (alpha >= kAlphaMin);
          if (__ballot(comp) == 0) continue;  // uniform
          any = true;
          const float am = comp ? alpha : 0.0f;
          const float ti = T[p] * __builtin_amdgcn_rcpf(1.0f - am);
          const float w = am * ti;
          a_r = fmaf(g0[p], w, a_r);
          a_g = fmaf(g1[p], w, a_g);
          a_b = fmaf(g2[p], w, a_b);
          const float d0 = q2.z - R0[p], d1 = q2.w - R1[p], d2 = cb - R2[p];
          const float dla = ti * fmaf(g0[p], d0, fmaf(g1[p], d1, g2[p] * d2));
          R0[p] = fmaf(am, d0, R0[p]);
          R1[p] = fmaf(am, d1, R1[p]);
          R2[p] = fmaf(am, d2, R2[p]);
          T[p] = ti;
          // below the 0.99 cap alpha = opacity 2^q; at the cap its
          // derivative in opacity and q is zero
          const bool uncapped = comp & (oe <= kAlphaMax);
          const float eg = uncapped ? e : 0.0f;
          const float dq = uncapped ? dla * alpha : 0.0f;
          a_o = fmaf(eg, dla, a_o);
          const float du = dq * u;
          a_u += du;
          a_dy = fmaf(dq, dy, a_dy);
          a_qa = fmaf(dq, u2, a_qa);
          a_udy = fmaf(du, dy, a_udy);
          a_qc = fmaf(dq, dy2, a_qc);
        }
        if (any) {
          const float v9[9] = {a_u, a_dy, a_qa, a_udy, a_qc, a_o, a_r, a_g, a_b};
          const float sum = wave_sum9_packed(v9);  // value l in lane l < 8, value 8 in lane 32
          if (lane < 8 || lane == 32) L.g[((size_t)jj * NW + wv) * 9 + (lane < 8 ? lane : 8)] = sum;
        }
      }
    }
    group_sync<WG>();
    for (uint32_t e = t; e < mc; e += NT) {
      float s9[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) s9[c] = 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w)
#pragma unroll
        for (int c = 0; c < 9; ++c) s9[c] += L.g[((size_t)e * NW + w) * 9 + c];
      // q = qa u^2 + qc dy^2, u = dx + qb dy, dx = ... - offx, dy = ... - offy:
      //   dL/dqb = 2 qa sum(dq u dy),  dL/doffx = -2 qa sum(dq u),
      //   dL/doffy = -(2 qa qb sum(dq u) + 2 qc sum(dq dy))   (times ln 2)
      const uint32_t slot = L.out[e];
      const float qa2 = 2.0f * L.p1[e].z, qb = L.p1[e].w, qc2 = 2.0f * L.p2[e].x;
      const float d_offx = -qa2 * s9[0], d_offy = -fmaf(qa2 * qb, s9[0], qc2 * s9[1]);
      const float v[9] = {d_offx * kLn2, d_offy * kLn2, s9[2] * kLn2, qa2 * s9[3] * kLn2, s9[4] * kLn2,
                          s9[5],          s9[6],          s9[7],          s9[8]};
      store_partial(ws, slot, v);
    }
    hi = lo;
  }
}

// 16 px tiles, persistent (see ItemQueue).  Tiles whose list has at least
// Sizes::long_list entries (a prefix of the longest-first order, autotuned)
// are one work item each, for the whole workgroup: four waves, each an
// 8 x 8 quadrant with one pixel per lane, sharing 128-record LDS batches, so
// a long list is walked four times faster.  The remaining tiles are items of
// four, one wave each (16 x 16 pixels, four per lane), so each record's wave
// reduction is paid once per tile; neighbours in the longest-first order
// have similar lengths, so the four waves finish together.

union BwdLds16 {
  BwdLds<128, 4> quad;
  BwdLds<64, 1> wave[4];
};

// Five waves per SIMD: 96 VGPRs instead of 110 (four waves), with 14 values
// kept in scratch, and measured 8% faster than four waves without spills.
// Six would need more than the CU's 160 KB of LDS.
template <bool P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_raster_bwd16(
    const ViewInfo *__restrict__ views, Ws ws, Sizes sz, const float *__restrict__ t_final,
    const uint32_t *__restrict__ last_pos, const float *__restrict__ dL_dimage) {
  __shared__ BwdLds16 S;
  __shared__ uint32_t take;
  if (ws.scalars[kOverflow]) return;
  uint32_t *queue = ws.queues + kQueueLanes * kQueueStride;
  const uint32_t n_long = ws.scalars[kNumLong];
  const uint32_t n_items = n_long + (sz.t_tot - n_long + 3u) / 4u;
  const int t = threadIdx.x;
  ItemQueue<P> q(queue);
  for (uint32_t it = blockIdx.x; it < n_items; it = q.next(&take)) {
    if (it < n_long) {
      bwd_walk<16, 256, 1, true, 128>(views, ws, sz, ws.tile_order[it], t, S.quad, t_final, last_pos, dL_dimage,
                                      [](int tt, int, int &x, int &y) {
                                        const int l = tt & 63, w = tt >> 6;
                                        x = (w & 1) * 8 + (l & 7);
                                        y = (w >> 1) * 8 + (l >> 3);
                                      });
    } else {
      const uint32_t i = n_long + (it - n_long) * 4u + (uint32_t)wave_id();
      if (i < sz.t_tot)
        bwd_walk<16, 64, 4, false, 64>(views, ws, sz, ws.tile_order[i], lane_id(), S.wave[wave_id()], t_final,
                                       last_pos, dL_dimage, [](int tt, int p, int &x, int &y) {
                                         x = (tt & 7) + (p & 1) * 8;
                                         y = (tt >> 3) + (p >> 1) * 8;
                                       });
    }
  }
}

// 8 and 32 px tiles, persistent: one tile per work item, longest lists
// first (one wave at 8 px with one pixel per lane; four waves
// at 32 px, one 16 x 16 quadrant each).
template <int TS, bool P>
__global__ __launch_bounds__(TileCfg<TS>::NT) __attribute__((amdgpu_waves_per_eu(TS == 32 ? 4 : 6))) void k_raster_bwd(const ViewInfo *__restrict__ views, Ws ws,
                                                                Sizes sz, const float *__restrict__ t_final,
                                                                const uint32_t *__restrict__ last_pos,
                                                                const float *__restrict__ dL_dimage) {
  constexpr int NT = TileCfg<TS>::NT, PPT = TileCfg<TS>::PPT;
  constexpr int B = NT >= 128 ? 128 : NT;
  __shared__ BwdLds<B, NT / kWave> S;
  __shared__ uint32_t take;
  if (ws.scalars[kOverflow]) return;
  ItemQueue<P> q(ws.queues + kQueueLanes * kQueueStride);
  for (uint32_t i = blockIdx.x; i < sz.t_tot; i = q.next(&take))
    bwd_walk<TS, NT, PPT, true, B>(views, ws, sz, ws.tile_order[i], threadIdx.x, S, t_final, last_pos, dL_dimage,
                                   [](int tt, int p, int &x, int &y) { pixel_of<TS>(tt, p, x, y); });
}

// Sum each record's per-tile partials (contiguous, record-major) into its
// reduced gradient.  Each wave takes 64 consecutive records: a lane sums a
// record of at most kBig pairs alone, two pairs per step so their loads
// overlap; larger footprints are summed by the whole wave (lane l takes
// pairs l, l + 64, ...) and reduced across lanes, so one big record does not
// hold its wave for hundreds of dependent loads.
constexpr uint32_t kBig = 16;

__device__ __forceinline__ void add_partial(const float *__restrict__ src, float (&v)[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) v[k] += src[k];
}

// step (optional): the Adam step counter, incremented here (before the
// per-Gaussian kernel that reads it) rather than by a launch of its own.  On
// a capacity overflow nothing is updated (the per-Gaussian kernel skips its
// Adam step too), so the counter stays with the moments.
__global__ __launch_bounds__(256) void k_reduce_pairs(Ws ws, int32_t *step) {
  // the next backward's work queue starts from zero
  if (blockIdx.x == 0 && threadIdx.x < kQueueLanes)
    ws.queues[(kQueueLanes + threadIdx.x) * kQueueStride] = 0u;
  if (ws.scalars[kOverflow]) return;
  if (step && blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
  const uint32_t nrec = ws.scalars[kNumRecords];
  const int lane = lane_id();
  const uint32_t wave_stride = gridDim.x * (blockDim.x / kWave) * kWave;
  for (uint32_t wbase = (blockIdx.x * (blockDim.x / kWave) + wave_id()) * kWave; wbase < nrec;
       wbase += wave_stride) {
    const uint32_t r = wbase + lane;
    uint32_t cnt = 0, p0 = 0;
    if (r < nrec) {
      const uint4 rc = ws.rec_rect[r];
      cnt = ((rc.x >> 16) - (rc.x & 0xFFFFu) + 1) * ((rc.y >> 16) - (rc.y & 0xFFFFu) + 1);
      p0 = ws.rec_pairoff[r];
    }
    if (r < nrec && cnt <= kBig) {
      float a[9], b[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) a[k] = b[k] = 0.0f;
      // even pairs into a, odd ones into b, in order; four pairs' loads are
      // issued before their sums
      uint32_t k = 0;
      for (; k + 3 < cnt; k += 4) {
        const float *src = ws.partials + (size_t)(p0 + k) * 9;
        float x[36];
#pragma unroll
        for (int c = 0; c < 36; ++c) x[c] = src[c];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          a[c] += x[c];
          b[c] += x[9 + c];
          a[c] += x[18 + c];
          b[c] += x[27 + c];
        }
      }
      for (; k + 1 < cnt; k += 2) {
        add_partial(ws.partials + (size_t)(p0 + k) * 9, a);
        add_partial(ws.partials + (size_t)(p0 + k + 1) * 9, b);
      }
      if (k < cnt) add_partial(ws.partials + (size_t)(p0 + k) * 9, a);
#pragma unroll
      for (int c = 0; c < 9; ++c) a[c] += b[c];
      ws.g2d[(size_t)r * 3 + 0] = make_float4(a[0], a[1], a[2], a[3]);
      ws.g2d[(size_t)r * 3 + 1] = make_float4(a[4], a[5], a[6], a[7]);
      ws.g2d[(size_t)r * 3 + 2] = make_float4(a[8], 0.0f, 0.0f, 0.0f);
    }
    uint64_t big = __ballot(r < nrec && cnt > kBig);
    while (big) {
      const int l = __ffsll((unsigned long long)big) - 1;
      big &= big - 1;
      const uint32_t bc = __shfl(cnt, l, kWave), bp = __shfl(p0, l, kWave);
      float v[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = 0.0f;
      for (uint32_t k = lane; k < bc; k += kWave) add_partial(ws.partials + (size_t)(bp + k) * 9, v);
      const float sum = wave_sum9_packed(v);  // value l in lane l < 8, value 8 in lane 32
      float *dst = reinterpret_cast<float *>(ws.g2d + (size_t)(wbase + l) * 3);
      if (lane < 8) dst[lane] = sum;
      if (lane == 32) {
        dst[8] = sum;
        dst[9] = dst[10] = dst[11] = 0.0f;
      }
    }
  }
}

// Grid or persistent schedule, as the forward (launch_items there).
template <bool P, class K, class... A>
static void launch_items(K kernel, uint32_t t_tot, int threads, hipStream_t st, A... args) {
  uint32_t grid = t_tot;
  if (P) {
    static const uint32_t pgrid = persistent_grid(kernel, threads);
    grid = pgrid;
  }
  kernel<<<grid, threads, 0, st>>>(args...);
}

void launch_raster_bwd(const ViewInfo *views, const Ws &ws, const Sizes &sz, const float *t_final,
                       const uint32_t *last_pos, const float *dL_dimage, hipStream_t st) {
  if (sz.t_tot == 0) return;
#define BWD_ARGS views, ws, sz, t_final, last_pos, dL_dimage
  switch ((sz.ts << 1) | (sz.persistent ? 1 : 0)) {
    case 16: launch_items<false>(k_raster_bwd<8, false>, sz.t_tot, TileCfg<8>::NT, st, BWD_ARGS); break;
    case 17: launch_items<true>(k_raster_bwd<8, true>, sz.t_tot, TileCfg<8>::NT, st, BWD_ARGS); break;
    case 64: launch_items<false>(k_raster_bwd<32, false>, sz.t_tot, TileCfg<32>::NT, st, BWD_ARGS); break;
    case 65: launch_items<true>(k_raster_bwd<32, true>, sz.t_tot, TileCfg<32>::NT, st, BWD_ARGS); break;
    case 33: launch_items<true>(k_raster_bwd16<true>, sz.t_tot, 256, st, BWD_ARGS); break;
    default: launch_items<false>(k_raster_bwd16<false>, sz.t_tot, 256, st, BWD_ARGS); break;
  }
#undef BWD_ARGS
}

void launch_reduce_pairs(const Ws &ws, const Sizes &sz, int32_t *step, hipStream_t st) {
  const uint32_t blocks = std::min<uint32_t>((sz.cap_rec + 255) / 256, 4096u);
  k_reduce_pairs<<<std::max(blocks, 1u), 256, 0, st>>>(ws, step);
}

}  // namespace gsr

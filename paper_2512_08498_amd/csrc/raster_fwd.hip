// Forward compositing: front-to-back alpha blending of each tile's sorted
// list, with per-pixel early termination once transmittance would fall
// below 1e-4 and a workgroup-level exit once every pixel has stopped.
//
// Records are staged in LDS in batches (one per thread, four float4 each,
// stored as four arrays so all lanes read the same address: LDS broadcast).
// Each wave then walks only the records whose box meets one of its 8 x 8
// pixel blocks (bit masks in scalar registers), and there every pixel not
// yet stopped evaluates alpha: outside the box alpha < 1/255, so the
// per-pixel alpha test alone decides which entries composite.
// Per pixel the kernel keeps T, the colour and the position one past the
// last composited entry, which the backward pass starts from.  With a
// target image the L1 loss is fused into the epilogue: dL/dimage per pixel
// and |image - target| summed per tile (a fixed butterfly per wave, then the
// waves in order), one partial per tile, added up in tile order by k_l1_sum.
// Both compositing passes are persistent launches that take tiles from a
// work queue (ItemQueue in raster.hpp).
#include "kernels.hpp"
#include "raster.hpp"
#include "util.hpp"

namespace gsr {

// Barrier over the threads that share one tile's LDS: the workgroup, or a
// single wave (whose LDS accesses are performed in order).
template <bool WG>
__device__ __forceinline__ void fwd_sync() {
  if (WG) {
    __syncthreads();
  } else {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
  }
}

template <bool WG>
__device__ __forceinline__ bool group_any(bool x) {
  if (WG) return __syncthreads_or(x ? 1 : 0) != 0;
  fwd_sync<false>();
  return __ballot(x) != 0;
}

template <int B>
struct FwdLds {
  float4 p0[B], p1[B], p2[B], p3[B];
};

// Front-to-back walk over one tile's list by a group of NT threads (a
// workgroup when WG, else one wave), each thread holding PPT pixels given by
// `pix(t, p, x, y)` relative to the tile origin; records are staged in LDS
// in batches of B.
template <int TS, int NT, int PPT, bool WG, int B, class Pix>
__device__ __forceinline__ void fwd_walk(const ViewInfo *__restrict__ views, const Ws &ws, const Sizes &sz,
                                         uint32_t tile, int t, FwdLds<B> &L, float *__restrict__ image,
                                         float *__restrict__ t_final, uint32_t *__restrict__ last_pos,
                                         uint32_t *__restrict__ n_contrib, const LossArgs &la, float &acc,
                                         Pix pix) {
  const int v = view_of_tile(views, sz.n_views, tile);
  const ViewInfo vi = views[v];
  const uint32_t lt = tile - vi.tile_base;
  const int tx = (int)(lt % (uint32_t)vi.tiles_x), ty = (int)(lt / (uint32_t)vi.tiles_x);
  const uint32_t start = ws.tile_start[tile], n = ws.tile_count[tile];
  const uint32_t nrec = ws.scalars[kNumRecords];

  int px[PPT], py[PPT];
  float fx[PPT], fy[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
  // live[p]: 1 while pixel p composites (a 32-bit word rather than a bool,
  // so testing it is one compare instead of lane-mask bookkeeping)
  uint32_t last[PPT], cnt[PPT], live[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    int x, y;
    pix(t, p, x, y);
    px[p] = tx * TS + x;
    py[p] = ty * TS + y;
    fx[p] = (float)px[p];
    fy[p] = (float)py[p];
    live[p] = (px[p] < vi.w && py[p] < vi.h) ? 1u : 0u;
    T[p] = 1.0f;
    C0[p] = C1[p] = C2[p] = 0.0f;
    last[p] = 0;
    cnt[p] = 0;
  }

  for (uint32_t b0 = 0; b0 < n; b0 += B) {
    uint32_t alive = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) alive |= live[p];
    if (!group_any<WG>(alive != 0u)) break;
    const uint32_t m = min((uint32_t)B, n - b0);
    if ((uint32_t)t < m) {
      uint32_t rec = ws.tile_recs[start + b0 + t];
      if (rec >= nrec) {  // corrupt list: flag it, stay in bounds
        ws.scalars[kOverflow] = 4u;
        rec = 0;
      }
      const float4 *src = ws.rec_payload + (size_t)rec * 4;
      L.p0[t] = src[0];
      L.p1[t] = src[1];
      L.p2[t] = src[2];
      L.p3[t] = src[3];
    }
    fwd_sync<WG>();
    // records by 8 x 8 pixel block (wave-uniform bit masks): a wave visits
    // only the records that can composite in one of its blocks
    constexpr int NC = (B + kWave - 1) / kWave;
    uint64_t mk[PPT][NC];
    block_masks<PPT, NC, true>(L.p0, L.p1, L.p2, m, t, (float)(tx * TS), (float)(ty * TS), pix, mk);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      uint64_t any = 0;
#pragma unroll
      for (int p = 0; p < PPT; ++p) any |= mk[p][c];
      while (any) {
        const uint32_t jj = (uint32_t)__builtin_ctzll(any);
        any &= any - 1;
        const uint32_t j = (uint32_t)c * kWave + jj;
        const float4 box = L.p0[j], q1 = L.p1[j], q2 = L.p2[j];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          // per 8 x 8 block: skipped (wave-uniform) unless one of its
          // pixels is still compositing and reaches alpha >= 1/255; then
          // branch-free, lanes that do not composite leaving their state
          // as it is
          if (!((mk[p][c] >> jj) & 1u)) continue;
          if (__ballot(live[p] != 0u) == 0) continue;
          const float dx = (fx[p] - box.x) - q1.x;
          const float dy = (fy[p] - box.z) - q1.y;
          const float u = fmaf(q1.w, dy, dx);
          const float q = fmaf(q1.z, u * u, q2.x * (dy * dy));
          const float alpha = fminf(kAlphaMax, q2.y * __builtin_amdgcn_exp2f(q));
          const bool hit = (live[p] != 0u) & (alpha >= kAlphaMin);
          if (__ballot(hit) == 0) continue;
          // stop before the entry that would take T below 1e-4
          const float tn = T[p] * (1.0f - alpha);
          const bool stop = hit & (tn < kTMin);
          const bool comp = hit & !stop;
          live[p] = stop ? 0u : live[p];
          const float w = comp ? alpha * T[p] : 0.0f;
          const float b = L.p3[j].x;
          C0[p] = fmaf(w, q2.z, C0[p]);
          C1[p] = fmaf(w, q2.w, C1[p]);
          C2[p] = fmaf(w, b, C2[p]);
          T[p] = comp ? tn : T[p];
          last[p] = comp ? b0 + j + 1 : last[p];
          cnt[p] += comp ? 1u : 0u;
        }
      }
    }
  }

#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    if (px[p] < vi.w && py[p] < vi.h) {
      const uint32_t hw = (uint32_t)vi.w * (uint32_t)vi.h;
      const uint32_t pixi = (uint32_t)py[p] * (uint32_t)vi.w + (uint32_t)px[p];
      float *img = image + (size_t)3 * vi.pix_off;
      const float c0 = C0[p] + T[p] * sz.bg[0], c1 = C1[p] + T[p] * sz.bg[1], c2 = C2[p] + T[p] * sz.bg[2];
      img[pixi] = c0;
      img[hw + pixi] = c1;
      img[2 * hw + pixi] = c2;
      if (la.target) {
        const float *tg = la.target + (size_t)3 * vi.pix_off;
        float *dl = la.dl + (size_t)3 * vi.pix_off;
        const float d0 = c0 - tg[pixi], d1 = c1 - tg[hw + pixi], d2 = c2 - tg[2 * hw + pixi];
        auto sgn = [&](float d) { return d > 0.0f ? la.inv_n : (d < 0.0f ? -la.inv_n : 0.0f); };
        dl[pixi] = sgn(d0);
        dl[hw + pixi] = sgn(d1);
        dl[2 * hw + pixi] = sgn(d2);
        acc += (fabsf(d0) + fabsf(d1)) + fabsf(d2);
      }
      t_final[vi.pix_off + pixi] = T[p];
      last_pos[vi.pix_off + pixi] = last[p];
      n_contrib[vi.pix_off + pixi] = cnt[p];
    }
  }
}

// The fused loss keeps one partial per tile (its item in the longest-first
// order), so its fixed-order sum does not depend on which workgroup took
// which tile.  A workgroup's tile: a butterfly per wave, then the waves in
// order (every thread takes part); a wave's tile: its butterfly alone.
template <int NW>
__device__ __forceinline__ void tile_loss_group(const LossArgs &la, float acc, float *red, uint32_t item) {
  if (!la.target) return;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (lane_id() == 0) red[wave_id()] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += red[w];
    la.part[item] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ void tile_loss_wave(const LossArgs &la, float acc, uint32_t item) {
  if (!la.target) return;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (lane_id() == 0) la.part[item] = acc;
}

// 16 px tiles, persistent: lists of at least long_list entries (a prefix
// of the longest-first order) are one work item each, shared by the four
// waves of the workgroup, one 8 x 8 quadrant each with one pixel per lane;
// the other tiles are items of four, one per wave (16 x 16 pixels, four per
// lane), so each record is tested once per tile rather than once per
// quadrant, and neighbours in the longest-first order (of similar length)
// finish together.
union FwdLds16 {
  FwdLds<256> quad;
  FwdLds<64> wave[4];
};

template <bool P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_raster_fwd16(
    const ViewInfo *__restrict__ views, Ws ws, Sizes sz, float *__restrict__ image, float *__restrict__ t_final,
    uint32_t *__restrict__ last_pos, uint32_t *__restrict__ n_contrib, LossArgs la) {
  __shared__ FwdLds16 S;
  __shared__ float red[4];
  __shared__ uint32_t take;
  if (ws.scalars[kOverflow]) return;
  uint32_t *queue = ws.queues;
  // items: the n_long long tiles one by one, then the others four at a time
  const uint32_t n_long = ws.scalars[kNumLong];
  const uint32_t n_items = n_long + (sz.t_tot - n_long + 3u) / 4u;
  const int t = threadIdx.x;
  ItemQueue<P> q(queue);
  for (uint32_t it = blockIdx.x; it < n_items; it = q.next(&take)) {
    if (it < n_long) {
      float acc = 0.0f;
      fwd_walk<16, 256, 1, true, 256>(views, ws, sz, ws.tile_order[it], t, S.quad, image, t_final, last_pos,
                                      n_contrib, la, acc, [](int tt, int, int &x, int &y) {
                                        const int l = tt & 63, w = tt >> 6;
                                        x = (w & 1) * 8 + (l & 7);
                                        y = (w >> 1) * 8 + (l >> 3);
                                      });
      tile_loss_group<4>(la, acc, red, it);
    } else {
      const uint32_t i = n_long + (it - n_long) * 4u + (uint32_t)wave_id();
      if (i < sz.t_tot) {
        float acc = 0.0f;
        fwd_walk<16, 64, 4, false, 64>(views, ws, sz, ws.tile_order[i], lane_id(), S.wave[wave_id()], image,
                                       t_final, last_pos, n_contrib, la, acc, [](int tt, int p, int &x, int &y) {
                                         x = (tt & 7) + (p & 1) * 8;
                                         y = (tt >> 3) + (p >> 1) * 8;
                                       });
        tile_loss_wave(la, acc, i);
      }
    }
  }
}

// 8 and 32 px tiles, persistent: a workgroup (FwdTile) takes one tile at a
// time, longest lists first.
template <int TS, bool P>
__global__ __launch_bounds__(FwdTile<TS>::NT) __attribute__((amdgpu_waves_per_eu(TS == 8 ? 8 : 6))) void k_raster_fwd(
    const ViewInfo *__restrict__ views, Ws ws, Sizes sz, float *__restrict__ image, float *__restrict__ t_final,
    uint32_t *__restrict__ last_pos, uint32_t *__restrict__ n_contrib, LossArgs la) {
  constexpr int NT = FwdTile<TS>::NT, PPT = FwdTile<TS>::PPT;
  __shared__ FwdLds<NT> S;
  __shared__ float red[NT / 64];
  __shared__ uint32_t take;
  if (ws.scalars[kOverflow]) return;
  ItemQueue<P> q(ws.queues);
  for (uint32_t i = blockIdx.x; i < sz.t_tot; i = q.next(&take)) {
    float acc = 0.0f;
    fwd_walk<TS, NT, PPT, true, NT>(views, ws, sz, ws.tile_order[i], threadIdx.x, S, image, t_final, last_pos,
                                    n_contrib, la, acc,
                                    [](int tt, int p, int &x, int &y) { fwd_pixel<TS>(tt, p, x, y); });
    tile_loss_group<NT / 64>(la, acc, red, i);
  }
}

// Loss partials of the forward: one per tile.
uint32_t raster_fwd_grid(const Sizes &sz) { return sz.t_tot; }

// Grid schedule: one workgroup per item, at most t_tot (at 16 px one per
// long tile, then one per four tiles; the count of long tiles is known on
// the device only).  Persistent: the device's resident workgroups.
template <bool P, class K, class... A>
static void launch_items(K kernel, uint32_t t_tot, int threads, hipStream_t st, A... args) {
  uint32_t grid = t_tot;
  if (P) {
    static const uint32_t pgrid = persistent_grid(kernel, threads);
    grid = pgrid;
  }
  kernel<<<grid, threads, 0, st>>>(args...);
}

void launch_raster_fwd(const ViewInfo *views, const Ws &ws, const Sizes &sz, float *image, float *t_final,
                       uint32_t *last_pos, uint32_t *n_contrib, const LossArgs &la, hipStream_t st) {
  if (sz.t_tot == 0) return;
#define FWD_ARGS views, ws, sz, image, t_final, last_pos, n_contrib, la
  switch ((sz.ts << 1) | (sz.persistent ? 1 : 0)) {
    case 16: launch_items<false>(k_raster_fwd<8, false>, sz.t_tot, FwdTile<8>::NT, st, FWD_ARGS); break;
    case 17: launch_items<true>(k_raster_fwd<8, true>, sz.t_tot, FwdTile<8>::NT, st, FWD_ARGS); break;
    case 64: launch_items<false>(k_raster_fwd<32, false>, sz.t_tot, FwdTile<32>::NT, st, FWD_ARGS); break;
    case 65: launch_items<true>(k_raster_fwd<32, true>, sz.t_tot, FwdTile<32>::NT, st, FWD_ARGS); break;
    case 33: launch_items<true>(k_raster_fwd16<true>, sz.t_tot, 256, st, FWD_ARGS); break;
    default: launch_items<false>(k_raster_fwd16<false>, sz.t_tot, 256, st, FWD_ARGS); break;
  }
#undef FWD_ARGS
}

}  // namespace gsr

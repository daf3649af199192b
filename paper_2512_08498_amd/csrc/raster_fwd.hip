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
// and |image - target| summed per workgroup (a fixed butterfly per wave, then
// the waves in order), one partial per workgroup, added up in order by
// k_l1_sum.
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
    block_masks<PPT, NC>(L.p0, m, t, (float)(tx * TS), (float)(ty * TS), pix, mk);
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

// Sum of the loss accumulators of a workgroup of NW waves into its partial
// slot: a butterfly per wave, then the waves in order (every thread of the
// workgroup must take part).
template <int NW>
__device__ __forceinline__ void loss_partial(const LossArgs &la, float acc, float *red) {
  if (!la.target) return;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (lane_id() == 0) red[wave_id()] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += red[w];
    la.part[blockIdx.x] = s;
  }
}

// 16 px tiles: lists of at least long_list entries (a prefix of the
// longest-first order) are shared by four waves, one 8 x 8 quadrant each
// with one pixel per lane; the other tiles take one wave each (16 x 16
// pixels, four per lane), four tiles per workgroup, so each record is tested
// once per tile rather than once per quadrant.
union FwdLds16 {
  FwdLds<256> quad;
  FwdLds<64> wave[4];
};

__global__ __launch_bounds__(256) void k_raster_fwd16(const ViewInfo *__restrict__ views, Ws ws, Sizes sz,
                                                      float *__restrict__ image, float *__restrict__ t_final,
                                                      uint32_t *__restrict__ last_pos,
                                                      uint32_t *__restrict__ n_contrib, LossArgs la) {
  __shared__ FwdLds16 S;
  __shared__ float red[4];
  if (ws.scalars[kOverflow]) return;
  const uint32_t n_long = ws.scalars[kNumLong];
  const int t = threadIdx.x;
  float acc = 0.0f;
  if (blockIdx.x < n_long) {
    fwd_walk<16, 256, 1, true, 256>(views, ws, sz, ws.tile_order[blockIdx.x], t, S.quad, image, t_final, last_pos,
                                    n_contrib, la, acc, [](int tt, int, int &x, int &y) {
                                      const int l = tt & 63, w = tt >> 6;
                                      x = (w & 1) * 8 + (l & 7);
                                      y = (w >> 1) * 8 + (l >> 3);
                                    });
  } else {
    const uint32_t i = n_long + (blockIdx.x - n_long) * 4u + (uint32_t)wave_id();
    if (i < sz.t_tot)
      fwd_walk<16, 64, 4, false, 64>(views, ws, sz, ws.tile_order[i], lane_id(), S.wave[wave_id()], image, t_final,
                                     last_pos, n_contrib, la, acc, [](int tt, int p, int &x, int &y) {
                                       x = (tt & 7) + (p & 1) * 8;
                                       y = (tt >> 3) + (p >> 1) * 8;
                                     });
  }
  loss_partial<4>(la, acc, red);
}

// 8 and 32 px tiles: one workgroup per tile (FwdTile), longest lists first.
template <int TS>
__global__ __launch_bounds__(FwdTile<TS>::NT) void k_raster_fwd(const ViewInfo *__restrict__ views, Ws ws,
                                                                Sizes sz, float *__restrict__ image,
                                                                float *__restrict__ t_final,
                                                                uint32_t *__restrict__ last_pos,
                                                                uint32_t *__restrict__ n_contrib, LossArgs la) {
  constexpr int NT = FwdTile<TS>::NT, PPT = FwdTile<TS>::PPT;
  __shared__ FwdLds<NT> S;
  __shared__ float red[NT / 64];
  if (ws.scalars[kOverflow]) return;
  float acc = 0.0f;
  if (blockIdx.x < sz.t_tot)
    fwd_walk<TS, NT, PPT, true, NT>(views, ws, sz, ws.tile_order[blockIdx.x], threadIdx.x, S, image, t_final,
                                    last_pos, n_contrib, la, acc,
                                    [](int tt, int p, int &x, int &y) { fwd_pixel<TS>(tt, p, x, y); });
  loss_partial<NT / 64>(la, acc, red);
}

// Workgroups of the forward launch (the fused loss has one partial per workgroup).
uint32_t raster_fwd_grid(const Sizes &sz) { return sz.ts == 16 ? sz.t_tot : tile_grid(sz.t_tot); }

void launch_raster_fwd(const ViewInfo *views, const Ws &ws, const Sizes &sz, float *image, float *t_final,
                       uint32_t *last_pos, uint32_t *n_contrib, const LossArgs &la, hipStream_t st) {
  const uint32_t grid = raster_fwd_grid(sz);
  if (grid == 0) return;
  switch (sz.ts) {
    case 8:
      k_raster_fwd<8><<<grid, FwdTile<8>::NT, 0, st>>>(views, ws, sz, image, t_final, last_pos, n_contrib, la);
      break;
    case 32:
      k_raster_fwd<32><<<grid, FwdTile<32>::NT, 0, st>>>(views, ws, sz, image, t_final, last_pos, n_contrib, la);
      break;
    default:
      // at most t_tot workgroups: one per long tile, then one per four tiles
      k_raster_fwd16<<<grid, 256, 0, st>>>(views, ws, sz, image, t_final, last_pos, n_contrib, la);
      break;
  }
}

}  // namespace gsr

// Forward compositing: front-to-back alpha blending of each tile's sorted
// list, with per-pixel early termination once transmittance would fall
// below 1e-4 and a workgroup-level exit once every pixel has stopped.
//
// Records are staged in LDS in batches of NT (one per thread, four float4
// each, stored as four arrays so all lanes read the same address: LDS
// broadcast).  Per pixel the kernel keeps T, the colour and the position one
// past the last composited entry, which the backward pass starts from.
#include "kernels.hpp"
#include "raster.hpp"
#include "util.hpp"

namespace gsr {

template <int TS>
__global__ __launch_bounds__(FwdTile<TS>::NT) void k_raster_fwd(const ViewInfo *__restrict__ views, Ws ws,
                                                                Sizes sz, float *__restrict__ image,
                                                                float *__restrict__ t_final,
                                                                uint32_t *__restrict__ last_pos,
                                                                uint32_t *__restrict__ n_contrib) {
  constexpr int NT = FwdTile<TS>::NT, PPT = FwdTile<TS>::PPT, B = NT;
  __shared__ float4 s_p0[B], s_p1[B], s_p2[B], s_p3[B];
  if (ws.scalars[kOverflow]) return;
  if (blockIdx.x >= sz.t_tot) return;
  const uint32_t tile = ws.tile_order[blockIdx.x];
  const int t = threadIdx.x;
  const int v = view_of_tile(views, sz.n_views, tile);
  const ViewInfo vi = views[v];
  const uint32_t lt = tile - vi.tile_base;
  const int tx = (int)(lt % (uint32_t)vi.tiles_x), ty = (int)(lt / (uint32_t)vi.tiles_x);
  const uint32_t start = ws.tile_start[tile], n = ws.tile_count[tile];
  const uint32_t nrec = ws.scalars[kNumRecords];

  int px[PPT], py[PPT];
  float fx[PPT], fy[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
  uint32_t last[PPT], cnt[PPT];
  bool done[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    int x, y;
    fwd_pixel<TS>(t, p, x, y);
    px[p] = tx * TS + x;
    py[p] = ty * TS + y;
    fx[p] = (float)px[p];
    fy[p] = (float)py[p];
    done[p] = !(px[p] < vi.w && py[p] < vi.h);
    T[p] = 1.0f;
    C0[p] = C1[p] = C2[p] = 0.0f;
    last[p] = 0;
    cnt[p] = 0;
  }

  for (uint32_t b0 = 0; b0 < n; b0 += B) {
    int alive = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) alive |= done[p] ? 0 : 1;
    if (!__syncthreads_or(alive)) break;
    const uint32_t m = min((uint32_t)B, n - b0);
    if ((uint32_t)t < m) {
      uint32_t rec = ws.tile_recs[start + b0 + t];
      if (rec >= nrec) {  // corrupt list: flag it, stay in bounds
        ws.scalars[kOverflow] = 4u;
        rec = 0;
      }
      const float4 *src = ws.rec_payload + (size_t)rec * 4;
      s_p0[t] = src[0];
      s_p1[t] = src[1];
      s_p2[t] = src[2];
      s_p3[t] = src[3];
    }
    __syncthreads();
    for (uint32_t j = 0; j < m; ++j) {
      const float4 box = s_p0[j];
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        const bool in = !done[p] && fx[p] >= box.x && fx[p] <= box.y && fy[p] >= box.z && fy[p] <= box.w;
        if (in) {
          const float4 q1 = s_p1[j], q2 = s_p2[j];
          const float dx = (fx[p] - box.x) - q1.x;
          const float dy = (fy[p] - box.z) - q1.y;
          const float u = fmaf(q1.w, dy, dx);
          const float q = fmaf(q1.z, u * u, q2.x * (dy * dy));
          const float alpha = fminf(kAlphaMax, q2.y * __builtin_amdgcn_exp2f(q));
          if (alpha >= kAlphaMin) {
            const float tn = T[p] * (1.0f - alpha);
            if (tn < kTMin) {
              done[p] = true;
            } else {
              const float w = alpha * T[p];
              const float b = s_p3[j].x;
              C0[p] = fmaf(w, q2.z, C0[p]);
              C1[p] = fmaf(w, q2.w, C1[p]);
              C2[p] = fmaf(w, b, C2[p]);
              T[p] = tn;
              last[p] = b0 + j + 1;
              cnt[p] += 1;
            }
          }
        }
      }
    }
  }

#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    if (px[p] < vi.w && py[p] < vi.h) {
      const uint32_t hw = (uint32_t)vi.w * (uint32_t)vi.h;
      const uint32_t pix = (uint32_t)py[p] * (uint32_t)vi.w + (uint32_t)px[p];
      float *img = image + (size_t)3 * vi.pix_off;
      img[pix] = C0[p] + T[p] * sz.bg[0];
      img[hw + pix] = C1[p] + T[p] * sz.bg[1];
      img[2 * hw + pix] = C2[p] + T[p] * sz.bg[2];
      t_final[vi.pix_off + pix] = T[p];
      last_pos[vi.pix_off + pix] = last[p];
      n_contrib[vi.pix_off + pix] = cnt[p];
    }
  }
}

void launch_raster_fwd(const ViewInfo *views, const Ws &ws, const Sizes &sz, float *image, float *t_final,
                       uint32_t *last_pos, uint32_t *n_contrib, hipStream_t st) {
  const uint32_t grid = tile_grid(sz.t_tot);
  if (grid == 0) return;
  switch (sz.ts) {
    case 8:
      k_raster_fwd<8><<<grid, FwdTile<8>::NT, 0, st>>>(views, ws, sz, image, t_final, last_pos, n_contrib);
      break;
    case 32:
      k_raster_fwd<32><<<grid, FwdTile<32>::NT, 0, st>>>(views, ws, sz, image, t_final, last_pos, n_contrib);
      break;
    default:
      k_raster_fwd<16><<<grid, FwdTile<16>::NT, 0, st>>>(views, ws, sz, image, t_final, last_pos, n_contrib);
      break;
  }
}

}  // namespace gsr

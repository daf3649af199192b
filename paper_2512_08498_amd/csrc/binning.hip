// Tile binning: per-tile list lengths from the difference grids, list
// offsets, and emission of the (depth | record) entries into their tiles.
#include <algorithm>

#include "kernels.hpp"
#include "util.hpp"

namespace gsr {

// One workgroup per view: 2D prefix sum of the difference grid gives every
// tile's list length; an exclusive scan in row-major tile order gives the
// list starts relative to the view.  The view total goes to
// view_pair_base[v + 1] until k_view_scan turns the totals into offsets.
__global__ __launch_bounds__(1024) void k_tile_prefix(const ViewInfo *__restrict__ views, Ws ws) {
  __shared__ uint32_t s_scan[16];
  if (ws.scalars[kOverflow]) return;
  const int v = blockIdx.x;
  const ViewInfo vi = views[v];
  int32_t *D = ws.diff + vi.diff_base;
  const int tx = vi.tiles_x, ty = vi.tiles_y, stride = tx + 1;
  for (int r = threadIdx.x; r < ty; r += blockDim.x) {
    int acc = 0;
    for (int c = 0; c < tx; ++c) {
      acc += D[r * stride + c];
      D[r * stride + c] = acc;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < tx; c += blockDim.x) {
    int acc = 0;
    for (int r = 0; r < ty; ++r) {
      acc += D[r * stride + c];
      D[r * stride + c] = acc;
    }
  }
  __syncthreads();
  const uint32_t tv = (uint32_t)tx * (uint32_t)ty;
  const uint32_t per = (tv + blockDim.x - 1) / blockDim.x;
  const uint32_t lo = min(tv, threadIdx.x * per), hi = min(tv, lo + per);
  uint32_t sum = 0;
  for (uint32_t t = lo; t < hi; ++t) sum += (uint32_t)D[(t / tx) * stride + (t % tx)];
  uint32_t total;
  uint32_t run = block_excl_scan<1024>(sum, s_scan, total);
  for (uint32_t t = lo; t < hi; ++t) {
    const uint32_t c = (uint32_t)D[(t / tx) * stride + (t % tx)];
    ws.tile_count[vi.tile_base + t] = c;
    ws.tile_start[vi.tile_base + t] = run;
    run += c;
  }
  if (threadIdx.x == 0) ws.view_pair_base[v + 1] = total;
}

// Per-view totals -> exclusive offsets; cross-checks the pair count.
__global__ void k_view_scan(Ws ws, Sizes sz) {
  if (threadIdx.x != 0 || ws.scalars[kOverflow]) return;
  uint32_t acc = 0;
  ws.view_pair_base[0] = 0;
  for (int v = 0; v < sz.n_views; ++v) {
    acc += ws.view_pair_base[v + 1];
    ws.view_pair_base[v + 1] = acc;
  }
  if (acc != ws.scalars[kNumPairs]) ws.scalars[kOverflow] = 3u;  // inconsistent counts
}

// List starts relative to the view -> absolute.
__global__ void k_tile_abs(const ViewInfo *__restrict__ views, Ws ws, Sizes sz) {
  if (ws.scalars[kOverflow]) return;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= sz.t_tot) return;
  const int v = view_of_tile(views, sz.n_views, t);
  ws.tile_start[t] += ws.view_pair_base[v];
}

// Tiles by decreasing list length (1024 buckets of 4 entries; order within
// a bucket is arbitrary), so the compositing kernels start the longest lists
// first and the short ones fill in behind them.
__global__ __launch_bounds__(1024) void k_tile_order(Ws ws, Sizes sz, uint32_t long_list) {
  constexpr uint32_t NB = 1024;
  __shared__ uint32_t hist[NB];
  __shared__ uint32_t s_scan[16];
  if (ws.scalars[kOverflow]) return;
  const uint32_t t = threadIdx.x;
  hist[t] = 0;
  __syncthreads();
  auto bucket = [&](uint32_t tile) { return NB - 1 - min(ws.tile_count[tile] >> 2, NB - 1); };
  for (uint32_t i = t; i < sz.t_tot; i += blockDim.x) atomicAdd(&hist[bucket(i)], 1u);
  __syncthreads();
  uint32_t total;
  const uint32_t base = block_excl_scan<1024>(hist[t], s_scan, total);
  __syncthreads();
  hist[t] = base;
  __syncthreads();
  for (uint32_t i = t; i < sz.t_tot; i += blockDim.x) ws.tile_order[atomicAdd(&hist[bucket(i)], 1u)] = i;
  // tiles with at least long_list entries come first (when long_list is a
  // multiple of the bucket width, 4); the backward splits them over four waves
  uint32_t nl = 0;
  for (uint32_t i = t; i < sz.t_tot; i += blockDim.x) nl += ws.tile_count[i] >= long_list ? 1u : 0u;
  uint32_t tot_long;
  block_excl_scan<1024>(nl, s_scan, tot_long);
  if (t == 0) ws.scalars[kNumLong] = tot_long;
}

// Each wave expands 64 consecutive records into their (record, tile) pairs:
// lane l takes pair b + l of the wave's concatenated tile rectangles, finds
// its record by a binary search over the wave's prefix sums, and claims a
// slot in the tile's list.  Big footprints are thus spread over the lanes.
__global__ __launch_bounds__(256) void k_emit(const ViewInfo *__restrict__ views, Ws ws, Sizes sz) {
  if (ws.scalars[kOverflow]) return;
  const uint32_t nrec = ws.scalars[kNumRecords];
  const int lane = lane_id();
  const uint32_t wave_stride = gridDim.x * (blockDim.x / kWave) * kWave;
  for (uint32_t wbase = (blockIdx.x * (blockDim.x / kWave) + wave_id()) * kWave; wbase < nrec;
       wbase += wave_stride) {
    const uint32_t r = wbase + lane;
    const bool valid = r < nrec;
    uint32_t tx0 = 0, w = 1, ty0 = 0, cnt = 0, v = 0, zb = 0;
    if (valid) {
      const uint2 rc = ws.rec_rect[r];
      tx0 = rc.x & 0xFFFFu;
      w = (rc.x >> 16) - tx0 + 1;
      ty0 = rc.y & 0xFFFFu;
      cnt = w * ((rc.y >> 16) - ty0 + 1);
      v = ws.rec_view[r];
      zb = ws.rec_zbits[r];
    }
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t excl = incl - cnt;
    const uint32_t total = __shfl(incl, kWave - 1, kWave);
    for (uint32_t b = 0; b < total; b += kWave) {
      const uint32_t p = b + lane;
      int o = 0;
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1) {
        const uint32_t e = __shfl(excl, o + s, kWave);
        if (e <= p) o += s;
      }
      const uint32_t o_tx0 = __shfl(tx0, o, kWave), o_w = __shfl(w, o, kWave);
      const uint32_t o_ty0 = __shfl(ty0, o, kWave), o_v = __shfl(v, o, kWave);
      const uint32_t o_zb = __shfl(zb, o, kWave), o_ex = __shfl(excl, o, kWave);
      if (p < total) {
        const uint32_t k = p - o_ex;
        const uint32_t tx = o_tx0 + k % o_w, ty = o_ty0 + k / o_w;
        const ViewInfo vi = views[o_v];
        const uint32_t tile = vi.tile_base + ty * (uint32_t)vi.tiles_x + tx;
        const uint32_t slot = atomicAdd(ws.tile_cursor + tile, 1u);
        if (slot < ws.tile_count[tile]) {
          ws.pairs[ws.tile_start[tile] + slot] = ((uint64_t)o_zb << 32) | (uint64_t)(wbase + o);
        } else {
          ws.scalars[kOverflow] = 3u;
        }
      }
    }
  }
}

void launch_binning(const ViewInfo *views, const Ws &ws, const Sizes &sz, hipStream_t st) {
  k_tile_prefix<<<sz.n_views, 1024, 0, st>>>(views, ws);
  k_view_scan<<<1, 64, 0, st>>>(ws, sz);
  k_tile_abs<<<(sz.t_tot + 255) / 256, 256, 0, st>>>(views, ws, sz);
  k_tile_order<<<1, 1024, 0, st>>>(ws, sz, sz.long_list);
  const uint32_t waves = (sz.cap_rec + kWave - 1) / kWave;
  const uint32_t blocks = std::min<uint32_t>((waves + 3) / 4, 8192u);
  k_emit<<<std::max(blocks, 1u), 256, 0, st>>>(views, ws, sz);
}

}  // namespace gsr

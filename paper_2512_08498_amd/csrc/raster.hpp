// Tile geometry shared by the forward and backward compositing kernels.
//
// A tile of TS x TS pixels is walked by one workgroup, or at 16 px by one
// wave of it: one workgroup per work item, or (a tuning option) persistent
// workgroups taking items from a work queue.  Records are staged in LDS in
// batches and read back as broadcasts; per 8 x 8 pixel block a wave visits
// only the records whose box (in the forward, whose falloff) can reach it
// (block_masks), so a record that misses a block costs nothing there.  The
// forward and the
// backward split a tile differently (FwdTile / TileCfg below): the forward
// spreads a tile over four waves (one pixel per lane), the backward keeps a
// 16 x 16 block in one wave (four pixels per lane) so the per-record wave
// reduction is paid once per block.  Tiles are visited longest list first.
//
// Per pixel and Gaussian, with the record's payload (see common.hpp):
//   dx = (px - i0) - offx,  dy = (py - j0) - offy
//   u  = dx + qb dy
//   q  = qa u^2 + qc dy^2            (= log2 of the Gaussian falloff)
//   alpha = min(0.99, opacity * 2^q)
// which is the conic quadratic form -(a dx^2 + 2 b dx dy + c dy^2)/2 written
// as a sum of squares, free of the cancellation the expanded form suffers
// for elongated footprints.
//
// The tile lists hold every tile of a record's binning rectangle, but the
// alpha >= 1/255 ellipse of an elongated or tilted footprint misses many of
// them.  The backward therefore compacts each batch in LDS to the records
// that can reach the threshold somewhere in the tile (tile_reaches); the
// others cost one lane's test instead of box tests and failed alpha
// evaluations in every pixel slot.  The test is conservative, so the
// composited sequence of every pixel, and with it every gradient bit, is
// unchanged.  (In the forward the test's registers cost more occupancy than
// the skipped records save.)
#pragma once

#include "common.hpp"
#include "util.hpp"

namespace gsr {

// Whether the record (box, p1, p2 of its payload) can reach alpha >= 1/255 at
// a pixel of the tile whose pixels span [x0, x0 + ts - 1] x [y0, y0 + ts - 1].
// With A = -qa, C = -qc, k = qb the falloff is f = A (dx + k dy)^2 + C dy^2
// (alpha = opacity 2^-f), convex, and a pixel composites only if
// f <= log2(255 opacity).  Its exact minimum over the rectangle tile ∩ box
// (continuous, so it bounds every pixel centre in it) is 0 when the
// rectangle holds the centre, else the least of the four edge minima: at
// fixed dy the minimiser is dx = -k dy, at fixed dx it is
// dy = -A k dx / (A k^2 + C), each clamped to the edge.  The record is
// dropped only if that minimum exceeds the threshold by a margin covering the
// rounding of this evaluation and of the per-pixel one (a relative 2^-18 of
// the largest value f takes on the rectangle, plus 1/16 for the hardware
// exp2 and log2); NaN keeps it.
__device__ __forceinline__ bool tile_reaches(const float4 box, const float4 p1, const float4 p2, float x0, float y0,
                                             float ts) {
  const float X0 = fmaxf(x0, box.x), X1 = fminf(x0 + (ts - 1.0f), box.y);
  const float Y0 = fmaxf(y0, box.z), Y1 = fminf(y0 + (ts - 1.0f), box.w);
  if (X0 > X1 || Y0 > Y1) return false;
  const float dx0 = (X0 - box.x) - p1.x, dx1 = (X1 - box.x) - p1.x;
  const float dy0 = (Y0 - box.z) - p1.y, dy1 = (Y1 - box.z) - p1.y;
  const float A = -p1.z, k = p1.w, C = -p2.x;
  auto f = [&](float dx, float dy) {
    const float u = fmaf(k, dy, dx);
    return fmaf(A, u * u, C * (dy * dy));
  };
  auto clampf = [](float v, float lo, float hi) { return fminf(fmaxf(v, lo), hi); };
  float fmin = 0.0f;
  if (!(dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f)) {
    const float r = (A * k) / fmaf(A * k, k, C);
    const float e0 = f(clampf(-k * dy0, dx0, dx1), dy0), e1 = f(clampf(-k * dy1, dx0, dx1), dy1);
    const float e2 = f(dx0, clampf(-r * dx0, dy0, dy1)), e3 = f(dx1, clampf(-r * dx1, dy0, dy1));
    fmin = fminf(fminf(e0, e1), fminf(e2, e3));
  }
  const float mx = fmaxf(fabsf(dx0), fabsf(dx1)), my = fmaxf(fabsf(dy0), fabsf(dy1));
  const float um = fmaf(fabsf(k), my, mx);
  const float big = fmaf(A, um * um, C * (my * my));
  const float thr = __builtin_amdgcn_logf(p2.y) + 0x1.ffa37cp+2f;  // log2(opacity) + log2(255)
  return !(fmin > thr + (0.0625f + 0x1p-18f * big));
}

// Which staged records each 8 x 8 pixel block of the calling thread's wave
// can composite.  Every pixel mapping of the compositing kernels gives a wave
// one 8 x 8 block per pixel slot p, lane l at (l & 7, l >> 3) within it, so
// the block origin is the pixel of the wave's lane 0.  mk[p][c] bit b: batch
// record 64 c + b (c < NC, 64 c + b < m) may composite in block p.  Outside
// the record's compositing box alpha < 1/255 at every pixel centre (the box
// is the alpha >= 1/255 region's bounding box, with a margin); with ELLIPSE
// the block must also pass the exact test of tile_reaches (the falloff's
// minimum over block ∩ box against the threshold, with its rounding margin),
// which drops the blocks in the corners of a tilted or elongated footprint's
// box.  Both tests are conservative, so a record whose bit is clear
// composites nowhere in the block, and within a block the per-pixel alpha
// test alone decides.  The masks are wave-uniform, so the record loops branch
// on them in scalar registers and skip records without touching LDS.  Every
// thread of the group must call this after the batch's payloads are in LDS.
template <int PPT, int NC, bool ELLIPSE, class Pix>
__device__ __forceinline__ void block_masks(const float4 *p0, const float4 *p1, const float4 *p2, uint32_t m, int t,
                                            float ox, float oy, Pix pix, uint64_t (&mk)[PPT][NC]) {
  float bx[PPT], by[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    int x, y;
    pix(t & ~(kWave - 1), p, x, y);
    bx[p] = ox + (float)x;
    by[p] = oy + (float)y;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const uint32_t j = (uint32_t)(c * kWave + lane_id());
    const bool live = j < m;
    const float4 b = p0[live ? j : 0u];
    if (!ELLIPSE) {
#pragma unroll
      for (int p = 0; p < PPT; ++p)
        mk[p][c] = __ballot(live & (b.x <= bx[p] + 7.0f) & (b.y >= bx[p]) & (b.z <= by[p] + 7.0f) & (b.w >= by[p]));
    } else {
      const float4 q1 = p1[live ? j : 0u], q2 = p2[live ? j : 0u];
#pragma unroll
      for (int p = 0; p < PPT; ++p) mk[p][c] = __ballot(live && tile_reaches(b, q1, q2, bx[p], by[p], 8.0f));
    }
  }
}

// Slot of this thread's record in the compacted batch: the kept records
// numbered in thread order.  A workgroup (WG) exchanges its NW per-wave
// counts through wc with one barrier; a single wave needs none.  Returns the
// slot (meaningful where keep) and the number kept in `total`.  Every thread
// of the group must call it.
template <bool WG, int NW>
__device__ __forceinline__ uint32_t compact_slot(bool keep, uint32_t *wc, uint32_t &total) {
  const uint64_t b = __ballot(keep);
  const uint32_t before = (uint32_t)__popcll(b & lanemask_lt());
  if (!WG) {
    total = (uint32_t)__popcll(b);
    return before;
  }
  if (lane_id() == 0) wc[wave_id()] = (uint32_t)__popcll(b);
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t c = wc[w];
    off += w < wave_id() ? c : 0u;
    tot += c;
  }
  total = tot;
  return off + before;
}

// Forward at 8 and 32 px (and for long lists at 16 px): all waves of the
// workgroup share the tile's LDS batch, each wave an 8 x 8 block with one
// pixel per lane (four pixels per lane, one per 16 x 16 quadrant, at
// TS = 32).  Sharing a tile over four waves shortens the critical path of
// long lists.
template <int TS>
struct FwdTile {
  static constexpr int NT = TS == 8 ? 64 : 256;
  static constexpr int PPT = TS == 32 ? 4 : 1;
};

template <int TS>
__device__ __forceinline__ void fwd_pixel(int t, int p, int &x, int &y) {
  const int l = t & 63, w = t >> 6;
  if (TS == 8) {
    x = l & 7;
    y = l >> 3;
  } else {
    x = (w & 1) * 8 + (l & 7);
    y = (w >> 1) * 8 + (l >> 3);
    if (TS == 32) {
      x += (p & 1) * 16;
      y += (p >> 1) * 16;
    }
  }
}

// Backward: one wave per 16 x 16 block with four pixels per lane, so the
// 9-value wave reduction of each record is paid once per block.
template <int TS>
struct TileCfg {
  static constexpr int NT = TS == 32 ? 256 : 64;
  static constexpr int PPT = TS == 8 ? 1 : 4;
  static constexpr int NW = NT / 64;
};

template <int TS>
__device__ __forceinline__ void pixel_of(int t, int p, int &x, int &y) {
  const int l = t & 63, w = t >> 6;
  x = l & 7;
  y = l >> 3;
  if (TS != 8) {
    x += (p & 1) * 8;
    y += (p >> 1) * 8;
  }
  if (TS == 32) {
    x += (w & 1) * 16;
    y += (w >> 1) * 16;
  }
}

// Persistent compositing launches: as many workgroups as the chip holds at
// once, each walking work items (tiles, or groups of tiles, in the
// longest-first order) until none is left; taking an item never waits for
// another workgroup, so the balance adapts at run time to the actual cost of
// each list.  Item i belongs to lane i % 8 of the queue, and workgroup b
// serves lane b % 8: its first item is b itself, later ones come from that
// lane's counter, one atomic add per item (lane-local index gridDim.x / 8 +
// count).  The grid is a multiple of eight, so every lane has workgroups and
// every item is taken exactly once, however the workgroups are placed.  The
// chip dispatches workgroups to its eight XCDs round-robin, so each counter
// (on a 128-byte line of its own) is used from one XCD: the eight are served
// in parallel, where a single counter for all workgroups serialised the
// atomics and doubled the compositing time.  The add for the next item is
// issued when the current one starts (a wave's memory returns complete in
// order, so it is still waited for at the walk's first load, which overlaps
// most of its latency).  A workgroup stops at its first item past the end;
// the claim it still has in flight then lies past the end too (a lane's
// items grow with its count), so no item is lost.  The counters start at
// zero: the forward's first kernel zeroes both queues, and the pair
// reduction that follows every compositing backward zeroes the backward's
// again.
// Without persistence (P = false) the grid has one workgroup per item and
// next() ends the walk after the first; the kernels are instantiated for
// both, so the grid schedule carries no queue state.
template <bool P>
struct ItemQueue {
  uint32_t *ctr;   // the lane's counter
  uint32_t claim;  // thread 0: lane-local count claimed for the next item

  __device__ __forceinline__ explicit ItemQueue(uint32_t *queue)
      : ctr(queue + (blockIdx.x & (kQueueLanes - 1u)) * kQueueStride), claim(0u) {
    if (P && threadIdx.x == 0) claim = atomicAdd(ctr, 1u);
  }

  // Next item of the calling workgroup (uniform); every thread must call it,
  // after its last access to the LDS of the current item.
  __device__ __forceinline__ uint32_t next(uint32_t *slot) {
    if (!P) return 0xFFFFFFFFu;
    if (threadIdx.x == 0) *slot = claim;
    __syncthreads();
    const uint32_t k = *slot;
    __syncthreads();
    if (threadIdx.x == 0) claim = atomicAdd(ctr, 1u);
    return (gridDim.x / kQueueLanes + k) * kQueueLanes + (blockIdx.x & (kQueueLanes - 1u));
  }
};

// Workgroups of a persistent launch: compute units times the workgroups of
// `kernel` (of `threads` threads) that one holds at once, a multiple of the
// queue's lanes.
template <typename K>
inline uint32_t persistent_grid(K kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1) per = 1;
  const uint32_t g = (uint32_t)(cus * per) / kQueueLanes * kQueueLanes;
  return g < (uint32_t)kQueueLanes ? (uint32_t)kQueueLanes : g;
}

}  // namespace gsr

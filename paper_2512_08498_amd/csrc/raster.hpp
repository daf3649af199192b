// Tile geometry shared by the forward and backward compositing kernels.
//
// A tile of TS x TS pixels is processed by one workgroup.  Records are staged
// in LDS in batches and read back as broadcasts; a record whose pixel box
// misses a lane's pixel costs only the box test (the per-lane test clears
// the exec mask and the body is branched over).  The forward and the
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
#pragma once

#include "common.hpp"

namespace gsr {

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

}  // namespace gsr

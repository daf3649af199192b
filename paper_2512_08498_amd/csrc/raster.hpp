// Tile geometry shared by the forward and backward compositing kernels.
//
// A tile of TS x TS pixels is processed by one workgroup of NW waves.  Each
// wave owns a 16 x 16 block (an 8 x 8 block for TS = 8) and each lane holds
// PPT pixels, one in each 8 x 8 quadrant of the block (lane l -> (l & 7,
// l >> 3) within the quadrant).  A record is read from LDS once per wave and
// tested against each quadrant; a quadrant its pixel box misses costs only
// the test, since the per-lane test clears the exec mask and the body is
// branched over.  Per-entry costs that are paid per wave (LDS reads, loop
// control, and in the backward the 9-value wave reduction) are thus shared by
// up to 256 pixels.
//   TS = 8  :  64 threads, 1 pixel per lane
//   TS = 16 :  64 threads, 4 pixels per lane
//   TS = 32 : 256 threads, 4 pixels per lane (one wave per 16 x 16 quadrant)
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

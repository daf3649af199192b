// Tile geometry shared by the forward and backward compositing kernels.
//
// A tile of TS x TS pixels is processed by one workgroup.  Each wave owns
// 8 x 8 pixel blocks (lane l -> (l & 7, l >> 3)), so a Gaussian whose pixel
// box misses a wave's block costs that wave only the box test: the per-lane
// test clears the whole exec mask and the body is branched over.
//   TS = 8  :  64 threads, 1 pixel per thread
//   TS = 16 : 256 threads, 1 pixel per thread (waves = quadrants)
//   TS = 32 : 256 threads, 4 pixels per thread (one per 16 x 16 quadrant)
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
  static constexpr int NT = TS == 8 ? 64 : 256;
  static constexpr int PPT = TS == 32 ? 4 : 1;
};

template <int TS>
__device__ __forceinline__ void pixel_of(int t, int p, int &x, int &y) {
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

}  // namespace gsr

// Wavefront (64 lanes) and workgroup scan / reduction helpers.
#pragma once

#include "common.hpp"

namespace gsr {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

// Inclusive prefix sum over the wave.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive prefix sum over a workgroup of NT threads; `total` gets the sum.
// `lds` must hold NT / 64 elements.  Contains two barriers.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *lds, T &total) {
  constexpr int NW = NT / kWave;
  const T incl = wave_incl_scan(x);
  if (lane_id() == kWave - 1) lds[wave_id()] = incl;
  __syncthreads();
  T before = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const T s = lds[w];
    if (w < wave_id()) before += s;
    sum += s;
  }
  __syncthreads();
  total = sum;
  return before + incl - x;
}

template <typename T>
__device__ __forceinline__ T wave_reduce_or(T x) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) x |= __shfl_xor(x, d, kWave);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_reduce_and(T x) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) x &= __shfl_xor(x, d, kWave);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_reduce_max(T x) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = __shfl_xor(x, d, kWave);
    x = x > y ? x : y;
  }
  return x;
}

// Sum over the wave with DPP row operations; the total is valid in lane 63.
// Must be called with all 64 lanes active.
// Swap-and-add of two row-summed values a, b: lanes 0..31 get
// a[l] + a[l + 32], lanes 32..63 get b[l - 32] + b[l].
__device__ __forceinline__ float fold32(float a, float b) {
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(h[0]) + __uint_as_float(h[1]);
}

// Swap-and-add of two fold32 results x (values A | B) and y (C | D): lanes
// 0..15 get A, 16..31 get C, 32..47 get B, 48..63 get D, each summed over
// the whole wave.
__device__ __forceinline__ float fold16(float x, float y) {
  const auto h = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(h[0]) + __uint_as_float(h[1]);
}

// keep + (send of the DPP partner CTRL), in float.
template <int CTRL>
__device__ __forceinline__ float dpp_add(float keep, float send) {
  return keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), CTRL, 0xF, 0xF, false));
}

// Exchange-and-add of two values between DPP partners that differ in lane
// bit `hi`: the lane with the bit clear keeps a, the other keeps b, and each
// adds its partner's copy of the value it keeps.
template <int CTRL>
__device__ __forceinline__ float pack_add(float a, float b, bool hi) {
  return dpp_add<CTRL>(hi ? b : a, hi ? a : b);
}

// Wave sums of nine values, with the values packed as the butterfly goes:
// in-row steps xor 1, xor 2 (quad permutes) and rotate 4 each halve the
// registers by keeping one value of a pair per lane (9 -> 5 -> 3 -> 2),
// rotate 8 completes the row sums, and the 32- and 16-lane swaps add the
// rows.  On return lane l < 8 holds the sum of v[l] and lanes 32..47 the sum
// of v[8].  Fixed order (deterministic); every lane must be active.
__device__ __forceinline__ float wave_sum9_packed(const float (&v)[9]) {
  const int l = lane_id();
  const bool b0 = l & 1, b1 = (l >> 1) & 1, b2 = (l >> 2) & 1;
  constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kRor4 = 0x124, kRor8 = 0x128;
  // xor 1: value 2k + b0 in register k
  const float p0 = pack_add<kXor1>(v[0], v[1], b0), p1 = pack_add<kXor1>(v[2], v[3], b0);
  const float p2 = pack_add<kXor1>(v[4], v[5], b0), p3 = pack_add<kXor1>(v[6], v[7], b0);
  const float p4 = dpp_add<kXor1>(v[8], v[8]);
  // xor 2: value 4k + 2 b1 + b0 in register k
  const float q0 = pack_add<kXor2>(p0, p1, b1), q1 = pack_add<kXor2>(p2, p3, b1);
  const float q2 = dpp_add<kXor2>(p4, p4);
  // rotate 4: value 4 b2 + 2 b1 + b0 (= l & 7) in r0
  const float r0 = pack_add<kRor4>(q0, q1, b2);
  const float r1 = dpp_add<kRor4>(q2, q2);
  // rotate 8: row sums
  const float s0 = dpp_add<kRor8>(r0, r0), s1 = dpp_add<kRor8>(r1, r1);
  // rows: s0 in lanes 0..31, s1 in lanes 32..63, then all four rows
  const float f = fold32(s0, s1);
  return fold16(f, f);
}


// Lanes below this one in the wave.
__device__ __forceinline__ uint64_t lanemask_lt() { return (uint64_t(1) << lane_id()) - 1u; }

// Atomic increment of *p for every lane with `pred`, issued once per wave:
// each such lane gets a distinct old value (in lane order within the wave).
// Must be reached by all lanes of the wave.
__device__ __forceinline__ uint32_t wave_atomic_inc(uint32_t *p, bool pred) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return 0u;
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0u;
  if (lane_id() == leader) base = atomicAdd(p, (uint32_t)__popcll(m));
  base = __shfl(base, leader, kWave);
  return base + (uint32_t)__popcll(m & lanemask_lt());
}

// Tile visited by workgroup `bid` of a grid of `grid` workgroups over `total`
// tiles.  Consecutive workgroups are dispatched round-robin over the 8 XCDs;
// this mapping gives each XCD one contiguous run of tiles so neighbouring
// tiles, which share most of their Gaussians, hit the same L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t grid) {
  const uint32_t per_xcd = grid / 8u;  // grid is a multiple of 8
  return (bid % 8u) * per_xcd + bid / 8u;
}

__device__ __forceinline__ int view_of_tile(const ViewInfo *__restrict__ views, int n_views, uint32_t tile) {
  int v = 0;
  while (v + 1 < n_views && views[v + 1].tile_base <= tile) ++v;
  return v;
}

}  // namespace gsr

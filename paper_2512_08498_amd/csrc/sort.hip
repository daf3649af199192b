// Per-tile sort of the (depth bits << 32 | record) entries.
//
// Each tile's list is sorted in LDS by a least-significant-digit radix sort
// over the depth bits (4-bit digits; digits equal across the whole list are
// skipped), followed by an odd-even transposition pass that orders entries of
// equal depth by record index (record order = Gaussian order within a view).
// The result is the list sorted by (depth, record), as the compositing order
// requires.  Lists longer than the LDS capacity use the same ranking in
// chunks, streaming through global memory.
//
// Size classes (one workgroup per tile):
//   n <= 256   :  64 threads x 4 items, grid over all tiles (one wave, so
//                its barriers are cheap)
//   n <= 2048  : 256 threads x 8 items, tiles queued by the first kernel
//   n <= 8192  : 512 threads x 16 items
//   larger     : 1024 threads, 8192-entry chunks through global memory
#include "kernels.hpp"
#include "util.hpp"

namespace gsr {

constexpr uint64_t kPadKey = ~0ull;

template <int NT>
__device__ __forceinline__ void block_or_and(uint32_t x_or, uint32_t x_and, uint32_t *red, uint32_t &o,
                                             uint32_t &a) {
  x_or = wave_reduce_or(x_or);
  x_and = wave_reduce_and(x_and);
  if (lane_id() == 0) {
    red[wave_id() * 2] = x_or;
    red[wave_id() * 2 + 1] = x_and;
  }
  __syncthreads();
  o = 0;
  a = ~0u;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) {
    o |= red[w * 2];
    a &= red[w * 2 + 1];
  }
  __syncthreads();
}

// Rank the IPT items of each thread (blocked layout: thread t owns items
// t*IPT .. t*IPT+IPT-1) by their 4-bit digit, stably.  On return pos[i] is
// the item's rank in the workgroup's digit-sorted order and, for d < 16,
// cnt[d*NT] holds the number of items with digit < d.  valid[i] = false
// items are not counted and get no position.
template <int NT, int IPT>
__device__ __forceinline__ void block_rank(const uint32_t (&dig)[IPT], const bool (&valid)[IPT],
                                           uint16_t *cnt, uint32_t *scan_lds, uint32_t (&pos)[IPT]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < 16; ++d) cnt[d * NT + t] = 0;
  uint32_t sub[IPT];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    if (valid[i]) {
      const uint32_t c = cnt[dig[i] * NT + t];
      sub[i] = c;
      cnt[dig[i] * NT + t] = (uint16_t)(c + 1);
    }
  }
  __syncthreads();
  // exclusive scan over the 16*NT counters in digit-major order; thread t
  // owns the 16 consecutive counters 16t .. 16t+15
  uint32_t loc[16];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    loc[k] = cnt[16 * t + k];
    s += loc[k];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan<NT>(s, scan_lds, tot);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    cnt[16 * t + k] = (uint16_t)run;
    run += loc[k];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IPT; ++i)
    if (valid[i]) pos[i] = cnt[dig[i] * NT + t] + sub[i];
}

template <int NT, int IPT>
struct SortLds {
  uint64_t keys[NT * IPT];
  uint64_t tmp[NT * IPT];
  uint16_t cnt[16 * NT];
  uint32_t scan[NT / kWave * 2];
  uint32_t red[NT / kWave * 2];
  int flag;
};

// Sort n <= NT*IPT entries of one tile in LDS and write the record indices.
template <int NT, int IPT>
__device__ void sort_tile_lds(SortLds<NT, IPT> &S, const Ws &ws, uint32_t start, uint32_t n) {
  const int t = threadIdx.x;
  uint32_t zo = 0, za = ~0u;
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint32_t idx = t * IPT + i;
    const uint64_t k = idx < n ? ws.pairs[start + idx] : kPadKey;
    S.keys[idx] = k;
    if (idx < n) {
      zo |= (uint32_t)(k >> 32);
      za &= (uint32_t)(k >> 32);
    }
  }
  uint32_t o, a;
  block_or_and<NT>(zo, za, S.red, o, a);
  const uint32_t vary = o ^ a;
  uint64_t *src = S.keys, *dst = S.tmp;
  for (int sh = 0; sh < 32; sh += 4) {
    if (((vary >> sh) & 0xFu) == 0) continue;
    uint32_t dig[IPT], pos[IPT];
    bool val[IPT];
    uint64_t kk[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      kk[i] = src[t * IPT + i];
      dig[i] = (uint32_t)(kk[i] >> (32 + sh)) & 0xFu;
      val[i] = true;
    }
    block_rank<NT, IPT>(dig, val, S.cnt, S.scan, pos);
#pragma unroll
    for (int i = 0; i < IPT; ++i) dst[pos[i]] = kk[i];
    __syncthreads();
    uint64_t *x = src;
    src = dst;
    dst = x;
  }
  // equal depths: order by record (odd-even transposition; the list is
  // already sorted by depth, so only ties can be out of order)
  for (;;) {
    int swapped = 0;
    for (int ph = 0; ph < 2; ++ph) {
      for (uint32_t k = t; 2 * k + ph + 1 < n; k += NT) {
        const uint32_t i = 2 * k + ph;
        const uint64_t x = src[i], y = src[i + 1];
        if (x > y) {
          src[i] = y;
          src[i + 1] = x;
          swapped = 1;
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(swapped)) break;
  }
  for (uint32_t i = t; i < n; i += NT) ws.tile_recs[start + i] = (uint32_t)src[i];
}

// Lists of at most small_max entries (the others were queued for the larger
// sorts by the binning).
__global__ __launch_bounds__(64) void k_sort_small(Ws ws, Sizes sz, uint32_t small_max) {
  __shared__ SortLds<64, 4> S;
  if (ws.scalars[kOverflow]) return;
  const uint32_t tile = blockIdx.x;
  const uint32_t n = ws.tile_count[tile];
  const uint32_t start = ws.tile_start[tile];
  if (n == 0 || n > small_max) return;
  if (n == 1) {
    if (threadIdx.x == 0) ws.tile_recs[start] = (uint32_t)ws.pairs[start];
    return;
  }
  sort_tile_lds<64, 4>(S, ws, start, n);
}

template <int NT, int IPT>
__global__ __launch_bounds__(NT) void k_sort_queue(Ws ws, Sizes sz, int q) {
  __shared__ SortLds<NT, IPT> S;
  if (ws.scalars[kOverflow]) return;
  const uint32_t count = ws.scalars[kQueueMid + q];
  for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
    const uint32_t tile = ws.queues[q * sz.t_tot + i];
    sort_tile_lds<NT, IPT>(S, ws, ws.tile_start[tile], ws.tile_count[tile]);
    __syncthreads();
  }
}

// Lists longer than 8192: LSD radix passes through global memory, chunk by
// chunk in order (stable), ping-ponging between pairs and pairs_tmp.
constexpr int kHugeNT = 1024, kHugeIPT = 8, kHugeChunk = kHugeNT * kHugeIPT;

struct HugeLds {
  uint64_t keys[kHugeChunk];
  uint16_t cnt[16 * kHugeNT];
  uint32_t scan[kHugeNT / kWave * 2];
  uint32_t red[kHugeNT / kWave * 2];
  uint32_t hist[16];
  uint32_t base[17];
  uint32_t chunk_start[17];
};

__device__ void sort_tile_global(HugeLds &S, const Ws &ws, uint32_t start, uint32_t n) {
  const int t = threadIdx.x;
  uint32_t zo = 0, za = ~0u;
  for (uint32_t i = t; i < n; i += kHugeNT) {
    const uint32_t z = (uint32_t)(ws.pairs[start + i] >> 32);
    zo |= z;
    za &= z;
  }
  uint32_t o, a;
  block_or_and<kHugeNT>(zo, za, S.red, o, a);
  const uint32_t vary = o ^ a;
  uint64_t *src = ws.pairs + start, *dst = ws.pairs_tmp + start;
  for (int sh = 0; sh < 32; sh += 4) {
    if (((vary >> sh) & 0xFu) == 0) continue;
    if (t < 16) S.hist[t] = 0;
    __syncthreads();
    for (uint32_t i = t; i < n; i += kHugeNT) atomicAdd(&S.hist[(uint32_t)(src[i] >> (32 + sh)) & 0xFu], 1u);
    __syncthreads();
    if (t == 0) {
      uint32_t acc = 0;
      for (int d = 0; d < 16; ++d) {
        S.base[d] = acc;
        acc += S.hist[d];
      }
    }
    __syncthreads();
    for (uint32_t c0 = 0; c0 < n; c0 += kHugeChunk) {
      uint32_t dig[kHugeIPT], pos[kHugeIPT];
      bool val[kHugeIPT];
      uint64_t kk[kHugeIPT];
#pragma unroll
      for (int i = 0; i < kHugeIPT; ++i) {
        const uint32_t idx = c0 + t * kHugeIPT + i;
        val[i] = idx < n;
        kk[i] = val[i] ? src[idx] : kPadKey;
        dig[i] = (uint32_t)(kk[i] >> (32 + sh)) & 0xFu;
      }
      block_rank<kHugeNT, kHugeIPT>(dig, val, S.cnt, S.scan, pos);
      if (t < 16) S.chunk_start[t] = S.cnt[t * kHugeNT];
      if (t == 0) {
        const uint32_t m = min<uint32_t>(kHugeChunk, n - c0);
        S.chunk_start[16] = m;
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kHugeIPT; ++i) {
        if (val[i]) {
          const uint32_t d = dig[i];
          dst[S.base[d] + (pos[i] - S.chunk_start[d])] = kk[i];
        }
      }
      __syncthreads();
      if (t < 16) S.base[t] += S.chunk_start[t + 1] - S.chunk_start[t];
      __syncthreads();
    }
    uint64_t *x = src;
    src = dst;
    dst = x;
    __threadfence_block();
    __syncthreads();
  }
  // equal depths: each run is sorted by record by the thread at its start
  for (uint32_t i = t; i < n; i += kHugeNT) {
    const uint32_t z = (uint32_t)(src[i] >> 32);
    const bool head = (i == 0 || (uint32_t)(src[i - 1] >> 32) != z);
    if (head && i + 1 < n && (uint32_t)(src[i + 1] >> 32) == z) {
      uint32_t e = i + 1;
      while (e < n && (uint32_t)(src[e] >> 32) == z) ++e;
      for (uint32_t a2 = i + 1; a2 < e; ++a2) {
        const uint64_t key = src[a2];
        uint32_t b2 = a2;
        while (b2 > i && src[b2 - 1] > key) {
          src[b2] = src[b2 - 1];
          --b2;
        }
        src[b2] = key;
      }
    }
  }
  __syncthreads();
  for (uint32_t i = t; i < n; i += kHugeNT) ws.tile_recs[start + i] = (uint32_t)src[i];
}

__global__ __launch_bounds__(kHugeNT) void k_sort_huge(Ws ws, Sizes sz) {
  __shared__ HugeLds S;
  if (ws.scalars[kOverflow]) return;
  const uint32_t count = ws.scalars[kQueueHuge];
  for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
    const uint32_t tile = ws.queues[2 * sz.t_tot + i];
    sort_tile_global(S, ws, ws.tile_start[tile], ws.tile_count[tile]);
    __syncthreads();
  }
}

// lds_small_max < 256 (a debug option, applied by the binning's size
// classes as well) pushes shorter lists into the larger sorts so every path
// can be exercised on small inputs.
void launch_sort(const ViewInfo *views, const Ws &ws, const Sizes &sz, uint32_t lds_small_max, hipStream_t st) {
  (void)views;
  if (sz.t_tot == 0) return;
  k_sort_small<<<sz.t_tot, 64, 0, st>>>(ws, sz, lds_small_max);
  k_sort_queue<256, 8><<<1024, 256, 0, st>>>(ws, sz, 0);
  k_sort_queue<512, 16><<<512, 512, 0, st>>>(ws, sz, 1);
  k_sort_huge<<<256, kHugeNT, 0, st>>>(ws, sz);
}

}  // namespace gsr

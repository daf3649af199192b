// Tile binning without global atomics on contended addresses:
//
//  1. emission   every (record, tile) pair is written at its record-major
//                position (the record's pair offset from the preprocess
//                scan plus its index in the record's tile rectangle): the
//                global tile id as key, the record as value;
//  2. tile sort  stable LSD counting passes on 8-bit digits of the tile id:
//                per-block digit histograms, a device-wide scan, and a
//                scatter that ranks each block's items by digit with wave
//                ballots (stable, so a tile's entries stay in record order,
//                which is Gaussian order within a view); the last pass
//                writes the (depth bits << 32 | record) entries the per-tile
//                depth sorts take;
//  3. bounds     list start and length of every tile from the sorted ids;
//  4. classify   size class of each tile for the depth sorts and its
//                longest-first sort key; the longest-first tile order is two
//                more counting passes over 16-bit keys.
//
// Far-away Gaussians crowd into the few tiles around the vanishing point of
// a street scene; per-pair atomic slot claims on those tiles serialise, the
// counting passes do not.
#include <algorithm>

#include "kernels.hpp"
#include "util.hpp"

namespace gsr {

constexpr int kRdxNT = 256;                        // threads per counting-pass block
constexpr int kRdxRounds = 32;                     // rounds of 256 items per block
constexpr uint32_t kRdxChunk = kRdxNT * kRdxRounds;  // items per block
constexpr int kScanNT = 256, kScanIPT = 16;
constexpr uint32_t kScanChunk = kScanNT * kScanIPT;

__device__ __forceinline__ uint32_t n_items(const uint32_t *count_dev, uint32_t cap) {
  return count_dev ? min(*count_dev, cap) : cap;
}

// 1. Each wave expands 64 consecutive records into their pairs: lane l takes
// pair b + l of the wave's concatenated tile rectangles and finds its record
// by a binary search over the wave's prefix sums, so a big footprint is
// spread over the lanes.  Positions are record-major and contiguous per wave.
__global__ __launch_bounds__(256) void k_emit(const ViewInfo *__restrict__ views, Ws ws, Sizes sz,
                                              uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  if (ws.scalars[kOverflow]) return;
  const uint32_t nrec = ws.scalars[kNumRecords];
  const int lane = lane_id();
  const uint32_t wave_stride = gridDim.x * (blockDim.x / kWave) * kWave;
  for (uint32_t wbase = (blockIdx.x * (blockDim.x / kWave) + wave_id()) * kWave; wbase < nrec;
       wbase += wave_stride) {
    const uint32_t r = wbase + lane;
    const bool valid = r < nrec;
    uint32_t tx0 = 0, w = 1, ty0 = 0, cnt = 0, v = 0, off = 0;
    if (valid) {
      const uint2 rc = ws.rec_rect[r];
      tx0 = rc.x & 0xFFFFu;
      w = (rc.x >> 16) - tx0 + 1;
      ty0 = rc.y & 0xFFFFu;
      cnt = w * ((rc.y >> 16) - ty0 + 1);
      v = ws.rec_view[r];
      off = ws.rec_pairoff[r];
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
      const uint32_t o_off = __shfl(off, o, kWave), o_ex = __shfl(excl, o, kWave);
      if (p < total) {
        const uint32_t k = p - o_ex;
        const uint32_t tx = o_tx0 + k % o_w, ty = o_ty0 + k / o_w;
        const ViewInfo vi = views[o_v];
        const uint32_t pos = o_off + k;
        if (pos < sz.cap_pairs) {
          keys[pos] = vi.tile_base + ty * (uint32_t)vi.tiles_x + tx;
          vals[pos] = wbase + (uint32_t)o;
        } else {
          ws.scalars[kOverflow] = 3u;  // inconsistent pair offsets
        }
      }
    }
  }
}

// 2a. Digit histogram of one block's chunk, stored digit-major:
// hist[d * gridDim.x + block].
__global__ __launch_bounds__(kRdxNT) void k_digit_hist(const uint32_t *__restrict__ scalars,
                                                       const uint32_t *__restrict__ keys,
                                                       const uint32_t *__restrict__ count_dev, uint32_t cap,
                                                       int shift, uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[256];
  const uint32_t t = threadIdx.x;
  h[t] = 0u;
  __syncthreads();
  if (!scalars[kOverflow]) {
    const uint32_t n = n_items(count_dev, cap);
    const uint32_t lo = blockIdx.x * kRdxChunk, hi = min(n, lo + kRdxChunk);
    for (uint32_t i = lo + t; i < hi; i += kRdxNT) atomicAdd(&h[(keys[i] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[t * gridDim.x + blockIdx.x] = h[t];
}

// Device-wide exclusive scan of data[0, len): chunk sums, a single-block
// scan of the sums, then each chunk scanned with its offset.
__global__ __launch_bounds__(kScanNT) void k_scan_reduce(const uint32_t *__restrict__ data, uint32_t len,
                                                         uint32_t *__restrict__ part) {
  __shared__ uint32_t s[kScanNT / kWave];
  const uint32_t lo = blockIdx.x * kScanChunk + threadIdx.x * kScanIPT;
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) acc += lo + i < len ? data[lo + i] : 0u;
  uint32_t total;
  block_excl_scan<kScanNT>(acc, s, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *__restrict__ part, uint32_t nb) {
  __shared__ uint32_t s[1024 / kWave];
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t x = i < nb ? part[i] : 0u;
    uint32_t total;
    const uint32_t e = block_excl_scan<1024>(x, s, total);
    if (i < nb) part[i] = carry + e;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanNT) void k_scan_down(uint32_t *__restrict__ data, uint32_t len,
                                                       const uint32_t *__restrict__ part) {
  __shared__ uint32_t s[kScanNT / kWave];
  const uint32_t lo = blockIdx.x * kScanChunk + threadIdx.x * kScanIPT;
  uint32_t x[kScanIPT], acc = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    x[i] = lo + i < len ? data[lo + i] : 0u;
    acc += x[i];
  }
  uint32_t total;
  uint32_t run = part[blockIdx.x] + block_excl_scan<kScanNT>(acc, s, total);
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    if (lo + i < len) data[lo + i] = run;
    run += x[i];
  }
}

// 2b. Stable scatter of one block's chunk by digit.  Per round of 256 items
// (item = lane order), lanes of a wave with equal digits are found with 8
// ballots; a lane's rank is the number of such lanes below it plus the
// counts of the same digit in the lower waves and in earlier rounds.
// FINAL: the output is the (depth bits << 32 | record) entry, and the
// sorted key.
template <bool FINAL>
__global__ __launch_bounds__(kRdxNT) void k_digit_scatter(
    const uint32_t *__restrict__ scalars, const uint32_t *__restrict__ keys_in,
    const uint32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
    uint64_t *__restrict__ pairs_out, const uint32_t *__restrict__ zbits, const uint32_t *__restrict__ count_dev,
    uint32_t cap, int shift, const uint32_t *__restrict__ hist) {
  constexpr int NW = kRdxNT / kWave;
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[NW][256];
  if (scalars[kOverflow]) return;
  const uint32_t t = threadIdx.x;
  const int w = wave_id(), lane = lane_id();
  base[t] = hist[t * gridDim.x + blockIdx.x];
#pragma unroll
  for (int k = 0; k < NW; ++k) wcnt[k][t] = 0u;
  __syncthreads();
  const uint32_t n = n_items(count_dev, cap);
  const uint32_t lo = blockIdx.x * kRdxChunk;
  const uint64_t lt = lanemask_lt();
  for (int r = 0; r < kRdxRounds; ++r) {
    const uint32_t r0 = lo + (uint32_t)r * kRdxNT;
    if (r0 >= n) break;  // uniform over the block
    const uint32_t i = r0 + t;
    const bool valid = i < n;
    const uint32_t key = valid ? keys_in[i] : 0u;
    const uint32_t val = valid ? vals_in[i] : 0u;
    const uint32_t d = (key >> shift) & 0xFFu;
    uint64_t eq = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      eq &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(eq & lt);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(eq);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + rank;
      for (int k = 0; k < w; ++k) pos += wcnt[k][d];
      if (pos < cap) {
        if (FINAL) {
          pairs_out[pos] = ((uint64_t)zbits[val] << 32) | (uint64_t)val;
          keys_out[pos] = key;
        } else {
          keys_out[pos] = key;
          vals_out[pos] = val;
        }
      }
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      s += wcnt[k][t];
      wcnt[k][t] = 0u;
    }
    base[t] += s;
    __syncthreads();
  }
}

// 3. List bounds from the sorted tile ids: the first entry of a tile writes
// its start, the last one its end (into tile_count, turned into the length
// by k_tile_classify).  Both arrays are zeroed by the forward beforehand.
__global__ void k_tile_bounds(Ws ws, Sizes sz, const uint32_t *__restrict__ tiles) {
  if (ws.scalars[kOverflow]) return;
  const uint32_t n = min(ws.scalars[kNumPairs], sz.cap_pairs);
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t t = tiles[i];
    if (t >= sz.t_tot) {
      ws.scalars[kOverflow] = 3u;
      continue;
    }
    if (i == 0 || tiles[i - 1] != t) ws.tile_start[t] = i;
    if (i == n - 1 || tiles[i + 1] != t) ws.tile_count[t] = i + 1;
  }
}

// 4. Per tile: the list length; the size class of its depth sort (lists
// longer than small_max go to a queue of the larger sorts, force_q pushes
// them to at least that class); the longest-first key; and the number of
// lists of at least long_list entries.  Queue slots are claimed once per
// wave.
__global__ __launch_bounds__(256) void k_tile_classify(Ws ws, Sizes sz, uint32_t small_max, int force_q,
                                                       uint32_t *__restrict__ order_keys,
                                                       uint32_t *__restrict__ order_vals) {
  if (ws.scalars[kOverflow]) return;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < sz.t_tot;
  uint32_t n = 0;
  if (valid) {
    const uint32_t end = ws.tile_count[t];
    n = end ? end - ws.tile_start[t] : 0u;
    ws.tile_count[t] = n;
    order_keys[t] = 0xFFFFu - min(n, 0xFFFFu);
    order_vals[t] = t;
  }
  int q = -1;
  if (valid && n > small_max) {
    q = n <= kMidMax ? 0 : (n <= kBigMax ? 1 : 2);
    if (force_q > q) q = force_q;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const uint32_t at = wave_atomic_inc(ws.scalars + kQueueMid + c, q == c);
    if (q == c) ws.queues[(uint32_t)c * sz.t_tot + at] = t;
  }
  (void)wave_atomic_inc(ws.scalars + kNumLong, valid && n >= sz.long_list);
}

namespace {

struct Pass {
  const uint32_t *keys_in, *vals_in;
  uint32_t *keys_out, *vals_out;
};

// Exclusive scan of len words in place, part holding ceil(len / 4096) words.
void scan_words(uint32_t *data, uint32_t len, uint32_t *part, hipStream_t st) {
  const uint32_t nb = (len + kScanChunk - 1) / kScanChunk;
  if (nb == 0) return;
  k_scan_reduce<<<nb, kScanNT, 0, st>>>(data, len, part);
  k_scan_top<<<1, 1024, 0, st>>>(part, nb);
  k_scan_down<<<nb, kScanNT, 0, st>>>(data, len, part);
}

// Stable sort of (keys, vals) by the low `bits` bits of the keys, `cap`
// items of which *count_dev (or all, if NULL) are live.  The last pass
// writes FINAL output when pairs_out is given, else to out_vals.
void counting_sort(const Ws &ws, const uint32_t *count_dev, uint32_t cap, int bits, uint32_t *ka, uint32_t *va,
                   uint32_t *kb, uint32_t *vb, uint32_t *out_keys, uint32_t *out_vals, uint64_t *pairs_out,
                   hipStream_t st) {
  const uint32_t nblk = std::max<uint32_t>((cap + kRdxChunk - 1) / kRdxChunk, 1u);
  const int passes = std::max(1, (bits + 7) / 8);
  const uint32_t *kin = ka, *vin = va;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    uint32_t *kout = last ? out_keys : (kin == ka ? kb : ka);
    uint32_t *vout = last ? out_vals : (kin == ka ? vb : va);
    k_digit_hist<<<nblk, kRdxNT, 0, st>>>(ws.scalars, kin, count_dev, cap, 8 * p, ws.radix_hist);
    scan_words(ws.radix_hist, 256u * nblk, ws.scan_part, st);
    if (last && pairs_out) {
      k_digit_scatter<true><<<nblk, kRdxNT, 0, st>>>(ws.scalars, kin, vin, kout, nullptr, pairs_out, ws.rec_zbits,
                                                     count_dev, cap, 8 * p, ws.radix_hist);
    } else {
      k_digit_scatter<false><<<nblk, kRdxNT, 0, st>>>(ws.scalars, kin, vin, kout, vout, nullptr, nullptr,
                                                      count_dev, cap, 8 * p, ws.radix_hist);
    }
    kin = kout;
    vin = vout;
  }
}

int bit_width(uint32_t x) { return x == 0 ? 0 : 32 - __builtin_clz(x); }

}  // namespace

void launch_binning(const ViewInfo *views, const Ws &ws, const Sizes &sz, uint32_t small_max, int force_q,
                    hipStream_t st) {
  if (sz.t_tot == 0) return;
  // pair buffers: (tile, record) ping-pong in pairs_tmp and in the
  // backward's partials (unused until the backward runs)
  uint32_t *ka = reinterpret_cast<uint32_t *>(ws.pairs_tmp), *va = ka + sz.cap_pairs;
  uint32_t *kb = reinterpret_cast<uint32_t *>(ws.partials), *vb = kb + sz.cap_pairs;
  const uint32_t waves = (sz.cap_rec + kWave - 1) / kWave;
  const uint32_t blocks = std::min<uint32_t>((waves + 3) / 4, 8192u);
  k_emit<<<std::max(blocks, 1u), 256, 0, st>>>(views, ws, sz, ka, va);
  const int bits = std::max(1, bit_width(sz.t_tot - 1));
  const int passes = (bits + 7) / 8;
  // the final pass leaves the sorted tile ids in the buffer not read by it
  uint32_t *sorted_tiles = (passes % 2 == 1) ? kb : ka;
  counting_sort(ws, ws.scalars + kNumPairs, sz.cap_pairs, bits, ka, va, kb, vb, sorted_tiles, nullptr, ws.pairs, st);
  const uint32_t bb = std::min<uint32_t>((sz.cap_pairs + 255) / 256, 16384u);
  k_tile_bounds<<<std::max(bb, 1u), 256, 0, st>>>(ws, sz, sorted_tiles);
  uint32_t *ok = ws.tile_tmp, *ov = ok + sz.t_tot, *ok2 = ov + sz.t_tot, *ov2 = ok2 + sz.t_tot;
  k_tile_classify<<<(sz.t_tot + 255) / 256, 256, 0, st>>>(ws, sz, small_max, force_q, ok, ov);
  // longest list first: 16-bit keys, two passes (the second reads ok2/ov2)
  counting_sort(ws, nullptr, sz.t_tot, 16, ok, ov, ok2, ov2, ok, ws.tile_order, nullptr, st);
}

// Exclusive scan of the list lengths: the CSR offsets of the tile lists
// (lists are contiguous in tile order), for the binning export.
__global__ void k_copy_counts(Ws ws, Sizes sz, uint32_t *__restrict__ csr) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < sz.t_tot) csr[t] = ws.tile_count[t];
  if (t == sz.t_tot) csr[t] = 0u;
}

void launch_tile_csr(const Ws &ws, const Sizes &sz, uint32_t *csr, hipStream_t st) {
  k_copy_counts<<<(sz.t_tot + 256) / 256, 256, 0, st>>>(ws, sz, csr);
  scan_words(csr, sz.t_tot + 1, ws.scan_part, st);
}

}  // namespace gsr

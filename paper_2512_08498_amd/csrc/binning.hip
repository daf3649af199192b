// Depth sort and tile binning, as stable counting (LSD radix) passes on
// 8- to 10-bit digits -- no global atomics on contended addresses:
//
//  sort      the visible records by their depth bits (four passes; stable,
//            so equal depths keep record order, which is Gaussian order
//            within a view);
//  emission  every (record, tile) pair in depth-sorted record order: the
//            global tile id as key, the record as value, at the record's
//            pair offset (a scan of the rectangle areas in that order);
//  tile sort the pairs by tile id (8-bit passes up to 2^16 tiles, two
//            9- or 10-bit passes up to 2^20 tiles): being stable, it
//            leaves each tile's list in (depth, record) order, the
//            compositing order, so no per-tile sort is needed -- together
//            the passes sort the 64-bit (tile | depth) keys;
//  bounds    list start and length of every tile from the sorted ids;
//  classify  the longest-first key of each tile (an 8-bit length code);
//            the longest-first tile order is one more pass over it.
//
// A pass is a per-block digit histogram, a device-wide scan of the
// histograms, and a scatter that ranks each block's items by digit with
// wave ballots and writes them through LDS in digit runs.  Far-away
// Gaussians crowd into the few tiles around the vanishing point of a street
// scene; per-pair atomic slot claims on those tiles would serialise, the
// counting passes do not.
#include <algorithm>

#include "kernels.hpp"
#include "util.hpp"

namespace gsr {

constexpr int kRdxNT = 256;  // threads per counting-pass block
// items per lane: 8 (2048 per block) for inputs below kRdxBig items, so a
// pass spreads over enough workgroups, else 32 (8192 per block)
constexpr uint32_t kRdxBig = 1u << 23;
constexpr int kScanNT = 256, kScanIPT = 16;
constexpr uint32_t kScanChunk = kScanNT * kScanIPT;

// Longest-first code of a list length: 16 steps per octave (the exponent
// and top four mantissa bits of the length as a float), inverted, so the
// longest lists come first; lengths from 2^16 up share the first code.
__device__ __forceinline__ uint32_t length_key(uint32_t n) {
  if (n == 0) return 255u;
  const uint32_t code = (__float_as_uint((float)n) >> 19) - (127u << 4);  // 0 for n = 1
  return 255u - min(code, 255u);
}

__device__ __forceinline__ uint32_t n_items(const uint32_t *count_dev, uint32_t cap) {
  return count_dev ? min(*count_dev, cap) : cap;
}

// Emission: each wave takes 64 consecutive records of the depth order (their
// indices perm[i] and tile records srect[i] are read in order); their pairs
// form one contiguous range (offs[i] is the first pair of sorted record i).
// A record of at most kEmitSmall pairs is written by its own lane, stepping
// through its tile rectangle; the lanes' stores fall into that one range.
// Bigger footprints are written by the whole wave, 64 pairs per step.
constexpr uint32_t kEmitSmall = 8;

__global__ __launch_bounds__(256) void k_emit(Ws ws, Sizes sz,
                                              const uint32_t *__restrict__ perm, const uint4 *__restrict__ srect,
                                              const uint32_t *__restrict__ offs,
                                              uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  if (ws.scalars[kOverflow]) return;
  const uint32_t nrec = ws.scalars[kNumRecords];
  const int lane = lane_id();
  const uint32_t wave_stride = gridDim.x * (blockDim.x / kWave) * kWave;
  for (uint32_t wbase = (blockIdx.x * (blockDim.x / kWave) + wave_id()) * kWave; wbase < nrec;
       wbase += wave_stride) {
    const uint32_t i = wbase + lane;
    uint32_t tx0 = 0, tx1 = 0, ty0 = 0, w = 1, cnt = 0, off = 0, rec = 0, tbase = 0, tpitch = 0;
    if (i < nrec) {
      rec = perm[i];
      const uint4 rc = srect[i];  // rectangle, first tile, row pitch
      tx0 = rc.x & 0xFFFFu;
      tx1 = rc.x >> 16;
      ty0 = rc.y & 0xFFFFu;
      w = tx1 - tx0 + 1;
      cnt = w * ((rc.y >> 16) - ty0 + 1);
      tbase = rc.z - ty0 * rc.w - tx0;  // so that tbase + ty * pitch + tx is the tile's id
      tpitch = rc.w;
      off = offs[i];
      if (off + cnt > sz.cap_pairs) {  // inconsistent pair offsets
        ws.scalars[kOverflow] = 3u;
        cnt = 0;
      }
    }
    if (cnt <= kEmitSmall) {
      uint32_t tx = tx0, row = tbase + ty0 * tpitch;
      for (uint32_t k = 0; k < cnt; ++k) {
        keys[off + k] = row + tx;
        vals[off + k] = rec;
        if (++tx > tx1) {
          tx = tx0;
          row += tpitch;
        }
      }
    }
    uint64_t big = __ballot(cnt > kEmitSmall);
    while (big) {
      const int l = __ffsll((unsigned long long)big) - 1;
      big &= big - 1;
      const uint32_t b_cnt = __shfl(cnt, l, kWave), b_off = __shfl(off, l, kWave), b_rec = __shfl(rec, l, kWave);
      const uint32_t b_tx0 = __shfl(tx0, l, kWave), b_w = __shfl(w, l, kWave);
      const uint32_t b_row0 = __shfl(tbase + ty0 * tpitch, l, kWave), b_pitch = __shfl(tpitch, l, kWave);
      for (uint32_t k = lane; k < b_cnt; k += kWave) {
        const uint32_t r = k / b_w, c = k - r * b_w;
        keys[b_off + k] = b_row0 + r * b_pitch + b_tx0 + c;
        vals[b_off + k] = b_rec;
      }
    }
  }
}

// Chunk of a counting-pass workgroup, given the number of chunks holding
// live items.  Workgroups go to the 8 XCDs in turn, so the live chunks are
// dealt out as 8 contiguous ranges, one per XCD: neighbouring chunks then
// share the cache lines of their digit-major histogram entries, and of their
// short digit runs in the output, in one XCD's L2 instead of writing parts
// of the same lines from different XCDs.  Chunks past the live ones keep
// their workgroup's index.
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t live_chunks) {
  const uint32_t b = blockIdx.x;
  if (b >= live_chunks) return b;
  const uint32_t x = b & 7u, q = live_chunks >> 3, r = live_chunks & 7u;
  return x * q + min(x, r) + (b >> 3);
}

// Lanes of the wave whose BITS-bit digit equals this lane's, among `live`:
// one ballot per bit; a lane differs from this one where the ballot of some
// bit differs from this lane's own bit (spread over a word as 0 or ~0), and
// those differences are OR-ed up per 32-lane half.
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool live) {
  uint32_t lo = 0u, hi = 0u;
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const uint32_t x = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
    const uint64_t m = __ballot(x != 0u);
    lo |= (uint32_t)m ^ x;
    hi |= (uint32_t)(m >> 32) ^ x;
  }
  return ((uint64_t)~hi << 32 | (uint64_t)~lo) & __ballot(live);
}

// 2a. Digit histogram of one block's chunk (IPL items per lane) for digits
// of BITS bits (8, 9 or 10: 2^BITS bins), stored digit-major:
// hist[d * gridDim.x + chunk].  Each wave loads its items first, then counts
// them 64 at a time: one LDS atomic when all 64 share a digit (as the high
// depth bits mostly do), else one per lane.
template <int IPL, int BITS>
__global__ __launch_bounds__(kRdxNT) void k_digit_hist(const uint32_t *__restrict__ scalars,
                                                       const uint32_t *__restrict__ keys,
                                                       const uint32_t *__restrict__ count_dev, uint32_t cap,
                                                       int shift, uint32_t *__restrict__ hist) {
  constexpr uint32_t CHUNK = kRdxNT * IPL;
  constexpr uint32_t RADIX = 1u << BITS, MASK = RADIX - 1u;
  __shared__ uint32_t h[RADIX];
  const uint32_t t = threadIdx.x;
  for (uint32_t d = t; d < RADIX; d += kRdxNT) h[d] = 0u;
  const uint32_t n = n_items(count_dev, cap);
  const uint32_t c = xcd_chunk(n / CHUNK + (n % CHUNK != 0u));
  __syncthreads();
  if (!scalars[kOverflow]) {
    const uint32_t lo = c * CHUNK + (uint32_t)wave_id() * (CHUNK / 4) + (uint32_t)lane_id();
    uint32_t d[IPL];
#pragma unroll
    for (int r = 0; r < IPL; ++r) {
      const uint32_t i = lo + (uint32_t)r * kWave;
      d[r] = i < n ? (keys[i] >> shift) & MASK : 0u;
    }
#pragma unroll
    for (int r = 0; r < IPL; ++r) {
      const bool live = lo + (uint32_t)r * kWave < n;  // lane 0 is live if any lane is
      const uint32_t d0 = __builtin_amdgcn_readfirstlane(d[r]);
      const uint64_t all = __ballot(live);
      if (__ballot(live && d[r] == d0) == all) {
        if (lane_id() == 0 && all) atomicAdd(&h[d0], (uint32_t)__popcll(all));
      } else if (live) {
        atomicAdd(&h[d[r]], 1u);
      }
    }
  }
  __syncthreads();
  for (uint32_t d = t; d < RADIX; d += kRdxNT) hist[d * gridDim.x + c] = h[d];
}

// Device-wide exclusive scan of data[0, len): chunk sums, then each chunk
// scanned with its offset, the sum of the totals before it (added up by the
// chunk's own workgroup, or over many chunks by a single-block scan).  Global
// accesses are coalesced; the per-thread runs of 16 words are read from LDS
// with a skew of one word per 16, so the 64 lanes hit distinct banks.
__device__ __forceinline__ uint32_t skew(uint32_t j) { return j + (j >> 4); }

__global__ __launch_bounds__(kScanNT) void k_scan_reduce(const uint32_t *__restrict__ data, uint32_t len,
                                                         uint32_t *__restrict__ part) {
  __shared__ uint32_t s[kScanNT / kWave];
  const uint32_t lo = blockIdx.x * kScanChunk;
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < kScanIPT; ++i) {
    const uint32_t j = lo + (uint32_t)i * kScanNT + threadIdx.x;
    acc += j < len ? data[j] : 0u;
  }
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

// Exclusive scan of NT*16 words at data + lo (words past len read as 0 and
// are not written), plus `carry`; returns the chunk total.
template <int NT>
__device__ __forceinline__ uint32_t scan_chunk(uint32_t *__restrict__ data, uint32_t lo, uint32_t len,
                                               uint32_t carry, uint32_t *lds, uint32_t *red) {
  constexpr uint32_t C = NT * 16;
  const uint32_t t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint32_t j = (uint32_t)i * NT + t;
    lds[skew(j)] = lo + j < len ? data[lo + j] : 0u;
  }
  __syncthreads();
  uint32_t x[16], acc = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    x[i] = lds[skew(t * 16 + i)];
    acc += x[i];
  }
  uint32_t total;
  uint32_t run = carry + block_excl_scan<NT>(acc, red, total);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    lds[skew(t * 16 + i)] = run;
    run += x[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint32_t j = (uint32_t)i * NT + t;
    if (lo + j < len) data[lo + j] = lds[skew(j)];
  }
  __syncthreads();
  (void)C;
  return total;
}

// Small scans in one workgroup of 1024 threads, 16K words per step.
__global__ __launch_bounds__(1024) void k_scan_one(uint32_t *__restrict__ data, uint32_t len) {
  __shared__ uint32_t lds[1024 * 16 + 1024];
  __shared__ uint32_t red[1024 / kWave];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < len; base += 1024u * 16u) carry += scan_chunk<1024>(data, base, len, carry, lds, red);
}

// SUM_BEFORE: part holds the chunk totals, and each workgroup adds up those
// before its chunk itself (at most kScanFusedMax words, read from L2), which
// saves the launch of the single-block scan of the totals.  Otherwise part
// holds the chunks' offsets.
template <bool SUM_BEFORE>
__global__ __launch_bounds__(kScanNT) void k_scan_down(uint32_t *__restrict__ data, uint32_t len,
                                                       const uint32_t *__restrict__ part) {
  __shared__ uint32_t lds[kScanChunk + kScanChunk / 16];
  __shared__ uint32_t red[kScanNT / kWave];
  uint32_t carry;
  if (SUM_BEFORE) {
    uint32_t c = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanNT) c += part[i];
    block_excl_scan<kScanNT>(c, red, carry);
  } else {
    carry = part[blockIdx.x];
  }
  scan_chunk<kScanNT>(data, blockIdx.x * kScanChunk, len, carry, lds, red);
}

// 2b. Stable scatter of one block's chunk by digit.  Wave w owns the w-th
// quarter of the chunk and loads all of it first (IPL items per lane).  It
// ranks its items by digit round by round (64 items, in order) with ballot
// matches and its own running digit counts in LDS, so no workgroup barrier
// is needed per round.  The block then places its items in LDS in local
// digit order (stable: waves and rounds in item order) and writes each
// digit's run to its global offset, contiguously.  vals_in = NULL: the
// values are the item indices.  With area_out, the values are records, and
// their tile-rectangle areas and tile records (rect_out) are written beside
// them.
template <int IPL, int BITS>
struct ScatterLds {
  uint32_t key[kRdxNT * IPL];
  uint32_t val[kRdxNT * IPL];
  uint32_t wcnt[kRdxNT / kWave][1u << BITS];  // running, then starting, counts per wave and digit
  uint32_t lstart[1u << BITS];                // local start of each digit
  uint32_t gbase[1u << BITS];                 // global start of each digit for this block
  uint32_t scan[kRdxNT / kWave];
};

template <int IPL, int BITS>
__global__ __launch_bounds__(kRdxNT) void k_digit_scatter(const uint32_t *__restrict__ scalars,
                                                          const uint32_t *__restrict__ keys_in,
                                                          const uint32_t *__restrict__ vals_in,
                                                          uint32_t *__restrict__ keys_out,
                                                          uint32_t *__restrict__ vals_out,
                                                          const uint32_t *__restrict__ count_dev, uint32_t cap,
                                                          int shift, const uint32_t *__restrict__ hist,
                                                          const uint4 *__restrict__ rect,
                                                          uint32_t *__restrict__ area_out,
                                                          uint4 *__restrict__ rect_out) {
  constexpr int NW = kRdxNT / kWave;
  constexpr uint32_t CHUNK = kRdxNT * IPL;
  constexpr uint32_t RADIX = 1u << BITS, MASK = RADIX - 1u;
  constexpr int DPT = (int)(RADIX / kRdxNT);  // digits per thread, consecutive: t * DPT + k
  __shared__ ScatterLds<IPL, BITS> S;
  if (scalars[kOverflow]) return;
  const uint32_t t = threadIdx.x;
  const int w = wave_id(), lane = lane_id();
  const uint32_t n = n_items(count_dev, cap);
  const uint32_t c = xcd_chunk(n / CHUNK + (n % CHUNK != 0u)), blo = c * CHUNK;
  if (blo >= n) return;  // uniform: nothing of this block is live
  const uint32_t m = min(CHUNK, n - blo);
#pragma unroll
  for (int e = 0; e < DPT; ++e) {
    const uint32_t d = t * DPT + (uint32_t)e;
#pragma unroll
    for (int k = 0; k < NW; ++k) S.wcnt[k][d] = 0u;
    S.gbase[d] = hist[d * gridDim.x + c];
  }
  const uint32_t lo = blo + (uint32_t)w * (CHUNK / NW);
  uint32_t key[IPL], val[IPL], rk[IPL];
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    const uint32_t i = lo + (uint32_t)r * kWave + (uint32_t)lane;
    key[r] = i < n ? keys_in[i] : 0u;
    val[r] = i < n ? (vals_in ? vals_in[i] : i) : 0u;
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    const uint32_t i = lo + (uint32_t)r * kWave + (uint32_t)lane;
    const bool live = i < n;
    const uint32_t d = (key[r] >> shift) & MASK;
    const uint64_t eq = match_digit<BITS>(d, live);
    const uint32_t before = (uint32_t)__popcll(eq & lt);
    const uint32_t prior = S.wcnt[w][d];
    rk[r] = prior + before;
    if (live && before == 0) S.wcnt[w][d] = prior + (uint32_t)__popcll(eq);
  }
  __syncthreads();
  {
    // the thread's DPT consecutive digits: local starts in digit order, then
    // per digit in wave order
    uint32_t cnt[DPT][NW], tot = 0;
#pragma unroll
    for (int e = 0; e < DPT; ++e)
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        cnt[e][k] = S.wcnt[k][t * DPT + (uint32_t)e];
        tot += cnt[e][k];
      }
    uint32_t total;
    uint32_t run = block_excl_scan<kRdxNT>(tot, S.scan, total);
#pragma unroll
    for (int e = 0; e < DPT; ++e) {
      const uint32_t d = t * DPT + (uint32_t)e;
      S.lstart[d] = run;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        S.wcnt[k][d] = run;
        run += cnt[e][k];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    const uint32_t i = lo + (uint32_t)r * kWave + (uint32_t)lane;
    if (i < n) {
      const uint32_t p = S.wcnt[w][(key[r] >> shift) & MASK] + rk[r];
      S.key[p] = key[r];
      S.val[p] = val[r];
    }
  }
  __syncthreads();
  for (uint32_t j = t; j < m; j += kRdxNT) {
    const uint32_t k = S.key[j], v = S.val[j];
    const uint32_t d = (k >> shift) & MASK;
    const uint32_t g = S.gbase[d] + (j - S.lstart[d]);
    if (g < cap) {
      keys_out[g] = k;
      vals_out[g] = v;
      if (area_out) {  // tile record and tile-rectangle area of record v
        const uint4 rc = rect[v];
        area_out[g] = ((rc.x >> 16) - (rc.x & 0xFFFFu) + 1) * ((rc.y >> 16) - (rc.y & 0xFFFFu) + 1);
        rect_out[g] = rc;
      }
    }
  }
}

// 3. List bounds from the sorted tile ids: the first entry of a tile writes
// its start, the last one its end (into tile_count, turned into the length
// by k_tile_classify).  Both arrays are zeroed by the forward beforehand.
// Each thread takes four consecutive ids with one 16-byte load.
__global__ void k_tile_bounds(Ws ws, Sizes sz, const uint32_t *__restrict__ tiles) {
  if (ws.scalars[kOverflow]) return;
  const uint32_t n = min(ws.scalars[kNumPairs], sz.cap_pairs);
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; 4 * q < n; q += stride) {
    const uint32_t i0 = 4 * q;
    uint32_t t[6];
    t[0] = i0 > 0 ? tiles[i0 - 1] : 0xFFFFFFFFu;
    if (i0 + 4 <= n) {
      const uint4 v = *reinterpret_cast<const uint4 *>(tiles + i0);  // i0 is a multiple of 4
      t[1] = v.x; t[2] = v.y; t[3] = v.z; t[4] = v.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) t[1 + k] = i0 + k < n ? tiles[i0 + k] : 0xFFFFFFFFu;
    }
    t[5] = i0 + 4 < n ? tiles[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
      const uint32_t i = i0 + (uint32_t)k - 1;
      if (i >= n) break;
      const uint32_t tl = t[k];
      if (tl >= sz.t_tot) {
        ws.scalars[kOverflow] = 3u;
        continue;
      }
      if (t[k - 1] != tl) ws.tile_start[tl] = i;
      if (t[k + 1] != tl) ws.tile_count[tl] = i + 1;
    }
  }
}

// Per tile: the list length, the longest-first key and the number of lists
// of at least long_list entries (counted once per wave).
__global__ __launch_bounds__(256) void k_tile_classify(Ws ws, Sizes sz, uint32_t *__restrict__ order_keys,
                                                       uint32_t *__restrict__ order_vals) {
  if (ws.scalars[kOverflow]) return;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < sz.t_tot;
  uint32_t n = 0;
  if (valid) {
    const uint32_t end = ws.tile_count[t];
    n = end ? end - ws.tile_start[t] : 0u;
    ws.tile_count[t] = n;
    order_keys[t] = length_key(n);
    order_vals[t] = t;
  }
  (void)wave_atomic_inc(ws.scalars + kNumLong, valid && n >= sz.long_list);
}

namespace {

constexpr uint32_t kScanOneMax = 1u << 16;  // scans up to this length take one workgroup
constexpr uint32_t kScanFusedMax = 1024;    // chunks up to which each adds up the totals before it

// Exclusive scan of len words in place, part holding ceil(len / 4096) words.
void scan_words(uint32_t *data, uint32_t len, uint32_t *part, hipStream_t st) {
  if (len == 0) return;
  if (len <= kScanOneMax) {
    k_scan_one<<<1, 1024, 0, st>>>(data, len);
    return;
  }
  const uint32_t nb = (len + kScanChunk - 1) / kScanChunk;
  k_scan_reduce<<<nb, kScanNT, 0, st>>>(data, len, part);
  if (nb <= kScanFusedMax) {
    k_scan_down<true><<<nb, kScanNT, 0, st>>>(data, len, part);
    return;
  }
  k_scan_top<<<1, 1024, 0, st>>>(part, nb);
  k_scan_down<false><<<nb, kScanNT, 0, st>>>(data, len, part);
}

uint32_t rdx_chunk(uint32_t cap) { return cap >= kRdxBig ? kRdxNT * 32u : kRdxNT * 8u; }

// Digit widths of a counting sort over `bits` key bits: 8-bit passes, except
// that 17 to 20 bits take two passes of 9 or 10 bits rather than three.
int sort_passes(int bits, int widths[4]) {
  if (bits > 16 && bits <= 20) {
    widths[0] = widths[1] = (bits + 1) / 2;
    return 2;
  }
  const int passes = std::max(1, (bits + 7) / 8);
  for (int p = 0; p < passes; ++p) widths[p] = 8;
  return passes;
}

template <int IPL, int BITS>
void count_pass(const Ws &ws, uint32_t nblk, const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                uint32_t *vout, const uint32_t *count_dev, uint32_t cap, int shift, uint32_t *aout, uint4 *rout,
                hipStream_t st) {
  k_digit_hist<IPL, BITS><<<nblk, kRdxNT, 0, st>>>(ws.scalars, kin, count_dev, cap, shift, ws.radix_hist);
  scan_words(ws.radix_hist, (1u << BITS) * nblk, ws.scan_part, st);
  k_digit_scatter<IPL, BITS><<<nblk, kRdxNT, 0, st>>>(ws.scalars, kin, vin, kout, vout, count_dev, cap, shift,
                                                      ws.radix_hist, ws.rec_rect, aout, rout);
}

// Stable sort of `cap` items, of which *count_dev (all if NULL) are live, by
// the low `bits` bits of their keys.  Input (k0, v0; v0 = NULL: values are
// the indices); pass p writes (kb, vb) for even p and (ka, va) for odd p,
// the last pass (out_k, out_v), which must not be its own input.  (ka, va)
// may be the input itself.  With area_out the last pass also writes the
// tile-rectangle areas of the (record) values, and their tile records to
// rect_out, in sorted order.
void counting_sort(const Ws &ws, const uint32_t *count_dev, uint32_t cap, int bits, const uint32_t *k0,
                   const uint32_t *v0, uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, uint32_t *out_k,
                   uint32_t *out_v, uint32_t *area_out, uint4 *rect_out, hipStream_t st) {
  const uint32_t chunk = rdx_chunk(cap);
  const uint32_t nblk = std::max<uint32_t>((cap + chunk - 1) / chunk, 1u);
  int widths[4];
  const int passes = sort_passes(bits, widths);
  const uint32_t *kin = k0, *vin = v0;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    uint32_t *kout = last ? out_k : (p % 2 == 0 ? kb : ka);
    uint32_t *vout = last ? out_v : (p % 2 == 0 ? vb : va);
    uint32_t *aout = last ? area_out : nullptr;
    uint4 *rout = last ? rect_out : nullptr;
    const bool big = chunk == kRdxNT * 32u;
    switch (widths[p] * 2 + (big ? 1 : 0)) {
      case 16: count_pass<8, 8>(ws, nblk, kin, vin, kout, vout, count_dev, cap, shift, aout, rout, st); break;
      case 17: count_pass<32, 8>(ws, nblk, kin, vin, kout, vout, count_dev, cap, shift, aout, rout, st); break;
      case 18: count_pass<8, 9>(ws, nblk, kin, vin, kout, vout, count_dev, cap, shift, aout, rout, st); break;
      case 19: count_pass<32, 9>(ws, nblk, kin, vin, kout, vout, count_dev, cap, shift, aout, rout, st); break;
      case 20: count_pass<8, 10>(ws, nblk, kin, vin, kout, vout, count_dev, cap, shift, aout, rout, st); break;
      default: count_pass<32, 10>(ws, nblk, kin, vin, kout, vout, count_dev, cap, shift, aout, rout, st); break;
    }
    shift += widths[p];
    kin = kout;
    vin = vout;
  }
}

int bit_width(uint32_t x) { return x == 0 ? 0 : 32 - __builtin_clz(x); }

}  // namespace

// Records by depth bits (four passes): the last pass reads rec_tmp[2..3]
// and writes the order to rec_tmp[0..1] (record indices in rec_tmp[1]), the
// records' tile-rectangle areas to rec_tmp[4] and their tile records to the
// start of the backward's partials (free until the tile sort, at least 48
// bytes per record), so that the emission reads them in order.
void launch_depth_sort(const Ws &ws, const Sizes &sz, hipStream_t st) {
  if (sz.cap_rec == 0) return;
  uint32_t *q[5];
  for (int k = 0; k < 5; ++k) q[k] = ws.rec_tmp + (size_t)k * sz.cap_rec;
  counting_sort(ws, ws.scalars + kNumRecords, sz.cap_rec, 32, ws.rec_zbits, nullptr, q[0], q[1], q[2], q[3], q[0],
                q[1], q[4], reinterpret_cast<uint4 *>(ws.partials), st);
}

void launch_binning(const ViewInfo *views, const Ws &ws, const Sizes &sz, hipStream_t st) {
  if (sz.t_tot == 0) return;
  const uint32_t *perm = ws.rec_tmp + sz.cap_rec;
  // areas -> pair offsets; entries past the live records are stale, which
  // affects no offset of a live record (an exclusive scan looks back only)
  uint32_t *offs = ws.rec_tmp + 4 * (size_t)sz.cap_rec;
  scan_words(offs, sz.cap_rec, ws.scan_part, st);
  // (tile, record) ping-pong in pairs_tmp and in the backward's partials
  // (unused until the backward runs)
  uint32_t *ka = ws.pairs_tmp, *va = ka + sz.cap_pairs;
  uint32_t *kb = reinterpret_cast<uint32_t *>(ws.partials), *vb = kb + sz.cap_pairs;
  const uint32_t waves = (sz.cap_rec + kWave - 1) / kWave;
  const uint32_t blocks = std::min<uint32_t>((waves + 3) / 4, 8192u);
  // the tile records in depth order, written by the depth sort's last pass
  const uint4 *srect = reinterpret_cast<const uint4 *>(ws.partials);
  k_emit<<<std::max(blocks, 1u), 256, 0, st>>>(ws, sz, perm, srect, offs, ka, va);
  const int bits = std::max(1, bit_width(sz.t_tot - 1));
  int widths[4];
  const int passes = sort_passes(bits, widths);
  // the last pass reads (kb, vb) when the pass count is even, else (ka, va)
  uint32_t *sorted_tiles = (passes % 2 == 1) ? kb : ka;
  counting_sort(ws, ws.scalars + kNumPairs, sz.cap_pairs, bits, ka, va, ka, va, kb, vb, sorted_tiles, ws.tile_recs,
                nullptr, nullptr, st);
  const uint32_t bb = std::min<uint32_t>((sz.cap_pairs + 255) / 256, 16384u);
  k_tile_bounds<<<std::max(bb, 1u), 256, 0, st>>>(ws, sz, sorted_tiles);
  uint32_t *ok = ws.tile_tmp, *ov = ok + sz.t_tot, *ok2 = ov + sz.t_tot, *ov2 = ok2 + sz.t_tot;
  k_tile_classify<<<(sz.t_tot + 255) / 256, 256, 0, st>>>(ws, sz, ok, ov);
  // longest list first: one pass over the 8-bit length codes
  counting_sort(ws, nullptr, sz.t_tot, 8, ok, ov, ok, ov, ok2, ov2, ok2, ws.tile_order, nullptr, nullptr, st);
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

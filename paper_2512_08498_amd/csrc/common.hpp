// Shared device/host definitions of the rasterizer: camera and per-view
// tables, workspace pointers, and the constants of the image model.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsr {

// Mirrors gsr_camera (72 bytes).
struct Cam {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t w, h;
};
static_assert(sizeof(Cam) == 72, "camera layout");

// Per-view tile table fixed by the plan.
struct ViewInfo {
  int32_t w, h;          // image size
  int32_t tiles_x, tiles_y;
  uint32_t tile_base;    // first global tile id of the view
  uint32_t pix_off;      // first pixel of the view in the flat outputs
  uint32_t pad[2];
};

// Scalars the kernels exchange through device memory.
enum Scalar : int {
  kNumRecords = 0,    // visible (view, Gaussian) records
  kNumPairs = 1,      // (record, tile) pairs
  kOverflow = 2,      // nonzero: capacity exceeded; later stages skip their work
  kNumLong = 7,       // 16 px tiles with a long list (a prefix of tile_order)
  kNumScalars = 16
};

// Workspace arrays (device pointers into the caller's workspace).
struct Ws {
  uint32_t *scalars;        // [kNumScalars]              zeroed per forward
  uint32_t *queues;         // [2][kQueueLanes][kQueueStride] compositing work queues (forward, backward),
                            //                            zeroed per forward
  uint32_t *tile_count;     // [T_tot] list length        zeroed per forward
  uint32_t *tile_start;     // [T_tot] list start         zeroed per forward
  uint2 *block_sums;        // [n_blocks] (records, pairs) -> exclusive offsets
  uint64_t *vis_mask;       // [vis_words][n] visible views of each Gaussian (bit v % 64 of word v / 64)
  uint32_t *rec_start;      // [n + 1] first record of each Gaussian
  float4 *rec_payload;      // [cap_rec][4] raster payload, see RecPayload
  uint32_t *rec_g;          // [cap_rec] Gaussian index
  uint32_t *rec_view;       // [cap_rec] view index
  uint32_t *rec_pairoff;    // [cap_rec] first gradient slot of the record (records in order, tiles row-major)
  uint4 *rec_rect;          // [cap_rec] (tx0 | tx1 << 16, ty0 | ty1 << 16, global id of tile (tx0, ty0),
                            //   tiles per row of the view): one 16-byte line part per record
  uint32_t *rec_zbits;      // [cap_rec] depth bits
  uint32_t *rec_tmp;        // [5][cap_rec] depth sort of the records, pair offsets
  uint32_t *tile_order;     // [T_tot] tiles by decreasing list length
  uint32_t *tile_tmp;       // [4][T_tot] keys and values of the tile-order sort
  uint32_t *radix_hist;     // [radix][blocks] digit histograms of the counting passes (radix <= 1024)
  uint32_t *scan_part;      // chunk sums of the device-wide scans
  uint32_t *pairs_tmp;      // [2][cap_pairs] tile ids and records of the tile sort
  uint32_t *tile_recs;      // [cap_pairs] record list of every tile, in depth order
  float *partials;          // [cap_pairs][9] backward partial gradients per pair, 36 bytes each
  float4 *g2d;              // [cap_rec][3] per-record reduced gradients
  float *loss_partials;     // [kLossBlocks]
};

struct Sizes {
  int64_t n;
  int32_t n_views;
  int32_t sh_k;
  int32_t ts;
  uint32_t t_tot;
  uint32_t cap_rec;
  uint32_t cap_pairs;
  uint32_t n_blocks;        // ceil(n / kPreBlock)
  uint32_t long_list;       // 16 px tiles: lists this long are walked by four waves in the backward
  uint32_t persistent;      // compositing: 1 = persistent workgroups over a work queue (ItemQueue)
  uint32_t vis_words;       // ceil(n_views / 64)
  float bg[3];
};

constexpr int kPreBlock = 256;     // Gaussians per preprocess workgroup
constexpr int kQueueLanes = 8;     // counters per work queue: one per XCD
constexpr int kQueueStride = 32;   // words between counters (one 128-byte line each)
constexpr int kLossBlocks = 2048;  // loss reduction partials

// Image-model constants (float32 bit patterns written as hex literals).
constexpr float kNearZ = 0x1.99999ap-3f;       // 0.2
constexpr float kDilation = 0x1.333334p-2f;    // 0.3
constexpr float kSupportK = 0x1.62a4a8p+3f;    // 11.0826 >= 2 ln 255
constexpr float kClampFov = 0x1.4cccccp+0f;    // 1.3
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kLog2e = 0x1.715476p+0f;
constexpr float kHalfLog2e = 0x1.715476p-1f;   // log2(e) / 2

// Raster payload of one record, four float4 (64 bytes, staged in LDS by the
// compositing kernels):
//  p0 = (i0, i1, j0, j1)            inclusive pixel box the compositing tests,
//                                   as floats: the binning box narrowed to
//                                   d^2 <= 2 ln(255 opacity) (empty if the
//                                   opacity is below 1/255)
//  p1 = (offx, offy, qa, qb)        mean offset from that box's corner; conic
//  p2 = (qc, opacity, r, g)         in Cholesky form (see raster.hpp)
//  p3 = (b, i0 | i1 << 16, j0 | j1 << 16, pass)   the binning box, as packed
//                                   16-bit integers, and bits 0..2 set where
//                                   colour channel ch was not clamped at 0
//                                   (bit patterns)
// offx = mu'_x - i0 - 0.5, so dx = (px - i0) - offx is the centre offset of
// pixel px, exact up to the rounding of offx.

}  // namespace gsr

// Shared by the forward and backward blend kernels: tile/lane geometry, the XCD-aware tile
// order and wave64 reductions through DPP (no LDS crossbar traffic).
#pragma once

#include "project.h"

namespace flod {

constexpr int kXcds = 8;
constexpr int kBlendThreads = 64;                          // one wave64 per 16x16 tile
constexpr int kPix = (kTile * kTile) / kBlendThreads;      // 4 pixels per lane
constexpr int kRowStep = kBlendThreads / kTile;            // lane rows 0..3, then +4, +8, +12
constexpr int kBatch = 256;                                // list entries staged in LDS at once

// Tile of workgroup `bid`. Workgroups go to the 8 XCDs round-robin (XCD = bid % 8); XCD x
// takes the tile rows r with r % 8 == x, each row left to right. Every XCD so gets an even
// share of the frame (the work concentrates in its middle rows: contiguous blocks of rows per
// XCD left one XCD with 1.4-1.5x the mean list length at 1080p), and the tiles it holds in
// flight are horizontal neighbours that share Gaussians in its L2. Returns -1 for the padding
// workgroups of the last row group.
__device__ __forceinline__ int xcd_tile(int bid, int tiles_x, int tiles_y) {
  const int x = bid % kXcds, j = bid / kXcds;
  const int row = x + kXcds * (j / tiles_x);
  return row < tiles_y ? row * tiles_x + j % tiles_x : -1;
}

// Workgroups that xcd_tile() maps onto every tile of a tiles_x x tiles_y grid.
inline int xcd_grid(int tiles_x, int tiles_y) { return kXcds * tiles_x * ((tiles_y + kXcds - 1) / kXcds); }

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_or_zero(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, true));
}

// Sum over the 16 lanes of each DPP row; every lane of the row receives its row's sum.
__device__ __forceinline__ float row_sum16(float x) {
  x += dpp_or_zero<0xB1>(x);         // quad_perm [1,0,3,2]
  x += dpp_or_zero<0x4E>(x);         // quad_perm [2,3,0,1]
  x += dpp_or_zero<0x141>(x);        // row_half_mirror
  x += dpp_or_zero<0x140>(x);        // row_mirror
  return x;
}


}  // namespace flod

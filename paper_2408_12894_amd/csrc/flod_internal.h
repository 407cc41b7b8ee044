// Internal declarations shared by the kernels and the host orchestration of libflod.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/flod.h"

namespace flod {

constexpr int kTile = FLOD_TILE;          // 16x16 pixel tiles
constexpr int kBlock = 256;               // threads per workgroup (4 wave64)
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;   // 256 buckets per radix pass
constexpr int kSortItems = 12;            // keys per thread in a radix pass (measured 8 / 12 / 16)
constexpr int kSortTile = kBlock * kSortItems;   // 3072 keys per workgroup
constexpr int kSortItemsSmall = 8;        // 2048-key workgroups for sorts below kRadixBigSort (2 / 4 / 8)
constexpr int64_t kRadixBigSort = 4 << 20;
constexpr int kSortItemsHuge = 16;        // 4096-key workgroups for sorts of kRadixHugeSort keys or more
constexpr int64_t kRadixHugeSort = 32 << 20;
constexpr size_t kGaussianBytes = (3 + 3 + 4 + 1 + FLOD_SH_COEFFS * 3) * 4;   // 236 B per stored Gaussian
constexpr unsigned long long kPruneMaxScan = 1ull << 36;   // overlap-pruning neighbour-scan limit

// Rasterizer conventions (3DGS framework): near plane, EWA dilation, Jacobian clamp at 1.3x the half field of view, alpha clamp, alpha floor,
// transmittance floor, support cut q <= 9.
constexpr float kNearZ = 0.2f;
constexpr float kDilate = 0.3f;
constexpr float kFovClamp = 1.3f;
// Depth key of a candidate that is not rendered (culled or not selected): above every FP32
// depth bits of a positive depth, and skipped by the depth sort's first pass.
constexpr uint32_t kDepthNone = 0xFFFFFFFFu;
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kQCut = 9.0f;
constexpr double kNearZD = 0.2;
constexpr double kDilateD = 0.3;
constexpr double kFovClampD = 1.3;

struct DevCamera {
  float R[9], t[3], campos[3];
  float fx, fy, cx, cy;
  int W, H, tiles_x, tiles_y;
};

struct DevLevel {
  const float *means, *log_scales, *quats, *logits, *sh;
  int64_t offset, n;
  float s_min;
  float lo2, hi2;     // eq. 6 band, squared; used only when selecting
};

struct PreParams {
  DevLevel lv[FLOD_MAX_LEVELS];
  int n_levels;
  int select;
  int sh_degree;
  float logit_min;    // opacity cull: logit < logit_min  <=>  opacity < 1/255
  float centre[3];
  DevCamera cam;
  int64_t n_total;
};

// Per-candidate outputs of the preprocess (structure of arrays).
struct PreOut {
  float4 *xyab;       // mu'x, mu'y, conic a, conic b
  float4 *cop;        // conic c, opacity, red, green
  float2 *blue;       // blue, packed bf16 residuals of mu' (bits)
  uint32_t *depth;    // FP32 bits of the view-space depth
  float4 *bin;        // binning record, two per candidate: (mu'x, mu'y, conic a, conic b) and
                      // (conic c, support bound Q_g, bits of x0 | y0 << 16, bits of x1 | y1 << 16)
  uint32_t *tiles;    // tiles touched, 0 when culled or not selected
  uint32_t *block_vis;  // per-workgroup count of visible candidates
  uint32_t *zero_sums;  // one word per workgroup, zeroed (the depth sort's tile-count sums; may be null)
  unsigned long long *n_selected;   // per-level selected counts (may be null)
  float4 *shjac;      // three planes of n_total float4, per visible candidate the colour's Jacobian in
                      // the unit view direction, J[ch][a] row-major, then the three colours before the
                      // clamp (J00 J01 J02 J10 | J11 J12 J20 J21 | J22 c0 c1 c2); may be null
};

// One attribute array of a level in an Adam step: parameter, gradient and the two moment
// arrays (same length), its first float4 slot in the launch and its learning rate.
struct AdamSeg {
  float *p;
  const float *g;
  float *m, *v;
  int64_t len;      // floats
  int64_t first4;   // first float4 slot of the segment
  float lr;         // for the SH segment: the degree-0 rate
  int vec;          // all four arrays 16-byte aligned
};

struct AdamArgs {
  AdamSeg seg[5];   // means, log_scales, quats, opacity logits, SH
  float lr_sh_rest;
  float b1, b2, omb1, omb2;   // beta1, beta2, 1 - beta1, 1 - beta2
  float inv_bc1, inv_bc2;     // 1 / (1 - beta^t), formed in FP64 and rounded once
  float eps;
  int64_t total4;
};

// Counters in device memory (one small array per context).
enum : int {
  kCntVisible = 0,      // u32 count of visible candidates
  kCntInstances = 1,    // u32 count of instances; 0 when it exceeds the instance buffers
  kCntTotal64 = 2,      // u64 scratch for totals (two u32 slots: 2, 3)
  kCntSlots = 8
};

// ---- launches (each file defines its own) ----
hipError_t launch_preprocess(const PreParams &p, const PreOut &o, hipStream_t s);
hipError_t launch_scan_blocks(const uint32_t *in, const uint32_t *n_items, int items_per_block,
                              unsigned long long *prefix, uint32_t *total32,
                              unsigned long long *total64, int max_blocks, hipStream_t s,
                              unsigned long long cap32 = 0xFFFFFFFFull, unsigned long long *host_out = nullptr,
                              uint32_t host_seq = 0);
int radix_items(int64_t n_max);        // keys per thread the radix sort of n_max keys uses
size_t radix_hist_bytes(int64_t n_max);  // bytes of each of its hist and scan arrays
// With tiles_of (tile count per value), the last pass also writes tiles_out[pos] =
// tiles_of[sorted value] and adds the counts into block_sum[pos / 256] (zeroed beforehand).
// With first_keys, the first pass reads first_keys[0, n_max) instead of keys[0] and vals[0],
// takes each key's index as its value and skips keys equal to kDepthNone; it writes the count
// it kept to *n_ptr, which the later passes read.
hipError_t launch_radix_sort(uint32_t *keys[2], uint32_t *vals[2], uint32_t *n_ptr,
                             int64_t n_max, int bits, uint32_t *hist, uint32_t *scan,
                             uint32_t *tot, int *result_buf, hipStream_t s, const uint32_t *tiles_of = nullptr,
                             uint32_t *tiles_out = nullptr, uint32_t *block_sum = nullptr,
                             const uint32_t *first_keys = nullptr);
hipError_t launch_emit(const uint32_t *sorted_ids, const uint32_t *n_ptr, const uint32_t *k_ptr,
                       int64_t n_max, int64_t k_max, const uint32_t *sorted_tiles, const float4 *bin,
                       const unsigned long long *prefix, int tiles_x, int tiles_y, uint32_t *tile_ids,
                       uint32_t *values, uint2 *ranges, hipStream_t s);   // also zeroes ranges
// zeroed: ranges already zeroed (by the emission); otherwise zeroed here first
hipError_t launch_ranges(const uint32_t *tile_ids, const uint32_t *k_ptr, int64_t k_max, int n_tiles,
                         uint2 *ranges, bool zeroed, hipStream_t s);
// blended: per tile, the (list position, Gaussian) pairs of the entries the forward blended
// into some pixel, in list order at the start of the tile's range; tile_blended: their count
// (both may be null: the render keeps no backward state)
hipError_t launch_blend(const uint2 *ranges, const uint32_t *values, const float4 *xyab,
                        const float4 *cop, const float2 *blue, const DevCamera &cam,
                        const float bg[3], float *image, float *final_T, int32_t *n_contrib,
                        int32_t *n_blended, uint2 *blended, uint32_t *tile_blended, const uint32_t *order,
                        hipStream_t s);
// order: n_tiles + 2 words of scratch (the backward's tile order and its counts of split tiles);
// g2d: the n_g2d floats of gradient sums, zeroed here first; the kernel is timed by the events
// (if given), its tile order and the zeroing are not
hipError_t launch_blend_bwd(const uint2 *ranges, const float4 *xyab, const float4 *cop, const float2 *blue,
                            const DevCamera &cam, const float bg[3], const float *final_T,
                            const int32_t *n_contrib, const float *dL_dimage, float *g2d, int64_t n_g2d,
                            const uint2 *blended, const uint32_t *tile_blended, uint32_t *order,
                            hipStream_t s, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// the most blocks the backward's split tiles add beyond one per tile
int bwd_split_extra(int n_tiles);
hipError_t launch_tile_order_by_length(const uint2 *ranges, int n_tiles, uint32_t *order, hipStream_t s);
// The blend backward's per-Gaussian moment sums into dL/d(mu', conic) in place (inspection).
hipError_t launch_g2d_from_moments(int64_t n, const uint32_t *tiles, const float4 *xyab, const float4 *cop,
                                   float *g2d, hipStream_t s);
// shjac: the forward preprocess's Jacobians and pre-clamp colours (PreOut::shjac)
hipError_t launch_preprocess_bwd(const PreParams &p, const uint32_t *tiles, const float *g2d,
                                 const float4 *shjac, const flod_grads &g, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_select_count(const float *means, int64_t n, const float centre[3], float lo2, float hi2,
                               uint32_t *block_cnt, hipStream_t s);
hipError_t launch_select_copy(const flod_level &in, const float centre[3], float lo2, float hi2,
                              const unsigned long long *prefix, const flod_level &out, hipStream_t s);
hipError_t launch_mask_count(const uint8_t *mask, int64_t n, uint32_t *block_cnt, hipStream_t s);
hipError_t launch_mask_copy(const flod_level &in, const uint8_t *mask, const unsigned long long *prefix,
                            const flod_level &out, hipStream_t s);
hipError_t launch_level_transition(const flod_level &in, float s_min_next, const flod_level &out, hipStream_t s);
hipError_t launch_adam(const AdamArgs &a, hipStream_t s);
int64_t ssim_blocks(int C, int H, int W);   // workgroups (and loss partials) of the SSIM kernels
hipError_t launch_ssim_forward(const float *x, const float *y, int C, int H, int W, float lam, double *loss,
                               float *gmap, double2 *partials, hipStream_t s);
hipError_t launch_ssim_backward(const float *x, const float *y, int C, int H, int W, float lam, const float *gmap,
                                const double *dloss, float *dx, hipStream_t s);
int64_t l1_blocks();   // workgroups (and loss partials) of the L1 forward
hipError_t launch_l1_forward(const float *x, const float *y, int64_t n, double *loss, double2 *partials,
                             hipStream_t s);
hipError_t launch_l1_backward(const float *x, const float *y, int64_t n, const double *dloss, float *dx,
                              hipStream_t s);
int prune_table_bits(int64_t n);   // log2 of the overlap-pruning hash table size for n points
hipError_t launch_prune_keys(const float *means, int64_t n, float d_op, uint32_t *keys, uint32_t *vals,
                             hipStream_t s);
hipError_t launch_prune_gather(const float *means, const uint32_t *sorted_vals, int64_t n, float4 *pts,
                               hipStream_t s);
hipError_t launch_prune_cost(const float4 *pts, const uint2 *ranges, int64_t n, float d_op,
                             unsigned long long *cost, hipStream_t s);
hipError_t launch_prune_query(const float4 *pts, const uint2 *ranges, int64_t n, float d_op, uint8_t *keep,
                              double *d_avg, hipStream_t s);

}  // namespace flod

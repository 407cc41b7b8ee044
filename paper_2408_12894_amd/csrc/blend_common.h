// Shared by the forward and backward blend kernels: the staged list entry and the
// longest-first tile orders.
#pragma once

#include "project.h"

namespace flod {

constexpr int kBatch = 256;                                // list entries staged in LDS at once

// A list entry as both blend kernels stage it in LDS, decoded once per entry instead of in
// every lane: (mu'x - x0, mu'y - y0, r = b / c, k det / c), (k c, log2 o, red, green) and
// (the threshold on l = k q + log2 o, blue, 1 when the opacity exceeds kClampOpacity, 0), with
// k = kExpScale (the completed square of q, see conic_stage) and (x0, y0) the tile's corner.
// The mean relative to the corner is the FP32 mean minus the corner (exact while the two are
// within a factor of two, otherwise rounded to the difference's ulp) plus the bf16 residual of
// mu': a pixel's offsets from the mean are then one subtraction from its tile-local centre,
// (px - x0) + 1/2. Every float4 holds values the decision needs, so that each is read whole
// before it and a blending pixel finds its colour in registers (a colour read only by
// blending pixels would make each of them wait for LDS).
//
// An opacity up to kClampOpacity cannot reach the 0.99 clamp: q >= 0 gives l <= log2 o, so
// 2^l <= o (1 + a few ulp) < 0.99; such entries take alpha = 2^l without the clamp where that
// saves work (the backward's decision).
constexpr float kClampOpacity = 0.98f;

__device__ __forceinline__ void stage_entry(const float4 *xyab, const float4 *cop, const float2 *blue, uint32_t g,
                                            int x0, int y0, float4 &a, float4 &b, float4 &c) {
  const float4 A = xyab[g];
  const float2 BL = blue[g];
  const uint32_t lo = __float_as_uint(BL.y);
  const float4 C = cop[g];
  // the decision: q <= 9 and o exp(-q/2) >= 1/255, i.e. l >= max(log2(1/255), 9 k + log2 o)
  const float l2o = log2f(C.y);
  const float thr = fmaxf(kLog2AlphaMin, kQCutScaled + l2o);
  float r, ek, ck;
  conic_stage(A.z, A.w, C.x, r, ek, ck);
  a = make_float4((A.x - (float)x0) + mu_lo_x(lo), (A.y - (float)y0) + mu_lo_y(lo), r, ek);
  b = make_float4(ck, l2o, C.z, C.w);
  c = make_float4(thr, BL.x, C.y > kClampOpacity ? 1.0f : 0.0f, 0.0f);
}

// Tile orders, longest first (LPT order). The blend kernels' cost per tile varies by orders of
// magnitude between tiles; dispatched in frame order, tiles with much work often started last
// and a kernel ended in a long ramp with most wave slots idle. The forward orders its tiles by
// list length, the backward by the entries the forward blended into some pixel of the tile
// (the entries it processes). One workgroup: a histogram over 256 buckets of the cost (8 per
// octave), descending bucket offsets, then a scatter; the order inside a bucket is whatever
// the LDS atomics give, which changes only the schedule, never a result. Consecutive
// workgroups go to different XCDs (round-robin), so every XCD receives an even share.
// For the backward (split.cap2 >= 0) it also writes, at order[n] and order[n + 1], how many tiles
// lead the order with a cost in a bucket above that of split.f2 (respectively split.f4) times
// the mean cost, at most split.cap2 (split.cap4 <= split.cap2); none for a factor <= 0: the
// tiles the backward splits between two and between four waves.
struct TileSplit {
  float f2, f4;
  int cap2, cap4;
};
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 256;
constexpr int kOrderLoads = 8;

__device__ __forceinline__ int cost_bucket(uint32_t c) {
  if (c < 8u) return (int)c;
  const int e = 31 - __clz(c);                     // c in [2^e, 2^(e+1)), e >= 3
  const int m = (int)((c >> (e - 3)) & 7u);        // next three bits
  return min(kOrderBuckets - 1, 8 + (e - 3) * 8 + m);
}

struct ListLengthCost {   // forward: entries in the tile's list
  const uint2 *ranges;
  __device__ __forceinline__ uint32_t operator()(int t) const { return ranges[t].y - ranges[t].x; }
};

struct CountCost {        // backward: entries the forward blended somewhere in the tile
  const uint32_t *count;
  __device__ __forceinline__ uint32_t operator()(int t) const { return count[t]; }
};

// The tile order as one workgroup of kOrderThreads threads (the body of k_tile_order, which
// the backward also runs beside other work in one launch).
template <class Cost>
__device__ __forceinline__ void tile_order(Cost cost, int n, uint32_t *__restrict__ order, TileSplit split) {
  constexpr int W = kOrderThreads / 64;
  // per-wave bucket counts (contention only inside a wave), then per (bucket, wave) offsets
  __shared__ uint32_t s_cnt[W][kOrderBuckets];
  __shared__ uint32_t s_wsum[kOrderBuckets / 64];
  __shared__ unsigned long long s_csum[W];
  __shared__ uint32_t s_split[2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int k = tid; k < W * kOrderBuckets; k += kOrderThreads) (&s_cnt[0][0])[k] = 0u;
  if (tid < 2) s_split[tid] = 0u;
  __syncthreads();
  const int chunk = (n + W - 1) / W;
  const int t0 = w * chunk, t1 = min(n, t0 + chunk);
  // kOrderLoads costs per lane loaded before any is used (one loop trip at 1080p: each wave
  // takes at most 512 tiles there), the indices clamped into the wave's range rather than
  // guarded (a guard made each load a branch that waited for it); loaded one at a time, each
  // trip waited for its load
  unsigned long long csum = 0ull;
  for (int base = t0 + lane; base < t1; base += 64 * kOrderLoads) {
    uint32_t c[kOrderLoads];
#pragma unroll
    for (int u = 0; u < kOrderLoads; ++u) c[u] = cost(min(base + 64 * u, t1 - 1));   // in bounds: base < t1
#pragma unroll
    for (int u = 0; u < kOrderLoads; ++u)
      if (base + 64 * u < t1) {
        csum += c[u];
        atomicAdd(&s_cnt[w][cost_bucket(c[u])], 1u);
      }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) csum += __shfl_xor(csum, o, 64);
  if (lane == 0) s_csum[w] = csum;
  __syncthreads();
  // thread d < 256 takes bucket b = 255 - d (descending cost): its count over the waves, with
  // each wave's count replaced by the running sum before it
  uint32_t tot = 0u;
  if (tid < kOrderBuckets) {
    const int b = kOrderBuckets - 1 - tid;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const uint32_t c = s_cnt[k][b];
      s_cnt[k][b] = tot;
      tot += c;
    }
  }
  // exclusive scan of the bucket totals in descending bucket order (threads 0..255)
  uint32_t inc = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t x = __shfl_up(inc, o, 64);
    if (lane >= o) inc += x;
  }
  if (tid < kOrderBuckets && lane == 63) s_wsum[w] = inc;
  __syncthreads();
  if (tid < kOrderBuckets) {
    uint32_t base = inc - tot;
    for (int k = 0; k < w; ++k) base += s_wsum[k];
    const int b = kOrderBuckets - 1 - tid;
#pragma unroll
    for (int k = 0; k < W; ++k) s_cnt[k][b] += base;
    if (split.cap2 > 0) {
      // the tiles in the buckets above a threshold's lead the order: base + tot of the bucket
      // just above it
      unsigned long long total = 0ull;
#pragma unroll
      for (int k = 0; k < W; ++k) total += s_csum[k];
      const double mean = (double)total / (double)max(n, 1);
      const float fs[2] = {split.f2, split.f4};
      const int caps[2] = {split.cap2, split.cap4};
#pragma unroll
      for (int i = 0; i < 2; ++i)
        if (fs[i] > 0.0f && caps[i] > 0) {
          const int bthr = cost_bucket((uint32_t)fmin((double)fs[i] * mean, 4.0e9)) + 1;
          if (b == bthr) s_split[i] = min(base + tot, (uint32_t)caps[i]);
        }
    }
  }
  __syncthreads();
  for (int base = t0 + lane; base < t1; base += 64 * kOrderLoads) {
    uint32_t c[kOrderLoads];
#pragma unroll
    for (int u = 0; u < kOrderLoads; ++u) c[u] = cost(min(base + 64 * u, t1 - 1));   // in bounds: base < t1
#pragma unroll
    for (int u = 0; u < kOrderLoads; ++u)
      if (base + 64 * u < t1) order[atomicAdd(&s_cnt[w][cost_bucket(c[u])], 1u)] = (uint32_t)(base + 64 * u);
  }
  if (split.cap2 >= 0 && tid < 2) order[n + tid] = s_split[tid];
}

template <class Cost>
__global__ __launch_bounds__(kOrderThreads) void k_tile_order(Cost cost, int n, uint32_t *__restrict__ order,
                                                              TileSplit split) {
  tile_order(cost, n, order, split);
}

}  // namespace flod

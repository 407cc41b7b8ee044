// Whole-level operations on the resident stack.
//
// Compaction keeps a subset of a level's Gaussians, in index order, in caller-provided
// arrays. The subset is either the eq. 6 band around a fixed centre (the predetermined
// selection set, section Selective Rendering: rendering the compacted levels together gives
// the same image as selective rendering around that centre, while only the kept Gaussians
// stay resident and can be stored) or a per-Gaussian keep mask (overlap pruning, section
// Overlap Pruning). Two passes: per-workgroup counts, then (after a scan) a copy of the
// kept Gaussians' 59 attributes (236 bytes; the SH row as 12 dwordx4 loads and stores).
//
// The level transition (section Training Method, eq. 5) clones a trained level into the
// initial state of the next one with s_opt = log(s^(l) - s_min^(l+1)), so that the next
// level's eq. 4 scale starts equal to s^(l).
#include "project.h"

namespace flod {

struct BandKeep {
  const float *means;
  float c[3];
  float lo2, hi2;
  __device__ __forceinline__ bool operator()(int64_t i) const {
    const float d2 = dist2(means[i * 3 + 0], means[i * 3 + 1], means[i * 3 + 2], c);
    return (lo2 <= d2) && (d2 < hi2);
  }
};

struct MaskKeep {
  const uint8_t *mask;
  __device__ __forceinline__ bool operator()(int64_t i) const { return mask[i] != 0; }
};

template <class Keep>
__global__ __launch_bounds__(kBlock) void k_keep_count(Keep keep_of, int64_t n, uint32_t *block_cnt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool keep = (i < n) && keep_of(i);
  const int cnt = __syncthreads_count(keep);
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = (uint32_t)cnt;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ void copy_gaussian(const flod_level &in, int64_t i, const flod_level &out, int64_t o) {
  float *om = const_cast<float *>(out.means), *ol = const_cast<float *>(out.log_scales);
  for (int k = 0; k < 3; ++k) {
    om[o * 3 + k] = in.means[i * 3 + k];
    ol[o * 3 + k] = in.log_scales[i * 3 + k];
  }
  reinterpret_cast<float4 *>(const_cast<float *>(out.quats))[o] = reinterpret_cast<const float4 *>(in.quats)[i];
  const_cast<float *>(out.opacity_logits)[o] = in.opacity_logits[i];
  const float4 *src = reinterpret_cast<const float4 *>(in.sh + i * (FLOD_SH_COEFFS * 3));
  float4 *dst = reinterpret_cast<float4 *>(const_cast<float *>(out.sh) + o * (FLOD_SH_COEFFS * 3));
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = src[k];
}

template <class Keep>
__global__ __launch_bounds__(kBlock) void k_keep_copy(Keep keep_of, flod_level in,
                                                      const unsigned long long *prefix, flod_level out) {
  __shared__ uint32_t s_w[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool keep = (i < in.n) && keep_of(i);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t v = keep ? 1u : 0u;
  const uint32_t inc = wave_incl_scan_u32(v);
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int k = 0; k < w; ++k) base += s_w[k];
  if (!keep) return;
  copy_gaussian(in, i, out, (int64_t)(prefix[blockIdx.x] + base + inc - v));
}

static unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_select_count(const float *means, int64_t n, const float centre[3], float lo2, float hi2,
                               uint32_t *block_cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const BandKeep k{means, {centre[0], centre[1], centre[2]}, lo2, hi2};
  hipLaunchKernelGGL(k_keep_count<BandKeep>, dim3(grid_of(n)), dim3(kBlock), 0, s, k, n, block_cnt);
  return hipGetLastError();
}

hipError_t launch_select_copy(const flod_level &in, const float centre[3], float lo2, float hi2,
                              const unsigned long long *prefix, const flod_level &out, hipStream_t s) {
  if (in.n <= 0) return hipSuccess;
  const BandKeep k{in.means, {centre[0], centre[1], centre[2]}, lo2, hi2};
  hipLaunchKernelGGL(k_keep_copy<BandKeep>, dim3(grid_of(in.n)), dim3(kBlock), 0, s, k, in, prefix, out);
  return hipGetLastError();
}

hipError_t launch_mask_count(const uint8_t *mask, int64_t n, uint32_t *block_cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_keep_count<MaskKeep>, dim3(grid_of(n)), dim3(kBlock), 0, s, MaskKeep{mask}, n, block_cnt);
  return hipGetLastError();
}

hipError_t launch_mask_copy(const flod_level &in, const uint8_t *mask, const unsigned long long *prefix,
                            const flod_level &out, hipStream_t s) {
  if (in.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_keep_copy<MaskKeep>, dim3(grid_of(in.n)), dim3(kBlock), 0, s, MaskKeep{mask}, in, prefix,
                     out);
  return hipGetLastError();
}

// eq. 5, one thread per Gaussian. s^(l) is formed as the rasterizer's eq. 4 forms it (exp in
// FP64 rounded once to FP32, plus s_min^(l) in FP64); the logarithm is FP64, rounded to FP32.
// Arrays the output shares with the input (in-place transition) are not copied.
__global__ __launch_bounds__(kBlock) void k_level_transition(flod_level in, double s_min_l, double s_min_next,
                                                             flod_level out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= in.n) return;
  float *ol = const_cast<float *>(out.log_scales);
  for (int k = 0; k < 3; ++k) {
    const double s = (double)exp_rn1(in.log_scales[i * 3 + k]) + s_min_l;
    ol[i * 3 + k] = (float)log(s - s_min_next);
  }
  if (out.means != in.means) {
    float *om = const_cast<float *>(out.means);
    for (int k = 0; k < 3; ++k) om[i * 3 + k] = in.means[i * 3 + k];
  }
  if (out.quats != in.quats)
    reinterpret_cast<float4 *>(const_cast<float *>(out.quats))[i] = reinterpret_cast<const float4 *>(in.quats)[i];
  if (out.opacity_logits != in.opacity_logits) const_cast<float *>(out.opacity_logits)[i] = in.opacity_logits[i];
  if (out.sh != in.sh) {
    const float4 *src = reinterpret_cast<const float4 *>(in.sh + i * (FLOD_SH_COEFFS * 3));
    float4 *dst = reinterpret_cast<float4 *>(const_cast<float *>(out.sh) + i * (FLOD_SH_COEFFS * 3));
#pragma unroll
    for (int k = 0; k < 12; ++k) dst[k] = src[k];
  }
}

hipError_t launch_level_transition(const flod_level &in, float s_min_next, const flod_level &out, hipStream_t s) {
  if (in.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_transition, dim3(grid_of(in.n)), dim3(kBlock), 0, s, in, (double)in.s_min,
                     (double)s_min_next, out);
  return hipGetLastError();
}

}  // namespace flod

// Predetermined selection set (section Selective Rendering, predetermined Gaussian set):
// evaluate the eq. 6 band predicate once around a fixed centre and compact each level's
// kept Gaussians, in index order, into caller-provided arrays. Rendering the compacted
// levels together gives the same image as selective rendering around that centre, while
// only the kept Gaussians stay resident (and can be stored).
//
// Two passes per level: flags and per-workgroup counts, then (after a scan) a copy of the
// kept Gaussians' 59 attributes (236 bytes; the SH row as 12 dwordx4 loads and stores).
#include "project.h"

namespace flod {

__global__ __launch_bounds__(kBlock) void k_select_count(const float *means, int64_t n, float cx, float cy, float cz,
                                                         float lo2, float hi2, uint32_t *block_cnt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool keep = false;
  if (i < n) {
    const float c[3] = {cx, cy, cz};
    const float d2 = dist2(means[i * 3 + 0], means[i * 3 + 1], means[i * 3 + 2], c);
    keep = (lo2 <= d2) && (d2 < hi2);
  }
  const int cnt = __syncthreads_count(keep);
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = (uint32_t)cnt;
}

__device__ __forceinline__ uint32_t wave_incl_scan_sel(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__global__ __launch_bounds__(kBlock) void k_select_copy(flod_level in, float cx, float cy, float cz, float lo2,
                                                        float hi2, const unsigned long long *prefix, flod_level out) {
  __shared__ uint32_t s_w[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool keep = false;
  if (i < in.n) {
    const float c[3] = {cx, cy, cz};
    const float d2 = dist2(in.means[i * 3 + 0], in.means[i * 3 + 1], in.means[i * 3 + 2], c);
    keep = (lo2 <= d2) && (d2 < hi2);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t v = keep ? 1u : 0u;
  const uint32_t inc = wave_incl_scan_sel(v);
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int k = 0; k < w; ++k) base += s_w[k];
  if (!keep) return;
  const int64_t o = (int64_t)(prefix[blockIdx.x] + base + inc - v);
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

hipError_t launch_select_count(const float *means, int64_t n, const float centre[3], float lo2, float hi2,
                               uint32_t *block_cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_select_count, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, means, n,
                     centre[0], centre[1], centre[2], lo2, hi2, block_cnt);
  return hipGetLastError();
}

hipError_t launch_select_copy(const flod_level &in, const float centre[3], float lo2, float hi2,
                              const unsigned long long *prefix, const flod_level &out, hipStream_t s) {
  if (in.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_select_copy, dim3((unsigned)((in.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, in,
                     centre[0], centre[1], centre[2], lo2, hi2, prefix, out);
  return hipGetLastError();
}

}  // namespace flod

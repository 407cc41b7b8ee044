// Adam step over every attribute array of a level (section Training Method, Algorithm 1: the
// per-level training loop updates means, scale parameters s_opt, rotations, colours and
// opacities with Adam after each rasterize-and-backpropagate iteration).
//
// One launch covers the five arrays (59 floats per Gaussian) as consecutive segments of
// float4 slots; a thread updates one slot: reads parameter, gradient and both moments and
// writes parameter and moments (28 bytes per float: HBM-bound elementwise work). Slots whose
// four arrays are 16-byte aligned and fully inside the segment use dwordx4 accesses, the
// rest fall back to scalar ones.
#include "flod_internal.h"

namespace flod {

__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, float lr, const AdamArgs &a) {
  m = a.b1 * m + a.omb1 * g;
  v = a.b2 * v + a.omb2 * g * g;
  const float mh = m * a.inv_bc1;
  const float vh = v * a.inv_bc2;
  p -= lr * mh / (sqrtf(vh) + a.eps);
}

// SH segment: the first 3 floats of each Gaussian's 48 are the degree-0 coefficients.
__device__ __forceinline__ float seg_rate(const AdamArgs &a, int s, int64_t e) {
  if (s != 4) return a.seg[s].lr;
  return (e % (FLOD_SH_COEFFS * 3)) < 3 ? a.seg[4].lr : a.lr_sh_rest;
}

__global__ __launch_bounds__(kBlock) void k_adam(AdamArgs a) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= a.total4) return;
  int s = 0;
#pragma unroll
  for (int k = 1; k < 5; ++k) s += (q >= a.seg[k].first4) ? 1 : 0;
  const AdamSeg &S = a.seg[s];
  const int64_t e = (q - S.first4) * 4;
  if (S.vec && e + 4 <= S.len) {
    float4 p = *reinterpret_cast<const float4 *>(S.p + e);
    const float4 g = *reinterpret_cast<const float4 *>(S.g + e);
    float4 m = *reinterpret_cast<const float4 *>(S.m + e);
    float4 v = *reinterpret_cast<const float4 *>(S.v + e);
    adam_one(p.x, g.x, m.x, v.x, seg_rate(a, s, e + 0), a);
    adam_one(p.y, g.y, m.y, v.y, seg_rate(a, s, e + 1), a);
    adam_one(p.z, g.z, m.z, v.z, seg_rate(a, s, e + 2), a);
    adam_one(p.w, g.w, m.w, v.w, seg_rate(a, s, e + 3), a);
    *reinterpret_cast<float4 *>(S.p + e) = p;
    *reinterpret_cast<float4 *>(S.m + e) = m;
    *reinterpret_cast<float4 *>(S.v + e) = v;
    return;
  }
  for (int c = 0; c < 4 && e + c < S.len; ++c) {
    float p = S.p[e + c], m = S.m[e + c], v = S.v[e + c];
    adam_one(p, S.g[e + c], m, v, seg_rate(a, s, e + c), a);
    S.p[e + c] = p;
    S.m[e + c] = m;
    S.v[e + c] = v;
  }
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t s) {
  if (a.total4 <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((a.total4 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace flod

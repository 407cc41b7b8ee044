// Front-to-back alpha compositing (Preliminary section: eq. 2 and blending in depth order).
//
// One workgroup (256 threads = 4 wave64) per 16x16 tile, one pixel per thread. The tile's
// sorted list is consumed in batches of 256 entries staged in LDS (36 bytes per entry:
// mu', conic, opacity, colour); every lane reads the same entry (LDS broadcast). Per pixel:
//   q = d^T conic d (d = pixel centre - mu'); skip if q > 9 (3-sigma support)
//   alpha = min(0.99, o exp(-q/2)); skip if alpha < 1/255
//   stop (without blending) once T (1 - alpha) < 1e-4
//   C += alpha T c; T *= 1 - alpha
// The workgroup leaves the list as soon as all its pixels have stopped.
//
// Workgroup -> tile mapping is XCD-aware: workgroups are dispatched round-robin over the 8
// XCDs, so workgroup i is sent to tile (i % 8) * chunk + i / 8 and each XCD's L2 serves a
// contiguous band of tiles, which share most of their Gaussians.
#include "project.h"

namespace flod {

constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_tile(int bid, int n_tiles) {
  const int chunk = (n_tiles + kXcds - 1) / kXcds;
  return (bid % kXcds) * chunk + bid / kXcds;
}

__global__ __launch_bounds__(kBlock) void k_blend(const uint2 *__restrict__ ranges,
                                                  const uint32_t *__restrict__ values,
                                                  const float4 *__restrict__ xyab,
                                                  const float4 *__restrict__ cop,
                                                  const float *__restrict__ blue, int W, int H, int tiles_x,
                                                  int n_tiles, float bg0, float bg1, float bg2,
                                                  float *__restrict__ image, float *__restrict__ final_T,
                                                  int32_t *__restrict__ n_contrib) {
  __shared__ float4 s_a[kBlock];
  __shared__ float4 s_b[kBlock];
  __shared__ float s_c[kBlock];
  const int tile = xcd_tile(blockIdx.x, n_tiles);
  if (tile >= n_tiles) return;
  const int tid = threadIdx.x;
  const int px = (tile % tiles_x) * kTile + (tid & (kTile - 1));
  const int py = (tile / tiles_x) * kTile + (tid >> 4);
  const bool inside = px < W && py < H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const int n = (int)(rg.y - rg.x);
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  int last = 0;
  bool done = !inside;
  for (int start = 0; start < n; start += kBlock) {
    if (__syncthreads_and(done)) break;
    const int k = start + tid;
    if (k < n) {
      const uint32_t g = values[rg.x + k];
      s_a[tid] = xyab[g];
      s_b[tid] = cop[g];
      s_c[tid] = blue[g];
    }
    __syncthreads();
    const int cnt = min(kBlock, n - start);
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const float4 A = s_a[j];
        const float4 B = s_b[j];
        const float dx = fx - A.x, dy = fy - A.y;
        const float q = conic_q(A.z, A.w, B.x, dx, dy);
        if (q > kQCut) continue;
        const float alpha = fminf(kAlphaMax, B.y * __expf(-0.5f * q));
        if (alpha < kAlphaMin) continue;
        const float Tn = T * (1.0f - alpha);
        if (Tn < kTMin) {
          done = true;
          break;
        }
        const float wgt = alpha * T;
        C0 = fmaf(wgt, B.z, C0);
        C1 = fmaf(wgt, B.w, C1);
        C2 = fmaf(wgt, s_c[j], C2);
        T = Tn;
        last = start + j + 1;
      }
    }
  }
  if (inside) {
    const size_t pix = (size_t)py * W + px;
    const size_t plane = (size_t)W * H;
    image[pix] = fmaf(T, bg0, C0);
    image[plane + pix] = fmaf(T, bg1, C1);
    image[2 * plane + pix] = fmaf(T, bg2, C2);
    final_T[pix] = T;
    n_contrib[pix] = last;
  }
}

hipError_t launch_blend(const uint2 *ranges, const uint32_t *values, const float4 *xyab, const float4 *cop,
                        const float *blue, const DevCamera &cam, const float bg[3], float *image, float *final_T,
                        int32_t *n_contrib, hipStream_t s) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  const int grid = ((n_tiles + kXcds - 1) / kXcds) * kXcds;
  hipLaunchKernelGGL(k_blend, dim3(grid), dim3(kBlock), 0, s, ranges, values, xyab, cop, blue, cam.W, cam.H,
                     cam.tiles_x, n_tiles, bg[0], bg[1], bg[2], image, final_T, n_contrib);
  return hipGetLastError();
}

}  // namespace flod

// Front-to-back alpha compositing (Preliminary section: eq. 2 and blending in depth order).
//
// One workgroup per 16x16 tile with PPT pixels per thread: thread t owns the pixels
// (t % 16, t / 16 + (256 / PPT / 16) k), k < PPT, so each list entry staged in LDS is read
// once per thread and applied to PPT pixels. The tile's
// sorted list is consumed in batches of 256 entries (48 bytes each in LDS: mu' and its
// residual, conic, opacity, colour, decoded once per entry). Per pixel:
//   q = d^T conic d (d = pixel centre - mu', mu' = hi + lo); skip if q > 9 (evaluated as
//   k q in the completed-square form of conic_stage, k the scale of exp2)
//   alpha = min(0.99, o exp(-q/2)); skip if alpha < 1/255
//   stop (without blending) once T (1 - alpha) < 1e-4
//   C += alpha T c; T *= 1 - alpha
// T and the colours are FP32: T takes one rounding per blended contributor, so after m of
// them its relative error grows like sqrt(m) ulp (about 2e-6 at a thousand), far inside the
// relative 1e-4 margin around the stop threshold that the parity checks flag.
// The workgroup leaves the list as soon as all 256 pixels have stopped.
//
// Workgroups take the tiles in order of decreasing list length (k_tile_order). Each tile also
// lists the entries it blended into some pixel, the only ones its backward pass processes:
// (list position, Gaussian) pairs in list order at the start of the tile's range, and their
// count, from which the backward orders its tiles.
#include "blend_common.h"

namespace flod {

constexpr int kFwdPix = 1;

// Appends the entries of the staged batch at list position bstart that some pixel blended
// (s_taken) to the tile's list of blended entries (out, n_bl entries so far; the count is the
// same in every thread). Called by every thread of the workgroup after a barrier that follows
// the batch's walk; thread t handles the entries t, t + NT, ...
template <int NT>
__device__ __forceinline__ void append_blended(const uint8_t *s_taken, const uint32_t *s_id, uint32_t *s_wcnt,
                                               int bstart, int n, uint2 *out, uint32_t &n_bl, int tid) {
  constexpr int W = NT / 64;
  const int lane = tid & 63, w = tid >> 6;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int e0 = 0; e0 < kBatch; e0 += NT) {
    const int e = e0 + tid;
    const bool f = bstart + e < n && s_taken[e] != 0;
    const unsigned long long m = __ballot(f);
    if (lane == 0) s_wcnt[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t off = n_bl, tot = 0;
#pragma unroll
    for (int v = 0; v < W; ++v) {
      const uint32_t c = s_wcnt[v];
      off += v < w ? c : 0u;
      tot += c;
    }
    if (f) out[off + (uint32_t)__popcll(m & below)] = make_uint2((uint32_t)(bstart + e), s_id[e]);
    n_bl += tot;
    if (e0 + NT < kBatch) __syncthreads();   // s_wcnt is written again
  }
}

// COUNT: the caller wants each pixel's count of blended entries (n_blended); without it the
// walk does not count (one VALU fewer per blending wave and entry).
template <int PPT, bool COUNT>
__global__ __launch_bounds__(kTile * kTile / PPT) void k_blend(const uint2 *__restrict__ ranges,
                                                              const uint32_t *__restrict__ values,
                                                              const float4 *__restrict__ xyab,
                                                              const float4 *__restrict__ cop,
                                                              const float2 *__restrict__ blue, int W, int H,
                                                              int tiles_x, int n_tiles, float bg0, float bg1,
                                                              float bg2, float *__restrict__ image,
                                                              float *__restrict__ final_T,
                                                              int32_t *__restrict__ n_contrib,
                                                              int32_t *__restrict__ n_blended,
                                                              uint2 *__restrict__ blended,
                                                              uint32_t *__restrict__ tile_blended,
                                                              const uint32_t *__restrict__ order) {
  constexpr int NT = kTile * kTile / PPT;   // threads per tile
  constexpr int ROWS = NT / kTile;          // pixel rows covered by one pass of the threads
  __shared__ float4 s_a[kBatch];
  __shared__ float4 s_b[kBatch];
  __shared__ float4 s_c[kBatch];
  __shared__ uint8_t s_taken[kBatch];
  __shared__ uint32_t s_id[kBatch];
  __shared__ uint32_t s_wcnt[NT / 64];
  const int tile = (int)order[blockIdx.x];
  const int tid = threadIdx.x;
  const int x0 = (tile % tiles_x) * kTile, y0 = (tile / tiles_x) * kTile;
  const int px = x0 + (tid & (kTile - 1));
  const float fx = (float)(tid & (kTile - 1)) + 0.5f;   // pixel centres relative to the tile's corner
  float fy[PPT];
  bool inside[PPT];
  float T[PPT];
  float C0[PPT], C1[PPT], C2[PPT];
  int last[PPT], nbl[PPT];
  bool done[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int py = y0 + (tid >> 4) + ROWS * k;
    fy[k] = (float)(py - y0) + 0.5f;
    inside[k] = px < W && py < H;
    T[k] = 1.0f; C0[k] = 0.0f; C1[k] = 0.0f; C2[k] = 0.0f;
    last[k] = 0;
    nbl[k] = 0;
    done[k] = !inside[k];
  }
  const uint2 rg = ranges[tile];
  const int n = (int)(rg.y - rg.x);
  int last_start = -1;   // start of the last batch walked
  uint32_t n_bl = 0;     // blended entries listed so far
  for (int start = 0; start < n; start += kBatch) {
    bool all_done = true;
#pragma unroll
    for (int k = 0; k < PPT; ++k) all_done = all_done && done[k];
    if (NT == 64) {
      if (__all(all_done)) break;
      __syncthreads();
    } else {
      if (__syncthreads_and(all_done)) break;
    }
    // the previous batch's blended entries join the list, this batch's flags start at zero
    if (blended && start > 0)
      append_blended<NT>(s_taken, s_id, s_wcnt, start - kBatch, n, blended + rg.x, n_bl, tid);
    for (int e = tid; e < kBatch; e += NT) {
      s_taken[e] = 0;
      if (start + e < n) {
        const uint32_t g = values[rg.x + start + e];
        s_id[e] = g;
        stage_entry(xyab, cop, blue, g, x0, y0, s_a[e], s_b[e], s_c[e]);
      }
    }
    __syncthreads();
    // the count is the same in every lane (read from the first: the loop's exit test is then a
    // scalar compare instead of a VALU one per entry)
    const int cnt = __builtin_amdgcn_readfirstlane(min(kBatch, n - start));
    // the staged entries are read at a vector-register base (jb, zero, opaque to the compiler)
    // plus constant offsets: with the base in a scalar register the compiler moved it into a
    // vector register again for every entry, since it reused that register for the reads (two
    // VALU per entry fewer with the exit test: 720p / 500k 0.1085 -> 0.1044 ms, 1080p / 1M
    // within the noise). Eight entries per iteration (measured 0.193 ms against 0.199 ms
    // unrolled by four, 0.215 ms by two and 0.260 ms not unrolled at 1080p / 1M)
    int jb = 0;
    asm volatile("" : "+v"(jb));
#pragma unroll 8
    for (int j = 0; j < cnt; ++j) {
      bool any_live = false;
#pragma unroll
      for (int k = 0; k < PPT; ++k) any_live = any_live || !done[k];
      if (!any_live) break;
      const float4 A = s_a[jb + j];
      const float4 B = s_b[jb + j];
      const float2 BL = *reinterpret_cast<const float2 *>(&s_c[jb + j]);   // threshold on l, blue
      const float dx = fx - A.x;
      const float t = conic_column(A.w, dx, B.y);
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if (done[k]) continue;
        const float l = conic_kq(B.x, A.z, dx, fy[k] - A.y, t);   // k q + log2 o
        if (l < BL.x) continue;                                   // q > 9 or alpha < 1/255
        const float alpha = fminf(kAlphaMax, alpha_from_log2(l));
        const float wgt = alpha * T[k];
        const float Tn = fmaf(-alpha, T[k], T[k]);   // T (1 - alpha), one rounding
        if (Tn < kTMin) {
          done[k] = true;
          continue;
        }
        C0[k] = fmaf(wgt, B.z, C0[k]);
        C1[k] = fmaf(wgt, B.w, C1[k]);
        C2[k] = fmaf(wgt, BL.y, C2[k]);
        T[k] = Tn;
        last[k] = start + j + 1;
        if (COUNT) ++nbl[k];
        s_taken[j] = 1;
      }
    }
    last_start = start;
  }
  // the blended entries of the last batch walked (the walk blends nothing after it)
  __syncthreads();
  if (blended && last_start >= 0)
    append_blended<NT>(s_taken, s_id, s_wcnt, last_start, n, blended + rg.x, n_bl, tid);
  if (tid == 0 && tile_blended) tile_blended[tile] = n_bl;
  const size_t plane = (size_t)W * H;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    if (!inside[k]) continue;
    const size_t pix = (size_t)(y0 + (tid >> 4) + ROWS * k) * W + px;
    const float Tf = T[k];
    image[pix] = fmaf(Tf, bg0, C0[k]);
    image[plane + pix] = fmaf(Tf, bg1, C1[k]);
    image[2 * plane + pix] = fmaf(Tf, bg2, C2[k]);
    final_T[pix] = Tf;
    n_contrib[pix] = last[k];
    if (COUNT) n_blended[pix] = nbl[k];
  }
}

hipError_t launch_blend(const uint2 *ranges, const uint32_t *values, const float4 *xyab, const float4 *cop,
                        const float2 *blue, const DevCamera &cam, const float bg[3], float *image, float *final_T,
                        int32_t *n_contrib, int32_t *n_blended, uint2 *blended, uint32_t *tile_blended,
                        const uint32_t *order, hipStream_t s) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  // 1 pixel per thread (4 waves per tile) measured fastest at 1080p / 1M: 0.218 ms against
  // 0.242 ms with 2 and 0.353 ms with 4 (entry loop unrolled by two in that comparison).
  auto kernel = n_blended ? k_blend<kFwdPix, true> : k_blend<kFwdPix, false>;
  hipLaunchKernelGGL(kernel, dim3(n_tiles), dim3(kTile * kTile / kFwdPix), 0, s, ranges, values, xyab, cop, blue,
                     cam.W, cam.H, cam.tiles_x, n_tiles, bg[0], bg[1], bg[2], image, final_T, n_contrib, n_blended,
                     blended, tile_blended, order);
  return hipGetLastError();
}

hipError_t launch_tile_order_by_length(const uint2 *ranges, int n_tiles, uint32_t *order, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_order<ListLengthCost>, dim3(1), dim3(kOrderThreads), 0, s, ListLengthCost{ranges},
                     n_tiles, order, TileSplit{0.0f, 0.0f, -1, -1});
  return hipGetLastError();
}

}  // namespace flod

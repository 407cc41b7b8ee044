// Backward pass of the rasterizer (the rasterize-and-backpropagate step of Algorithm 1).
//
// Blend backward: one wave per tile (4 pixels per lane), walking the tile list back to
// front from the last blended entry. The per-pixel transmittance before entry i is
// recovered from the saved final T as T_i = T_{i+1} / (1 - alpha_i) (alpha <= 0.99, FP32
// reciprocal: about one rounding per blended contributor, so the relative error after m of
// them grows like sqrt(m) ulp, far below the FP32 summation error of the gradients), and
//   dC/dc_i     = alpha_i T_i
//   dC/dalpha_i = T_i c_i - S_i / (1 - alpha_i),  S_i = sum_{j>i} alpha_j T_j c_j + T_final bg
//               = T_i (c_i - Shat_i),  Shat_i = S_i / T_{i+1}
// where the normalised colour behind entry i follows the convex update
//   Shat_{i-1} = alpha_i c_i + (1 - alpha_i) Shat_i,  Shat_last = bg,
// which avoids the cancellation between T_i c_i and S_i / (1 - alpha_i) in FP32.
// Then alpha -> (opacity, q) unless the 0.99 clamp is active, q -> (conic, mu'): per entry the
// wave sums nine per-Gaussian values through LDS (the moments of e = dL/dalpha alpha over its
// pixels, e dx, e dy, e dx^2, e dx dy, e dy^2 and e, and the colour gradient) and nine lanes
// issue one FP32 atomic each per (tile, Gaussian); the conic and opacity factors that turn the
// moments into dL/d(mu', conic, opacity) are applied per Gaussian in the preprocess backward.
//
// Preprocess backward: one thread per Gaussian, recomputing the forward projection (FP64)
// and applying the chain rule in FP64 to the mean (through mu', the EWA Jacobian and the SH view
// direction), log-scales (eq. 4: times exp(s_opt); s_min gets no gradient), quaternion
// (through the normalisation), opacity logit (times o (1 - o)) and SH coefficients. The SH
// colour's clamp and its view-direction Jacobian come from the forward, which keeps them per
// visible Gaussian, so the SH coefficients themselves are not read.
#include <hip/hip_ext.h>

#include <type_traits>

#include "blend_common.h"

namespace flod {

constexpr int kG2d = 9;   // mu'x, mu'y, conic a, b, c, opacity, red, green, blue
#ifndef FLOD_BWD_SPLIT
#define FLOD_BWD_SPLIT 1.75f
#endif
#ifndef FLOD_BWD_SPLIT4
#define FLOD_BWD_SPLIT4 3.0f
#endif
#ifndef FLOD_BWD_BATCH
#define FLOD_BWD_BATCH 64
#endif
// List entries staged in LDS per batch: 64 x 56 B = 3.5 KB per one-wave workgroup, plus the
// 3 KB of the per-entry reduction, so LDS does not cap the waves a CU holds below what the
// registers allow. At 1080p / 1M (with 72-byte entries then), 128-entry batches (9.3 KB per
// wave) took 0.268 ms, 96 0.241 ms and 64 0.232 ms.
constexpr int kBwdBatch = FLOD_BWD_BATCH;

// Sum over the 16 lanes of each DPP row, in every lane of the row (rotations by 8, 4, 2, 1).
template <int N>
__device__ __forceinline__ float add_row_ror(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + N, 0xF, 0xF, true));
}
__device__ __forceinline__ float row_sum16(float v) {
  return add_row_ror<1>(add_row_ror<2>(add_row_ror<4>(add_row_ror<8>(v))));
}

// Frames with at least this many tiles reduce each entry's gradient with a second LDS round,
// smaller ones with DPP (see the kernel). With heavy tiles split and the priority by remaining
// work, 720p (3,600 tiles) measured 0.141 ms with the LDS rounds against 0.144 with DPP (at
// 6144, the earlier threshold, it had been the other way round).
constexpr int kLdsRound2MinTiles = 3072;

// The per-pixel decision of one entry, repeating the forward's bit for bit: the pixel takes
// part when its walk has reached the entry and l = k q + log2 o reaches the entry's threshold
// (q <= 9 and alpha >= 1/255). A pixel that does not take part gets alpha 0 and a weight of 0:
// it then adds exact zeros, keeps its T (T / (1 - 0) = T) and its V. The weight gmv is the
// unclamped alpha o G, and 0 where the 0.99 clamp is active (alpha does not depend on opacity
// or q there); entries whose opacity cannot reach the clamp (see stage_entry) skip its test.
// Without CHECK the caller guarantees that the walk has reached the entry in every pixel of the
// wave.
template <int PPT, bool CLAMP, bool CHECK>
__device__ __forceinline__ bool decide(const float (&fy)[PPT], const int (&last)[PPT], int jpos, float my, float r,
                                       float dx, float ck, float thr, float t, float (&dyv)[PPT], float (&aev)[PPT],
                                       float (&gmv)[PPT]) {
  bool contrib = false;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const float dy = fy[k] - my;
    dyv[k] = dy;
    const float l = conic_kq(ck, r, dx, dy, t);   // k q + log2 o
    const float a0 = alpha_from_log2(l);          // o G
    const bool ok = (!CHECK || jpos < last[k]) && l >= thr;
    if (CLAMP) {
      aev[k] = ok ? fminf(kAlphaMax, a0) : 0.0f;
      gmv[k] = (ok && a0 <= kAlphaMax) ? a0 : 0.0f;
    } else {
      aev[k] = ok ? a0 : 0.0f;   // gmv: alpha itself (the caller reads aev)
    }
    contrib = contrib || ok;
  }
  return contrib;
}

// Per-entry reduction through LDS: component c of lane l at s_red[c * kRedStride + l]. The
// stride of 80 floats puts the four components a read instruction of the first round touches
// at once on four different 64-byte bank groups.
constexpr int kRedStride = 80;

// The wave's issue priority from the work it has left (entries to walk, weighted by their cost
// per wave: 3 for a whole tile, 2 for a half): level min(3, work / 128), set at every batch.
// The SIMD's arbiter otherwise serves the oldest ready wave first, so the youngest waves of
// the first dispatch round were starved until the older ones finished and then ran on nearly
// alone as the kernel's tail; serving the waves with the most work left first evens out when
// they finish (1080p / 1M 0.192 -> 0.184 ms; thresholds of 48 to 256 measured within 2%).
__device__ __forceinline__ void set_priority_by_work(int work) {
  const int level = min(3, work / 128);
  if (level >= 3) __builtin_amdgcn_s_setprio(3);
  else if (level == 2) __builtin_amdgcn_s_setprio(2);
  else if (level == 1) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// The LDS of one backward workgroup (one wave).
// The reduction's buffer comes first: its nine components then lie within reach of three
// base registers' 8-bit offsets (placed after the staged entries they took five, which the
// compiler rebuilt with an add each per entry).
struct __align__(16) BwdShared {
  float red[kG2d * kRedStride];                       // the per-entry reduction
  float4 a[kBwdBatch], b[kBwdBatch], c[kBwdBatch];   // the staged entries (see stage_entry;
                                                      // c.w holds the Gaussian's index)
  int pos[kBwdBatch];                                 // their positions in the tile's list
  float red2[4 * kG2d];                               // its first round's partials (LDS form)
};

// One wave walks one part of a tile: the pixel rows r0 + lane / 16 + 4 k, k < PPT (PPT = 4:
// the whole tile, 4 pixels per lane; PPT = 2: half of it). Per pixel the state is T
// (transmittance after the current entry), V = dL/dC . Shat (the upstream gradient dotted with
// the normalised colour behind the current entry) and dL/dC, all FP32 (V is a convex
// combination per step, so its error does not grow along the chain). Per entry each lane sums
// its pixels' 9 gradient components in registers and the wave reduces them (see below) before
// one atomic instruction adds the nine sums.
template <int PPT, bool LDS_ROUND2>
__device__ __forceinline__ void bwd_part(
    BwdShared &sh, int tile, int r0, const uint2 *__restrict__ ranges, const float4 *__restrict__ xyab,
    const float4 *__restrict__ cop, const float2 *__restrict__ blue, int W, int H, int tiles_x, float bg0,
    float bg1, float bg2, const float *__restrict__ final_T, const int32_t *__restrict__ n_contrib,
    const float *__restrict__ dimg, float *__restrict__ g2d, const uint2 *__restrict__ blended,
    const uint32_t *__restrict__ tile_blended) {
  constexpr int NT = 64;
  constexpr int ROWS = NT / kTile;
  static_assert(kBwdBatch == NT, "one staged entry per lane");
  float4 *s_a = sh.a, *s_b = sh.b, *s_c = sh.c;
  int *s_pos = sh.pos;
  float *s_red = sh.red, *s_red2 = sh.red2;
  constexpr int RS = LDS_ROUND2 ? kRedStride : 64;   // component stride of the reduction
  const int tid = threadIdx.x, lane = tid & 63;
  // float4 slots each lane reads in the reduction's rounds (clamped: lanes past the last
  // slot read a valid one and discard it). LDS form: lane 4 c + h (c < 9, h < 4) sums the
  // float4 slots h, h + 4, h + 8, h + 12 of component c in the first round, lane c < 9 the
  // four partials of component c in the second; DPP form: slots lane, lane + 64, lane + 128
  const int red_l36 = min(lane, 4 * kG2d - 1);
  const int red_r1 = (red_l36 >> 2) * (kRedStride / 4) + (red_l36 & 3);
  const int red_hi = min(lane + 128, kG2d * 16 - 1), red_lo9 = min(lane, kG2d - 1);
  // zero in a vector register, opaque to the compiler: added to the DPP form's lane-0 atomic
  // address, which the compiler would otherwise see as uniform and send through its atomic
  // combining path (a lane loop plus a wait for all outstanding memory operations per entry)
  int vzero = 0;
  asm volatile("" : "+v"(vzero));
  const int x0 = (tile % tiles_x) * kTile, y0 = (tile / tiles_x) * kTile;
  const int px = x0 + (tid & (kTile - 1));
  const float fx = (float)(tid & (kTile - 1)) + 0.5f;   // pixel centres relative to the tile's corner
  const size_t plane = (size_t)W * H;
  const uint2 rg = ranges[tile];
  // the walk covers the entries the forward blended into some pixel of the tile (the others
  // change no T, no suffix and no gradient), which it listed at the start of the tile's range;
  // a pixel takes part in those before its n_contrib (the count is clamped to the list, and
  // n_contrib, which comes from the caller's buffer, only enters comparisons)
  const int list_len = (int)(rg.y - rg.x);
  const int n_bl = min((int)tile_blended[tile], list_len);
  float fy[PPT], d0[PPT], d1[PPT], d2[PPT];
  float T[PPT], V[PPT];
  int last[PPT];
  int myfirst = list_len;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int py = y0 + r0 + (tid >> 4) + ROWS * k;
    fy[k] = (float)(py - y0) + 0.5f;
    T[k] = 1.0f; V[k] = 0.0f; d0[k] = 0.0f; d1[k] = 0.0f; d2[k] = 0.0f;
    last[k] = 0;
    if (px < W && py < H) {
      const size_t pix = (size_t)py * W + px;
      T[k] = final_T[pix];
      last[k] = min(max(n_contrib[pix], 0), list_len);
      d0[k] = dimg[pix];
      d1[k] = dimg[plane + pix];
      d2[k] = dimg[2 * plane + pix];
      V[k] = d0[k] * bg0 + d1[k] * bg1 + d2[k] * bg2;
    }
    myfirst = min(myfirst, last[k]);   // 0 for a pixel outside the image
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) myfirst = min(myfirst, __shfl_xor(myfirst, o, 64));
  // batches of 64 listed entries (one per lane), back to front. Listing them in the forward
  // instead of staging 64 list positions per batch and compacting those it blended: 9% of the
  // positions are listed at 1080p / 1M (92 of 1040 per tile on average), so a tile took about
  // 16 batches, each two dependent global loads and two barriers for a handful of entries
  for (int end = n_bl; end > 0; end -= kBwdBatch) {
    set_priority_by_work(end * (PPT == 4 ? 3 : PPT == 2 ? 2 : 1));
    const int start = max(0, end - kBwdBatch);
    const int cnt = end - start;
    __syncthreads();
    // the first nlow staged entries lie below every pixel's last entry (myfirst): there the
    // walk has reached the entry in every pixel and the decision skips that test
    const bool f = tid < cnt;
    int pos = 0;
    if (f) {
      const uint2 pe = blended[rg.x + start + tid];   // (list position, Gaussian)
      pos = (int)pe.x;
      s_pos[tid] = pos;
      float4 a, b, c;
      stage_entry(xyab, cop, blue, pe.y, x0, y0, a, b, c);
      c.w = __uint_as_float(pe.y);   // read with the entry, for the gradient's row
      s_a[tid] = a;
      s_b[tid] = b;
      s_c[tid] = c;
    }
    const int nlow = (int)__popcll(__ballot(f && pos < myfirst));
    __syncthreads();
    // back to front over the staged entries: first those that some pixel's walk may not have
    // reached (with the test of the position), then the rest without it (four compares per
    // entry fewer: 720p / 500k 0.221 -> 0.217 ms, 1080p / 1M unchanged). The two loops keep
    // their counters in vector registers: with scalar counters, or without the early return
    // below, the compiler copied the eight T and V registers on every iteration (8 more VALU
    // than the test saves)
    auto walk = [&](auto check_tag, int hi, int lo) {
      constexpr bool CHECK = decltype(check_tag)::value;
      for (int jl = hi - 1; jl >= lo; --jl) {
        const int jpos = CHECK ? s_pos[jl] : 0;
        const float4 A = s_a[jl];
        const float4 B = s_b[jl];
        const float4 BL = s_c[jl];   // threshold on l, blue, clamp flag, Gaussian
        const float dx = fx - A.x;
        const float t = conic_column(A.w, dx, B.y);
        // first only what decides whether a pixel takes part; the transmittance recovery and
        // the gradient run when some pixel of the wave does (always, in a consistent state: the
        // entry was staged because the forward blended it into some pixel of the tile, and the
        // decision repeats the forward's). The whole entry is instantiated with and without the
        // clamp's test (the flag is the same in every lane: a uniform branch), so that without
        // it alpha itself is the weight of the gradient
        auto entry = [&](auto clamp_tag) {
          constexpr bool CLAMP = decltype(clamp_tag)::value;
          float dyv[PPT], aev[PPT], gmv[PPT];
          if (!__any(decide<PPT, CLAMP, CHECK>(fy, last, jpos, A.y, A.z, dx, B.x, BL.x, t, dyv, aev, gmv))) return;
          {
          // the gradient arithmetic may contract into FMAs (the decision above must not: it
          // repeats the forward's, bit for bit)
#pragma clang fp contract(fast)
          float gr[kG2d];
          gr[6] = gr[7] = gr[8] = 0.0f;
          // with alpha = o G below the clamp, dalpha/do = alpha / o and dalpha/dq = -alpha / 2, so one
          // sum e = dL/dalpha alpha per pixel serves both: dL/do = sum e / o and dL/dq = -e / 2. With
          // q = a dx^2 + 2 b dx dy + c dy^2 every q-derivative is a moment of e times a factor of
          // the Gaussian: dL/d(a, b, c) = -(1 / 2) (sum e dx^2, 2 sum e dx dy, sum e dy^2) and
          // dL/dmu' = (a sum e dx + b sum e dy, b sum e dx + c sum e dy). A lane's pixels share
          // their column, so it needs only E0 = sum e, E1 = sum e dy and E2 = sum e dy^2 over them
          float E0 = 0.0f, E1 = 0.0f, E2 = 0.0f;
#pragma unroll
          for (int k = 0; k < PPT; ++k) {
            const float alpha = aev[k], dy = dyv[k];
            const float Ti = T[k] * __builtin_amdgcn_rcpf(1.0f - alpha);
            const float wT = alpha * Ti;
            const float dcc = d0[k] * B.z + d1[k] * B.w + d2[k] * BL.y;   // dL/dC . c
            const float diff = dcc - V[k];
            // dL/dalpha alpha (with alpha the weight, T_i alpha (c - Shat) is wT diff)
            const float e = CLAMP ? (Ti * diff) * gmv[k] : wT * diff;
            gr[6] = fmaf(wT, d0[k], gr[6]);
            gr[7] = fmaf(wT, d1[k], gr[7]);
            gr[8] = fmaf(wT, d2[k], gr[8]);
            V[k] = fmaf(alpha, diff, V[k]);                             // alpha dcc + (1 - alpha) V
            T[k] = Ti;
            const float ey = e * dy;
            E0 += e;
            E1 += ey;
            E2 = fmaf(ey, dy, E2);
          }
          // the moments sum e dx, e dy, e dx^2, e dx dy, e dy^2, e over the lane's pixels (dx is
          // the column's): the conic and opacity factors are the Gaussian's own and are applied
          // once per Gaussian after all its tiles (k_preprocess_bwd)
          gr[0] = dx * E0;
          gr[1] = E1;
          gr[2] = dx * gr[0];
          gr[3] = dx * E1;
          gr[4] = E2;
          gr[5] = E0;
          {
            // the nine components summed over the wave: each lane writes its nine values to LDS
            // component-major. LDS form: 36 lanes each add 16 values of one component (four float4
            // reads), then lane c < 9 adds the four partials of component c to the Gaussian's 36-byte
            // row (one atomic instruction). DPP form: each lane adds three float4 (4 lanes' values of
            // components l / 16, 4 + l / 16 and, lanes below 16, 8), DPP sums over each row of 16 lanes
            // follow (lanes 0, 16, 32, 48 then hold the sums; three atomic instructions). DPP costs
            // about two VALU issue slots per operation, an LDS round a wait: the LDS form for frames
            // with enough tiles to hide the wait (8 waves per SIMD at 1080p: 0.233 against 0.254 ms
            // with a three-float4 first round), DPP for small ones (720p, 3.5 waves per SIMD: 0.238
            // against 0.248 ms). The workgroup is one wave, so its barriers only order the LDS
            // accesses.
#pragma unroll
            for (int c = 0; c < kG2d; ++c) s_red[c * RS + lane] = gr[c];
            __syncthreads();
            const float4 *r4 = reinterpret_cast<const float4 *>(s_red);
            const size_t row = (size_t)__float_as_uint(BL.w) * kG2d;
            if (LDS_ROUND2) {
              // lane 4 c + h: 16 values of component c (lanes 4 h .. 4 h + 3 of each group of 16)
              const float4 q0 = r4[red_r1], q1 = r4[red_r1 + 4], q2 = r4[red_r1 + 8], q3 = r4[red_r1 + 12];
              const float p = (((q0.x + q0.y) + (q0.z + q0.w)) + ((q1.x + q1.y) + (q1.z + q1.w))) +
                              (((q2.x + q2.y) + (q2.z + q2.w)) + ((q3.x + q3.y) + (q3.z + q3.w)));
              if (lane < 4 * kG2d) s_red2[lane] = p;
              __syncthreads();
              const float4 q = reinterpret_cast<const float4 *>(s_red2)[red_lo9];   // component lane (lanes 0..8)
              const float x = (q.x + q.y) + (q.z + q.w);
              if (lane < kG2d && x != 0.0f) atomicAdd(&g2d[row + lane], x);
            } else {
              const float4 ra = r4[lane], rb = r4[lane + 64], rc = r4[red_hi];
              const float p0 = (ra.x + ra.y) + (ra.z + ra.w);   // component lane / 16
              const float p1 = (rb.x + rb.y) + (rb.z + rb.w);   // component 4 + lane / 16
              const float p2 = (rc.x + rc.y) + (rc.z + rc.w);   // component 8 (lanes 0..15)
              const float s0 = row_sum16(p0), s1 = row_sum16(p1), s2 = row_sum16(p2);
              if ((lane & 15) == 0) {
                if (s0 != 0.0f) atomicAdd(&g2d[row + (lane >> 4)], s0);
                if (s1 != 0.0f) atomicAdd(&g2d[row + 4 + (lane >> 4)], s1);
                if (lane == 0 && s2 != 0.0f) atomicAdd(&g2d[row + 8 + vzero], s2);
              }
            }
          }
          }
        };
        if (__builtin_amdgcn_readfirstlane(__float_as_int(BL.z)) != 0)
          entry(std::integral_constant<bool, true>{});
        else
          entry(std::integral_constant<bool, false>{});
      }
    };
    walk(std::true_type{}, cnt, nlow);
    walk(std::false_type{}, nlow, 0);
  }
}

// Tiles whose count of listed entries exceeds this many times the mean (by the tile order's
// buckets) are walked by two waves, one per half (8 rows each, 2 pixels per lane), at most a
// quarter of the tiles. One wave per tile leaves the heaviest ones as the kernel's tail: five
// waves share each SIMD, so a tile with twice the mean work runs about as long as a whole SIMD's
// share of the frame (1080p / 1M: the last tiles, started at once, ended 70 us after the
// last dispatch). With the priority below, 1.75 measured best at 1080p / 1M (0.176 ms against
// 0.181 at 2 and 0.189 at 1.65; 720p / 500k the same from 1.65 to 2).
constexpr float kBwdSplitFactor = FLOD_BWD_SPLIT;
// Tiles above this many times the mean are split in four instead (quarters of 4 rows, one pixel
// per lane): at 720p / 500k, with 3,600 tiles for 6,144 wave slots, the heaviest tiles' halves
// still set the kernel's span.
constexpr float kBwdSplit4Factor = FLOD_BWD_SPLIT4;

// The order leads with h4 = order[n_tiles + 1] tiles split in four (quarters of 4 rows, one
// pixel per lane), then h2 - h4 (h2 = order[n_tiles]) split in two; workgroups 0 .. 4 h4 - 1
// walk the quarters, the next 2 (h2 - h4) the halves, the next n_tiles - h2 whole tiles, and
// any past those have nothing to do.
template <bool LDS_ROUND2>
__global__ __launch_bounds__(64) void k_blend_bwd(
    const uint2 *__restrict__ ranges, const float4 *__restrict__ xyab, const float4 *__restrict__ cop,
    const float2 *__restrict__ blue, int W, int H, int tiles_x, int n_tiles, float bg0, float bg1, float bg2,
    const float *__restrict__ final_T, const int32_t *__restrict__ n_contrib, const float *__restrict__ dimg,
    float *__restrict__ g2d, const uint2 *__restrict__ blended, const uint32_t *__restrict__ tile_blended,
    const uint32_t *__restrict__ order) {
  __shared__ BwdShared sh;
  const int h2 = (int)order[n_tiles], h4 = (int)order[n_tiles + 1];
  const int b = (int)blockIdx.x;
  const int b2 = b - 4 * h4, b1 = b2 - 2 * (h2 - h4);
  if (b < 4 * h4)
    bwd_part<1, LDS_ROUND2>(sh, (int)order[b >> 2], (b & 3) * (kTile / 4), ranges, xyab, cop, blue, W, H, tiles_x,
                            bg0, bg1, bg2, final_T, n_contrib, dimg, g2d, blended, tile_blended);
  else if (b1 < 0)
    bwd_part<2, LDS_ROUND2>(sh, (int)order[h4 + (b2 >> 1)], (b2 & 1) * (kTile / 2), ranges, xyab, cop, blue, W, H,
                            tiles_x, bg0, bg1, bg2, final_T, n_contrib, dimg, g2d, blended, tile_blended);
  else if (b1 < n_tiles - h2)
    bwd_part<4, LDS_ROUND2>(sh, (int)order[h2 + b1], 0, ranges, xyab, cop, blue, W, H, tiles_x, bg0, bg1, bg2,
                            final_T, n_contrib, dimg, g2d, blended, tile_blended);
}

template <bool LDS_ROUND2>
static void launch_blend_bwd_t(const uint2 *ranges, const float4 *xyab, const float4 *cop, const float2 *blue,
                               const DevCamera &cam, const float bg[3], const float *final_T, const int32_t *n_contrib,
                               const float *dL_dimage, float *g2d, const uint2 *blended, const uint32_t *tile_blended,
                               const uint32_t *order, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  const int grid = n_tiles + bwd_split_extra(n_tiles);
  auto kernel = k_blend_bwd<LDS_ROUND2>;
  if (ev_start || ev_stop) {
    // timed from the kernel's own dispatch: no event packets between it and its neighbours
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(64), 0, s, ev_start, ev_stop, 0, ranges, xyab, cop, blue, cam.W,
                          cam.H, cam.tiles_x, n_tiles, bg[0], bg[1], bg[2], final_T, n_contrib, dL_dimage, g2d,
                          blended, tile_blended, order);
  } else {
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(64), 0, s, ranges, xyab, cop, blue, cam.W, cam.H, cam.tiles_x,
                       n_tiles, bg[0], bg[1], bg[2], final_T, n_contrib, dL_dimage, g2d, blended, tile_blended,
                       order);
  }
}

// at most a quarter of the tiles split in two or four, at most a sixteenth in four
static int split_cap2(int n_tiles) { return n_tiles / 4; }
static int split_cap4(int n_tiles) { return n_tiles / 16; }
int bwd_split_extra(int n_tiles) { return split_cap2(n_tiles) + 2 * split_cap4(n_tiles); }

// The backward's tile order (workgroup 0) and the zeroing of the n floats of the gradient
// sums at p (the other workgroups) in one launch: the order is one latency-bound workgroup, the
// fill is bound by bandwidth, and neither needs the other (one after the other they took 9 and
// 7 us at 1080p / 1M; together the step is 2.5 us shorter).
__global__ __launch_bounds__(kOrderThreads) void k_bwd_order_fill(CountCost cost, int n_tiles, uint32_t *order,
                                                                  TileSplit split, float *p, int64_t n) {
  if (blockIdx.x == 0) {
    tile_order(cost, n_tiles, order, split);
    return;
  }
  // the floats before the first 16-byte boundary, then whole uint4, then the rest
  const int64_t lead = min(n, (int64_t)(((16u - (uint32_t)(reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / 4u));
  const int64_t n4 = (n - lead) / 4;
  uint4 *q = reinterpret_cast<uint4 *>(p + lead);
  const int64_t stride = (int64_t)(gridDim.x - 1) * kOrderThreads;
  for (int64_t i = (int64_t)(blockIdx.x - 1) * kOrderThreads + threadIdx.x; i < n4; i += stride)
    q[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 1) {
    const int64_t tail = lead + 4 * n4;
    if (threadIdx.x < lead) p[threadIdx.x] = 0.0f;
    if (tail + threadIdx.x < n) p[tail + threadIdx.x] = 0.0f;
  }
}

hipError_t launch_blend_bwd(const uint2 *ranges, const float4 *xyab, const float4 *cop, const float2 *blue,
                            const DevCamera &cam, const float bg[3], const float *final_T, const int32_t *n_contrib,
                            const float *dL_dimage, float *g2d, int64_t n_g2d, const uint2 *blended,
                            const uint32_t *tile_blended, uint32_t *order, hipStream_t s, hipEvent_t ev_start,
                            hipEvent_t ev_stop) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  if (n_tiles <= 0) return launch_fill_u32(reinterpret_cast<uint32_t *>(g2d), 0u, n_g2d, s);
  // tiles in order of decreasing listed-entry count, the ones split in four and in two first,
  // beside the zeroing of the gradient sums the walk adds into
  const int64_t fill_blocks = std::max<int64_t>(1, std::min<int64_t>(512, (n_g2d / 4 + 4 * kOrderThreads - 1) /
                                                                               (4 * kOrderThreads)));
  hipLaunchKernelGGL(k_bwd_order_fill, dim3((unsigned)(1 + fill_blocks)), dim3(kOrderThreads), 0, s,
                     CountCost{tile_blended}, n_tiles, order,
                     TileSplit{kBwdSplitFactor, kBwdSplit4Factor, split_cap2(n_tiles), split_cap4(n_tiles)}, g2d,
                     n_g2d);
  if (n_tiles >= kLdsRound2MinTiles)
    launch_blend_bwd_t<true>(ranges, xyab, cop, blue, cam, bg, final_T, n_contrib, dL_dimage, g2d, blended,
                             tile_blended, order, s, ev_start, ev_stop);
  else
    launch_blend_bwd_t<false>(ranges, xyab, cop, blue, cam, bg, final_T, n_contrib, dL_dimage, g2d, blended,
                              tile_blended, order, s, ev_start, ev_stop);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------

// The chain rule for one visible Gaussian i; its SH gradient row goes to dsh (LDS).
__device__ __forceinline__ void preprocess_bwd_one(const PreParams &p, const DevLevel &L, int64_t i,
                                                        const float *__restrict__ g2d,
                                                        const float4 *__restrict__ shjac, const flod_grads &out,
                                                        float4 *dsh) {
  double g[kG2d];   // the blend backward's sums (moments of e, colour), turned into gradients below
#pragma unroll
  for (int c = 0; c < kG2d; ++c) g[c] = (double)g2d[i * kG2d + c];
  const float m0 = L.means[i * 3 + 0], m1 = L.means[i * 3 + 1], m2 = L.means[i * 3 + 2];
  float ls[3] = {L.log_scales[i * 3 + 0], L.log_scales[i * 3 + 1], L.log_scales[i * 3 + 2]};
  const float4 q4 = reinterpret_cast<const float4 *>(L.quats)[i];
  float q[4] = {q4.x, q4.y, q4.z, q4.w};
  const float logit = L.logits[i];
  Proj pr;
  view_transform(p.cam, m0, m1, m2, pr);
  project_cov(p.cam, ls, q, L.s_min, pr);
  const DevCamera &cam = p.cam;

  // opacity
  const float o = 1.0f / (1.0f + __expf(-logit));

  // conic -> dilated 2D covariance (a, b; b, c); FP64 because det can be far below a c
  const double a = pr.a, b = pr.b, c = pr.c;
  const double idet = 1.0 / pr.det;
  const double id2 = idet * idet;
  {
    // moments of e = dL/dalpha alpha -> dL/d(mu', conic a, b, c, opacity), with the conic
    // (c, -b, a) / det and the opacity
    const double ca = c * idet, cb = -b * idet, cc = a * idet;
    const double m_dx = g[0], m_dy = g[1];
    g[0] = ca * m_dx + cb * m_dy;
    g[1] = cb * m_dx + cc * m_dy;
    g[2] = -0.5 * g[2];
    g[3] = -g[3];
    g[4] = -0.5 * g[4];
    g[5] = g[5] / (double)o;
  }
  const float d_logit = (float)g[5] * o * (1.0f - o);
  const double gA = g[2], gB = g[3], gC = g[4];
  const double ga = (-c * c * gA + b * c * gB - b * b * gC) * id2;
  const double gb = (2.0 * b * c * gA - (a * c + b * b) * gB + 2.0 * a * b * gC) * id2;
  const double gc = (-b * b * gA + a * b * gB - a * a * gC) * id2;

  // Sigma' = T Sigma T^T with T rows T0, T1
  const double *T0 = pr.Tm, *T1 = pr.Tm + 3;
  const double *S = pr.S;
  double ST0[3], ST1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ST0[k] = S[k * 3 + 0] * T0[0] + S[k * 3 + 1] * T0[1] + S[k * 3 + 2] * T0[2];
    ST1[k] = S[k * 3 + 0] * T1[0] + S[k * 3 + 1] * T1[1] + S[k * 3 + 2] * T1[2];
  }
  double gT0[3], gT1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gT0[k] = 2.0 * ga * ST0[k] + gb * ST1[k];
    gT1[k] = 2.0 * gc * ST1[k] + gb * ST0[k];
  }
  // symmetric gradient of Sigma: Gs = 2 ga T0 T0^T + gb (T0 T1^T + T1 T0^T) + 2 gc T1 T1^T
  double Gs[9];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      Gs[k * 3 + l] = 2.0 * ga * T0[k] * T0[l] + gb * (T0[k] * T1[l] + T1[k] * T0[l]) + 2.0 * gc * T1[k] * T1[l];

  // T = J R_c
  double Rc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rc[k] = cam.R[k];
  double gJ00 = 0.0, gJ02 = 0.0, gJ11 = 0.0, gJ12 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    gJ00 += gT0[j] * Rc[j];
    gJ02 += gT0[j] * Rc[6 + j];
    gJ11 += gT1[j] * Rc[3 + j];
    gJ12 += gT1[j] * Rc[6 + j];
  }
  // J and mu' -> view-space mean
  const double fx = cam.fx, fy = cam.fy;
  const double tz = pr.tz, tx = pr.tx, ty = pr.ty;
  const double iz = 1.0 / tz, iz2 = iz * iz;
  double gtx = g[0] * fx * iz;
  double gty = g[1] * fy * iz;
  double gtz = g[0] * (-fx * tx * iz2) + g[1] * (-fy * ty * iz2) + gJ00 * (-fx * iz2) + gJ11 * (-fy * iz2) +
               gJ02 * (fx * pr.xc * iz2) + gJ12 * (fy * pr.yc * iz2);
  if (pr.unclamped_x) {
    gtx += gJ02 * (-fx * iz) * iz;
    gtz += gJ02 * (-fx * iz) * (-tx * iz2);
  }
  if (pr.unclamped_y) {
    gty += gJ12 * (-fy * iz) * iz;
    gtz += gJ12 * (-fy * iz) * (-ty * iz2);
  }
  double gm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gm[k] = Rc[k] * gtx + Rc[3 + k] * gty + Rc[6 + k] * gtz;

  // colour -> SH coefficients and view direction (FP32: colour is not on the key path), from
  // the forward's Jacobian of the colour in the unit view direction and its colours before the
  // clamp (the same values this recomputed from the SH coefficients)
  {
    const int deg = p.sh_degree;
    const int nk = (deg + 1) * (deg + 1);
    const float vx = m0 - cam.campos[0], vy = m1 - cam.campos[1], vz = m2 - cam.campos[2];
    const float nv = sqrtf((vx * vx + vy * vy) + vz * vz);
    const float inv = 1.0f / nv;
    const float x = vx * inv, y = vy * inv, z = vz * inv;
    float Y[16];
    sh_basis(deg, x, y, z, Y);
    const float4 j0 = shjac[i], j1 = shjac[L.n + i], j2 = shjac[2 * L.n + i];   // three planes of n float4
    const float J[9] = {j0.x, j0.y, j0.z, j0.w, j1.x, j1.y, j1.z, j1.w, j2.x};
    const float pre[3] = {j2.y, j2.z, j2.w};
    float gsh[48];
    float gdx = 0.f, gdy = 0.f, gdz = 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float gcol = (pre[ch] < 0.0f) ? 0.0f : (float)g[6 + ch];
#pragma unroll
      for (int k = 0; k < 16; ++k) gsh[k * 3 + ch] = k < nk ? gcol * Y[k] : 0.0f;
      gdx = fmaf(gcol, J[ch * 3 + 0], gdx);
      gdy = fmaf(gcol, J[ch * 3 + 1], gdy);
      gdz = fmaf(gcol, J[ch * 3 + 2], gdz);
    }
    const float dd = x * gdx + y * gdy + z * gdz;
    gm[0] += (double)((gdx - x * dd) * inv);
    gm[1] += (double)((gdy - y * dd) * inv);
    gm[2] += (double)((gdz - z * dd) * inv);
#pragma unroll
    for (int k = 0; k < 12; ++k)
      dsh[k] = make_float4(gsh[4 * k], gsh[4 * k + 1], gsh[4 * k + 2], gsh[4 * k + 3]);
  }

  // Sigma = M M^T, M = R diag(s): gM = Gs M
  double M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) M[r * 3 + cc] = pr.R[r * 3 + cc] * pr.s[cc];
  double gR[9], gs[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const double gMrc = Gs[r * 3 + 0] * M[0 * 3 + cc] + Gs[r * 3 + 1] * M[1 * 3 + cc] + Gs[r * 3 + 2] * M[2 * 3 + cc];
      gs[cc] += gMrc * pr.R[r * 3 + cc];
      gR[r * 3 + cc] = gMrc * pr.s[cc];
    }
  // eq. 4: ds/ds_opt = exp(s_opt)
#pragma unroll
  for (int k = 0; k < 3; ++k) out.d_log_scales[i * 3 + k] = (float)(gs[k] * (double)exp_rn1(ls[k]));

  // R(q_hat) -> q_hat -> q
  const double w = pr.w, x = pr.x, y = pr.y, z = pr.z;
  const double gw = 2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
  const double gx = 2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] + z * gR[6] +
                           w * gR[7] - 2.0 * x * gR[8]);
  const double gy = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                           z * gR[7] - 2.0 * y * gR[8]);
  const double gz = 2.0 * (-2.0 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * z * gR[4] + y * gR[5] +
                           x * gR[6] + y * gR[7]);
  const double dot = w * gw + x * gx + y * gy + z * gz;
  const double inq = 1.0 / pr.nq;
  reinterpret_cast<float4 *>(out.d_quats)[i] =
      make_float4((float)((gw - w * dot) * inq), (float)((gx - x * dot) * inq), (float)((gy - y * dot) * inq),
                  (float)((gz - z * dot) * inq));
#pragma unroll
  for (int k = 0; k < 3; ++k) out.d_means[i * 3 + k] = (float)gm[k];
  out.d_opacity_logits[i] = d_logit;
}

// The SH gradients leave through LDS: each thread stages its 192-byte row, then the workgroup
// writes its 256 consecutive rows with consecutive float4 stores (written row by row, every
// lane of a store instruction hit a different cache line: 0.126 -> 0.097 ms at 1080p / 1M).
constexpr int kShRow4 = FLOD_SH_COEFFS * 3 / 4;   // float4 per SH row

__global__ __launch_bounds__(kBlock) void k_preprocess_bwd(PreParams p, const uint32_t *__restrict__ tiles,
                                                           const float *__restrict__ g2d,
                                                           const float4 *__restrict__ shjac, flod_grads out) {
  __shared__ float4 s_sh[kBlock * kShRow4];   // 48 KB: the workgroup's SH gradient rows
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const DevLevel L = p.lv[0];
  float4 *dsh = s_sh + threadIdx.x * kShRow4;
  if (i < L.n && tiles[i] == 0u) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { out.d_means[i * 3 + k] = 0.f; out.d_log_scales[i * 3 + k] = 0.f; }
    reinterpret_cast<float4 *>(out.d_quats)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    out.d_opacity_logits[i] = 0.f;
    for (int k = 0; k < kShRow4; ++k) dsh[k] = make_float4(0.f, 0.f, 0.f, 0.f);
  } else if (i < L.n) {
    preprocess_bwd_one(p, L, i, g2d, shjac, out, dsh);
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kBlock;
  float4 *dst = reinterpret_cast<float4 *>(out.d_sh + base * (FLOD_SH_COEFFS * 3));
  const int nf = (int)(min((int64_t)kBlock, L.n - base) * kShRow4);
  for (int f = threadIdx.x; f < nf; f += kBlock) dst[f] = s_sh[f];
}

hipError_t launch_preprocess_bwd(const PreParams &p, const uint32_t *tiles, const float *g2d,
                                 const float4 *shjac, const flod_grads &g, hipStream_t s) {
  const int64_t n = p.lv[0].n;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_preprocess_bwd, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, tiles,
                     g2d, shjac, g);
  return hipGetLastError();
}

// The blend backward's per-Gaussian moment sums turned into dL/d(mu', conic a, b, c, opacity)
// in place, with the stored FP32 conic and opacity (for inspection: the preprocess backward
// applies the same factors with its FP64 conic).
__global__ __launch_bounds__(kBlock) void k_g2d_from_moments(int64_t n, const uint32_t *__restrict__ tiles,
                                                             const float4 *__restrict__ xyab,
                                                             const float4 *__restrict__ cop, float *__restrict__ g2d) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || tiles[i] == 0u) return;   // not rendered: zero sums, and no conic stored
  float *g = g2d + i * kG2d;
  const double a = xyab[i].z, b = xyab[i].w, c = cop[i].x, o = cop[i].y;
  const double m_dx = g[0], m_dy = g[1];
  g[0] = (float)(a * m_dx + b * m_dy);
  g[1] = (float)(b * m_dx + c * m_dy);
  g[2] = (float)(-0.5 * (double)g[2]);
  g[3] = (float)(-(double)g[3]);
  g[4] = (float)(-0.5 * (double)g[4]);
  g[5] = (float)((double)g[5] / o);
}

hipError_t launch_g2d_from_moments(int64_t n, const uint32_t *tiles, const float4 *xyab, const float4 *cop,
                                   float *g2d, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_g2d_from_moments, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, tiles,
                     xyab, cop, g2d);
  return hipGetLastError();
}

}  // namespace flod

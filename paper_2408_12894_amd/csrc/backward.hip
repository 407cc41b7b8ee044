// Backward pass of the rasterizer (the rasterize-and-backpropagate step of Algorithm 1).
//
// Blend backward: one workgroup per tile, one pixel per thread, walking the tile list back
// to front from the last blended entry. The per-pixel transmittance before entry i is
// recovered from the saved final T as T_i = T_{i+1} / (1 - alpha_i) (alpha <= 0.99), and
//   dC/dc_i     = alpha_i T_i
//   dC/dalpha_i = T_i c_i - S_i / (1 - alpha_i),  S_i = sum_{j>i} alpha_j T_j c_j + T_final bg
// then alpha -> (opacity, q) unless the 0.99 clamp is active, q -> (conic, mu').
// Per entry the 9 gradient components are reduced across each wave with shuffles, the 4
// waves' partial sums are combined in LDS and one FP32 atomic per component is issued per
// (tile, Gaussian).
//
// Preprocess backward: one thread per Gaussian, recomputing the forward projection and
// applying the chain rule to the mean (through mu', the EWA Jacobian and the SH view
// direction), log-scales (eq. 4: times exp(s_opt); s_min gets no gradient), quaternion
// (through the normalisation), opacity logit (times o (1 - o)) and SH coefficients.
#include "project.h"

namespace flod {

constexpr int kXcdsB = 8;
constexpr int kG2d = 9;   // mu'x, mu'y, conic a, b, c, opacity, red, green, blue

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kBlock) void k_blend_bwd(const uint2 *__restrict__ ranges,
                                                      const uint32_t *__restrict__ values,
                                                      const float4 *__restrict__ xyab,
                                                      const float4 *__restrict__ cop,
                                                      const float *__restrict__ blue, int W, int H, int tiles_x,
                                                      int n_tiles, float bg0, float bg1, float bg2,
                                                      const float *__restrict__ final_T,
                                                      const int32_t *__restrict__ n_contrib,
                                                      const float *__restrict__ dimg, float *__restrict__ g2d,
                                                      int64_t stride) {
  __shared__ float4 s_a[kBlock];
  __shared__ float4 s_b[kBlock];
  __shared__ float s_c[kBlock];
  __shared__ uint32_t s_id[kBlock];
  __shared__ float s_red[kBlock / 64][kG2d][kBlock];
  __shared__ int s_max[kBlock / 64];
  const int chunk = (n_tiles + kXcdsB - 1) / kXcdsB;
  const int tile = (blockIdx.x % kXcdsB) * chunk + blockIdx.x / kXcdsB;
  if (tile >= n_tiles) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int px = (tile % tiles_x) * kTile + (tid & (kTile - 1));
  const int py = (tile / tiles_x) * kTile + (tid >> 4);
  const bool inside = px < W && py < H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const size_t pix = (size_t)py * W + px, plane = (size_t)W * H;
  float T = 1.0f, dC0 = 0.f, dC1 = 0.f, dC2 = 0.f;
  int last = 0;
  if (inside) {
    T = final_T[pix];
    last = n_contrib[pix];
    dC0 = dimg[pix];
    dC1 = dimg[plane + pix];
    dC2 = dimg[2 * plane + pix];
  }
  float S0 = T * bg0, S1 = T * bg1, S2 = T * bg2;
  // longest prefix any pixel of the tile used
  int m = last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if (lane == 0) s_max[w] = m;
  __syncthreads();
  int maxlast = s_max[0];
#pragma unroll
  for (int k = 1; k < kBlock / 64; ++k) maxlast = max(maxlast, s_max[k]);
  for (int end = maxlast; end > 0; end -= kBlock) {
    const int start = max(0, end - kBlock);
    const int cnt = end - start;
    __syncthreads();
    if (tid < cnt) {
      const uint32_t g = values[rg.x + start + tid];
      s_id[tid] = g;
      s_a[tid] = xyab[g];
      s_b[tid] = cop[g];
      s_c[tid] = blue[g];
    }
    __syncthreads();
    for (int jl = cnt - 1; jl >= 0; --jl) {
      const int jpos = start + jl;
      float gr[kG2d];
#pragma unroll
      for (int c = 0; c < kG2d; ++c) gr[c] = 0.0f;
      bool contrib = false;
      if (jpos < last) {
        const float4 A = s_a[jl];
        const float4 B = s_b[jl];
        const float dx = fx - A.x, dy = fy - A.y;
        const float q = conic_q(A.z, A.w, B.x, dx, dy);
        if (q <= kQCut) {
          const float G = __expf(-0.5f * q);
          const float a0 = B.y * G;
          const float alpha = fminf(kAlphaMax, a0);
          if (alpha >= kAlphaMin) {
            contrib = true;
            const float om = 1.0f - alpha;
            const float Ti = T / om;
            const float c0 = B.z, c1 = B.w, c2 = s_c[jl];
            const float wT = alpha * Ti;
            gr[6] = wT * dC0;
            gr[7] = wT * dC1;
            gr[8] = wT * dC2;
            const float dalpha = dC0 * (Ti * c0 - S0 / om) + dC1 * (Ti * c1 - S1 / om) + dC2 * (Ti * c2 - S2 / om);
            S0 = fmaf(wT, c0, S0);
            S1 = fmaf(wT, c1, S1);
            S2 = fmaf(wT, c2, S2);
            T = Ti;
            if (a0 <= kAlphaMax) {
              gr[5] = dalpha * G;
              const float dq = -0.5f * alpha * dalpha;
              gr[2] = dq * dx * dx;
              gr[3] = dq * 2.0f * dx * dy;
              gr[4] = dq * dy * dy;
              gr[0] = dq * (-2.0f * (A.z * dx + A.w * dy));
              gr[1] = dq * (-2.0f * (A.w * dx + B.x * dy));
            }
          }
        }
      }
      if (__ballot(contrib) != 0ull) {
#pragma unroll
        for (int c = 0; c < kG2d; ++c) {
          const float v = wave_sum(gr[c]);
          if (lane == 0) s_red[w][c][jl] = v;
        }
      } else if (lane == 0) {
#pragma unroll
        for (int c = 0; c < kG2d; ++c) s_red[w][c][jl] = 0.0f;
      }
    }
    __syncthreads();
    if (tid < cnt) {
      const uint32_t g = s_id[tid];
#pragma unroll
      for (int c = 0; c < kG2d; ++c) {
        float v = s_red[0][c][tid];
#pragma unroll
        for (int k = 1; k < kBlock / 64; ++k) v += s_red[k][c][tid];
        if (v != 0.0f) atomicAdd(&g2d[c * stride + g], v);
      }
    }
  }
}

hipError_t launch_blend_bwd(const uint2 *ranges, const uint32_t *values, const float4 *xyab, const float4 *cop,
                            const float *blue, const DevCamera &cam, const float bg[3], const float *final_T,
                            const int32_t *n_contrib, const float *dL_dimage, float *g2d, int64_t g2d_stride,
                            hipStream_t s) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  const int grid = ((n_tiles + kXcdsB - 1) / kXcdsB) * kXcdsB;
  hipLaunchKernelGGL(k_blend_bwd, dim3(grid), dim3(kBlock), 0, s, ranges, values, xyab, cop, blue, cam.W, cam.H,
                     cam.tiles_x, n_tiles, bg[0], bg[1], bg[2], final_T, n_contrib, dL_dimage, g2d, g2d_stride);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_preprocess_bwd(PreParams p, const uint32_t *__restrict__ tiles,
                                                           const float *__restrict__ g2d, int64_t stride,
                                                           flod_grads out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const DevLevel L = p.lv[0];
  if (i >= L.n) return;
  float *dsh = out.d_sh + i * (FLOD_SH_COEFFS * 3);
  if (tiles[i] == 0u) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { out.d_means[i * 3 + k] = 0.f; out.d_log_scales[i * 3 + k] = 0.f; }
    reinterpret_cast<float4 *>(out.d_quats)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    out.d_opacity_logits[i] = 0.f;
    for (int k = 0; k < 12; ++k) reinterpret_cast<float4 *>(dsh)[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  float g[kG2d];
#pragma unroll
  for (int c = 0; c < kG2d; ++c) g[c] = g2d[c * stride + i];
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
  const float d_logit = g[5] * o * (1.0f - o);

  // conic -> dilated 2D covariance (a, b; b, c)
  const float a = pr.a, b = pr.b, c = pr.c;
  const float id2 = 1.0f / (pr.det * pr.det);
  const float gA = g[2], gB = g[3], gC = g[4];
  const float ga = (-c * c * gA + b * c * gB - b * b * gC) * id2;
  const float gb = (2.0f * b * c * gA - (a * c + b * b) * gB + 2.0f * a * b * gC) * id2;
  const float gc = (-b * b * gA + a * b * gB - a * a * gC) * id2;

  // Sigma' = T Sigma T^T with T rows T0, T1
  const float *T0 = pr.Tm, *T1 = pr.Tm + 3;
  const float *S = pr.S;
  float ST0[3], ST1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ST0[k] = S[k * 3 + 0] * T0[0] + S[k * 3 + 1] * T0[1] + S[k * 3 + 2] * T0[2];
    ST1[k] = S[k * 3 + 0] * T1[0] + S[k * 3 + 1] * T1[1] + S[k * 3 + 2] * T1[2];
  }
  float gT0[3], gT1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gT0[k] = 2.0f * ga * ST0[k] + gb * ST1[k];
    gT1[k] = 2.0f * gc * ST1[k] + gb * ST0[k];
  }
  // symmetric gradient of Sigma: Gs = 2 ga T0 T0^T + gb (T0 T1^T + T1 T0^T) + 2 gc T1 T1^T
  float Gs[9];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      Gs[k * 3 + l] = 2.0f * ga * T0[k] * T0[l] + gb * (T0[k] * T1[l] + T1[k] * T0[l]) + 2.0f * gc * T1[k] * T1[l];

  // T = J R_c
  const float *Rc = cam.R;
  float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    gJ00 += gT0[j] * Rc[j];
    gJ02 += gT0[j] * Rc[6 + j];
    gJ11 += gT1[j] * Rc[3 + j];
    gJ12 += gT1[j] * Rc[6 + j];
  }
  // J and mu' -> view-space mean
  const float tz = pr.tz, tx = pr.tx, ty = pr.ty;
  const float iz = 1.0f / tz, iz2 = iz * iz;
  float gtx = g[0] * cam.fx * iz;
  float gty = g[1] * cam.fy * iz;
  float gtz = g[0] * (-cam.fx * tx * iz2) + g[1] * (-cam.fy * ty * iz2) + gJ00 * (-cam.fx * iz2) +
              gJ11 * (-cam.fy * iz2) + gJ02 * (cam.fx * pr.xc * iz2) + gJ12 * (cam.fy * pr.yc * iz2);
  if (pr.unclamped_x) {
    gtx += gJ02 * (-cam.fx * iz) * iz;
    gtz += gJ02 * (-cam.fx * iz) * (-tx * iz2);
  }
  if (pr.unclamped_y) {
    gty += gJ12 * (-cam.fy * iz) * iz;
    gtz += gJ12 * (-cam.fy * iz) * (-ty * iz2);
  }
  float gm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gm[k] = Rc[k] * gtx + Rc[3 + k] * gty + Rc[6 + k] * gtz;

  // colour -> SH coefficients and view direction
  {
    const int deg = p.sh_degree;
    const int nk = (deg + 1) * (deg + 1);
    const float vx = m0 - cam.campos[0], vy = m1 - cam.campos[1], vz = m2 - cam.campos[2];
    const float nv = sqrtf((vx * vx + vy * vy) + vz * vz);
    const float inv = 1.0f / nv;
    const float x = vx * inv, y = vy * inv, z = vz * inv;
    float Y[16], Gx[16], Gy[16], Gz[16];
    sh_basis(deg, x, y, z, Y);
    sh_basis_grad(deg, x, y, z, Gx, Gy, Gz);
    const float4 *shv = reinterpret_cast<const float4 *>(L.sh + i * (FLOD_SH_COEFFS * 3));
    float sh[48];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      float4 v = shv[k];
      sh[4 * k + 0] = v.x; sh[4 * k + 1] = v.y; sh[4 * k + 2] = v.z; sh[4 * k + 3] = v.w;
    }
    float gsh[48];
    float gdx = 0.f, gdy = 0.f, gdz = 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < nk) acc = fmaf(sh[k * 3 + ch], Y[k], acc);
      const float gcol = (acc + 0.5f < 0.0f) ? 0.0f : g[6 + ch];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const bool on = k < nk;
        gsh[k * 3 + ch] = on ? gcol * Y[k] : 0.0f;
        if (on) {
          gdx += gcol * sh[k * 3 + ch] * Gx[k];
          gdy += gcol * sh[k * 3 + ch] * Gy[k];
          gdz += gcol * sh[k * 3 + ch] * Gz[k];
        }
      }
    }
    const float dd = x * gdx + y * gdy + z * gdz;
    gm[0] += (gdx - x * dd) * inv;
    gm[1] += (gdy - y * dd) * inv;
    gm[2] += (gdz - z * dd) * inv;
#pragma unroll
    for (int k = 0; k < 12; ++k)
      reinterpret_cast<float4 *>(dsh)[k] = make_float4(gsh[4 * k], gsh[4 * k + 1], gsh[4 * k + 2], gsh[4 * k + 3]);
  }

  // Sigma = M M^T, M = R diag(s): gM = Gs M
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) M[r * 3 + cc] = pr.R[r * 3 + cc] * pr.s[cc];
  float gR[9], gs[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const float gMrc = Gs[r * 3 + 0] * M[0 * 3 + cc] + Gs[r * 3 + 1] * M[1 * 3 + cc] + Gs[r * 3 + 2] * M[2 * 3 + cc];
      gs[cc] += gMrc * pr.R[r * 3 + cc];
      gR[r * 3 + cc] = gMrc * pr.s[cc];
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) out.d_log_scales[i * 3 + k] = gs[k] * exp_rn1(ls[k]);

  // R(q_hat) -> q_hat -> q
  const float w = pr.w, x = pr.x, y = pr.y, z = pr.z;
  const float gw = 2.0f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
  const float gx = 2.0f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0f * x * gR[4] - w * gR[5] + z * gR[6] +
                           w * gR[7] - 2.0f * x * gR[8]);
  const float gy = 2.0f * (-2.0f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                           z * gR[7] - 2.0f * y * gR[8]);
  const float gz = 2.0f * (-2.0f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0f * z * gR[4] + y * gR[5] +
                           x * gR[6] + y * gR[7]);
  const float dot = w * gw + x * gx + y * gy + z * gz;
  const float inq = 1.0f / pr.nq;
  reinterpret_cast<float4 *>(out.d_quats)[i] =
      make_float4((gw - w * dot) * inq, (gx - x * dot) * inq, (gy - y * dot) * inq, (gz - z * dot) * inq);
#pragma unroll
  for (int k = 0; k < 3; ++k) out.d_means[i * 3 + k] = gm[k];
  out.d_opacity_logits[i] = d_logit;
}

hipError_t launch_preprocess_bwd(const PreParams &p, const uint32_t *tiles, const float *g2d, int64_t g2d_stride,
                                 const flod_grads &g, hipStream_t s) {
  const int64_t n = p.lv[0].n;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_preprocess_bwd, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, tiles,
                     g2d, g2d_stride, g);
  return hipGetLastError();
}

}  // namespace flod

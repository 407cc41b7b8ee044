// Training loss: L1 plus SSIM (section Implementation: the backbone's L1 and SSIM losses).
//
//   F(z)     11 x 11 Gaussian window (sigma 1.5, normalised, separable), zeros outside the image
//   moments  mu_x = F(x), mu_y = F(y), E_xx = F(xx), E_yy = F(yy), E_xy = F(xy)
//   S        (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)),
//            s_xx = E_xx - mu_x^2, s_yy = E_yy - mu_y^2, s_xy = E_xy - mu_x mu_y
//   loss     (1 - lam) mean|x - y| + lam (1 - mean S)
//
// Forward: one workgroup per 16 x 16 output tile and channel. The 26 x 26 input halo goes to
// LDS, a horizontal pass writes the five windowed row sums of the 26 halo rows (FP64) to LDS,
// a vertical pass finishes the moments per pixel. Each pixel then writes the partial
// derivatives of S with respect to mu_x, E_xx and E_xy (FP32, 12 B per channel-pixel), and
// the workgroup writes its sums of S and |x - y| (FP64) for a fixed-order final reduction.
// Backward: the same tiling filters the three derivative maps (the window is symmetric, so F
// is its own adjoint) and combines them: dL/dx = c (F(d_mu) + 2 x F(d_xx) + y F(d_xy)) plus
// the L1 term (1 - lam) sign(x - y) / n, c = -lam / n, times the incoming loss gradient.
// All sums are FP64; inputs and outputs FP32.
#include "flod_internal.h"

namespace flod {

constexpr int kSsimTile = 16;
constexpr int kSsimR = 5;
constexpr int kSsimHalo = kSsimTile + 2 * kSsimR;   // 26
constexpr double kC1 = 0.01 * 0.01;
constexpr double kC2 = 0.03 * 0.03;

struct SsimArgs {
  const float *x, *y;
  int C, H, W, tiles_x;
  double lam, inv_n;
  double g[2 * kSsimR + 1];
};

__device__ __forceinline__ void ssim_load_halo(const float *src, int H, int W, int x0, int y0,
                                               float (*dst)[kSsimHalo]) {
  for (int e = threadIdx.x; e < kSsimHalo * kSsimHalo; e += kBlock) {
    const int r = e / kSsimHalo, c = e % kSsimHalo;
    const int gy = y0 - kSsimR + r, gx = x0 - kSsimR + c;
    dst[r][c] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? src[(int64_t)gy * W + gx] : 0.0f;
  }
}

template <bool WITH_GRAD>
__global__ __launch_bounds__(kBlock) void k_ssim_fwd(SsimArgs a, float *gmap, double2 *partials) {
  __shared__ float sx[kSsimHalo][kSsimHalo], sy[kSsimHalo][kSsimHalo];
  __shared__ double sh[5][kSsimHalo][kSsimTile];
  __shared__ double red[2][kBlock / 64];
  const int ch = blockIdx.y;
  const int x0 = (blockIdx.x % a.tiles_x) * kSsimTile, y0 = (blockIdx.x / a.tiles_x) * kSsimTile;
  const int64_t plane = (int64_t)a.H * a.W;
  ssim_load_halo(a.x + ch * plane, a.H, a.W, x0, y0, sx);
  ssim_load_halo(a.y + ch * plane, a.H, a.W, x0, y0, sy);
  __syncthreads();
  for (int e = threadIdx.x; e < kSsimHalo * kSsimTile; e += kBlock) {
    const int r = e / kSsimTile, c = e % kSsimTile;
    double m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0;
#pragma unroll
    for (int k = 0; k <= 2 * kSsimR; ++k) {
      const double xv = sx[r][c + k], yv = sy[r][c + k], w = a.g[k];
      m0 += w * xv;
      m1 += w * yv;
      m2 += w * (xv * xv);
      m3 += w * (yv * yv);
      m4 += w * (xv * yv);
    }
    sh[0][r][c] = m0; sh[1][r][c] = m1; sh[2][r][c] = m2; sh[3][r][c] = m3; sh[4][r][c] = m4;
  }
  __syncthreads();
  const int tx = threadIdx.x % kSsimTile, ty = threadIdx.x / kSsimTile;
  const int px = x0 + tx, py = y0 + ty;
  double s_sum = 0.0, l1_sum = 0.0;
  if (px < a.W && py < a.H) {
    double mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
#pragma unroll
    for (int k = 0; k <= 2 * kSsimR; ++k) {
      const double w = a.g[k];
      mx += w * sh[0][ty + k][tx];
      my += w * sh[1][ty + k][tx];
      exx += w * sh[2][ty + k][tx];
      eyy += w * sh[3][ty + k][tx];
      exy += w * sh[4][ty + k][tx];
    }
    const double sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
    const double A = 2.0 * mx * my + kC1, B = 2.0 * sxy + kC2;
    const double Cc = mx * mx + my * my + kC1, D = sxx + syy + kC2;
    const double CD = Cc * D;
    const double S = (A * B) / CD;
    s_sum = S;
    const double xv = sx[ty + kSsimR][tx + kSsimR], yv = sy[ty + kSsimR][tx + kSsimR];
    l1_sum = fabs(xv - yv);
    if (WITH_GRAD) {
      const double d_xx = -S / D;
      const double d_xy = 2.0 * A / CD;
      const double d_mu = 2.0 * my * B / CD - 2.0 * mx * S / Cc + 2.0 * mx * S / D - 2.0 * my * A / CD;
      const int64_t o = ch * plane + (int64_t)py * a.W + px, stride = (int64_t)a.C * plane;
      gmap[o] = (float)d_mu;
      gmap[stride + o] = (float)d_xx;
      gmap[2 * stride + o] = (float)d_xy;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    s_sum += __shfl_down(s_sum, off, 64);
    l1_sum += __shfl_down(l1_sum, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s_sum;
    red[1][threadIdx.x >> 6] = l1_sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0, l = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      s += red[0][w];
      l += red[1][w];
    }
    partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = make_double2(s, l);
  }
}

// Fixed-order reduction of the workgroup sums (one workgroup): deterministic loss.
__global__ __launch_bounds__(kBlock) void k_ssim_reduce(const double2 *partials, int64_t count, double lam,
                                                        double inv_n, double *loss) {
  __shared__ double red[2][kBlock / 64];
  double s = 0, l = 0;
  for (int64_t i = threadIdx.x; i < count; i += kBlock) {
    s += partials[i].x;
    l += partials[i].y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_down(s, off, 64);
    l += __shfl_down(l, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s;
    red[1][threadIdx.x >> 6] = l;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double st = 0, lt = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      st += red[0][w];
      lt += red[1][w];
    }
    loss[0] = (1.0 - lam) * (lt * inv_n) + lam * (1.0 - st * inv_n);
  }
}

__global__ __launch_bounds__(kBlock) void k_ssim_bwd(SsimArgs a, const float *gmap, const double *dloss,
                                                     float *dx) {
  __shared__ float sg[3][kSsimHalo][kSsimHalo];
  __shared__ double sh[3][kSsimHalo][kSsimTile];
  const int ch = blockIdx.y;
  const int x0 = (blockIdx.x % a.tiles_x) * kSsimTile, y0 = (blockIdx.x / a.tiles_x) * kSsimTile;
  const int64_t plane = (int64_t)a.H * a.W, stride = (int64_t)a.C * plane;
  for (int m = 0; m < 3; ++m) ssim_load_halo(gmap + m * stride + ch * plane, a.H, a.W, x0, y0, sg[m]);
  __syncthreads();
  for (int e = threadIdx.x; e < kSsimHalo * kSsimTile; e += kBlock) {
    const int r = e / kSsimTile, c = e % kSsimTile;
    double m0 = 0, m1 = 0, m2 = 0;
#pragma unroll
    for (int k = 0; k <= 2 * kSsimR; ++k) {
      const double w = a.g[k];
      m0 += w * (double)sg[0][r][c + k];
      m1 += w * (double)sg[1][r][c + k];
      m2 += w * (double)sg[2][r][c + k];
    }
    sh[0][r][c] = m0; sh[1][r][c] = m1; sh[2][r][c] = m2;
  }
  __syncthreads();
  const int tx = threadIdx.x % kSsimTile, ty = threadIdx.x / kSsimTile;
  const int px = x0 + tx, py = y0 + ty;
  if (px >= a.W || py >= a.H) return;
  double f0 = 0, f1 = 0, f2 = 0;
#pragma unroll
  for (int k = 0; k <= 2 * kSsimR; ++k) {
    const double w = a.g[k];
    f0 += w * sh[0][ty + k][tx];
    f1 += w * sh[1][ty + k][tx];
    f2 += w * sh[2][ty + k][tx];
  }
  const int64_t o = ch * plane + (int64_t)py * a.W + px;
  const double xv = a.x[o], yv = a.y[o];
  const double c = -a.lam * a.inv_n;
  const double t = xv - yv;
  const double sgn = (t > 0.0) ? 1.0 : ((t < 0.0) ? -1.0 : 0.0);
  const double g = c * (f0 + 2.0 * xv * f1 + yv * f2) + (1.0 - a.lam) * sgn * a.inv_n;
  dx[o] = (float)(dloss ? g * dloss[0] : g);
}

static SsimArgs ssim_args(const float *x, const float *y, int C, int H, int W, float lam) {
  SsimArgs a;
  a.x = x;
  a.y = y;
  a.C = C;
  a.H = H;
  a.W = W;
  a.tiles_x = (W + kSsimTile - 1) / kSsimTile;
  a.lam = (double)lam;
  a.inv_n = 1.0 / ((double)C * (double)H * (double)W);
  double sum = 0.0;
  for (int k = 0; k <= 2 * kSsimR; ++k) {
    const double d = (double)(k - kSsimR);
    a.g[k] = std::exp(-(d * d) / (2.0 * 1.5 * 1.5));
    sum += a.g[k];
  }
  for (int k = 0; k <= 2 * kSsimR; ++k) a.g[k] /= sum;
  return a;
}

int64_t ssim_blocks(int C, int H, int W) {
  return (int64_t)((W + kSsimTile - 1) / kSsimTile) * ((H + kSsimTile - 1) / kSsimTile) * C;
}

hipError_t launch_ssim_forward(const float *x, const float *y, int C, int H, int W, float lam, double *loss,
                               float *gmap, double2 *partials, hipStream_t s) {
  const SsimArgs a = ssim_args(x, y, C, H, W, lam);
  const dim3 grid((unsigned)(a.tiles_x * ((H + kSsimTile - 1) / kSsimTile)), (unsigned)C);
  if (gmap)
    hipLaunchKernelGGL(k_ssim_fwd<true>, grid, dim3(kBlock), 0, s, a, gmap, partials);
  else
    hipLaunchKernelGGL(k_ssim_fwd<false>, grid, dim3(kBlock), 0, s, a, gmap, partials);
  hipLaunchKernelGGL(k_ssim_reduce, dim3(1), dim3(kBlock), 0, s, partials, ssim_blocks(C, H, W), a.lam, a.inv_n,
                     loss);
  return hipGetLastError();
}

hipError_t launch_ssim_backward(const float *x, const float *y, int C, int H, int W, float lam, const float *gmap,
                                const double *dloss, float *dx, hipStream_t s) {
  const SsimArgs a = ssim_args(x, y, C, H, W, lam);
  const dim3 grid((unsigned)(a.tiles_x * ((H + kSsimTile - 1) / kSsimTile)), (unsigned)C);
  hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(kBlock), 0, s, a, gmap, dloss, dx);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Plain L1 loss, mean|x - y| over `count` elements (the image loss of the training step):
// a grid-stride FP64 sum per workgroup, then the fixed-order reduction above; the backward
// writes sign(x - y) / count times the incoming loss gradient.
// ---------------------------------------------------------------------------------------
constexpr int kL1Blocks = 1024;

__global__ __launch_bounds__(kBlock) void k_l1_fwd(const float4 *__restrict__ x, const float4 *__restrict__ y,
                                                   const float *__restrict__ xs, const float *__restrict__ ys,
                                                   int64_t n4, int64_t n, double2 *partials) {
  __shared__ double red[kBlock / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kBlock) {
    const float4 a = x[i], b = y[i];
    acc += (double)fabsf(a.x - b.x) + (double)fabsf(a.y - b.y) + (double)fabsf(a.z - b.z) +
           (double)fabsf(a.w - b.w);
  }
  if (blockIdx.x == 0)
    for (int64_t i = n4 * 4 + threadIdx.x; i < n; i += kBlock) acc += (double)fabsf(xs[i] - ys[i]);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    partials[blockIdx.x] = make_double2(0.0, t);
  }
}

__global__ __launch_bounds__(kBlock) void k_l1_bwd(const float *__restrict__ x, const float *__restrict__ y,
                                                   int64_t n, double inv_n, const double *dloss,
                                                   float *__restrict__ dx) {
  const float scale = (float)(dloss ? inv_n * dloss[0] : inv_n);
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const float t = x[i] - y[i];
    dx[i] = t > 0.0f ? scale : (t < 0.0f ? -scale : 0.0f);
  }
}

int64_t l1_blocks() { return kL1Blocks; }

hipError_t launch_l1_forward(const float *x, const float *y, int64_t n, double *loss, double2 *partials,
                             hipStream_t s) {
  const bool vec = (reinterpret_cast<uintptr_t>(x) % 16 == 0) && (reinterpret_cast<uintptr_t>(y) % 16 == 0);
  const int64_t n4 = vec ? n / 4 : 0;
  hipLaunchKernelGGL(k_l1_fwd, dim3(kL1Blocks), dim3(kBlock), 0, s, reinterpret_cast<const float4 *>(x),
                     reinterpret_cast<const float4 *>(y), x, y, n4, n, partials);
  // (1 - lam) L1 + lam (1 - S) with lam = 0 and the S sums zero: the mean of |x - y|
  hipLaunchKernelGGL(k_ssim_reduce, dim3(1), dim3(kBlock), 0, s, partials, (int64_t)kL1Blocks, 0.0,
                     1.0 / (double)n, loss);
  return hipGetLastError();
}

hipError_t launch_l1_backward(const float *x, const float *y, int64_t n, const double *dloss, float *dx,
                              hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_l1_bwd, dim3((unsigned)blocks), dim3(kBlock), 0, s, x, y, n, 1.0 / (double)n, dloss, dx);
  return hipGetLastError();
}

}  // namespace flod

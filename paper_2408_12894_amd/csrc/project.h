// Per-Gaussian projection used by the forward preprocess and recomputed by the backward.
//
// Evaluated in FP64 from the FP32 inputs (the preprocess is bound by HBM, so FP64 costs
// nothing here) with IEEE basic operations in a fixed order and no contraction (the library
// is built with -ffp-contract=off); the only transcendental, exp(s_opt), is evaluated in FP64
// and rounded to FP32 before use, so the whole chain is reproducible on any IEEE machine:
//   t = R_c mu + t_c                            view transform
//   s = float(exp(s_opt)) + s_min               eq. 4
//   q_hat = q / |q|;  R = R(q_hat)              unit quaternion (w, x, y, z)
//   Sigma = M M^T, M = R diag(s)                eq. 1
//   J = [[fx/tz, 0, -fx xc/tz], [0, fy/tz, -fy yc/tz]], xc, yc clamped to 1.3 half-FOV
//   Sigma' = (J R_c) Sigma (J R_c)^T + 0.3 I    EWA splat with dilation
//   tiles: per tile row, the columns where the ellipse q <= 9 (1 + 1e-3) reaches
// Each sum is evaluated left to right in the order written.
#pragma once

#include "flod_internal.h"

namespace flod {

struct Proj {
  double tx, ty, tz;
  double s[3];
  double w, x, y, z, nq;      // unit quaternion and the input's norm
  double R[9];
  double S[9];                // 3D covariance, full symmetric
  double u, v, xc, yc;
  bool unclamped_x, unclamped_y;
  double J00, J02, J11, J12;
  double Tm[6];               // J R_c
  double a, b, c, det;        // dilated 2D covariance and its determinant
  double ca, cb, cc;          // conic
  double mx, my;
};

// exp of an FP32 value in FP64, rounded once to FP32.
__device__ __forceinline__ float exp_rn1(float v) { return (float)exp((double)v); }

// Steps that depend only on the mean: view transform.
__device__ __forceinline__ void view_transform(const DevCamera &cam, float m0, float m1, float m2, Proj &p) {
  const double x = m0, y = m1, z = m2;
  p.tx = (((double)cam.R[0] * x + (double)cam.R[1] * y) + (double)cam.R[2] * z) + (double)cam.t[0];
  p.ty = (((double)cam.R[3] * x + (double)cam.R[4] * y) + (double)cam.R[5] * z) + (double)cam.t[1];
  p.tz = (((double)cam.R[6] * x + (double)cam.R[7] * y) + (double)cam.R[8] * z) + (double)cam.t[2];
}

// Everything after the view transform. Returns false for a zero-norm quaternion.
__device__ __forceinline__ bool project_cov(const DevCamera &cam, const float ls[3], const float q4[4],
                                            float s_min, Proj &p) {
  for (int i = 0; i < 3; ++i) p.s[i] = (double)exp_rn1(ls[i]) + (double)s_min;
  const double q0 = q4[0], q1 = q4[1], q2 = q4[2], q3 = q4[3];
  const double n2 = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
  const bool ok = n2 > 0.0;
  p.nq = sqrt(ok ? n2 : 1.0);
  p.w = q0 / p.nq;
  p.x = q1 / p.nq;
  p.y = q2 / p.nq;
  p.z = q3 / p.nq;
  const double w = p.w, x = p.x, y = p.y, z = p.z;
  double *R = p.R;
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
  double M[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i * 3 + j] = R[i * 3 + j] * p.s[j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const double v = (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];
      p.S[i * 3 + j] = v;
      p.S[j * 3 + i] = v;
    }
  const double fx = cam.fx, fy = cam.fy;
  p.u = p.tx / p.tz;
  p.v = p.ty / p.tz;
  const double limx = kFovClampD * ((0.5 * (double)cam.W) / fx);
  const double limy = kFovClampD * ((0.5 * (double)cam.H) / fy);
  p.xc = fmin(fmax(p.u, -limx), limx);
  p.yc = fmin(fmax(p.v, -limy), limy);
  p.unclamped_x = (p.u >= -limx) && (p.u <= limx);
  p.unclamped_y = (p.v >= -limy) && (p.v <= limy);
  p.J00 = fx / p.tz;
  p.J02 = -(fx * p.xc) / p.tz;
  p.J11 = fy / p.tz;
  p.J12 = -(fy * p.yc) / p.tz;
  double Rc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Rc[i] = cam.R[i];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    p.Tm[j] = p.J00 * Rc[j] + p.J02 * Rc[6 + j];
    p.Tm[3 + j] = p.J11 * Rc[3 + j] + p.J12 * Rc[6 + j];
  }
  double U[6];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      U[i * 3 + j] = (p.Tm[i * 3 + 0] * p.S[j] + p.Tm[i * 3 + 1] * p.S[3 + j]) + p.Tm[i * 3 + 2] * p.S[6 + j];
  const double s00 = (U[0] * p.Tm[0] + U[1] * p.Tm[1]) + U[2] * p.Tm[2];
  const double s01 = (U[0] * p.Tm[3] + U[1] * p.Tm[4]) + U[2] * p.Tm[5];
  const double s11 = (U[3] * p.Tm[3] + U[4] * p.Tm[4]) + U[5] * p.Tm[5];
  p.a = s00 + kDilateD;
  p.b = s01;
  p.c = s11 + kDilateD;
  p.det = p.a * p.c - p.b * p.b;
  const double inv = 1.0 / p.det;
  p.ca = p.c * inv;
  p.cb = -p.b * inv;
  p.cc = p.a * inv;
  p.mx = fx * p.u + (double)cam.cx;
  p.my = fy * p.v + (double)cam.cy;
  return ok;
}

// ---------------------------------------------------------------------------------------
// Tile footprint. A pixel blends a Gaussian only if q <= 9 and o exp(-q/2) >= 1/255, i.e.
// q <= Q_g = min(9, 2 ln(255 o)); Q_g is formed from the FP32 logit with exp and log in
// FP64, each result rounded to FP32, so that any last-bit difference between math libraries
// vanishes. A Gaussian is binned to a tile when the tile's pixel-centre rows meet the ellipse
// d^T conic d <= Q with Q = Q_g (1 + 1e-3) + 1e-3 (at that q the blend's alpha is below 1/255
// by a relative 5e-4, far above FP32 and fast-exp error): per tile row, the x-extent of the
// ellipse over the row's band of pixel centres is found in closed form (the right boundary
// is concave in dy, so its maximum over the band is the ellipse's rightmost point when that
// lies in the band, else a band end; the left boundary mirrors it). Computed in FP64 from the
// stored FP32 mu', conic and Q_g by the preprocess (to count) and the emission (to write), so
// both agree exactly.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ float support_q(float logit) {
  const float o = (float)(1.0 / (1.0 + exp(-(double)logit)));
  return (float)fmin(9.0, fmax(0.0, 2.0 * log(255.0 * (double)o)));
}

__device__ __forceinline__ double support_span(float qg) { return (double)qg * 1.001 + 1e-3; }


struct Footprint {
  double mx, my, a, b, c, det, ia, hx, hy, dyr, Q;
  int ty0, ty1;
};

__device__ __forceinline__ bool footprint(float mx, float my, float a, float b, float c, double Q, int tiles_y,
                                          Footprint &f) {
  f.mx = mx; f.my = my; f.a = a; f.b = b; f.c = c; f.Q = Q;
  f.det = f.a * f.c - f.b * f.b;
  if (!(f.det > 0.0) || !(f.a > 0.0)) return false;
  // reciprocals taken once; the rows multiply by them
  const double idet = 1.0 / f.det;
  f.ia = 1.0 / f.a;
  const double sxx = f.c * idet, syy = f.a * idet, sxy = -f.b * idet;
  f.hx = sqrt(Q * sxx);
  f.hy = sqrt(Q * syy);
  f.dyr = sxy * sqrt(Q / sxx);
  double y0 = floor((f.my - f.hy) * 0.0625);
  double y1 = floor((f.my + f.hy) * 0.0625);
  y0 = fmax(y0, 0.0);
  y1 = fmin(y1, (double)(tiles_y - 1));
  if (!(y0 <= y1)) return false;
  f.ty0 = (int)y0;
  f.ty1 = (int)y1;
  return true;
}

// Tiles [tx0, tx1] of tile row ty that the footprint reaches; false if none.
__device__ __forceinline__ bool row_span(const Footprint &f, int ty, int tiles_x, int &tx0, int &tx1) {
  const double dlo = fmax((16.0 * ty + 0.5) - f.my, -f.hy);
  const double dhi = fmin((16.0 * ty + 15.5) - f.my, f.hy);
  if (!(dlo <= dhi)) return false;
  const double qa = f.Q * f.a;
  const double rlo = sqrt(fmax(0.0, qa - f.det * dlo * dlo));
  const double rhi = sqrt(fmax(0.0, qa - f.det * dhi * dhi));
  const double right = (dlo <= f.dyr && f.dyr <= dhi) ? f.hx : fmax((-f.b * dlo + rlo) * f.ia, (-f.b * dhi + rhi) * f.ia);
  const double left = (dlo <= -f.dyr && -f.dyr <= dhi) ? -f.hx : fmin((-f.b * dlo - rlo) * f.ia, (-f.b * dhi - rhi) * f.ia);
  double x0 = floor((f.mx + left) * 0.0625);
  double x1 = floor((f.mx + right) * 0.0625);
  x0 = fmax(x0, 0.0);
  x1 = fmin(x1, (double)(tiles_x - 1));
  if (!(x0 <= x1)) return false;
  tx0 = (int)x0;
  tx1 = (int)x1;
  return true;
}

// bf16 (round to nearest even) of an FP32 value, in the upper half of a 32-bit word.
__device__ __forceinline__ uint32_t bf16_bits(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
}

// mu' = hi + lo with hi = float(mu') and lo the residual rounded to bf16; packed as
// (lo_x bits >> 16) | lo_y bits.
__device__ __forceinline__ uint32_t pack_mu_lo(double mx, double my, float hx, float hy) {
  const uint32_t lx = bf16_bits((float)(mx - (double)hx));
  const uint32_t ly = bf16_bits((float)(my - (double)hy));
  return (lx >> 16) | ly;
}

__device__ __forceinline__ float mu_lo_x(uint32_t packed) { return __uint_as_float(packed << 16); }
__device__ __forceinline__ float mu_lo_y(uint32_t packed) { return __uint_as_float(packed & 0xFFFF0000u); }

// Real spherical harmonics up to degree 3 (orthonormal, no Condon-Shortley phase),
// index l*l + l + m, evaluated at a unit direction.
__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float Y[16]) {
  const float C0 = 0.28209479177387814f;
  const float C1 = 0.4886025119029199f;
  const float C2a = 1.0925484305920792f, C20 = 0.31539156525252005f, C22 = 0.5462742152960396f;
  const float C33 = 0.5900435899266435f, C32b = 2.890611442640554f, C31 = 0.4570457994644658f,
              C30 = 0.3731763325901154f, C32 = 1.445305721320277f;
  Y[0] = C0;
  if (deg < 1) return;
  Y[1] = C1 * y;
  Y[2] = C1 * z;
  Y[3] = C1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = C2a * x * y;
  Y[5] = C2a * y * z;
  Y[6] = C20 * (3.0f * zz - 1.0f);
  Y[7] = C2a * x * z;
  Y[8] = C22 * (xx - yy);
  if (deg < 3) return;
  Y[9] = C33 * y * (3.0f * xx - yy);
  Y[10] = C32b * x * y * z;
  Y[11] = C31 * y * (5.0f * zz - 1.0f);
  Y[12] = C30 * z * (5.0f * zz - 3.0f);
  Y[13] = C31 * x * (5.0f * zz - 1.0f);
  Y[14] = C32 * z * (xx - yy);
  Y[15] = C33 * x * (xx - 3.0f * yy);
}

// Gradient of each basis polynomial with respect to (x, y, z).
__device__ __forceinline__ void sh_basis_grad(int deg, float x, float y, float z, float gx[16],
                                              float gy[16], float gz[16]) {
  const float C1 = 0.4886025119029199f;
  const float C2a = 1.0925484305920792f, C20 = 0.31539156525252005f, C22 = 0.5462742152960396f;
  const float C33 = 0.5900435899266435f, C32b = 2.890611442640554f, C31 = 0.4570457994644658f,
              C30 = 0.3731763325901154f, C32 = 1.445305721320277f;
  for (int k = 0; k < 16; ++k) { gx[k] = 0.f; gy[k] = 0.f; gz[k] = 0.f; }
  if (deg < 1) return;
  gy[1] = C1;
  gz[2] = C1;
  gx[3] = C1;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx[4] = C2a * y; gy[4] = C2a * x;
  gy[5] = C2a * z; gz[5] = C2a * y;
  gz[6] = C20 * 6.0f * z;
  gx[7] = C2a * z; gz[7] = C2a * x;
  gx[8] = C22 * 2.0f * x; gy[8] = -C22 * 2.0f * y;
  if (deg < 3) return;
  gx[9] = C33 * 6.0f * x * y;          gy[9] = C33 * 3.0f * (xx - yy);
  gx[10] = C32b * y * z;               gy[10] = C32b * x * z;          gz[10] = C32b * x * y;
  gy[11] = C31 * (5.0f * zz - 1.0f);   gz[11] = C31 * 10.0f * y * z;
  gz[12] = C30 * (15.0f * zz - 3.0f);
  gx[13] = C31 * (5.0f * zz - 1.0f);   gz[13] = C31 * 10.0f * x * z;
  gx[14] = C32 * 2.0f * x * z;         gy[14] = -C32 * 2.0f * y * z;   gz[14] = C32 * (xx - yy);
  gx[15] = C33 * 3.0f * (xx - yy);     gy[15] = -C33 * 6.0f * x * y;
}

// Level of a global candidate index, with constant-index access to the kernel arguments.
__device__ __forceinline__ int level_of(const PreParams &p, int64_t i) {
  int l = 0;
#pragma unroll
  for (int k = 1; k < FLOD_MAX_LEVELS; ++k)
    if (k < p.n_levels && i >= p.lv[k].offset) l = k;
  return l;
}

__device__ __forceinline__ DevLevel level_at(const PreParams &p, int l) {
  DevLevel L = p.lv[0];
#pragma unroll
  for (int k = 1; k < FLOD_MAX_LEVELS; ++k)
    if (k == l) L = p.lv[k];
  return L;
}

// Squared distance used by eq. 6, FP32, summed x, y, z.
__device__ __forceinline__ float dist2(float m0, float m1, float m2, const float c[3]) {
  float dx = m0 - c[0], dy = m1 - c[1], dz = m2 - c[2];
  return (dx * dx + dy * dy) + dz * dz;
}

// The blend kernels evaluate o exp(-q/2) as 2^(k q + log2 o), k = -log2(e) / 2, with the scale
// and log2 o folded into the staged terms below, so that each (pixel, entry) pair forms
// l = k q + log2 o (the log2 of the unclamped alpha) directly and takes one hardware exp2:
// within a few ulp of o exp(-q/2). The support cut q <= 9 becomes k q >= 9 k, the alpha floor
// o exp(-q/2) >= 1/255 becomes l >= log2(1/255): both are l >= max(log2(1/255), 9 k + log2 o),
// one threshold per entry.
constexpr float kExpScale = -0.72134752044448170f;
constexpr float kQCutScaled = kQCut * kExpScale;
constexpr float kLog2AlphaMin = -7.99435343685885793f;   // log2(1/255)
__device__ __forceinline__ float alpha_from_log2(float l) { return __builtin_amdgcn_exp2f(l); }

// q = a dx^2 + 2 b dx dy + c dy^2 completed to a square in dy:
//   q = c v^2 + (det / c) dx^2,  v = dy + (b / c) dx,  det = a c - b^2 > 0, c > 0,
// a sum of two non-negative terms. The expanded form cancels for elongated footprints far
// from the centre (terms of thousands summing to a q of a few units: about 1e-4 relative
// error in FP32); here the only cancellation is in v, whose error stays near an ulp of dy.
// An entry is staged as r = b / c, e = k det / c (det by Kahan's two-product method, from the
// stored FP32 conic) and c_k = k c, with mu' relative to the tile's corner (see stage_entry).
// Per column (a lane's pixels share dx = x - mu'x): t = e dx^2 + log2 o; per pixel, with
// dy = y - mu'y: v = dy + r dx (one FMA), l = c_k v^2 + t = k q + log2 o.
// Shared by both blend kernels so that they take the same decisions on the same bits.
__device__ __forceinline__ void conic_stage(float a, float b, float c, float &r, float &ek, float &ck) {
  const float p = b * b;
  const float perr = fmaf(b, b, -p);              // b^2 = p + perr exactly
  const float det = fmaf(a, c, -p) - perr;
  const float ic = 1.0f / c;
  r = b * ic;
  ek = kExpScale * (det * ic);
  ck = kExpScale * c;
}

__device__ __forceinline__ float conic_column(float ek, float dx, float lo) { return fmaf(ek * dx, dx, lo); }

__device__ __forceinline__ float conic_kq(float ck, float r, float dx, float dy, float t) {
  const float v = fmaf(r, dx, dy);
  return fmaf(ck * v, v, t);
}

}  // namespace flod

// Per-Gaussian projection used by the forward preprocess and recomputed by the backward.
//
// Key path (exact, IEEE FP32, no contraction: the library is built with -ffp-contract=off):
//   t = R_c mu + t_c                            view transform
//   s = exp(s_opt) + s_min                      eq. 4 (exp in FP64, rounded once)
//   q_hat = q / |q|;  R = R(q_hat)              unit quaternion (w, x, y, z)
//   Sigma = M M^T, M = R diag(s)                eq. 1
//   J = [[fx/tz, 0, -fx xc/tz], [0, fy/tz, -fy yc/tz]], xc, yc clamped to 1.3 half-FOV
//   Sigma' = (J R_c) Sigma (J R_c)^T + 0.3 I    EWA splat with dilation
//   r = ceil(3 sqrt(lambda_max)), lambda_max = m + sqrt(max(0.1, m^2 - det))
// Each sum is evaluated left to right in the order written; divisions and square roots are
// IEEE correctly rounded (HIP's default for FP32).
#pragma once

#include "flod_internal.h"

namespace flod {

struct Proj {
  float tx, ty, tz;
  float s[3];
  float w, x, y, z, nq;       // unit quaternion and the input's norm
  float R[9];
  float S[9];                 // 3D covariance, full symmetric
  float u, v, xc, yc;
  bool unclamped_x, unclamped_y;
  float J00, J02, J11, J12;
  float Tm[6];                // J R_c
  float a, b, c, det;         // dilated 2D covariance and its determinant
  float ca, cb, cc;           // conic
  float mx, my;
};

__device__ __forceinline__ float exp_rn1(float v) { return (float)exp((double)v); }

// Steps that depend only on the mean: view transform.
__device__ __forceinline__ void view_transform(const DevCamera &cam, float m0, float m1, float m2,
                                               Proj &p) {
  p.tx = ((cam.R[0] * m0 + cam.R[1] * m1) + cam.R[2] * m2) + cam.t[0];
  p.ty = ((cam.R[3] * m0 + cam.R[4] * m1) + cam.R[5] * m2) + cam.t[1];
  p.tz = ((cam.R[6] * m0 + cam.R[7] * m1) + cam.R[8] * m2) + cam.t[2];
}

// Everything after the view transform. Returns false for a zero-norm quaternion.
__device__ __forceinline__ bool project_cov(const DevCamera &cam, const float ls[3], const float q[4],
                                            float s_min, Proj &p) {
  for (int i = 0; i < 3; ++i) p.s[i] = exp_rn1(ls[i]) + s_min;
  float n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  bool ok = n2 > 0.0f;
  p.nq = sqrtf(ok ? n2 : 1.0f);
  p.w = q[0] / p.nq;
  p.x = q[1] / p.nq;
  p.y = q[2] / p.nq;
  p.z = q[3] / p.nq;
  const float w = p.w, x = p.x, y = p.y, z = p.z;
  float *R = p.R;
  R[0] = 1.0f - 2.0f * (y * y + z * z);
  R[1] = 2.0f * (x * y - w * z);
  R[2] = 2.0f * (x * z + w * y);
  R[3] = 2.0f * (x * y + w * z);
  R[4] = 1.0f - 2.0f * (x * x + z * z);
  R[5] = 2.0f * (y * z - w * x);
  R[6] = 2.0f * (x * z - w * y);
  R[7] = 2.0f * (y * z + w * x);
  R[8] = 1.0f - 2.0f * (x * x + y * y);
  float M[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i * 3 + j] = R[i * 3 + j] * p.s[j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      float v = (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];
      p.S[i * 3 + j] = v;
      p.S[j * 3 + i] = v;
    }
  p.u = p.tx / p.tz;
  p.v = p.ty / p.tz;
  const float limx = kFovClamp * ((0.5f * (float)cam.W) / cam.fx);
  const float limy = kFovClamp * ((0.5f * (float)cam.H) / cam.fy);
  p.xc = fminf(fmaxf(p.u, -limx), limx);
  p.yc = fminf(fmaxf(p.v, -limy), limy);
  p.unclamped_x = (p.u >= -limx) && (p.u <= limx);
  p.unclamped_y = (p.v >= -limy) && (p.v <= limy);
  p.J00 = cam.fx / p.tz;
  p.J02 = -(cam.fx * p.xc) / p.tz;
  p.J11 = cam.fy / p.tz;
  p.J12 = -(cam.fy * p.yc) / p.tz;
  const float *Rc = cam.R;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    p.Tm[j] = p.J00 * Rc[j] + p.J02 * Rc[6 + j];
    p.Tm[3 + j] = p.J11 * Rc[3 + j] + p.J12 * Rc[6 + j];
  }
  float U[6];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      U[i * 3 + j] = (p.Tm[i * 3 + 0] * p.S[j] + p.Tm[i * 3 + 1] * p.S[3 + j]) + p.Tm[i * 3 + 2] * p.S[6 + j];
  float s00 = (U[0] * p.Tm[0] + U[1] * p.Tm[1]) + U[2] * p.Tm[2];
  float s01 = (U[0] * p.Tm[3] + U[1] * p.Tm[4]) + U[2] * p.Tm[5];
  float s11 = (U[3] * p.Tm[3] + U[4] * p.Tm[4]) + U[5] * p.Tm[5];
  p.a = s00 + kDilate;
  p.b = s01;
  p.c = s11 + kDilate;
  p.det = p.a * p.c - p.b * p.b;
  float inv = 1.0f / p.det;
  p.ca = p.c * inv;
  p.cb = -p.b * inv;
  p.cc = p.a * inv;
  p.mx = cam.fx * p.u + cam.cx;
  p.my = cam.fy * p.v + cam.cy;
  return ok;
}

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

// q = d^T conic d, shared by the forward and backward blend so both take the same
// decisions (support cut, alpha floor) on the same bits.
__device__ __forceinline__ float conic_q(float a, float b, float c, float dx, float dy) {
  return fmaf(a * dx, dx, fmaf(c * dy, dy, 2.0f * b * dx * dy));
}

}  // namespace flod

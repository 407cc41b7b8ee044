// CPU oracle for the FLoD-3DGS rasterizer hot path.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the benchmark's
// CPU-baseline leg load this library. The product path (the HIP library) never links,
// loads or calls it, and the two share no code.
//
// Three parts, each a plain definition with no tiling, blocking or early-out beyond what
// the definition itself states:
//   O1  key mirror: per-Gaussian discrete decisions (selection, culls, depth bits, tile
//       footprint) and the stored FP32 projection (mu' and its bf16 residual,
//       conic), from the FP64 projection of the FP32 inputs in a fixed operation order with
//       no contraction and the scale's exp rounded once to FP32, followed by std::sort of
//       the (tile, depth bits, index) instance list.
//   O2  FP64 image: every pixel loops over all surviving Gaussians in O1 depth order
//       and composites front to back in double precision.
//   O3  FP64 gradient: per-pixel reverse compositing in double, then the per-Gaussian
//       chain rule from 2D to 3D parameters by forward-mode dual numbers over the same
//       projection code that O2 uses.
//
// Method sources (FLoD paper):
//   Preliminary section, eq. 1    Sigma = R S S^T R^T
//   Preliminary section, eq. 2    alpha(x,y) = o exp(-1/2 d^T Sigma'^-1 d)
//   Preliminary section           alpha blending in depth order
//   Section 3D Scale Constraint, eq. 3 and eq. 4   s = exp(s_opt) + s_min
//   Section Selective Rendering, eq. 6 and eq. 7   distance bands
//   Section Overlap Pruning                        three-nearest-neighbour mean distance
//   Section Training Method, eq. 5                 level-transition scale parameter
// The projection (EWA Jacobian, dilation, radius) and compositing constants are the
// conventions of the 3DGS framework the paper builds on; the paper does not restate them.
// Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>
#include <type_traits>

namespace {

constexpr int TILE = 16;
constexpr double PI = 3.14159265358979323846;

// Named conventions, per precision.
template <class T> struct K;
template <> struct K<float> {
  static constexpr float near_z = 0.2f, dilate = 0.3f, eig_floor = 0.1f, fov_clamp = 1.3f;
  static constexpr float half = 0.5f, three = 3.0f, tile_inv = 0.0625f;
};
template <> struct K<double> {
  static constexpr double near_z = 0.2, dilate = 0.3, eig_floor = 0.1, fov_clamp = 1.3;
  static constexpr double half = 0.5, three = 3.0, tile_inv = 0.0625;
};

// ---------------------------------------------------------------------------------
// Forward-mode dual numbers (value plus ND directional derivatives).
// Directions: 0-2 mean, 3-5 log-scale, 6-9 quaternion, 10 opacity logit.
// ---------------------------------------------------------------------------------
constexpr int ND = 11;
struct Dual {
  double v;
  double d[ND];
  Dual() : v(0) { for (int i = 0; i < ND; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < ND; ++i) d[i] = 0; }
  static Dual var(double x, int k) { Dual r(x); r.d[k] = 1.0; return r; }
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int i = 0; i < ND; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int i = 0; i < ND; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { return a * Dual(b); }
inline Dual operator*(double a, const Dual& b) { return Dual(a) * b; }
inline Dual operator/(const Dual& a, double b) { return a / Dual(b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }

inline float ex(float x) { return (float)std::exp((double)x); }   // FP64 exp, rounded once
inline double ex(double x) { return std::exp(x); }
inline Dual ex(const Dual& a) { double e = std::exp(a.v); Dual r(e); for (int i = 0; i < ND; ++i) r.d[i] = e * a.d[i]; return r; }
inline float sq(float x) { return std::sqrt(x); }
inline double sq(double x) { return std::sqrt(x); }
inline Dual sq(const Dual& a) { double s = std::sqrt(a.v); Dual r(s); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] / (2.0 * s); return r; }
inline double val(float x) { return x; }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
template <class T> inline T tmin(const T& a, const T& b) { return val(b) < val(a) ? b : a; }
template <class T> inline T tmax(const T& a, const T& b) { return val(a) < val(b) ? b : a; }

template <class T> struct Cam {
  T R[9], t[3], campos[3], fx, fy, cx, cy;
  int W, H;
};

struct CamIn {  // layout shared with the Python wrapper (ctypes)
  float R[9], t[3], campos[3], fx, fy, cx, cy;
  int32_t W, H;
};

template <class T> Cam<T> cam_as(const CamIn& c) {
  Cam<T> r;
  for (int i = 0; i < 9; ++i) r.R[i] = T(c.R[i]);
  for (int i = 0; i < 3; ++i) { r.t[i] = T(c.t[i]); r.campos[i] = T(c.campos[i]); }
  r.fx = T(c.fx); r.fy = T(c.fy); r.cx = T(c.cx); r.cy = T(c.cy);
  r.W = c.W; r.H = c.H;
  return r;
}

// ---------------------------------------------------------------------------------
// Real spherical harmonics, built from their definition (not from a constant table):
//   Y_l^0  = K_l^0 P_l(z)
//   Y_l^m  = sqrt2 K_l^m  Q_l^m(z) Re((x+iy)^m)     m > 0
//   Y_l^-m = sqrt2 K_l^m  Q_l^m(z) Im((x+iy)^m)     m > 0
// with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), Q_l^m = d^m P_l / dz^m (so that
// P_l^m = (1-z^2)^(m/2) Q_l^m, no Condon-Shortley phase), P_l by Bonnet's recursion.
// Coefficient index k = l*l + l + m.
// ---------------------------------------------------------------------------------
struct ShTables {
  double poly[4][4][4];   // poly[l][m][j]: coefficient of z^j in Q_l^m
  double norm[4][4];      // sqrt2 K_l^m for m > 0, K_l^0 for m = 0
  ShTables() {
    double P[4][4] = {{0}};
    P[0][0] = 1.0;
    P[1][1] = 1.0;
    for (int l = 1; l < 3; ++l)   // (l+1) P_{l+1} = (2l+1) z P_l - l P_{l-1}
      for (int j = 0; j < 4; ++j) {
        double zp = (j > 0) ? P[l][j - 1] : 0.0;
        P[l + 1][j] = ((2 * l + 1) * zp - l * P[l - 1][j]) / (l + 1);
      }
    for (int l = 0; l < 4; ++l) {
      double cur[4];
      for (int j = 0; j < 4; ++j) cur[j] = P[l][j];
      for (int m = 0; m <= l; ++m) {
        for (int j = 0; j < 4; ++j) poly[l][m][j] = cur[j];
        double nxt[4] = {0, 0, 0, 0};
        for (int j = 1; j < 4; ++j) nxt[j - 1] = j * cur[j];
        for (int j = 0; j < 4; ++j) cur[j] = nxt[j];
      }
      for (int m = 0; m <= l; ++m) {
        double f = 1.0;
        for (int i = l - m + 1; i <= l + m; ++i) f *= i;   // (l+m)!/(l-m)!
        double k = std::sqrt((2 * l + 1) / (4.0 * PI) / f);
        norm[l][m] = (m == 0) ? k : std::sqrt(2.0) * k;
      }
      for (int m = l + 1; m < 4; ++m) { norm[l][m] = 0; for (int j = 0; j < 4; ++j) poly[l][m][j] = 0; }
    }
  }
};
const ShTables& sh_tables() { static ShTables t; return t; }

template <class T> void sh_basis(int deg, const T& x, const T& y, const T& z, T out[16]) {
  const ShTables& tb = sh_tables();
  T re[4], im[4];   // (x + i y)^m
  re[0] = T(1.0); im[0] = T(0.0);
  for (int m = 1; m < 4; ++m) {
    re[m] = re[m - 1] * x - im[m - 1] * y;
    im[m] = re[m - 1] * y + im[m - 1] * x;
  }
  for (int k = 0; k < 16; ++k) out[k] = T(0.0);
  for (int l = 0; l <= deg; ++l)
    for (int m = 0; m <= l; ++m) {
      T q = T(0.0);
      for (int j = 3; j >= 0; --j) q = q * z + T(tb.poly[l][m][j]);
      T base = q * T(tb.norm[l][m]);
      if (m == 0) {
        out[l * l + l] = base;
      } else {
        out[l * l + l + m] = base * re[m];
        out[l * l + l - m] = base * im[m];
      }
    }
}

// ---------------------------------------------------------------------------------
// Projection of one Gaussian, written once for float (the O1 mirror), double (O2)
// and Dual (O3). The float instance is the exact operation order of the key path.
// ---------------------------------------------------------------------------------
template <class T> struct Proj {
  T tx, ty, tz;          // view-space mean
  T a, b, c;             // dilated 2D covariance Sigma' (a, b; b, c)
  T det;
  T ca, cb, cc;          // conic = inverse of Sigma'
  T mx, my;              // mu' in pixels
  T opac;
  T rgb[3];
  bool clamped[3];       // colour channel clamped at 0
  bool qzero;            // quaternion of zero norm
};

template <class T>
void project(const T mu[3], const T ls[3], const T qv[4], const T& logit, const T& smin,
             const double* sh, int deg, const Cam<T>& cam, bool with_colour, Proj<T>& p,
             bool scale_exp_fp32 = false) {
  const T* Rc = cam.R;
  // view transform t = R_c mu + t_c
  p.tx = ((Rc[0] * mu[0] + Rc[1] * mu[1]) + Rc[2] * mu[2]) + cam.t[0];
  p.ty = ((Rc[3] * mu[0] + Rc[4] * mu[1]) + Rc[5] * mu[2]) + cam.t[1];
  p.tz = ((Rc[6] * mu[0] + Rc[7] * mu[1]) + Rc[8] * mu[2]) + cam.t[2];
  // eq. 4: s = exp(s_opt) + s_min
  T s[3];
  for (int i = 0; i < 3; ++i) {
    if (scale_exp_fp32)   // exp evaluated in FP64 and rounded once to FP32 (the key mirror)
      s[i] = T(double((float)std::exp(val(ls[i])))) + smin;
    else
      s[i] = ex(ls[i]) + smin;
  }
  // unit quaternion (w, x, y, z)
  T n2 = ((qv[0] * qv[0] + qv[1] * qv[1]) + qv[2] * qv[2]) + qv[3] * qv[3];
  p.qzero = !(val(n2) > 0.0);
  T nq = sq(p.qzero ? T(1.0) : n2);
  T w = qv[0] / nq, x = qv[1] / nq, y = qv[2] / nq, z = qv[3] / nq;
  T one = T(1.0), two = T(2.0);
  T R[9];
  R[0] = one - two * (y * y + z * z);
  R[1] = two * (x * y - w * z);
  R[2] = two * (x * z + w * y);
  R[3] = two * (x * y + w * z);
  R[4] = one - two * (x * x + z * z);
  R[5] = two * (y * z - w * x);
  R[6] = two * (x * z - w * y);
  R[7] = two * (y * z + w * x);
  R[8] = one - two * (x * x + y * y);
  // eq. 1: Sigma = M M^T, M = R diag(s)
  T M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i * 3 + j] = R[i * 3 + j] * s[j];
  T S[9];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      S[i * 3 + j] = (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];
      S[j * 3 + i] = S[i * 3 + j];
    }
  // EWA: J at the view-space mean, image-plane coordinates clamped to 1.3x the half FOV
  T u = p.tx / p.tz, v = p.ty / p.tz;
  T limx = T(K<double>::fov_clamp) * ((T(K<double>::half) * T(double(cam.W))) / cam.fx);
  T limy = T(K<double>::fov_clamp) * ((T(K<double>::half) * T(double(cam.H))) / cam.fy);
  if constexpr (std::is_same<T, float>::value) {
    limx = K<float>::fov_clamp * ((K<float>::half * (float)cam.W) / cam.fx);
    limy = K<float>::fov_clamp * ((K<float>::half * (float)cam.H) / cam.fy);
  }
  T xc = tmin(tmax(u, -limx), limx);
  T yc = tmin(tmax(v, -limy), limy);
  T J00 = cam.fx / p.tz, J02 = -(cam.fx * xc) / p.tz;
  T J11 = cam.fy / p.tz, J12 = -(cam.fy * yc) / p.tz;
  // T = J R_c (2x3)
  T Tm[6];
  for (int j = 0; j < 3; ++j) {
    Tm[0 * 3 + j] = J00 * Rc[0 * 3 + j] + J02 * Rc[2 * 3 + j];
    Tm[1 * 3 + j] = J11 * Rc[1 * 3 + j] + J12 * Rc[2 * 3 + j];
  }
  // U = T Sigma, Sigma' = U T^T
  T U[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      U[i * 3 + j] = (Tm[i * 3 + 0] * S[0 * 3 + j] + Tm[i * 3 + 1] * S[1 * 3 + j]) + Tm[i * 3 + 2] * S[2 * 3 + j];
  T s00 = (U[0] * Tm[0] + U[1] * Tm[1]) + U[2] * Tm[2];
  T s01 = (U[0] * Tm[3] + U[1] * Tm[4]) + U[2] * Tm[5];
  T s11 = (U[3] * Tm[3] + U[4] * Tm[4]) + U[5] * Tm[5];
  T dil = std::is_same<T, float>::value ? T(K<float>::dilate) : T(K<double>::dilate);
  p.a = s00 + dil;
  p.b = s01;
  p.c = s11 + dil;
  p.det = p.a * p.c - p.b * p.b;
  T inv = T(1.0) / p.det;
  p.ca = p.c * inv;
  p.cb = -p.b * inv;
  p.cc = p.a * inv;
  p.mx = cam.fx * u + cam.cx;
  p.my = cam.fy * v + cam.cy;
  p.opac = T(1.0) / (T(1.0) + ex(-logit));
  if (with_colour) {
    T dx = mu[0] - cam.campos[0], dy = mu[1] - cam.campos[1], dz = mu[2] - cam.campos[2];
    T nrm = sq((dx * dx + dy * dy) + dz * dz);
    dx = dx / nrm; dy = dy / nrm; dz = dz / nrm;
    T Y[16];
    sh_basis<T>(deg, dx, dy, dz, Y);
    int nk = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
      T acc = T(0.0);
      for (int k = 0; k < nk; ++k) acc = acc + T(sh[k * 3 + ch]) * Y[k];
      acc = acc + T(0.5);
      p.clamped[ch] = val(acc) < 0.0;
      p.rgb[ch] = p.clamped[ch] ? T(0.0) : acc;
    }
  }
}

// O1 result for one Gaussian.
struct KeyOut {
  uint8_t visible;
  uint32_t depth_bits;   // bits of float(t_z)
  int32_t rect[4];       // xmin, ymin, xmax, ymax (inclusive tiles)
  uint32_t tiles;
  float radius;
  float qsup;                 // support bound Q_g of the opacity (see support_q)
  float mx, my, ca, cb, cc;   // FP32 roundings of mu' and the conic
  uint32_t mu_lo;        // bf16 residuals of mu': x in the low half, y in the high half
};

// Support of a Gaussian: a pixel blends only if q <= 9 and o exp(-q/2) >= 1/255, i.e.
// q <= Q_g = min(9, 2 ln(255 o)). Q_g is formed from o = 1/(1 + exp(-logit)) in FP64, each
// rounded to FP32 (so that last-bit differences between exp/log implementations vanish),
// and the footprint uses Q = Q_g (1 + 1e-3) + 1e-3: at q = Q, o exp(-q/2) <= (1/255) e^-5e-4,
// a margin far above FP32 and fast-exp error, so no pixel outside the footprint can blend.
float support_q(float logit) {
  const float o = (float)(1.0 / (1.0 + std::exp(-(double)logit)));
  return (float)std::min(9.0, std::max(0.0, 2.0 * std::log(255.0 * (double)o)));
}

double support_span(float qg) { return (double)qg * 1.001 + 1e-3; }

// Tile footprint of a Gaussian from its stored FP32 mu' and conic: per tile row, the tiles
// whose [16 tx, 16 tx + 16) meets the x-extent of the ellipse d^T conic d <= Q (Q from
// support_span) over the row's band of pixel centres. FP64, fixed operation order.
struct Span { int ty, tx0, tx1; };

int footprint_spans(float mxf, float myf, float af, float bf, float cf, double kQSpan, int tiles_x, int tiles_y,
                    Span* out, int max_rows, int* row0, int* row1) {
  const double mx = mxf, my = myf, a = af, b = bf, c = cf;
  const double det = a * c - b * b;
  if (!(det > 0.0) || !(a > 0.0)) return 0;
  // reciprocals taken once: every row then multiplies (the footprint is inflated by 1e-3 in
  // Q, far above the rounding this changes)
  const double idet = 1.0 / det, ia = 1.0 / a;
  const double sxx = c * idet, syy = a * idet, sxy = -b * idet;
  const double hx = std::sqrt(kQSpan * sxx);
  const double hy = std::sqrt(kQSpan * syy);
  const double dyr = sxy * std::sqrt(kQSpan / sxx);
  double y0 = std::floor((my - hy) * 0.0625);
  double y1 = std::floor((my + hy) * 0.0625);
  y0 = std::max(y0, 0.0);
  y1 = std::min(y1, (double)(tiles_y - 1));
  if (!(y0 <= y1)) return 0;
  *row0 = (int)y0;
  *row1 = (int)y1;
  int n = 0;
  for (int ty = (int)y0; ty <= (int)y1 && n < max_rows; ++ty) {
    // band of pixel-centre offsets in this row, clipped to the ellipse's y-extent
    const double dlo = std::max((16.0 * ty + 0.5) - my, -hy);
    const double dhi = std::min((16.0 * ty + 15.5) - my, hy);
    if (!(dlo <= dhi)) continue;
    const double qa = kQSpan * a;
    const double rlo = std::sqrt(std::max(0.0, qa - det * dlo * dlo));
    const double rhi = std::sqrt(std::max(0.0, qa - det * dhi * dhi));
    // x = (-b dy +/- sqrt(Q a - det dy^2)) / a; the extreme points sit at dy = +/- dyr
    const double right = (dlo <= dyr && dyr <= dhi) ? hx : std::max((-b * dlo + rlo) * ia, (-b * dhi + rhi) * ia);
    const double left = (dlo <= -dyr && -dyr <= dhi) ? -hx : std::min((-b * dlo - rlo) * ia, (-b * dhi - rhi) * ia);
    double x0 = std::floor((mx + left) * 0.0625);
    double x1 = std::floor((mx + right) * 0.0625);
    x0 = std::max(x0, 0.0);
    x1 = std::min(x1, (double)(tiles_x - 1));
    if (!(x0 <= x1)) continue;
    out[n++] = Span{ty, (int)x0, (int)x1};
  }
  return n;
}

// Round to nearest even to bf16, kept in the upper 16 bits (finite inputs).
uint32_t bf16_rne(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  uint32_t lsb = (u >> 16) & 1u;
  return (u + 0x7FFFu + lsb) & 0xFFFF0000u;
}

void key_one(const float* muf, const float* lsf, const float* qf, float logit, float smin,
             const Cam<double>& cam, int tiles_x, int tiles_y, KeyOut& o) {
  std::memset(&o, 0, sizeof(o));
  double mu[3], ls[3], q[4];
  for (int i = 0; i < 3; ++i) { mu[i] = muf[i]; ls[i] = lsf[i]; }
  for (int i = 0; i < 4; ++i) q[i] = qf[i];
  Proj<double> p;
  project<double>(mu, ls, q, (double)logit, (double)smin, nullptr, 0, cam, false, p, true);
  // culls: near plane, opacity below 1/255 (logit compared in FP32), zero quaternion
  const float logit_min = (float)(-std::log(254.0));
  if (!(p.tz > K<double>::near_z)) return;
  if (logit < logit_min) return;
  if (p.qzero) return;
  if (!(p.det > 0.0)) return;
  double m = K<double>::half * (p.a + p.c);
  double disc = m * m - p.det;
  double lam = m + std::sqrt(std::max(K<double>::eig_floor, disc));
  double r = std::ceil(K<double>::three * std::sqrt(lam));
  o.mx = (float)p.mx; o.my = (float)p.my;
  o.ca = (float)p.ca; o.cb = (float)p.cb; o.cc = (float)p.cc;
  std::vector<Span> sp((size_t)tiles_y);
  int row0 = 0, row1 = -1;
  o.qsup = support_q(logit);
  int ns = footprint_spans(o.mx, o.my, o.ca, o.cb, o.cc, support_span(o.qsup), tiles_x, tiles_y, sp.data(), tiles_y,
                           &row0, &row1);
  uint32_t count = 0;
  int rx0 = 0xFFFF, rx1 = 0;
  for (int k = 0; k < ns; ++k) {
    count += (uint32_t)(sp[k].tx1 - sp[k].tx0 + 1);
    rx0 = std::min(rx0, sp[k].tx0);
    rx1 = std::max(rx1, sp[k].tx1);
  }
  if (count == 0) return;
  // rectangle reported: tile rows of the footprint's y-extent, columns of the spans
  o.visible = 1;
  float tzf = (float)p.tz;
  std::memcpy(&o.depth_bits, &tzf, 4);
  o.rect[0] = rx0; o.rect[1] = row0; o.rect[2] = rx1; o.rect[3] = row1;
  o.tiles = count;
  o.radius = (float)r;
  uint32_t lx = bf16_rne((float)(p.mx - (double)o.mx)), ly = bf16_rne((float)(p.my - (double)o.my));
  o.mu_lo = (lx >> 16) | ly;
}

inline bool near_rel(double x, double thr) { return std::fabs(x - thr) <= 1e-4 * std::fabs(thr); }

struct Gauss64 { double mx, my, ca, cb, cc, opac, rgb[3]; };

void project64_all(int64_t nv, const int64_t* order, const double* means, const double* ls, const double* q,
                   const double* logits, const double* smin, const double* sh, int deg, const Cam<double>& cam,
                   std::vector<Gauss64>& out) {
  out.resize(nv);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nv; ++k) {
    int64_t g = order[k];
    double mu[3], s[3], qq[4];
    for (int i = 0; i < 3; ++i) { mu[i] = means[g * 3 + i]; s[i] = ls[g * 3 + i]; }
    for (int i = 0; i < 4; ++i) qq[i] = q[g * 4 + i];
    Proj<double> p;
    project<double>(mu, s, qq, logits[g], smin[g], sh + g * 48, deg, cam, true, p);
    Gauss64& o = out[k];
    o.mx = p.mx; o.my = p.my; o.ca = p.ca; o.cb = p.cb; o.cc = p.cc; o.opac = p.opac;
    for (int ch = 0; ch < 3; ++ch) o.rgb[ch] = p.rgb[ch];
  }
}

// One pixel, front to back over all Gaussians in O1 order (preliminary section: alpha
// by eq. 2, blending in depth order). Steps: support cut q <= 9, alpha = min(0.99, o e^{-q/2}),
// skip alpha < 1/255, stop before blending when T(1 - alpha) < 1e-4.
// Flags (bits): 1 = a decision that changes the image lies within a relative 1e-4 of its
// threshold, where FP32 arithmetic may take it the other way: the support cut (only when the
// alpha test would pass at q = 9, else the Gaussian is skipped either way), the alpha floor or
// the stop; 2 = the unclamped alpha lies within a relative 1e-4 of the 0.99 clamp, whose kink
// changes the gradient but not the image (alpha is continuous there).
struct Contrib { int64_t k; double alpha, G, T; bool clamp; double dx, dy; };

template <bool RECORD>
void composite_pixel(double px, double py, const std::vector<Gauss64>& G, const double bg[3],
                     double rgb[3], double& Tout, int64_t& last, uint8_t& flag, int32_t& nblend,
                     std::vector<Contrib>* rec) {
  double T = 1.0, C[3] = {0, 0, 0};
  last = -1; flag = 0; nblend = 0;
  const double a_min = 1.0 / 255.0, t_min = 1e-4, a_max = 0.99, q_cut = 9.0;
  const double g_cut = std::exp(-0.5 * q_cut);
  for (size_t k = 0; k < G.size(); ++k) {
    const Gauss64& g = G[k];
    double dx = px - g.mx, dy = py - g.my;
    double q = g.ca * dx * dx + 2.0 * g.cb * dx * dy + g.cc * dy * dy;
    if (near_rel(q, q_cut) && g.opac * g_cut >= a_min * (1.0 - 1e-4)) flag |= 1;
    if (q > q_cut) continue;
    double Gv = std::exp(-0.5 * q);
    double a0 = g.opac * Gv;
    double alpha = std::min(a_max, a0);
    if (near_rel(a0, a_max)) flag |= 2;    // the clamp's kink: gradients differ on each side
    if (near_rel(alpha, a_min)) flag |= 1;
    if (alpha < a_min) continue;
    double Tn = T * (1.0 - alpha);
    if (near_rel(Tn, t_min)) flag |= 1;
    if (Tn < t_min) break;
    if (RECORD) rec->push_back(Contrib{(int64_t)k, alpha, Gv, T, a0 > a_max, dx, dy});
    for (int ch = 0; ch < 3; ++ch) C[ch] += alpha * T * g.rgb[ch];
    T = Tn;
    last = (int64_t)k;
    ++nblend;
  }
  for (int ch = 0; ch < 3; ++ch) rgb[ch] = C[ch] + T * bg[ch];
  Tout = T;
}

}  // namespace

extern "C" {

void or_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int or_get_threads(void) { return omp_get_max_threads(); }

// Real SH basis at a unit direction (pins and tests).
void or_sh_basis(int deg, const double* dir, double* out16) {
  sh_basis<double>(deg, dir[0], dir[1], dir[2], out16);
}

// eq. 6 selection for one level: keep iff lo2 <= |mu - c|^2 < hi2, FP32, summed x, y, z.
void or_select_level(int64_t n, const float* means, const float* centre, float lo2, float hi2, uint8_t* keep) {
  for (int64_t i = 0; i < n; ++i) {
    float dx = means[i * 3 + 0] - centre[0];
    float dy = means[i * 3 + 1] - centre[1];
    float dz = means[i * 3 + 2] - centre[2];
    float d2 = (dx * dx + dy * dy) + dz * dz;
    keep[i] = (lo2 <= d2 && d2 < hi2) ? 1 : 0;
  }
}

// Overlap pruning (section Overlap Pruning): d_avg of Gaussian i is the mean of its
// distances to the three nearest other Gaussians, d_1 <= d_2 <= d_3, each the FP64
// Euclidean distance between the FP32 means (differences taken as double(x_j) - double(x_i),
// squares summed x, y, z), the three added in ascending order and divided by 3. Gaussian i
// is removed when d_avg < d_op (d_op = s_min / 2 of the level being trained). With fewer
// than four Gaussians nobody has three neighbours: d_avg = +inf, all kept. Brute force over
// all pairs; coincident means are distinct neighbours at distance 0.
// ids: NULL for every Gaussian, else the m Gaussians to evaluate (outputs indexed 0..m-1).
void or_overlap_prune(int64_t n, const float* means, double d_op, int64_t m, const int64_t* ids, uint8_t* keep,
                      double* d_avg) {
  const int64_t count = ids ? m : n;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t t = 0; t < count; ++t) {
    const int64_t i = ids ? ids[t] : t;
    double best[3] = {INFINITY, INFINITY, INFINITY};
    const double xi = means[i * 3 + 0], yi = means[i * 3 + 1], zi = means[i * 3 + 2];
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = (double)means[j * 3 + 0] - xi;
      const double dy = (double)means[j * 3 + 1] - yi;
      const double dz = (double)means[j * 3 + 2] - zi;
      const double d = std::sqrt((dx * dx + dy * dy) + dz * dz);
      if (d < best[2]) {
        best[2] = d;
        if (best[2] < best[1]) std::swap(best[1], best[2]);
        if (best[1] < best[0]) std::swap(best[0], best[1]);
      }
    }
    const double avg = ((best[0] + best[1]) + best[2]) / 3.0;
    d_avg[t] = avg;
    keep[t] = (avg < d_op) ? 0 : 1;
  }
}

// Level transition (section Training Method, eq. 5): the next level's scale parameter is
// log(s^(l) - s_min^(l+1)), with s^(l) = exp(s_opt) + s_min^(l) as the rasterizer forms it
// (exp rounded once to FP32, sum in FP64). Result in FP64.
void or_level_transition(int64_t n, const float* log_scales, double s_min_l, double s_min_next, double* out) {
  for (int64_t i = 0; i < n * 3; ++i) {
    const double s = (double)(float)std::exp((double)log_scales[i]) + s_min_l;
    out[i] = std::log(s - s_min_next);
  }
}

// O1: per-Gaussian key mirror. keep may be NULL (all candidates). Outputs per Gaussian.
void or_keys(int64_t n, const float* means, const float* ls, const float* q, const float* logits,
             const float* smin, const uint8_t* keep, const CamIn* camin,
             uint8_t* visible, uint32_t* depth_bits, int32_t* rect, uint32_t* tiles, float* radius,
             float* mxy, float* conic, uint32_t* mu_lo, float* qsup) {
  Cam<double> cam = cam_as<double>(*camin);
  int tx = (cam.W + TILE - 1) / TILE, ty = (cam.H + TILE - 1) / TILE;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    KeyOut o;
    if (keep && !keep[i]) {
      std::memset(&o, 0, sizeof(o));
    } else {
      key_one(means + i * 3, ls + i * 3, q + i * 4, logits[i], smin[i], cam, tx, ty, o);
    }
    visible[i] = o.visible;
    depth_bits[i] = o.depth_bits;
    for (int j = 0; j < 4; ++j) rect[i * 4 + j] = o.rect[j];
    tiles[i] = o.tiles;
    radius[i] = o.radius;
    qsup[i] = o.qsup;
    mxy[i * 2 + 0] = o.mx; mxy[i * 2 + 1] = o.my;
    conic[i * 3 + 0] = o.ca; conic[i * 3 + 1] = o.cb; conic[i * 3 + 2] = o.cc;
    mu_lo[i] = o.mu_lo;
  }
}

// O1: instance list sorted by (tile, depth bits, index); each visible Gaussian's footprint
// enumerated row by row. Returns K; writes at most cap entries. ranges: [2 * n_tiles].
int64_t or_instances(int64_t n, const uint8_t* visible, const uint32_t* depth_bits, const float* mxy,
                     const float* conic, const float* qsup, int32_t tiles_x, int32_t tiles_y, int64_t cap,
                     uint32_t* out_tile,
                     uint32_t* out_val, uint32_t* ranges) {
  struct E { uint32_t tile, depth, idx; };
  const int32_t n_tiles = tiles_x * tiles_y;
  std::vector<E> v;
  std::vector<Span> sp((size_t)tiles_y);
  for (int64_t i = 0; i < n; ++i) {
    if (!visible[i]) continue;
    int r0 = 0, r1 = -1;
    int ns = footprint_spans(mxy[2 * i], mxy[2 * i + 1], conic[3 * i], conic[3 * i + 1], conic[3 * i + 2],
                             support_span(qsup[i]), tiles_x, tiles_y, sp.data(), tiles_y, &r0, &r1);
    for (int k = 0; k < ns; ++k)
      for (int x = sp[k].tx0; x <= sp[k].tx1; ++x)
        v.push_back(E{(uint32_t)(sp[k].ty * tiles_x + x), depth_bits[i], (uint32_t)i});
  }
  std::sort(v.begin(), v.end(), [](const E& a, const E& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.depth != b.depth) return a.depth < b.depth;
    return a.idx < b.idx;
  });
  int64_t K = (int64_t)v.size();
  for (int64_t k = 0; k < K && k < cap; ++k) { out_tile[k] = v[k].tile; out_val[k] = v[k].idx; }
  for (int32_t t = 0; t < n_tiles; ++t) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
  for (int64_t k = 0; k < K; ++k) {
    uint32_t t = v[k].tile;
    if (k == 0 || v[k - 1].tile != t) ranges[2 * t] = (uint32_t)k;
    if (k == K - 1 || v[k + 1].tile != t) ranges[2 * t + 1] = (uint32_t)(k + 1);
  }
  return K;
}

// FP64 per-Gaussian projection (mu', conic, opacity, colour) for the listed ids.
void or_project64(int64_t nv, const int64_t* ids, const double* means, const double* ls, const double* q,
                  const double* logits, const double* smin, const double* sh, int deg, const CamIn* camin,
                  double* out9) {
  Cam<double> cam = cam_as<double>(*camin);
  std::vector<Gauss64> G;
  project64_all(nv, ids, means, ls, q, logits, smin, sh, deg, cam, G);
  for (int64_t k = 0; k < nv; ++k) {
    double* o = out9 + k * 9;
    o[0] = G[k].mx; o[1] = G[k].my; o[2] = G[k].ca; o[3] = G[k].cb; o[4] = G[k].cc; o[5] = G[k].opac;
    o[6] = G[k].rgb[0]; o[7] = G[k].rgb[1]; o[8] = G[k].rgb[2];
  }
}

// O2: FP64 image at the listed pixels. order: surviving ids in O1 depth order.
// Outputs per pixel: rgb[3], final T, last blended id (-1 if none), flag, blended count.
void or_image(int64_t nv, const int64_t* order, const double* means, const double* ls, const double* q,
              const double* logits, const double* smin, const double* sh, int deg, const CamIn* camin,
              const float* bg, int64_t npix, const int32_t* pix_xy,
              double* rgb, double* finalT, int64_t* last, uint8_t* flag, int32_t* nblend) {
  Cam<double> cam = cam_as<double>(*camin);
  std::vector<Gauss64> G;
  project64_all(nv, order, means, ls, q, logits, smin, sh, deg, cam, G);
  double bgd[3] = {bg[0], bg[1], bg[2]};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < npix; ++p) {
    double px = pix_xy[2 * p] + 0.5, py = pix_xy[2 * p + 1] + 0.5;
    int64_t lk;
    composite_pixel<false>(px, py, G, bgd, rgb + 3 * p, finalT[p], lk, flag[p], nblend[p], nullptr);
    last[p] = lk < 0 ? -1 : order[lk];
  }
}

// O3: FP64 gradient of L = sum_p sum_ch dL_dpix[p,ch] * I[p,ch] with respect to every
// Gaussian's raw parameters (grads for ids outside `order` stay zero). When s_means is not
// NULL, s_* receive the summation scale of each entry: the per-pixel 2D terms' magnitudes
// (with dL/dalpha taken at the size of the two parts it is the difference of), summed, and
// carried through the absolute value of the projection Jacobian. An FP32
// evaluation of the same sums can only be trusted to a small multiple of eps times this.
// g2d / s2d (may be NULL): [n, 9] gradient with respect to (mu'x, mu'y, conic a, b, c,
// opacity, r, g, b) and its summation scale, by Gaussian id.
// g_means [n,3], g_ls [n,3], g_q [n,4], g_logit [n], g_sh [n,48]; all zeroed here.
void or_grad(int64_t n, int64_t nv, const int64_t* order, const double* means, const double* ls, const double* q,
             const double* logits, const double* smin, const double* sh, int deg, const CamIn* camin,
             const float* bg, int64_t npix, const int32_t* pix_xy, const double* dL_dpix,
             double* g_means, double* g_ls, double* g_q, double* g_logit, double* g_sh, double* s_means,
             double* s_ls, double* s_q, double* s_logit, double* s_sh, double* g2d, double* s2d) {
  Cam<double> cam = cam_as<double>(*camin);
  std::vector<Gauss64> G;
  project64_all(nv, order, means, ls, q, logits, smin, sh, deg, cam, G);
  double bgd[3] = {bg[0], bg[1], bg[2]};
  // accumulators of dL/d(mx, my, ca, cb, cc, opac, r, g, b) in list order, and of the
  // magnitudes of the per-pixel terms summed into them (the scale of the summation)
  const bool want_scale = s_means != nullptr;
  std::vector<double> acc((size_t)nv * 9, 0.0);
  std::vector<double> accm(want_scale ? (size_t)nv * 9 : 0, 0.0);
#pragma omp parallel
  {
    double* A = acc.data();
    double* Am = want_scale ? accm.data() : nullptr;
    std::vector<Contrib> rec;
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; ++p) {
      const double* dC = dL_dpix + 3 * p;
      if (dC[0] == 0.0 && dC[1] == 0.0 && dC[2] == 0.0) continue;
      double px = pix_xy[2 * p] + 0.5, py = pix_xy[2 * p + 1] + 0.5;
      double rgb[3], Tf; int64_t lk; uint8_t fl; int32_t nb;
      rec.clear();
      composite_pixel<true>(px, py, G, bgd, rgb, Tf, lk, fl, nb, &rec);
      // reverse pass: C = sum_i alpha_i T_i c_i + T_final bg
      double S[3] = {Tf * bgd[0], Tf * bgd[1], Tf * bgd[2]};
      for (size_t r = rec.size(); r-- > 0;) {
        const Contrib& e = rec[r];
        const Gauss64& g = G[e.k];
        double* a = A + (size_t)e.k * 9;
        double* am = Am ? Am + (size_t)e.k * 9 : nullptr;
        double dalpha = 0.0, dalpha_mag = 0.0;
        double t[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int ch = 0; ch < 3; ++ch) {
          t[6 + ch] = e.alpha * e.T * dC[ch];
          dalpha += dC[ch] * (e.T * g.rgb[ch] - S[ch] / (1.0 - e.alpha));
          dalpha_mag += std::fabs(dC[ch]) * (e.T * std::fabs(g.rgb[ch]) + std::fabs(S[ch]) / (1.0 - e.alpha));
          S[ch] += e.alpha * e.T * g.rgb[ch];
        }
        // magnitudes of the same terms with dL/dalpha replaced by the size of the two parts
        // it is the difference of (the scale at which a float evaluation can resolve it)
        double tm[9];
        for (int j = 0; j < 9; ++j) tm[j] = std::fabs(t[j]);
        if (!e.clamp) {   // alpha = 0.99 does not depend on o or q
          t[5] = dalpha * e.G;
          double dq = dalpha * (-0.5 * e.alpha);
          // q = ca dx^2 + 2 cb dx dy + cc dy^2, dx = px - mx
          t[0] = dq * (-2.0 * (g.ca * e.dx + g.cb * e.dy));
          t[1] = dq * (-2.0 * (g.cb * e.dx + g.cc * e.dy));
          t[2] = dq * e.dx * e.dx;
          t[3] = dq * 2.0 * e.dx * e.dy;
          t[4] = dq * e.dy * e.dy;
          const double dqm = dalpha_mag * 0.5 * e.alpha;
          tm[5] = dalpha_mag * e.G;
          tm[0] = dqm * 2.0 * (std::fabs(g.ca * e.dx) + std::fabs(g.cb * e.dy));
          tm[1] = dqm * 2.0 * (std::fabs(g.cb * e.dx) + std::fabs(g.cc * e.dy));
          tm[2] = dqm * e.dx * e.dx;
          tm[3] = dqm * 2.0 * std::fabs(e.dx * e.dy);
          tm[4] = dqm * e.dy * e.dy;
        }
        for (int j = 0; j < 9; ++j) {
#pragma omp atomic
          a[j] += t[j];
          if (am) {
#pragma omp atomic
            am[j] += tm[j];
          }
        }
      }
    }
  }
  std::memset(g_means, 0, sizeof(double) * n * 3);
  std::memset(g_ls, 0, sizeof(double) * n * 3);
  std::memset(g_q, 0, sizeof(double) * n * 4);
  std::memset(g_logit, 0, sizeof(double) * n);
  std::memset(g_sh, 0, sizeof(double) * n * 48);
  if (g2d) std::memset(g2d, 0, sizeof(double) * n * 9);
  if (s2d) std::memset(s2d, 0, sizeof(double) * n * 9);
  if (want_scale) {
    std::memset(s_means, 0, sizeof(double) * n * 3);
    std::memset(s_ls, 0, sizeof(double) * n * 3);
    std::memset(s_q, 0, sizeof(double) * n * 4);
    std::memset(s_logit, 0, sizeof(double) * n);
    std::memset(s_sh, 0, sizeof(double) * n * 48);
  }
  Cam<Dual> camd = cam_as<Dual>(*camin);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nv; ++k) {
    double d2[9] = {0}, m2[9] = {0};
    for (int j = 0; j < 9; ++j) {
      d2[j] = acc[(size_t)k * 9 + j];
      if (want_scale) m2[j] = accm[(size_t)k * 9 + j];
    }
    int64_t g = order[k];
    if (g2d)
      for (int j = 0; j < 9; ++j) g2d[g * 9 + j] = d2[j];
    if (s2d && want_scale)
      for (int j = 0; j < 9; ++j) s2d[g * 9 + j] = m2[j];
    bool any = false;
    for (int j = 0; j < 9; ++j) any = any || d2[j] != 0.0;
    if (!any) continue;
    Dual mu[3], s[3], qq[4], lg;
    for (int i = 0; i < 3; ++i) { mu[i] = Dual::var(means[g * 3 + i], i); s[i] = Dual::var(ls[g * 3 + i], 3 + i); }
    for (int i = 0; i < 4; ++i) qq[i] = Dual::var(q[g * 4 + i], 6 + i);
    lg = Dual::var(logits[g], 10);
    Proj<Dual> p;
    project<Dual>(mu, s, qq, lg, Dual(smin[g]), sh + g * 48, deg, camd, true, p);
    const Dual* outs[9] = {&p.mx, &p.my, &p.ca, &p.cb, &p.cc, &p.opac, &p.rgb[0], &p.rgb[1], &p.rgb[2]};
    double gr[ND] = {0};
    for (int j = 0; j < 9; ++j)
      for (int i = 0; i < ND; ++i) gr[i] += d2[j] * outs[j]->d[i];
    for (int i = 0; i < 3; ++i) { g_means[g * 3 + i] = gr[i]; g_ls[g * 3 + i] = gr[3 + i]; }
    for (int i = 0; i < 4; ++i) g_q[g * 4 + i] = gr[6 + i];
    g_logit[g] = gr[10];
    if (want_scale) {
      double sc[ND] = {0};
      for (int j = 0; j < 9; ++j)
        for (int i = 0; i < ND; ++i) sc[i] += m2[j] * std::fabs(outs[j]->d[i]);
      for (int i = 0; i < 3; ++i) { s_means[g * 3 + i] = sc[i]; s_ls[g * 3 + i] = sc[3 + i]; }
      for (int i = 0; i < 4; ++i) s_q[g * 4 + i] = sc[6 + i];
      s_logit[g] = sc[10];
    }
    // colour is linear in the SH coefficients: d c_ch / d k_{j,ch} = Y_j(dir) unless clamped
    double dir[3] = {means[g * 3 + 0] - cam.campos[0], means[g * 3 + 1] - cam.campos[1],
                     means[g * 3 + 2] - cam.campos[2]};
    double nr = std::sqrt((dir[0] * dir[0] + dir[1] * dir[1]) + dir[2] * dir[2]);
    for (int i = 0; i < 3; ++i) dir[i] /= nr;
    double Y[16];
    sh_basis<double>(deg, dir[0], dir[1], dir[2], Y);
    for (int ch = 0; ch < 3; ++ch) {
      if (p.clamped[ch]) continue;
      for (int j = 0; j < (deg + 1) * (deg + 1); ++j) {
        g_sh[g * 48 + j * 3 + ch] = d2[6 + ch] * Y[j];
        if (want_scale) s_sh[g * 48 + j * 3 + ch] = m2[6 + ch] * std::fabs(Y[j]);
      }
    }
  }
}

}  // extern "C"

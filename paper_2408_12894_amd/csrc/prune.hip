// Overlap pruning (section Overlap Pruning): a Gaussian is removed when the mean distance to
// its three nearest other Gaussians, d_avg = (d_1 + d_2 + d_3) / 3, is below d_op.
//
// Only the decision d_avg < d_op is needed, and it depends on neighbours within R = 3 d_op
// alone: if the third-nearest lies at R or beyond, d_avg >= R / 3 = d_op and the Gaussian
// stays. So a uniform grid of cell edge c slightly above R (the search radius is widened by
// a relative 1e-9 so that the rounded comparison stays on the safe side) finds every
// neighbour that can matter in the 27 cells around a Gaussian's own.
//
//   1. cell of each mean (FP64 floor of x / c, clamped to 21 bits per axis: a monotone map,
//      so points closer than c along an axis stay in the same or adjacent cells), hashed to
//      a table of T = 2^b >= n buckets (MurmurHash3's 64-bit finaliser, top b bits);
//   2. stable radix sort of (bucket, index), then the means gathered into bucket order
//      (16 B per point, index in the fourth word), and per-bucket [start, end);
//   3. one thread per point, in bucket order so that a wave's threads read the same
//      buckets: scan the 27 neighbour buckets, keep the three smallest squared distances
//      (FP64, from the FP32 means, summed x, y, z), skipping itself and any point already
//      kept (two neighbour cells can share a bucket);
//   4. d_avg = ((d_1 + d_2) + d_3) / 3 in FP64 when d_3 < R (then these are the true three
//      nearest), +inf otherwise; keep = !(d_avg < d_op).
// Distances, their order of summation and the comparison are the same FP64 operations a
// brute-force evaluation performs, so the decisions match it bit for bit.
#include "flod_internal.h"

namespace flod {

constexpr int kCellBits = 21;
constexpr double kCellHalf = (double)(1 << (kCellBits - 1));

struct Grid {
  double inv_c;
  int shift;    // 64 - table bits
};

__device__ __forceinline__ int32_t cell_of(float x, double inv_c) {
  double f = floor((double)x * inv_c);
  f = fmin(fmax(f, -kCellHalf), kCellHalf - 1.0);
  return (int32_t)f;
}

// MurmurHash3 fmix64 finaliser over the packed cell coordinates.
__device__ __forceinline__ uint32_t bucket_of(int32_t ix, int32_t iy, int32_t iz, int shift) {
  const uint64_t m = (1ull << kCellBits) - 1;
  uint64_t k = (((uint64_t)(ix + (1 << (kCellBits - 1))) & m) << (2 * kCellBits)) |
               (((uint64_t)(iy + (1 << (kCellBits - 1))) & m) << kCellBits) |
               ((uint64_t)(iz + (1 << (kCellBits - 1))) & m);
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return (uint32_t)(k >> shift);
}

__global__ __launch_bounds__(kBlock) void k_prune_keys(const float *means, int64_t n, Grid g, uint32_t *keys,
                                                       uint32_t *vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t ix = cell_of(means[i * 3 + 0], g.inv_c);
  const int32_t iy = cell_of(means[i * 3 + 1], g.inv_c);
  const int32_t iz = cell_of(means[i * 3 + 2], g.inv_c);
  keys[i] = bucket_of(ix, iy, iz, g.shift);
  vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_prune_gather(const float *means, const uint32_t *sorted_vals, int64_t n,
                                                         float4 *pts) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const uint32_t j = sorted_vals[p];
  pts[p] = make_float4(means[(int64_t)j * 3 + 0], means[(int64_t)j * 3 + 1], means[(int64_t)j * 3 + 2],
                       __uint_as_float(j));
}

__global__ __launch_bounds__(kBlock) void k_prune_query(const float4 *__restrict__ pts, const uint2 *__restrict__ ranges,
                                                        int64_t n, Grid g, double radius, double d_op,
                                                        uint8_t *keep, double *d_avg) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const float4 a = pts[p];
  const int32_t cx = cell_of(a.x, g.inv_c), cy = cell_of(a.y, g.inv_c), cz = cell_of(a.z, g.inv_c);
  const double ax = a.x, ay = a.y, az = a.z;
  double b0 = INFINITY, b1 = INFINITY, b2 = INFINITY;
  uint32_t q0 = 0xFFFFFFFFu, q1 = 0xFFFFFFFFu, q2 = 0xFFFFFFFFu;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const uint2 r = ranges[bucket_of(cx + dx, cy + dy, cz + dz, g.shift)];
        for (uint32_t q = r.x; q < r.y; ++q) {
          if (q == (uint32_t)p) continue;
          const float4 b = pts[q];
          const double ex = (double)b.x - ax, ey = (double)b.y - ay, ez = (double)b.z - az;
          const double d2 = (ex * ex + ey * ey) + ez * ez;
          if (!(d2 < b2) || q == q0 || q == q1 || q == q2) continue;
          if (d2 < b1) {
            b2 = b1; q2 = q1;
            if (d2 < b0) {
              b1 = b0; q1 = q0;
              b0 = d2; q0 = q;
            } else {
              b1 = d2; q1 = q;
            }
          } else {
            b2 = d2; q2 = q;
          }
        }
      }
  double avg = INFINITY;
  const double d3 = sqrt(b2);
  if (d3 < radius) avg = ((sqrt(b0) + sqrt(b1)) + d3) / 3.0;
  const uint32_t j = __float_as_uint(a.w);
  keep[j] = (avg < d_op) ? 0 : 1;
  if (d_avg) d_avg[j] = avg;
}

// Size of the neighbour scan: the sum over points of their 27 buckets' occupancy.
__global__ __launch_bounds__(kBlock) void k_prune_cost(const float4 *__restrict__ pts, const uint2 *__restrict__ ranges,
                                                       int64_t n, Grid g, unsigned long long *cost) {
  __shared__ unsigned long long s_sum[kBlock / 64];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  unsigned long long c = 0;
  if (p < n) {
    const float4 a = pts[p];
    const int32_t cx = cell_of(a.x, g.inv_c), cy = cell_of(a.y, g.inv_c), cz = cell_of(a.z, g.inv_c);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const uint2 r = ranges[bucket_of(cx + dx, cy + dy, cz + dz, g.shift)];
          c += r.y - r.x;
        }
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += s_sum[w];
    atomicAdd(cost, t);
  }
}

__global__ __launch_bounds__(kBlock) void k_prune_none(int64_t n, uint8_t *keep, double *d_avg) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  keep[i] = 1;
  if (d_avg) d_avg[i] = INFINITY;
}

static unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int prune_table_bits(int64_t n) {
  int b = 8;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

static Grid make_grid(double radius, int64_t n) {
  Grid g;
  g.inv_c = 1.0 / (radius * 1.001);
  g.shift = 64 - prune_table_bits(n);
  return g;
}

double prune_radius(float d_op) { return 3.0 * (double)d_op * (1.0 + 1e-9); }

hipError_t launch_prune_keys(const float *means, int64_t n, float d_op, uint32_t *keys, uint32_t *vals,
                             hipStream_t s) {
  if (n <= 0 || !(d_op > 0.0f)) return hipSuccess;
  hipLaunchKernelGGL(k_prune_keys, dim3(grid_of(n)), dim3(kBlock), 0, s, means, n, make_grid(prune_radius(d_op), n),
                     keys, vals);
  return hipGetLastError();
}

hipError_t launch_prune_gather(const float *means, const uint32_t *sorted_vals, int64_t n, float4 *pts,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prune_gather, dim3(grid_of(n)), dim3(kBlock), 0, s, means, sorted_vals, n, pts);
  return hipGetLastError();
}

hipError_t launch_prune_cost(const float4 *pts, const uint2 *ranges, int64_t n, float d_op,
                             unsigned long long *cost, hipStream_t s) {
  if (n <= 0 || !(d_op > 0.0f)) return hipSuccess;
  hipLaunchKernelGGL(k_prune_cost, dim3(grid_of(n)), dim3(kBlock), 0, s, pts, ranges, n,
                     make_grid(prune_radius(d_op), n), cost);
  return hipGetLastError();
}

hipError_t launch_prune_query(const float4 *pts, const uint2 *ranges, int64_t n, float d_op, uint8_t *keep,
                              double *d_avg, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (!(d_op > 0.0f)) {
    hipLaunchKernelGGL(k_prune_none, dim3(grid_of(n)), dim3(kBlock), 0, s, n, keep, d_avg);
    return hipGetLastError();
  }
  const double radius = prune_radius(d_op);
  hipLaunchKernelGGL(k_prune_query, dim3(grid_of(n)), dim3(kBlock), 0, s, pts, ranges, n, make_grid(radius, n),
                     radius, (double)d_op, keep, d_avg);
  return hipGetLastError();
}

}  // namespace flod

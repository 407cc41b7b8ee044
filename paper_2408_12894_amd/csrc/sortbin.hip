// Binning: visible-set compaction, depth sort, instance emission, stable tile sort, ranges.
//
// Order of the instance list: ascending (tile, depth bits, Gaussian index). It is built as
//   1. stable LSD radix sort of (depth bits, index) over the visible Gaussians (N keys); its
//      first pass reads every candidate's depth key in index order and drops the candidates
//      not rendered (key kDepthNone), so it also compacts the visible set,
//   2. emit each Gaussian's tiles in that depth order (row-major over its footprint),
//   3. stable LSD radix sort of the K instances by tile id only.
// Stability makes step 3 keep the (depth, index) order inside each tile, so only the tile
// digits of the K-long list are sorted: ceil(log2(tiles) / 8) passes instead of a full
// 64-bit key sort.
//
// The radix pass is a reduce-then-scan design (no inter-workgroup spinning, which would
// need cross-XCD coherent flags): per-workgroup digit histograms, a per-digit scan over
// workgroups, then a scatter in which each workgroup ranks its 3072 (or 2048) keys stably in LDS
// (wave64 ballots over the digit bits), reorders them by digit in LDS and writes each
// digit run contiguously.
#include <algorithm>

#include "project.h"

namespace flod {

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exclusive scan over a kBlock-thread workgroup; *total receives the sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t s_w[kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    uint32_t t = s_w[k];
    base += (k < w) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// ---------------------------------------------------------------------------------------
// Scan of per-workgroup counts (one workgroup): 64-bit exclusive prefixes and the total.
// total32 receives the total when it is at most cap32 and 0 otherwise: kernels sized for
// cap32 items read it as their item count and then do nothing. host_out (coherent host
// memory, or null) receives four 64-bit words, each host_seq in its high half and in its low
// half the item count, total32, and the low and high halves of the total: system-scope
// stores of whole words, so a host that polls them sees every word either old or complete
// and needs neither a copy nor an event.
// ---------------------------------------------------------------------------------------
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const uint32_t *in, const uint32_t *n_items,
                                                              int items_per_block, unsigned long long *prefix,
                                                              uint32_t *total32, unsigned long long *total64,
                                                              unsigned long long cap32, int max_blocks,
                                                              unsigned long long *host_out, uint32_t host_seq) {
  __shared__ unsigned long long s_w[kScanThreads / 64];
  int nb = max_blocks;
  const uint32_t items = n_items ? *n_items : 0u;
  if (n_items) nb = (int)(((unsigned long long)items + items_per_block - 1) / items_per_block);
  // thread t owns the contiguous counts [t per, (t + 1) per): its sum, a workgroup scan of the
  // sums, then its exclusive prefixes (a second read of its counts, from cache)
  const int per = (nb + kScanThreads - 1) / kScanThreads;
  const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, lo + per);
  // up to kScanHeld counts per thread are loaded together and kept for the prefixes (one memory
  // round trip instead of one per count); more (above kScanHeld x 1024 workgroups) are re-read
  constexpr int kScanHeld = 8;
  uint32_t held[kScanHeld];
#pragma unroll
  for (int i = 0; i < kScanHeld; ++i) held[i] = lo + i < hi ? in[lo + i] : 0u;
  unsigned long long mine = 0;
#pragma unroll
  for (int i = 0; i < kScanHeld; ++i) mine += held[i];
  for (int k = lo + kScanHeld; k < hi; ++k) mine += in[k];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned long long inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  unsigned long long run = inc - mine, total = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k) {
    const unsigned long long t = s_w[k];
    run += (k < w) ? t : 0ull;
    total += t;
  }
#pragma unroll
  for (int i = 0; i < kScanHeld; ++i) {
    if (lo + i < hi) prefix[lo + i] = run;
    run += held[i];
  }
  for (int k = lo + kScanHeld; k < hi; ++k) {
    prefix[k] = run;
    run += in[k];
  }
  if (threadIdx.x == 0) {
    const uint32_t t32 = total > cap32 ? 0u : (uint32_t)total;
    if (total64) *total64 = total;
    if (total32) *total32 = t32;
    if (host_out) {
      const unsigned long long tag = (unsigned long long)host_seq << 32;
      const unsigned long long w[4] = {tag | items, tag | t32, tag | (total & 0xFFFFFFFFull), tag | (total >> 32)};
#pragma unroll
      for (int k = 0; k < 4; ++k) __hip_atomic_store(&host_out[k], w[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

hipError_t launch_scan_blocks(const uint32_t *in, const uint32_t *n_items, int items_per_block,
                              unsigned long long *prefix, uint32_t *total32, unsigned long long *total64,
                              int max_blocks, hipStream_t s, unsigned long long cap32,
                              unsigned long long *host_out, uint32_t host_seq) {
  if (cap32 > 0xFFFFFFFFull) cap32 = 0xFFFFFFFFull;
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanThreads), 0, s, in, n_items, items_per_block, prefix,
                     total32, total64, cap32, max_blocks, host_out, host_seq);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Radix pass: histogram, per-digit scan, stable scatter.
// hist[d * stride + b] = count of digit d in block b; scan = exclusive prefix over b. The row
// stride is the block count rounded up to a multiple of 8 (32-byte aligned rows).
//
// Block of a histogram or scatter workgroup: workgroups go to the 8 XCDs round-robin, and
// each XCD takes runs of kXcdRun consecutive blocks. The counts of adjacent blocks share
// cache lines; written and read from one XCD's L2 they move as whole lines (spread over the
// 8 XCDs every line went out as 8 partial writes: 8x the histogram's bytes).
// ---------------------------------------------------------------------------------------
constexpr uint32_t kXcdRun = 16;

__device__ __forceinline__ uint32_t radix_block(uint32_t wg) {
  const uint32_t x = wg % 8u, j = wg / 8u;
  return (j / kXcdRun) * (8u * kXcdRun) + x * kXcdRun + (j % kXcdRun);
}

static unsigned radix_grid(int nb_max) {
  const int g = 8 * (int)kXcdRun;
  return (unsigned)(((nb_max + g - 1) / g) * g);
}
// All of a workgroup's keys are loaded before the first LDS update, so its loads are in
// flight together. The count n is read first: grids are sized for the buffers' capacity,
// which can far exceed n, and workgroups past n leave without reading their keys (loading
// keys and values together with n, bounded by the capacity, here and in the scatter made the
// tile sort at 1080p / 1M 10% slower).
//
// FIRST (the depth sort's first pass): the keys are all n_all candidates' depth keys, read
// directly, and keys equal to kDepthNone (candidates not rendered) are not counted.
template <int ITEMS, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t *keys, const uint32_t *n_ptr, uint32_t n_all,
                                                    int shift, uint32_t dmask, uint32_t *hist, int stride) {
  constexpr uint32_t TILE = kBlock * ITEMS;
  __shared__ uint32_t h[kRadix];
  const uint32_t n = FIRST ? n_all : *n_ptr;
  const uint32_t nb = (n + TILE - 1) / TILE;
  const uint32_t b = radix_block(blockIdx.x);
  if (b >= nb) return;
  const uint32_t base = b * TILE;
  uint32_t kr[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint32_t idx = base + r * kBlock + threadIdx.x;
    kr[r] = idx < n ? keys[idx] : 0u;
  }
  h[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r)
    if (base + r * kBlock + threadIdx.x < n && (!FIRST || kr[r] != kDepthNone))
      atomicAdd(&h[(kr[r] >> shift) & dmask], 1u);
  __syncthreads();
  hist[(size_t)threadIdx.x * stride + b] = h[threadIdx.x];
}

// One workgroup per digit. Rounds of 2048 counts: each thread takes 8 consecutive ones (two
// 16-byte loads), the next round's loads are issued before this round's scan.
__global__ __launch_bounds__(kBlock) void k_rs_scan(const uint32_t *n_ptr, uint32_t n_all, const uint32_t *hist,
                                                    uint32_t *scan, uint32_t *tot, int stride, int tile) {
  constexpr uint32_t kPer = 8, kRound = kBlock * kPer;
  const uint32_t n = n_ptr ? *n_ptr : n_all;   // null: the first pass over all candidates
  const uint32_t nb = (n + tile - 1) / tile;
  const int d = blockIdx.x;
  const uint32_t *row = hist + (size_t)d * stride;
  uint32_t *out = scan + (size_t)d * stride;
  // k < nb implies k + 3 < stride: a 16-byte group that starts below nb lies inside the row
  auto load = [&](uint32_t k, uint4 &lo, uint4 &hi) {
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    lo = k < nb ? *reinterpret_cast<const uint4 *>(row + k) : z;
    hi = k + 4 < nb ? *reinterpret_cast<const uint4 *>(row + k + 4) : z;
  };
  uint32_t run = 0;
  uint32_t k = threadIdx.x * kPer;
  uint4 lo, hi;
  load(k, lo, hi);
  for (uint32_t base = 0; base < nb; base += kRound, k += kRound) {
    uint32_t v[kPer] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    load(k + kRound, lo, hi);
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) {
      if (k + i >= nb) v[i] = 0u;
      sum += v[i];
    }
    uint32_t t;
    uint32_t e = run + block_excl_scan(sum, &t);
    uint32_t o[kPer];
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) {
      o[i] = e;
      e += v[i];
    }
    if (k < nb) *reinterpret_cast<uint4 *>(out + k) = make_uint4(o[0], o[1], o[2], o[3]);
    if (k + 4 < nb) *reinterpret_cast<uint4 *>(out + k + 4) = make_uint4(o[4], o[5], o[6], o[7]);
    run += t;
  }
  if (threadIdx.x == 0) tot[d] = run;
}

// Stable scatter of one workgroup's TILE keys. Wave w owns the contiguous keys
// [w * 64 ITEMS, (w + 1) * 64 ITEMS) of the tile, read round by round (64 consecutive keys per
// round), so (wave, round, lane) order is the input order. Each key's rank among equal digits
// of its wave comes from ballots over the digit bits plus a wave-private LDS count carried
// across rounds (a wave's LDS accesses complete in program order, so no barrier is needed
// between rounds); one barrier then turns the per-wave counts into offsets, keys are placed
// in LDS in digit order, and each digit's run is written out contiguously.
//
// With TILES (the last pass of the depth sort) the scatter also writes, at each output
// position, the tile count of the Gaussian its value names (tiles_out[pos] = tiles_of[val]),
// and adds the counts into sums over 256 consecutive output positions (block_sum[pos / 256],
// zeroed beforehand): the emission's per-workgroup counts, in depth order. Output positions
// grow with the local index across the workgroup (digit runs in digit order, each at its
// digit's base), so the lanes of one write round that share a 256-block are consecutive: a
// segmented sum over the wave leaves one atomic per segment.
struct TileTail {
  const uint32_t *tiles_of;   // tile count per Gaussian (indexed by value)
  uint32_t *tiles_out;        // tile count per sorted position
  uint32_t *block_sum;        // per 256 sorted positions
};

// With FIRST (the depth sort's first pass) the keys are all n_all candidates' depth keys, each
// key's value is its index, keys equal to kDepthNone are dropped (the output is the rendered
// candidates, compacted and ordered by the first digit), and workgroup 0 writes the count kept
// to *n_out for the later passes.
template <int ITEMS, bool TILES, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t *__restrict__ keys_in,
                                                       const uint32_t *__restrict__ vals_in,
                                                       uint32_t *__restrict__ keys_out,
                                                       uint32_t *__restrict__ vals_out, const uint32_t *n_ptr,
                                                       uint32_t n_all, uint32_t *n_out, int shift, uint32_t dmask,
                                                       const uint32_t *hist, const uint32_t *scan,
                                                       const uint32_t *tot, int stride, TileTail tail) {
  constexpr uint32_t TILE = kBlock * ITEMS;
  constexpr int WAVES = kBlock / 64;
  constexpr uint32_t WTILE = 64 * ITEMS;
  __shared__ uint32_t s_keys[TILE];
  __shared__ uint32_t s_vals[TILE];
  __shared__ uint32_t s_goff[kRadix];
  __shared__ uint32_t s_wcnt[WAVES][kRadix];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the count first (grids are sized for the capacity, which can far exceed it); then the
  // tile's keys and values, loaded together with the digit offsets below, so that their
  // latencies overlap (the offsets issued ahead of the count, with the scan's first counts
  // likewise, made the tile sort at 1080p / 1M 8% slower: a wait for the count then waits for
  // the scattered offset rows too)
  const uint32_t n = FIRST ? n_all : *n_ptr;
  const uint32_t nb = (n + TILE - 1) / TILE;
  const uint32_t b = radix_block(blockIdx.x);
  if (b >= nb) return;
  const uint32_t base = b * TILE;
  const uint32_t count = min(TILE, n - base);
  uint32_t kr[ITEMS], vr[ITEMS], rr[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint32_t li = (uint32_t)w * WTILE + (uint32_t)r * 64u + (uint32_t)lane;
    kr[r] = li < count ? keys_in[base + li] : (FIRST ? kDepthNone : 0u);
    vr[r] = FIRST ? base + li : (li < count ? vals_in[base + li] : 0u);
  }
  // digit bases over the whole array and this workgroup's local digit bases (the three
  // loads issued together, ahead of the scans' barriers)
  const uint32_t tot_d = tot[tid];
  const uint32_t cnt = hist[(size_t)tid * stride + b];
  const uint32_t sc = scan[(size_t)tid * stride + b];
  uint32_t t_all;
  const uint32_t dbase = block_excl_scan(tot_d, &t_all);
  uint32_t t_loc;   // the keys this workgroup writes (FIRST: the rendered ones)
  const uint32_t lbase = block_excl_scan(cnt, &t_loc);
  if (FIRST && b == 0 && tid == 0) *n_out = t_all;
  s_goff[tid] = dbase + sc - lbase;
#pragma unroll
  for (int k = 0; k < WAVES; ++k) s_wcnt[k][tid] = 0;
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint32_t li = (uint32_t)w * WTILE + (uint32_t)r * 64u + (uint32_t)lane;
    const bool valid = li < count && (!FIRST || kr[r] != kDepthNone);
    const uint32_t key = kr[r];
    const uint32_t d = (key >> shift) & dmask;   // bits above the pass's digit are zero
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const bool set = (d >> bit) & 1u;
      const unsigned long long bb = __ballot(set);
      peers &= set ? bb : ~bb;
    }
    const uint32_t in_round = (uint32_t)__popcll(peers & lt);
    const uint32_t prev = s_wcnt[w][d];
    rr[r] = prev + in_round;
    if (valid && in_round == 0) s_wcnt[w][d] = prev + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    uint32_t acc = lbase;   // this thread's digit is tid
#pragma unroll
    for (int k = 0; k < WAVES; ++k) {
      const uint32_t c = s_wcnt[k][tid];
      s_wcnt[k][tid] = acc;
      acc += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint32_t li = (uint32_t)w * WTILE + (uint32_t)r * 64u + (uint32_t)lane;
    if (li < count && (!FIRST || kr[r] != kDepthNone)) {
      const uint32_t pos = s_wcnt[w][(kr[r] >> shift) & dmask] + rr[r];
      s_keys[pos] = kr[r];
      s_vals[pos] = vr[r];
    }
  }
  __syncthreads();
  const uint32_t kept = FIRST ? t_loc : count;
  if (!TILES) {
    for (uint32_t li = tid; li < kept; li += kBlock) {
      const uint32_t key = s_keys[li];
      const uint32_t d = (key >> shift) & dmask;
      const uint32_t pos = s_goff[d] + li;
      keys_out[pos] = key;
      vals_out[pos] = s_vals[li];
    }
  } else {
    // whole rounds of the workgroup, so that every lane takes part in the segmented sum (the
    // tile count gathered in each round: gathering all of a thread's counts before the first
    // round measured 3.5 us slower at 1080p / 1M)
    for (uint32_t l0 = 0; l0 < kept; l0 += kBlock) {
      const uint32_t li = l0 + tid;
      const bool valid = li < kept;
      uint32_t c = 0u, seg = 0xFFFFFFFFu;
      if (valid) {
        const uint32_t key = s_keys[li];
        const uint32_t v = s_vals[li];
        const uint32_t pos = s_goff[(key >> shift) & dmask] + li;
        keys_out[pos] = key;
        vals_out[pos] = v;
        c = tail.tiles_of[v];
        tail.tiles_out[pos] = c;
        seg = pos / (uint32_t)kBlock;
      }
      // inclusive sums over runs of equal seg (seg does not decrease over the lanes; invalid
      // lanes, all past the valid ones, form a run of their own)
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t cu = __shfl_up(c, o, 64);
        const uint32_t su = __shfl_up(seg, o, 64);
        if (lane >= o && su == seg) c += cu;
      }
      const uint32_t seg_next = __shfl_down(seg, 1, 64);
      if (valid && (lane == 63 || seg_next != seg) && c != 0u) atomicAdd(&tail.block_sum[seg], c);
    }
  }
}

// Keys per thread from the sort's capacity (measured: 16 takes the 161M-key tile sort of level 5
// at 3840x2160 from 2.05 to 1.83 ms, but is slower than 12 at 8.5M keys).
int radix_items(int64_t n_max) {
  return n_max >= kRadixHugeSort ? kSortItemsHuge : n_max >= kRadixBigSort ? kSortItems : kSortItemsSmall;
}

static int64_t radix_stride(int64_t n_max) {
  const int64_t tile = (int64_t)kBlock * radix_items(n_max);
  return ((n_max + tile - 1) / tile + 7) & ~(int64_t)7;
}

size_t radix_hist_bytes(int64_t n_max) { return 4 * (size_t)kRadix * (size_t)radix_stride(n_max); }

// Sort (keys, vals) by the low `bits` bits of the keys; stable. Ping-pongs between
// buffers [0] and [1]; *result_buf receives the index holding the result. hist and scan
// hold radix_hist_bytes(n_max) each (16-byte aligned). Workgroups take 2048 keys below
// kRadixBigSort keys of capacity, 3072 up to kRadixHugeSort and 4096 beyond. With a tail, the
// last pass also writes the values' tile counts in sorted order and their 256-position sums
// (see k_rs_scatter).
template <int ITEMS>
static void radix_passes(uint32_t *keys[2], uint32_t *vals[2], uint32_t *n_ptr, int64_t n_max, int bits,
                         uint32_t *hist, uint32_t *scan, uint32_t *tot, int *cur_out, const TileTail *tail,
                         const uint32_t *first_keys, hipStream_t s) {
  constexpr int TILE = kBlock * ITEMS;
  const int nb_max = (int)((n_max + TILE - 1) / TILE);
  const int stride = (int)radix_stride(n_max);
  const uint32_t n_all = (uint32_t)n_max;
  const TileTail none{nullptr, nullptr, nullptr};
  const unsigned grid = radix_grid(nb_max);
  int cur = 0;
  // the fewest passes of at most kRadixBits digit bits, the bits spread evenly over them (the
  // 13-bit tile ids of a 1080p frame as 7 + 6 rather than 8 + 5 bits)
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  for (int pass = 0, shift = 0; pass < passes; ++pass) {
    const int nbits = bits / passes + (pass < bits % passes ? 1 : 0);
    const uint32_t dmask = (1u << nbits) - 1u;
    const bool first = pass == 0 && first_keys;
    const bool last = pass == passes - 1;
    const uint32_t *kin = first ? first_keys : keys[cur];
    if (first)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rs_hist<ITEMS, true>), dim3(grid), dim3(kBlock), 0, s, kin, n_ptr, n_all,
                         shift, dmask, hist, stride);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rs_hist<ITEMS, false>), dim3(grid), dim3(kBlock), 0, s, kin, n_ptr, n_all,
                         shift, dmask, hist, stride);
    // the first pass's workgroups cover all candidates; the later passes' the count it kept
    hipLaunchKernelGGL(k_rs_scan, dim3(kRadix), dim3(kBlock), 0, s, first ? nullptr : n_ptr, n_all, hist, scan, tot,
                       stride, TILE);
    const TileTail &tt = (last && tail) ? *tail : none;
    if (first && last && tail) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rs_scatter<ITEMS, true, true>), dim3(grid), dim3(kBlock), 0, s, kin,
                         vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_ptr, n_all, n_ptr, shift, dmask, hist, scan, tot, stride,
                         tt);
    } else if (first) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rs_scatter<ITEMS, false, true>), dim3(grid), dim3(kBlock), 0, s, kin,
                         vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_ptr, n_all, n_ptr, shift, dmask, hist, scan, tot, stride,
                         tt);
    } else if (last && tail) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rs_scatter<ITEMS, true, false>), dim3(grid), dim3(kBlock), 0, s, kin,
                         vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_ptr, n_all, n_ptr, shift, dmask, hist, scan, tot, stride,
                         tt);
    } else {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rs_scatter<ITEMS, false, false>), dim3(grid), dim3(kBlock), 0, s, kin,
                         vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_ptr, n_all, n_ptr, shift, dmask, hist, scan, tot, stride,
                         tt);
    }
    cur ^= 1;
    shift += nbits;
  }
  *cur_out = cur;
}

hipError_t launch_radix_sort(uint32_t *keys[2], uint32_t *vals[2], uint32_t *n_ptr, int64_t n_max,
                             int bits, uint32_t *hist, uint32_t *scan, uint32_t *tot, int *result_buf,
                             hipStream_t s, const uint32_t *tiles_of, uint32_t *tiles_out, uint32_t *block_sum,
                             const uint32_t *first_keys) {
  *result_buf = 0;
  if (n_max <= 0) return hipSuccess;
  const TileTail t{tiles_of, tiles_out, block_sum};
  const TileTail *tail = tiles_of ? &t : nullptr;
  switch (radix_items(n_max)) {
    case kSortItemsHuge: radix_passes<kSortItemsHuge>(keys, vals, n_ptr, n_max, bits, hist, scan, tot, result_buf, tail, first_keys, s); break;
    case kSortItems: radix_passes<kSortItems>(keys, vals, n_ptr, n_max, bits, hist, scan, tot, result_buf, tail, first_keys, s); break;
    default: radix_passes<kSortItemsSmall>(keys, vals, n_ptr, n_max, bits, hist, scan, tot, result_buf, tail, first_keys, s); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Instance emission in depth order. Each Gaussian writes its footprint (tile rows and the
// span of tiles in each row, as the preprocess counted them) row-major at its offset. A
// workgroup's 256 Gaussians own one contiguous output range; it is assembled in LDS in
// windows of kEmitCap instances and each window is then written out with consecutive stores.
//  - Footprints that fill their bounding rectangle (tile count = rectangle area) are placed by
//    the whole wave: output slot v of the wave's rectangles finds its Gaussian by a binary
//    search over the lanes' inclusive counts.
//  - Other footprints of up to kEmitSolo tiles are placed by their own thread, row spans
//    recomputed in FP64 exactly as the preprocess computed them.
//  - Larger ones are placed by the whole wave, one row span per lane, then the same search
//    over the row widths.
// A Gaussian whose range does not meet the current window is skipped for that window.
// ---------------------------------------------------------------------------------------
constexpr uint32_t kEmitSolo = 256;  // measured: 64 -> 256 halves emission of 75-tile footprints (4K)
constexpr uint32_t kEmitCap = 4096;   // instances staged per window (32 KB of LDS)
constexpr uint32_t kEmitSplit = 8;    // at most this many workgroups share one block's windows,
constexpr uint32_t kEmitSplitHuge = 64;  // or this many when a block may fill kEmitHugeWindows or more
constexpr uint32_t kEmitHugeWindows = 32;

struct RectSpan {
  int x0, y0, x1, y1;
  bool full;   // the footprint is the whole rectangle
};

__device__ __forceinline__ RectSpan rect_of(uint2 r, uint32_t count) {
  RectSpan q;
  q.x0 = (int)(r.x & 0xFFFFu);
  q.y0 = (int)(r.x >> 16);
  q.x1 = (int)(r.y & 0xFFFFu);
  q.y1 = (int)(r.y >> 16);
  q.full = (uint32_t)((q.x1 - q.x0 + 1) * (q.y1 - q.y0 + 1)) == count;
  return q;
}

// Lane that owns slot v: the number of lanes whose inclusive count is <= v (incl is
// non-decreasing over the lanes and v < incl of lane 63). All lanes must take part.
__device__ __forceinline__ int owner_lane(uint32_t incl, uint32_t v) {
  int lo = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1) {
    const uint32_t x = __shfl(incl, lo + step - 1, 64);
    if (x <= v) lo += step;
  }
  return lo;
}

struct EmitWindow {
  uint32_t w0, w1;         // local positions [w0, w1) of this window
  uint32_t *t, *v;         // LDS staging, indexed by position - w0
  __device__ __forceinline__ bool meets(uint32_t lo, uint32_t hi) const { return lo < w1 && hi > w0; }
  __device__ __forceinline__ void put(uint32_t p, uint32_t tile, uint32_t g) const {
    if (p >= w0 && p < w1) {
      t[p - w0] = tile;
      v[p - w0] = g;
    }
  }
};

__global__ __launch_bounds__(kBlock) void k_emit(const uint32_t *sorted_ids, const uint32_t *n_ptr,
                                                 const uint32_t *k_ptr, const uint32_t *sorted_tiles,
                                                 const float4 *bin, const unsigned long long *prefix,
                                                 int tiles_x, int tiles_y, uint32_t *__restrict__ tile_ids,
                                                 uint32_t *__restrict__ values, uint2 *__restrict__ ranges) {
  __shared__ uint32_t s_tile[kEmitCap];
  __shared__ uint32_t s_val[kEmitCap];
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  // the tile ranges start empty (k_ranges writes the tiles that have instances): zeroed here,
  // by the first workgroup of each block, before any workgroup leaves, instead of by a launch
  // of their own
  if (blockIdx.y == 0) {
    const int n_tiles = tiles_x * tiles_y;
    for (int t = (int)j; t < n_tiles; t += (int)(gridDim.x * kBlock)) ranges[t] = make_uint2(0u, 0u);
  }
  // the counts first (the grid covers every candidate, of which n are visible); then the
  // Gaussian, its tile count and the block's offsets, loaded together
  const uint32_t n = *n_ptr;
  const uint32_t K = *k_ptr;
  if (blockIdx.x * kBlock >= n || K == 0u) return;   // no instances, or more than the buffers hold
  const bool valid = j < n;
  const uint32_t nblk = (n + kBlock - 1) / kBlock;
  const uint32_t g = valid ? sorted_ids[j] : 0u;
  const uint32_t c = valid ? sorted_tiles[j] : 0u;
  const unsigned long long obase = prefix[blockIdx.x];
  const unsigned long long block_end = (blockIdx.x + 1 < nblk) ? prefix[blockIdx.x + 1] : (unsigned long long)K;
  // workgroup (block, split) takes the block's windows split, split + gridDim.y, ...: a block
  // of huge footprints fills hundreds of windows, most blocks fill one
  const uint32_t split = blockIdx.y;
  if ((unsigned long long)split * kEmitCap >= block_end - obase) return;
  uint32_t tot;
  const uint32_t off = block_excl_scan(c, &tot);     // local position of this Gaussian's first instance
  const int lane = threadIdx.x & 63;
  // the Gaussian's binning record: one 32-byte gather (mu', conic, support bound, rectangle)
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
  if (c > 0) {
    r0 = bin[2 * (size_t)g];
    r1 = bin[2 * (size_t)g + 1];
  }
  RectSpan rs{0, 0, 0, 0, false};
  if (c > 0) rs = rect_of(make_uint2(__float_as_uint(r1.z), __float_as_uint(r1.w)), c);
  const uint32_t cf = rs.full ? c : 0u;
  const uint32_t incl_f = wave_incl_scan(cf);
  const uint32_t total_f = __shfl(incl_f, 63, 64);
  const uint32_t wf = rs.full ? (uint32_t)(rs.x1 - rs.x0 + 1) : 1u;
  const uint32_t first_f = (uint32_t)(rs.y0 * tiles_x + rs.x0);
  const uint32_t wave_lo = __shfl(off, 0, 64), wave_hi = __shfl(off + c, 63, 64);
  const unsigned long long big_all = __ballot(c > kEmitSolo && !rs.full);

  for (uint32_t w0 = split * kEmitCap; w0 < tot; w0 += gridDim.y * kEmitCap) {
    const EmitWindow win{w0, min(w0 + kEmitCap, tot), s_tile, s_val};
    if (win.meets(wave_lo, wave_hi)) {
      // full rectangles, the whole wave at once. A lane's full slots take consecutive
      // positions, and positions grow with the slot index v over the wave, so the slots that
      // land in this window are the range [va, vb): the slots before each window edge, summed
      // over the lanes. (Walking every slot in every window made huge footprints quadratic.)
      const uint32_t va = wave_sum_u32(cf ? min(cf, (uint32_t)max(0ll, (long long)win.w0 - (long long)off)) : 0u);
      const uint32_t vb = wave_sum_u32(cf ? min(cf, (uint32_t)max(0ll, (long long)win.w1 - (long long)off)) : 0u);
      for (uint32_t v0 = va; v0 < vb; v0 += 64) {
        const uint32_t v = min(v0 + (uint32_t)lane, vb - 1u);
        const int o = owner_lane(incl_f, v);
        const uint32_t t = v - (__shfl(incl_f, o, 64) - __shfl(cf, o, 64));
        const uint32_t wo = __shfl(wf, o, 64);
        const uint32_t row = t / wo;
        const uint32_t tile = __shfl(first_f, o, 64) + row * (uint32_t)tiles_x + (t - row * wo);
        const uint32_t pos = __shfl(off, o, 64) + t;
        const uint32_t go = __shfl(g, o, 64);
        if (v0 + (uint32_t)lane < vb) win.put(pos, tile, go);
      }
      // small footprints that do not fill their rectangle, one thread each
      if (c > 0 && c <= kEmitSolo && !rs.full && win.meets(off, off + c)) {
        Footprint fp;
        footprint(r0.x, r0.y, r0.z, r0.w, r1.x, support_span(r1.y), tiles_y, fp);
        uint32_t pos = off;
        for (int ty = fp.ty0; ty <= fp.ty1; ++ty) {
          int tx0, tx1;
          if (!row_span(fp, ty, tiles_x, tx0, tx1)) continue;
          for (int tx = tx0; tx <= tx1; ++tx) win.put(pos++, (uint32_t)(ty * tiles_x + tx), g);
        }
      }
      // large footprints that do not fill their rectangle, one at a time per wave
      unsigned long long big = big_all;
      while (big) {
        const int src = __ffsll((long long)big) - 1;
        big &= big - 1;
        const uint32_t os = __shfl(off, src, 64);
        const uint32_t cs = __shfl(c, src, 64);
        if (!win.meets(os, os + cs)) continue;
        const uint32_t gs = __shfl(g, src, 64);
        Footprint fp;
        footprint(__shfl(r0.x, src, 64), __shfl(r0.y, src, 64), __shfl(r0.z, src, 64), __shfl(r0.w, src, 64),
                  __shfl(r1.x, src, 64), support_span(__shfl(r1.y, src, 64)), tiles_y, fp);
        const int nrows = fp.ty1 - fp.ty0 + 1;
        uint32_t base = os;
        for (int rb = 0; rb < nrows; rb += 64) {
          const int ty = fp.ty0 + rb + lane;
          int tx0 = 0, tx1 = -1;
          if (rb + lane < nrows) row_span(fp, ty, tiles_x, tx0, tx1);
          const uint32_t wr = (uint32_t)(tx1 - tx0 + 1);
          const uint32_t incl = wave_incl_scan(wr);
          const uint32_t total = __shfl(incl, 63, 64);
          const uint32_t first = (uint32_t)(ty * tiles_x + tx0);
          // only the slots of these rows whose positions fall in the window
          const uint32_t va = (uint32_t)min((long long)total, max(0ll, (long long)win.w0 - (long long)base));
          const uint32_t vb = (uint32_t)min((long long)total, max(0ll, (long long)win.w1 - (long long)base));
          for (uint32_t v0 = va; v0 < vb; v0 += 64) {
            const uint32_t v = min(v0 + (uint32_t)lane, vb - 1u);
            const int o = owner_lane(incl, v);
            const uint32_t t = v - (__shfl(incl, o, 64) - __shfl(wr, o, 64));
            const uint32_t tile = __shfl(first, o, 64) + t;
            if (v0 + (uint32_t)lane < vb) win.put(base + v, tile, gs);
          }
          base += total;
          if (base >= win.w1) break;   // later rows land past the window
        }
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < win.w1 - win.w0; i += kBlock) {
      tile_ids[obase + w0 + i] = s_tile[i];
      values[obase + w0 + i] = s_val[i];
    }
    __syncthreads();
  }
}

hipError_t launch_emit(const uint32_t *sorted_ids, const uint32_t *n_ptr, const uint32_t *k_ptr, int64_t n_max,
                       int64_t k_max, const uint32_t *sorted_tiles, const float4 *bin,
                       const unsigned long long *prefix, int tiles_x, int tiles_y, uint32_t *tile_ids,
                       uint32_t *values, uint2 *ranges, hipStream_t s) {
  if (n_max <= 0) return hipSuccess;
  // workgroups per block: enough for the windows an average block of up to k_max instances
  // fills (1 when blocks fit a window, as they do for small footprints). Coarse levels, whose
  // few blocks each fill hundreds of windows, get up to 64 (level 1 at 3840x2160: 1.42 ->
  // 1.04 ms); others at most 8, since the surplus workgroups of a small frame on a context
  // whose capacity a large frame set still cost their launch.
  const int64_t blocks = (n_max + kBlock - 1) / kBlock;
  const int64_t windows = (k_max + blocks * (int64_t)kEmitCap - 1) / (blocks * (int64_t)kEmitCap);
  const int64_t cap_split = windows >= (int64_t)kEmitHugeWindows ? kEmitSplitHuge : kEmitSplit;
  const unsigned split = (unsigned)std::min<int64_t>(cap_split, std::max<int64_t>(1, windows));
  hipLaunchKernelGGL(k_emit, dim3((unsigned)blocks, split), dim3(kBlock), 0, s, sorted_ids, n_ptr, k_ptr,
                     sorted_tiles, bin, prefix, tiles_x, tiles_y, tile_ids, values, ranges);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Tile ranges from the sorted tile ids (ranges zeroed beforehand); the id count is read on
// the device, the grid covers k_max ids.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_ranges(const uint32_t *__restrict__ tile_ids, const uint32_t *k_ptr,
                                                   uint2 *__restrict__ ranges) {
  const uint32_t K = *k_ptr;
  const uint32_t k0 = 4u * (blockIdx.x * kBlock + threadIdx.x);   // four ids per thread
  if (k0 >= K) return;
  uint32_t t[4];
  if (k0 + 4u <= K) {
    const uint4 v = *reinterpret_cast<const uint4 *>(tile_ids + k0);
    t[0] = v.x; t[1] = v.y; t[2] = v.z; t[3] = v.w;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = (k0 + i < K) ? tile_ids[k0 + i] : 0u;
  }
  uint32_t prev = (k0 > 0u) ? tile_ids[k0 - 1u] : 0xFFFFFFFFu;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t k = k0 + i;
    if (k >= K) break;
    if (t[i] != prev) {
      ranges[t[i]].x = k;
      if (k > 0u) ranges[prev].y = k;
    }
    prev = t[i];
  }
  if (k0 + 4u >= K) ranges[prev].y = K;   // the last id closes its tile
}

// 16-byte stores over the aligned body (grid-stride), single words before and after it.
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  const int64_t lead = min(n, (int64_t)(((16u - (uint32_t)(reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / 4u));
  const int64_t n4 = (n - lead) / 4;
  uint4 *q = reinterpret_cast<uint4 *>(p + lead);
  const uint4 vv = make_uint4(v, v, v, v);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) q[i] = vv;
  if (blockIdx.x == 0) {
    const int64_t tail = lead + 4 * n4;
    if ((int64_t)threadIdx.x < lead) p[threadIdx.x] = v;
    if ((int64_t)threadIdx.x < n - tail) p[tail + threadIdx.x] = v;
  }
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t groups = (n / 4 + kBlock - 1) / kBlock;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(groups, 4096));
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t *tile_ids, const uint32_t *k_ptr, int64_t k_max, int n_tiles,
                         uint2 *ranges, bool zeroed, hipStream_t s) {
  hipError_t e = zeroed ? hipSuccess : launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u, 2 * (int64_t)n_tiles, s);
  if (e != hipSuccess || k_max <= 0) return e;
  const int64_t threads = (k_max + 3) / 4;
  hipLaunchKernelGGL(k_ranges, dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, tile_ids,
                     k_ptr, ranges);
  return hipGetLastError();
}

}  // namespace flod

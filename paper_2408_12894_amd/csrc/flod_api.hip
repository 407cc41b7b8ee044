// C ABI of libflod: argument validation, workspace management and stage orchestration on
// the caller's stream. Every arithmetic step runs in the kernels of this library.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <mutex>
#include <new>

#include "flod_internal.h"

using namespace flod;

// Fixed scratch of flod_l1_ssim_forward_noalloc: the SSIM forward's per-workgroup partial
// sums (one double2 per workgroup). Each device holds its own copy until the process ends.
// Host code never passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol): the device address is looked up once per device, with that device
// current, when a context is created on it, and kept in g_scratch_dev.
constexpr size_t kNoAllocScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch_dev[kMaxDevices];
std::mutex g_scratch_mu;

// Look up the device address of `scratch` on `device`, which must be current.
bool resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return true;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return false;
  }
  g_scratch_dev[device] = ptr;
  return true;
}

void *scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[device];
}
}  // namespace

namespace {

struct Buf {
  void *p = nullptr;
  size_t cap = 0;
};

enum BufId {
  B_XYAB, B_COP, B_BLUE, B_DEPTH, B_BIN, B_TILES, B_BLOCKVIS, B_PREFIX,
  B_DKEY0, B_DKEY1, B_DVAL0, B_DVAL1, B_TBSUM, B_TPREFIX,
  B_TKEY0, B_TKEY1, B_TVAL0, B_TVAL1, B_HIST, B_SCAN, B_TOT, B_RANGES, B_COUNTERS,
  B_G2D, B_SSIM, B_BLENDED, B_TILE_BLENDED, B_TILE_ORDER, B_STILES, B_SHJAC, B_COUNT
};

struct Saved {
  bool valid = false;
  bool is_level = false;
  flod_level level{};
  int sh_degree = 0;
  DevCamera cam{};
  float bg[3] = {0, 0, 0};
  const float *final_T = nullptr;
  const int32_t *n_contrib = nullptr;
  int sorted_vals = 0;   // which of B_TVAL0/B_TVAL1 holds the sorted values
  int sorted_keys = 0;
  int depth_buf = 0;
  bool has_grad2d = false;
  bool grad2d_moments = false;   // B_G2D still holds the backward's moment sums (see flod_ctx_view)
  bool has_blended = false;      // the render listed its blended entries (the backward needs them)
};

}  // namespace

struct flod_ctx {
  int device = 0;
  flod_alloc_fn alloc = nullptr;
  flod_free_fn release = nullptr;
  void *user = nullptr;
  Buf buf[B_COUNT];
  hipStream_t last_stream = nullptr;   // stream of the last call that used the workspace
  bool has_stream = false;
  hipEvent_t ev_switch = nullptr;       // orders a call on a new stream after the last one
  size_t required = 0;
  unsigned long long *host_counters = nullptr;   // pinned: [visible u32 | K u32], [K u64]
  // coherent pinned memory the offsets scan writes the counts into, as four 64-bit words
  // tagged with the render's sequence number (null: copy instead), and its device address
  unsigned long long *host_counts = nullptr;
  unsigned long long *host_counts_dev = nullptr;
  uint32_t count_seq = 0;
  Saved saved;
  bool keep_backward = true;          // renders list their blended entries (flod_ctx_keep_backward_state)
  flod_stats stats{};
  // timing
  bool timing = false;
  uint32_t timing_mask = 0;           // stages recorded when timing is on
  hipEvent_t ev_sync = nullptr;       // marks the instance-count read-back
  hipEvent_t ev[FLOD_NUM_STAGES][2];
  bool ev_pending[FLOD_NUM_STAGES];
  double ms[FLOD_NUM_STAGES];
  int64_t calls[FLOD_NUM_STAGES];
  bool events_made = false;
};

namespace {

size_t ws_bytes(const flod_ctx *c) {
  size_t t = 0;
  for (int i = 0; i < B_COUNT; ++i) t += c->buf[i].cap;
  return t;
}

void release_buf(flod_ctx *c, Buf &b, hipStream_t s) {
  if (!b.p) return;
  if (c->release)
    c->release(c->user, b.p, b.cap, (void *)s);
  else
    (void)hipFreeAsync(b.p, s);
  b.p = nullptr;
  b.cap = 0;
}

// Grow-only buffers: reallocate with 25% headroom when too small.
flod_status ensure(flod_ctx *c, BufId id, size_t bytes, hipStream_t s, size_t *extra_needed) {
  Buf &b = c->buf[id];
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return FLOD_OK;
  size_t want = bytes + bytes / 4;
  want = (want + 255) & ~(size_t)255;
  release_buf(c, b, s);
  void *p = nullptr;
  if (c->alloc) {
    p = c->alloc(c->user, want, (void *)s);
  } else {
    if (hipMallocAsync(&p, want, s) != hipSuccess) p = nullptr;
  }
  if (!p) {
    *extra_needed += want;
    return FLOD_ERR_WORKSPACE;
  }
  b.p = p;
  b.cap = want;
  return FLOD_OK;
}

template <class T> T *P(flod_ctx *c, BufId id) { return reinterpret_cast<T *>(c->buf[id].p); }

flod_status dev(hipError_t e) { return e == hipSuccess ? FLOD_OK : FLOD_ERR_DEVICE; }

void timing_flush(flod_ctx *c) {
  if (!c->events_made) return;
  for (int k = 0; k < FLOD_NUM_STAGES; ++k) {
    if (!c->ev_pending[k]) continue;
    float ms = 0.f;
    if (hipEventSynchronize(c->ev[k][1]) == hipSuccess && hipEventElapsedTime(&ms, c->ev[k][0], c->ev[k][1]) == hipSuccess) {
      c->ms[k] += ms;
      c->calls[k] += 1;
    }
    c->ev_pending[k] = false;
  }
}

struct StageTimer {
  flod_ctx *c;
  hipStream_t s;
  int stage = -1;
  StageTimer(flod_ctx *c_, hipStream_t s_) : c(c_), s(s_) {}
  void begin(int k) {
    if (!c->timing || !((c->timing_mask >> k) & 1u)) return;
    stage = k;
    (void)hipEventRecord(c->ev[k][0], s);
  }
  void end() {
    if (!c->timing || stage < 0) return;
    (void)hipEventRecord(c->ev[stage][1], s);
    c->ev_pending[stage] = true;
    stage = -1;
  }
  // A one-kernel stage timed by its kernel's dispatch: the stage's events for the launch (null
  // when the stage is not recorded), so that no event packet sits between it and its neighbours.
  void dispatch(int k, hipEvent_t *start, hipEvent_t *stop) {
    *start = *stop = nullptr;
    if (!c->timing || !((c->timing_mask >> k) & 1u)) return;
    *start = c->ev[k][0];
    *stop = c->ev[k][1];
    c->ev_pending[k] = true;
  }
};

// Every call that uses the context's workspace runs on its caller's stream. When that stream
// differs from the one the context last used, the new stream first waits for the work already
// enqueued on the old one (an event, no host wait), so buffers are never reused, grown or
// released while an earlier call may still read or write them.
hipError_t use_stream(flod_ctx *c, hipStream_t s) {
  if (c->has_stream && s != c->last_stream) {
    if (!c->ev_switch && hipEventCreateWithFlags(&c->ev_switch, hipEventDisableTiming) != hipSuccess) {
      c->ev_switch = nullptr;
      return hipErrorOutOfMemory;
    }
    hipError_t e = hipEventRecord(c->ev_switch, c->last_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->ev_switch, 0);
    if (e != hipSuccess) return e;
  }
  c->last_stream = s;
  c->has_stream = true;
  return hipSuccess;
}

// Mark the work enqueued on s so far; wait_marked() returns once it has finished.
hipError_t mark_stream(flod_ctx *c, hipStream_t s) {
  if (!c->ev_sync && hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming) != hipSuccess) {
    c->ev_sync = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipEventRecord(c->ev_sync, s);
}

// Poll an event (a few microseconds of wake-up instead of a blocking wait's), falling back to
// a blocking wait after ~20000 polls.
hipError_t wait_event(hipEvent_t ev) {
  hipError_t e = hipSuccess;
  for (int spin = 0; spin < 20000; ++spin) {
    e = hipEventQuery(ev);
    if (e != hipErrorNotReady) return e;
  }
  return hipEventSynchronize(ev);
}

hipError_t wait_marked(flod_ctx *c) { return wait_event(c->ev_sync); }

// Wait until all four count words carry `seq` (the scan kernel writes them whole): polling,
// and after about 2 s a blocking wait for the stream, then one last look.
hipError_t wait_counts(flod_ctx *c, hipStream_t s, uint32_t seq) {
  const volatile unsigned long long *w = c->host_counts;
  auto ready = [&]() {
    for (int k = 0; k < 4; ++k)
      if ((uint32_t)(w[k] >> 32) != seq) return false;
    return true;
  };
  const auto t0 = std::chrono::steady_clock::now();
  for (uint64_t spin = 0;; ++spin) {
    if (ready()) return hipSuccess;
    if ((spin & 1023u) == 1023u && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) break;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  return ready() ? hipSuccess : hipErrorUnknown;
}

int ceil_log2(int64_t v) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < v) ++b;
  return b;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

flod_status check_level(const flod_level *lv) {
  if (!lv || lv->n < 0) return FLOD_ERR_INVALID_ARG;
  if (lv->n == 0) return FLOD_OK;
  if (!lv->means || !lv->log_scales || !lv->quats || !lv->opacity_logits || !lv->sh) return FLOD_ERR_INVALID_ARG;
  if (!aligned(lv->quats, 16) || !aligned(lv->sh, 16) || !aligned(lv->means, 4) || !aligned(lv->log_scales, 4) ||
      !aligned(lv->opacity_logits, 4))
    return FLOD_ERR_INVALID_ARG;
  if (!(lv->s_min >= 0.0f) || !isfinite(lv->s_min)) return FLOD_ERR_INVALID_ARG;
  return FLOD_OK;
}

flod_status check_camera(const flod_camera *cam) {
  if (!cam) return FLOD_ERR_INVALID_ARG;
  if (cam->width <= 0 || cam->height <= 0 || cam->width > 16384 || cam->height > 16384) return FLOD_ERR_INVALID_ARG;
  if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f) || !isfinite(cam->fx) || !isfinite(cam->fy)) return FLOD_ERR_INVALID_ARG;
  return FLOD_OK;
}

DevCamera dev_camera(const flod_camera *cam) {
  DevCamera d;
  memcpy(d.R, cam->R, sizeof(d.R));
  memcpy(d.t, cam->t, sizeof(d.t));
  memcpy(d.campos, cam->campos, sizeof(d.campos));
  d.fx = cam->fx; d.fy = cam->fy; d.cx = cam->cx; d.cy = cam->cy;
  d.W = cam->width; d.H = cam->height;
  d.tiles_x = (cam->width + kTile - 1) / kTile;
  d.tiles_y = (cam->height + kTile - 1) / kTile;
  return d;
}

float sq32(float d) { return isinf(d) ? INFINITY : (float)((double)d * (double)d); }

// Instances the tail buffers (tile keys and values, both ping-pong halves, the list of blended
// entries) hold.
int64_t instance_capacity(const flod_ctx *c) {
  size_t b = c->buf[B_TKEY0].cap;
  for (BufId id : {B_TKEY1, B_TVAL0, B_TVAL1}) b = b < c->buf[id].cap ? b : c->buf[id].cap;
  int64_t k = (int64_t)(b / 4);
  if (c->keep_backward) {
    const int64_t t = (int64_t)(c->buf[B_BLENDED].cap / 8);
    if (t < k) k = t;
  }
  if (k > 0xFFFFFFFEll) k = 0xFFFFFFFEll;
  return k > 0 ? k : 0;
}

size_t hist_bytes(int64_t n_max) { return radix_hist_bytes(n_max); }

// The forward pipeline over the candidate set described by p.
//
// The instance count K is known on the device only after the tile-count scan. The emission,
// tile sort, ranges and blend that follow are enqueued at once, sized for the instances the
// context's buffers hold (cap); the scan hands them K when K <= cap and 0 otherwise, in which
// case they do nothing. Meanwhile the host reads K back (stream-ordered, 16 bytes) for the
// statistics and the capacity check: when K > cap it grows the buffers and enqueues the scan's
// count and the tail again. A context's first render (cap = 0) waits for K before enqueuing.
// level: a single-level render, which keeps what its backward needs (when the context keeps
// backward state)
flod_status render_common(flod_ctx *c, PreParams &p, int64_t *n_selected, const float bg[3],
                          flod_frame *out, hipStream_t s, bool level = false) {
  c->required = 0;
  if (use_stream(c, s) != hipSuccess) return FLOD_ERR_DEVICE;
  c->saved.valid = false;
  c->saved.has_grad2d = false;
  timing_flush(c);
  StageTimer tm(c, s);
  const int64_t N = p.n_total;
  const DevCamera &cam = p.cam;
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  const int nb = (int)((N + kBlock - 1) / kBlock);
  int64_t cap = instance_capacity(c);
  size_t extra = 0;
  flod_status st = FLOD_OK;
  auto need = [&](BufId id, size_t bytes) {
    flod_status r = ensure(c, id, bytes, s, &extra);
    if (r != FLOD_OK) st = r;
  };
  const size_t hist = hist_bytes(N) > hist_bytes(cap) ? hist_bytes(N) : hist_bytes(cap);
  need(B_XYAB, 16 * (size_t)N);
  need(B_COP, 16 * (size_t)N);
  need(B_BLUE, 8 * (size_t)N);
  need(B_DEPTH, 4 * (size_t)N);
  need(B_BIN, 32 * (size_t)N);
  need(B_TILES, 4 * (size_t)N);
  need(B_BLOCKVIS, 4 * (size_t)nb);
  need(B_PREFIX, 8 * (size_t)nb);
  need(B_DKEY0, 4 * (size_t)N);
  need(B_DKEY1, 4 * (size_t)N);
  need(B_DVAL0, 4 * (size_t)N);
  need(B_DVAL1, 4 * (size_t)N);
  need(B_TBSUM, 4 * (size_t)nb);
  need(B_TPREFIX, 8 * (size_t)nb);
  need(B_STILES, 4 * (size_t)N);
  need(B_HIST, hist);
  need(B_SCAN, hist);
  need(B_TOT, 4 * (size_t)kRadix);
  need(B_RANGES, 8 * (size_t)n_tiles);
  need(B_TILE_BLENDED, 4 * (size_t)n_tiles);
  need(B_TILE_ORDER, 4 * ((size_t)n_tiles + 2));
  need(B_COUNTERS, 8 * (size_t)kCntSlots);
  const bool jac = level && c->keep_backward;   // the colour Jacobians for the backward
  if (jac) need(B_SHJAC, 48 * (size_t)N);
  if (st != FLOD_OK) {
    c->required = ws_bytes(c) + extra;
    return st;
  }
  uint32_t *counters = P<uint32_t>(c, B_COUNTERS);
  const bool speculate = N > 0 && cap > 0;
  int dres = 0;
  uint32_t *sorted_tiles = nullptr;
  // tile counts in depth order and their scan; K (guarded by `guard`) to counters[kCntInstances]
  // and, when `to_host`, the counts straight to the host, tagged with this render's number
  const bool direct = c->host_counts_dev != nullptr;
  if (direct && ++c->count_seq == 0u) c->count_seq = 1u;   // 0 is the buffer's initial tag
  const uint32_t seq = direct ? c->count_seq : 0u;
  auto offsets = [&](int64_t guard, bool to_host) -> hipError_t {
    return launch_scan_blocks(P<uint32_t>(c, B_TBSUM), counters + kCntVisible, kBlock,
                              P<unsigned long long>(c, B_TPREFIX), counters + kCntInstances,
                              reinterpret_cast<unsigned long long *>(counters + kCntTotal64), nb, s,
                              (unsigned long long)guard, to_host ? c->host_counts_dev : nullptr, seq);
  };
  if (N > 0) {
    PreOut o;
    o.xyab = P<float4>(c, B_XYAB);
    o.cop = P<float4>(c, B_COP);
    o.blue = P<float2>(c, B_BLUE);
    o.depth = P<uint32_t>(c, B_DEPTH);
    o.bin = P<float4>(c, B_BIN);
    o.tiles = P<uint32_t>(c, B_TILES);
    o.block_vis = P<uint32_t>(c, B_BLOCKVIS);
    o.zero_sums = P<uint32_t>(c, B_TBSUM);
    o.n_selected = reinterpret_cast<unsigned long long *>(n_selected);
    o.shjac = jac ? P<float4>(c, B_SHJAC) : nullptr;
    tm.begin(FLOD_STAGE_PREPROCESS);
    if (launch_preprocess(p, o, s) != hipSuccess) return FLOD_ERR_DEVICE;
    tm.end();
    tm.begin(FLOD_STAGE_DEPTH_SORT);
    uint32_t *dk[2] = {P<uint32_t>(c, B_DKEY0), P<uint32_t>(c, B_DKEY1)};
    uint32_t *dv[2] = {P<uint32_t>(c, B_DVAL0), P<uint32_t>(c, B_DVAL1)};
    // the first pass reads every candidate's depth key and keeps the rendered ones (the
    // compaction of the visible set; their count goes to counters[kCntVisible]); the last pass
    // also writes the tile counts in depth order and their sums per workgroup of the emission
    // (zeroed by the preprocess)
    sorted_tiles = P<uint32_t>(c, B_STILES);
    if (launch_radix_sort(dk, dv, counters + kCntVisible, N, 32, P<uint32_t>(c, B_HIST), P<uint32_t>(c, B_SCAN),
                          P<uint32_t>(c, B_TOT), &dres, s, o.tiles, sorted_tiles, P<uint32_t>(c, B_TBSUM),
                          o.depth) != hipSuccess)
      return FLOD_ERR_DEVICE;
    tm.end();
    tm.begin(FLOD_STAGE_OFFSETS);
    if (offsets(speculate ? cap : 0xFFFFFFFEll, direct) != hipSuccess) return FLOD_ERR_DEVICE;
    // the count read-back, [visible u32 | guarded K u32], [K u64]: written by the scan itself
    // (direct), else copied
    if (!direct && (hipMemcpyAsync(c->host_counters, counters, 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    mark_stream(c, s) != hipSuccess))
      return FLOD_ERR_DEVICE;
    tm.end();
  }
  int tres = 0;
  // emission, tile sort, ranges and blend for at most k_max instances
  auto tail = [&](int64_t k_max) -> flod_status {
    uint32_t *tk[2] = {P<uint32_t>(c, B_TKEY0), P<uint32_t>(c, B_TKEY1)};
    uint32_t *tv[2] = {P<uint32_t>(c, B_TVAL0), P<uint32_t>(c, B_TVAL1)};
    tres = 0;
    if (k_max > 0) {
      uint32_t *dv = dres ? P<uint32_t>(c, B_DVAL1) : P<uint32_t>(c, B_DVAL0);
      tm.begin(FLOD_STAGE_EMIT);
      if (launch_emit(dv, counters + kCntVisible, counters + kCntInstances, N, k_max, sorted_tiles, P<float4>(c, B_BIN),
                      P<unsigned long long>(c, B_TPREFIX), cam.tiles_x, cam.tiles_y, tk[0], tv[0],
                      P<uint2>(c, B_RANGES), s) != hipSuccess)
        return FLOD_ERR_DEVICE;
      tm.end();
      tm.begin(FLOD_STAGE_TILE_SORT);
      const int bits = ceil_log2(n_tiles);
      if (bits > 0 && launch_radix_sort(tk, tv, counters + kCntInstances, k_max, bits, P<uint32_t>(c, B_HIST),
                                        P<uint32_t>(c, B_SCAN), P<uint32_t>(c, B_TOT), &tres, s) != hipSuccess)
        return FLOD_ERR_DEVICE;
      tm.end();
    }
    tm.begin(FLOD_STAGE_RANGES);
    // the emission zeroed the ranges when it ran
    if (launch_ranges(tk[tres], counters + kCntInstances, k_max, n_tiles, P<uint2>(c, B_RANGES), k_max > 0, s) !=
        hipSuccess)
      return FLOD_ERR_DEVICE;
    tm.end();
    tm.begin(FLOD_STAGE_BLEND);
    uint32_t *order = P<uint32_t>(c, B_TILE_ORDER);
    if (launch_tile_order_by_length(P<uint2>(c, B_RANGES), n_tiles, order, s) != hipSuccess ||
        launch_blend(P<uint2>(c, B_RANGES), tv[tres], P<float4>(c, B_XYAB), P<float4>(c, B_COP),
                     P<float2>(c, B_BLUE), cam, bg, out->image, out->final_T, out->n_contrib, out->n_blended,
                     c->keep_backward ? P<uint2>(c, B_BLENDED) : nullptr,
                     c->keep_backward ? P<uint32_t>(c, B_TILE_BLENDED) : nullptr, order, s) != hipSuccess)
      return FLOD_ERR_DEVICE;
    tm.end();
    return FLOD_OK;
  };
  if (speculate && (st = tail(cap)) != FLOD_OK) return st;
  int64_t n_vis = 0;
  unsigned long long K = 0;
  if (N > 0) {
    if (direct) {
      if (wait_counts(c, s, seq) != hipSuccess) return FLOD_ERR_DEVICE;
      const volatile unsigned long long *w = c->host_counts;
      n_vis = (uint32_t)w[0];
      K = (unsigned long long)(uint32_t)w[2] | ((unsigned long long)(uint32_t)w[3] << 32);
    } else {
      if (wait_marked(c) != hipSuccess) return FLOD_ERR_DEVICE;
      n_vis = reinterpret_cast<const uint32_t *>(c->host_counters)[kCntVisible];
      K = c->host_counters[1];
    }
  }
  c->stats.n_candidates = N;
  c->stats.n_visible = n_vis;
  c->stats.n_instances = (int64_t)K;
  c->stats.tiles_x = cam.tiles_x;
  c->stats.tiles_y = cam.tiles_y;
  c->stats.width = cam.W;
  c->stats.height = cam.H;
  if (K >= 0xFFFFFFFFull) return FLOD_ERR_OVERFLOW;
  if (!speculate || (int64_t)K > cap) {
    if ((int64_t)K > cap) {
      const int64_t Kn = (int64_t)K;
      need(B_TKEY0, 4 * (size_t)Kn);
      need(B_TKEY1, 4 * (size_t)Kn);
      need(B_TVAL0, 4 * (size_t)Kn);
      need(B_TVAL1, 4 * (size_t)Kn);
      if (c->keep_backward) need(B_BLENDED, 8 * (size_t)Kn);
      if (st == FLOD_OK) {
        cap = instance_capacity(c);
        need(B_HIST, hist_bytes(cap));
        need(B_SCAN, hist_bytes(cap));
      }
      if (st != FLOD_OK) {
        c->required = ws_bytes(c) + extra;
        return st;
      }
      if (speculate && offsets(cap, false) != hipSuccess) return FLOD_ERR_DEVICE;
    }
    if ((st = tail(N > 0 ? cap : 0)) != FLOD_OK) return st;
  }
  Saved &sv = c->saved;
  sv.valid = true;
  sv.cam = cam;
  sv.bg[0] = bg[0]; sv.bg[1] = bg[1]; sv.bg[2] = bg[2];
  sv.final_T = out->final_T;
  sv.n_contrib = out->n_contrib;
  sv.sorted_vals = tres;
  sv.sorted_keys = tres;
  sv.depth_buf = dres;
  sv.sh_degree = p.sh_degree;
  sv.has_blended = c->keep_backward;
  return FLOD_OK;
}

PreParams base_params(const DevCamera &cam, int sh_degree) {
  PreParams p;
  memset(&p, 0, sizeof(p));
  p.cam = cam;
  p.sh_degree = sh_degree;
  p.logit_min = (float)(-log(254.0));
  return p;
}

bool frame_ok(const flod_frame *out) { return out && out->image && out->final_T && out->n_contrib; }

}  // namespace

extern "C" {

flod_status flod_ctx_create(flod_ctx **ctx, int device, flod_alloc_fn alloc, flod_free_fn release, void *user) {
  if (!ctx || (alloc == nullptr) != (release == nullptr)) return FLOD_ERR_INVALID_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return FLOD_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return FLOD_ERR_DEVICE;
  // the allocation-free entry point's scratch on this device (failure only disables it)
  (void)resolve_scratch(device);
  flod_ctx *c = new (std::nothrow) flod_ctx();
  if (!c) return FLOD_ERR_WORKSPACE;
  c->device = device;
  c->alloc = alloc;
  c->release = release;
  c->user = user;
  if (hipHostMalloc((void **)&c->host_counters, 64, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return FLOD_ERR_DEVICE;
  }
  // counts written by a kernel straight into coherent host memory; without it (or with
  // FLOD_COUNT_COPY=1 in the environment) the render copies them
  const char *force_copy = getenv("FLOD_COUNT_COPY");
  if (!(force_copy && force_copy[0] == '1') &&
      hipHostMalloc((void **)&c->host_counts, 64, hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess) {
    memset(c->host_counts, 0, 64);   // sequence 0 is never a render's
    if (hipHostGetDevicePointer((void **)&c->host_counts_dev, c->host_counts, 0) != hipSuccess) {
      (void)hipHostFree(c->host_counts);
      c->host_counts = nullptr;
    }
  }
  if (!c->host_counts) {
    c->host_counts_dev = nullptr;
    (void)hipGetLastError();
  }
  memset(c->ms, 0, sizeof(c->ms));
  memset(c->calls, 0, sizeof(c->calls));
  memset(c->ev_pending, 0, sizeof(c->ev_pending));
  *ctx = c;
  return FLOD_OK;
}

void flod_ctx_destroy(flod_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->last_stream;
  (void)hipStreamSynchronize(s);
  for (int i = 0; i < B_COUNT; ++i) release_buf(ctx, ctx->buf[i], s);
  (void)hipStreamSynchronize(s);
  if (ctx->events_made)
    for (int k = 0; k < FLOD_NUM_STAGES; ++k) {
      (void)hipEventDestroy(ctx->ev[k][0]);
      (void)hipEventDestroy(ctx->ev[k][1]);
    }
  if (ctx->ev_sync) (void)hipEventDestroy(ctx->ev_sync);
  if (ctx->ev_switch) (void)hipEventDestroy(ctx->ev_switch);
  if (ctx->host_counters) (void)hipHostFree(ctx->host_counters);
  if (ctx->host_counts) (void)hipHostFree(ctx->host_counts);
  delete ctx;
}

size_t flod_ctx_workspace_bytes(const flod_ctx *ctx) { return ctx ? ws_bytes(ctx) : 0; }

size_t flod_ctx_required_bytes(const flod_ctx *ctx) { return ctx ? ctx->required : 0; }

flod_status flod_ctx_trim(flod_ctx *ctx, void *stream) {
  if (!ctx) return FLOD_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  hipStream_t s = (hipStream_t)stream;
  if (use_stream(ctx, s) != hipSuccess) return FLOD_ERR_DEVICE;
  for (int i = 0; i < B_COUNT; ++i) release_buf(ctx, ctx->buf[i], s);
  ctx->saved.valid = false;
  return FLOD_OK;
}

flod_status flod_render_level(flod_ctx *ctx, const flod_level *level, int sh_degree, const flod_camera *cam,
                              const float bg[3], flod_frame *out, void *stream) {
  if (!ctx || !bg || !frame_ok(out) || sh_degree < 0 || sh_degree > 3) return FLOD_ERR_INVALID_ARG;
  flod_status st = check_level(level);
  if (st != FLOD_OK) return st;
  if ((st = check_camera(cam)) != FLOD_OK) return st;
  if (level->n > 0xFFFFFFF0ll) return FLOD_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  PreParams p = base_params(dev_camera(cam), sh_degree);
  p.n_levels = 1;
  p.select = 0;
  DevLevel &L = p.lv[0];
  L.means = level->means; L.log_scales = level->log_scales; L.quats = level->quats;
  L.logits = level->opacity_logits; L.sh = level->sh;
  L.offset = 0; L.n = level->n; L.s_min = level->s_min;
  L.lo2 = 0.0f; L.hi2 = INFINITY;
  p.n_total = level->n;
  st = render_common(ctx, p, nullptr, bg, out, (hipStream_t)stream, true);
  if (st == FLOD_OK) {
    ctx->saved.is_level = true;
    ctx->saved.level = *level;
  }
  return st;
}

flod_status flod_render_selective(flod_ctx *ctx, const flod_level *levels, int n_levels, int l_start, int l_end,
                                  const float *d_proj, const float centre[3], int sh_degree, const flod_camera *cam,
                                  const float bg[3], flod_frame *out, int64_t *n_selected, void *stream) {
  if (!ctx || !levels || !d_proj || !centre || !bg || !frame_ok(out) || sh_degree < 0 || sh_degree > 3)
    return FLOD_ERR_INVALID_ARG;
  if (n_levels < 1 || n_levels > FLOD_MAX_LEVELS || l_start < 1 || l_end < l_start || l_end > n_levels)
    return FLOD_ERR_INVALID_ARG;
  flod_status st = check_camera(cam);
  if (st != FLOD_OK) return st;
  for (int l = l_start; l <= l_end; ++l)
    if ((st = check_level(&levels[l - 1])) != FLOD_OK) return st;
  for (int l = 0; l < n_levels; ++l)
    if (!(d_proj[l] >= 0.0f)) return FLOD_ERR_INVALID_ARG;
  if (!isfinite(centre[0]) || !isfinite(centre[1]) || !isfinite(centre[2])) return FLOD_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  PreParams p = base_params(dev_camera(cam), sh_degree);
  p.select = 1;
  p.centre[0] = centre[0]; p.centre[1] = centre[1]; p.centre[2] = centre[2];
  int64_t off = 0;
  int k = 0;
  for (int l = l_start; l <= l_end; ++l, ++k) {
    const flod_level &lv = levels[l - 1];
    DevLevel &L = p.lv[k];
    L.means = lv.means; L.log_scales = lv.log_scales; L.quats = lv.quats;
    L.logits = lv.opacity_logits; L.sh = lv.sh;
    L.offset = off; L.n = lv.n; L.s_min = lv.s_min;
    // eq. 6 with d_proj^(l_end) = 0 and d_proj^(l_start - 1) = infinity
    const float hi = (l == l_start) ? INFINITY : d_proj[l - 2];
    const float lo = (l == l_end) ? 0.0f : d_proj[l - 1];
    L.lo2 = sq32(lo);
    L.hi2 = sq32(hi);
    off += lv.n;
  }
  p.n_levels = k;
  p.n_total = off;
  if (off > 0xFFFFFFF0ll) return FLOD_ERR_INVALID_ARG;
  // the kernel's level index is relative to l_start
  int64_t *nsel = n_selected;
  if (nsel) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(nsel), 0u, 2 * (int64_t)n_levels, (hipStream_t)stream);
    if (e != hipSuccess) return FLOD_ERR_DEVICE;
    nsel += (l_start - 1);
  }
  st = render_common(ctx, p, nsel, bg, out, (hipStream_t)stream);
  if (st == FLOD_OK) ctx->saved.is_level = false;
  return st;
}

flod_status flod_render_merged(flod_ctx *ctx, const flod_level *levels, int n_levels, int sh_degree,
                               const flod_camera *cam, const float bg[3], flod_frame *out, void *stream) {
  if (!ctx || !levels || !bg || !frame_ok(out) || sh_degree < 0 || sh_degree > 3) return FLOD_ERR_INVALID_ARG;
  if (n_levels < 1 || n_levels > FLOD_MAX_LEVELS) return FLOD_ERR_INVALID_ARG;
  flod_status st = check_camera(cam);
  if (st != FLOD_OK) return st;
  for (int l = 0; l < n_levels; ++l)
    if ((st = check_level(&levels[l])) != FLOD_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  PreParams p = base_params(dev_camera(cam), sh_degree);
  p.select = 0;
  int64_t off = 0;
  for (int l = 0; l < n_levels; ++l) {
    const flod_level &lv = levels[l];
    DevLevel &L = p.lv[l];
    L.means = lv.means; L.log_scales = lv.log_scales; L.quats = lv.quats;
    L.logits = lv.opacity_logits; L.sh = lv.sh;
    L.offset = off; L.n = lv.n; L.s_min = lv.s_min;
    L.lo2 = 0.0f; L.hi2 = INFINITY;
    off += lv.n;
  }
  p.n_levels = n_levels;
  p.n_total = off;
  if (off > 0xFFFFFFF0ll) return FLOD_ERR_INVALID_ARG;
  st = render_common(ctx, p, nullptr, bg, out, (hipStream_t)stream);
  if (st == FLOD_OK) ctx->saved.is_level = false;
  return st;
}

}  // extern "C"

namespace {

bool level_arrays_ok(const flod_level &o) {
  if (o.n < 0) return false;
  return o.n == 0 || (o.means && o.log_scales && o.quats && o.opacity_logits && o.sh && aligned(o.quats, 16) &&
                      aligned(o.sh, 16) && aligned(o.means, 4) && aligned(o.log_scales, 4) &&
                      aligned(o.opacity_logits, 4));
}

// Count the kept Gaussians of one level (per-workgroup counts, scan, a 4-byte read back)
// and, when `out` is given, copy them in index order. count(block_cnt) and copy(prefix, out)
// enqueue the two passes.
template <class CountFn, class CopyFn>
flod_status compact_pass(flod_ctx *ctx, int64_t n, hipStream_t s, CountFn count, CopyFn copy, flod_level *out,
                         float s_min, int64_t *kept_out) {
  *kept_out = 0;
  if (n == 0) {
    if (out) {
      out->n = 0;
      out->s_min = s_min;
    }
    return FLOD_OK;
  }
  const int nb = (int)((n + kBlock - 1) / kBlock);
  size_t extra = 0;
  if (ensure(ctx, B_BLOCKVIS, 4 * (size_t)nb, s, &extra) != FLOD_OK ||
      ensure(ctx, B_PREFIX, 8 * (size_t)nb, s, &extra) != FLOD_OK ||
      ensure(ctx, B_COUNTERS, 8 * (size_t)kCntSlots, s, &extra) != FLOD_OK) {
    ctx->required = ws_bytes(ctx) + extra;
    return FLOD_ERR_WORKSPACE;
  }
  uint32_t *counters = P<uint32_t>(ctx, B_COUNTERS);
  if (count(P<uint32_t>(ctx, B_BLOCKVIS)) != hipSuccess ||
      launch_scan_blocks(P<uint32_t>(ctx, B_BLOCKVIS), nullptr, kBlock, P<unsigned long long>(ctx, B_PREFIX),
                         counters + kCntVisible, nullptr, nb, s) != hipSuccess ||
      hipMemcpyAsync(ctx->host_counters, counters, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FLOD_ERR_DEVICE;
  const int64_t kept = reinterpret_cast<const uint32_t *>(ctx->host_counters)[kCntVisible];
  *kept_out = kept;
  if (!out) return FLOD_OK;
  if (out->n < kept) {
    ctx->required = (size_t)kept * kGaussianBytes;
    return FLOD_ERR_WORKSPACE;
  }
  if (copy(P<unsigned long long>(ctx, B_PREFIX), *out) != hipSuccess) return FLOD_ERR_DEVICE;
  out->n = kept;
  out->s_min = s_min;
  return FLOD_OK;
}

flod_status begin_level_op(flod_ctx *ctx, hipStream_t s) {
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  if (use_stream(ctx, s) != hipSuccess) return FLOD_ERR_DEVICE;
  ctx->required = 0;
  ctx->saved.valid = false;
  return FLOD_OK;
}

}  // namespace

extern "C" {

flod_status flod_select_compact(flod_ctx *ctx, const flod_level *levels, int n_levels, int l_start, int l_end,
                                const float *d_proj, const float centre[3], flod_level *out, int64_t *n_out,
                                void *stream) {
  if (!ctx || !levels || !d_proj || !centre || !n_out) return FLOD_ERR_INVALID_ARG;
  if (n_levels < 1 || n_levels > FLOD_MAX_LEVELS || l_start < 1 || l_end < l_start || l_end > n_levels)
    return FLOD_ERR_INVALID_ARG;
  flod_status st;
  for (int l = l_start; l <= l_end; ++l)
    if ((st = check_level(&levels[l - 1])) != FLOD_OK) return st;
  for (int l = 0; l < n_levels; ++l)
    if (!(d_proj[l] >= 0.0f)) return FLOD_ERR_INVALID_ARG;
  if (!isfinite(centre[0]) || !isfinite(centre[1]) || !isfinite(centre[2])) return FLOD_ERR_INVALID_ARG;
  if (out)
    for (int l = l_start; l <= l_end; ++l)
      if (!level_arrays_ok(out[l - 1])) return FLOD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if ((st = begin_level_op(ctx, s)) != FLOD_OK) return st;
  for (int l = 0; l < n_levels; ++l) n_out[l] = 0;
  for (int l = l_start; l <= l_end; ++l) {
    const flod_level &lv = levels[l - 1];
    // eq. 6 band of level l, with d_proj^(l_end) = 0 and d_proj^(l_start - 1) = infinity
    const float hi = (l == l_start) ? INFINITY : d_proj[l - 2];
    const float lo = (l == l_end) ? 0.0f : d_proj[l - 1];
    const float lo2 = sq32(lo), hi2 = sq32(hi);
    auto count = [&](uint32_t *bc) { return launch_select_count(lv.means, lv.n, centre, lo2, hi2, bc, s); };
    auto copy = [&](const unsigned long long *prefix, const flod_level &o) {
      return launch_select_copy(lv, centre, lo2, hi2, prefix, o, s);
    };
    if ((st = compact_pass(ctx, lv.n, s, count, copy, out ? &out[l - 1] : nullptr, lv.s_min, &n_out[l - 1])) !=
        FLOD_OK)
      return st;
  }
  if (out)
    for (int l = 1; l <= n_levels; ++l)
      if (l < l_start || l > l_end) out[l - 1].n = 0;
  return FLOD_OK;
}

flod_status flod_compact_level(flod_ctx *ctx, const flod_level *in, const uint8_t *keep, flod_level *out,
                               int64_t *n_out, void *stream) {
  if (!ctx || !in || !n_out || (in->n > 0 && !keep)) return FLOD_ERR_INVALID_ARG;
  flod_status st = check_level(in);
  if (st != FLOD_OK) return st;
  if (out) {
    if (!level_arrays_ok(*out)) return FLOD_ERR_INVALID_ARG;
    if (out->n > 0 && (out->means == in->means || out->log_scales == in->log_scales || out->quats == in->quats ||
                       out->opacity_logits == in->opacity_logits || out->sh == in->sh))
      return FLOD_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  if ((st = begin_level_op(ctx, s)) != FLOD_OK) return st;
  auto count = [&](uint32_t *bc) { return launch_mask_count(keep, in->n, bc, s); };
  auto copy = [&](const unsigned long long *prefix, const flod_level &o) {
    return launch_mask_copy(*in, keep, prefix, o, s);
  };
  return compact_pass(ctx, in->n, s, count, copy, out, in->s_min, n_out);
}

flod_status flod_overlap_prune(flod_ctx *ctx, const flod_level *level, float d_op, uint8_t *keep, double *d_avg,
                               int64_t *n_keep, void *stream) {
  if (!ctx || !level || !n_keep) return FLOD_ERR_INVALID_ARG;
  flod_status st = check_level(level);
  if (st != FLOD_OK) return st;
  const int64_t n = level->n;
  if (n > ((int64_t)1 << 30) || !(d_op >= 0.0f) || !isfinite(d_op)) return FLOD_ERR_INVALID_ARG;
  if (n > 0 && (!keep || (d_avg && !aligned(d_avg, 8)))) return FLOD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if ((st = begin_level_op(ctx, s)) != FLOD_OK) return st;
  *n_keep = 0;
  if (n == 0) return FLOD_OK;
  const int bits = prune_table_bits(n);
  const int64_t buckets = (int64_t)1 << bits;
  size_t extra = 0;
  auto need = [&](BufId id, size_t bytes) {
    if (ensure(ctx, id, bytes, s, &extra) != FLOD_OK) st = FLOD_ERR_WORKSPACE;
  };
  if (d_op > 0.0f) {
    need(B_DKEY0, 4 * (size_t)n);
    need(B_DKEY1, 4 * (size_t)n);
    need(B_DVAL0, 4 * (size_t)n);
    need(B_DVAL1, 4 * (size_t)n);
    need(B_XYAB, 16 * (size_t)n);
    need(B_RANGES, 8 * (size_t)buckets);
    need(B_HIST, radix_hist_bytes(n));
    need(B_SCAN, radix_hist_bytes(n));
    need(B_TOT, 4 * (size_t)kRadix);
  }
  need(B_COUNTERS, 8 * (size_t)kCntSlots);
  if (st != FLOD_OK) {
    ctx->required = ws_bytes(ctx) + extra;
    return st;
  }
  uint32_t *counters = P<uint32_t>(ctx, B_COUNTERS);
  const float4 *pts = P<float4>(ctx, B_XYAB);
  const uint2 *ranges = P<uint2>(ctx, B_RANGES);
  if (d_op > 0.0f) {
    uint32_t *dk[2] = {P<uint32_t>(ctx, B_DKEY0), P<uint32_t>(ctx, B_DKEY1)};
    uint32_t *dv[2] = {P<uint32_t>(ctx, B_DVAL0), P<uint32_t>(ctx, B_DVAL1)};
    int res = 0;
    if (launch_fill_u32(counters + kCntVisible, (uint32_t)n, 1, s) != hipSuccess ||
        launch_fill_u32(counters + kCntTotal64, 0u, 2, s) != hipSuccess ||
        launch_prune_keys(level->means, n, d_op, dk[0], dv[0], s) != hipSuccess ||
        launch_radix_sort(dk, dv, counters + kCntVisible, n, bits, P<uint32_t>(ctx, B_HIST),
                          P<uint32_t>(ctx, B_SCAN), P<uint32_t>(ctx, B_TOT), &res, s) != hipSuccess ||
        launch_prune_gather(level->means, dv[res], n, P<float4>(ctx, B_XYAB), s) != hipSuccess ||
        launch_ranges(dk[res], counters + kCntVisible, n, (int)buckets, P<uint2>(ctx, B_RANGES), false, s) !=
            hipSuccess ||
        launch_prune_cost(pts, ranges, n, d_op, reinterpret_cast<unsigned long long *>(counters + kCntTotal64),
                          s) != hipSuccess ||
        hipMemcpyAsync(ctx->host_counters, counters, 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FLOD_ERR_DEVICE;
    if (ctx->host_counters[1] > kPruneMaxScan) return FLOD_ERR_UNSUPPORTED;
  }
  if (launch_prune_query(pts, ranges, n, d_op, keep, d_avg, s) != hipSuccess) return FLOD_ERR_DEVICE;
  auto count = [&](uint32_t *bc) { return launch_mask_count(keep, n, bc, s); };
  auto no_copy = [&](const unsigned long long *, const flod_level &) { return hipSuccess; };
  return compact_pass(ctx, n, s, count, no_copy, nullptr, level->s_min, n_keep);
}

flod_status flod_l1_ssim_forward(flod_ctx *ctx, const float *image, const float *target, int channels, int height,
                                 int width, float lambda, double *loss, float *dmaps, void *stream) {
  if (!ctx || !image || !target || !loss) return FLOD_ERR_INVALID_ARG;
  if (channels < 1 || height < 1 || width < 1 || height > 65536 || width > 65536 || channels > 64)
    return FLOD_ERR_INVALID_ARG;
  if (!(lambda >= 0.0f && lambda <= 1.0f) || !aligned(loss, 8)) return FLOD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  if (use_stream(ctx, s) != hipSuccess) return FLOD_ERR_DEVICE;
  ctx->required = 0;
  size_t extra = 0;
  if (ensure(ctx, B_SSIM, 16 * (size_t)ssim_blocks(channels, height, width), s, &extra) != FLOD_OK) {
    ctx->required = ws_bytes(ctx) + extra;
    return FLOD_ERR_WORKSPACE;
  }
  return dev(launch_ssim_forward(image, target, channels, height, width, lambda, loss, dmaps,
                                 P<double2>(ctx, B_SSIM), s));
}

flod_status flod_l1_ssim_forward_noalloc(flod_ctx *ctx, const float *image, const float *target, int channels,
                                         int height, int width, float lambda, double *loss, float *dmaps,
                                         void *stream) {
  if (!ctx || !image || !target || !loss) return FLOD_ERR_INVALID_ARG;
  if (channels < 1 || height < 1 || width < 1 || height > 65536 || width > 65536 || channels > 64)
    return FLOD_ERR_INVALID_ARG;
  if (!(lambda >= 0.0f && lambda <= 1.0f) || !aligned(loss, 8)) return FLOD_ERR_INVALID_ARG;
  if ((size_t)ssim_blocks(channels, height, width) * sizeof(double2) > kNoAllocScratchBytes)
    return FLOD_ERR_TOO_LARGE;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  double2 *partials = reinterpret_cast<double2 *>(scratch_on(ctx->device));
  if (!partials) return FLOD_ERR_DEVICE;
  // every workgroup writes its own partial and the reduction reads exactly those: nothing
  // left in the scratch by an earlier call is read, so nothing is cleared
  return dev(launch_ssim_forward(image, target, channels, height, width, lambda, loss, dmaps, partials,
                                 (hipStream_t)stream));
}

flod_status flod_l1_ssim_backward(flod_ctx *ctx, const float *image, const float *target, int channels, int height,
                                  int width, float lambda, const float *dmaps, const double *dloss, float *d_image,
                                  void *stream) {
  if (!ctx || !image || !target || !dmaps || !d_image) return FLOD_ERR_INVALID_ARG;
  if (channels < 1 || height < 1 || width < 1 || height > 65536 || width > 65536 || channels > 64)
    return FLOD_ERR_INVALID_ARG;
  if (!(lambda >= 0.0f && lambda <= 1.0f) || (dloss && !aligned(dloss, 8))) return FLOD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  if (use_stream(ctx, s) != hipSuccess) return FLOD_ERR_DEVICE;
  ctx->required = 0;
  return dev(launch_ssim_backward(image, target, channels, height, width, lambda, dmaps, dloss, d_image, s));
}

flod_status flod_l1_loss_forward(flod_ctx *ctx, const float *image, const float *target, int64_t count,
                                 double *loss, void *stream) {
  if (!ctx || !image || !target || !loss || count < 1 || !aligned(loss, 8)) return FLOD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  if (use_stream(ctx, s) != hipSuccess) return FLOD_ERR_DEVICE;
  ctx->required = 0;
  size_t extra = 0;
  if (ensure(ctx, B_SSIM, 16 * (size_t)l1_blocks(), s, &extra) != FLOD_OK) {
    ctx->required = ws_bytes(ctx) + extra;
    return FLOD_ERR_WORKSPACE;
  }
  return dev(launch_l1_forward(image, target, count, loss, P<double2>(ctx, B_SSIM), s));
}

flod_status flod_l1_loss_backward(flod_ctx *ctx, const float *image, const float *target, int64_t count,
                                  const double *dloss, float *d_image, void *stream) {
  if (!ctx || !image || !target || !d_image || count < 1 || (dloss && !aligned(dloss, 8)))
    return FLOD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  if (use_stream(ctx, s) != hipSuccess) return FLOD_ERR_DEVICE;
  ctx->required = 0;
  return dev(launch_l1_backward(image, target, count, dloss, d_image, s));
}

flod_status flod_adam_step(flod_ctx *ctx, const flod_level_state *params, const flod_grads *grads,
                           const flod_level_state *m, const flod_level_state *v, int64_t n,
                           const flod_adam_params *hp, void *stream) {
  if (!ctx || !params || !grads || !m || !v || !hp || n < 0) return FLOD_ERR_INVALID_ARG;
  if (hp->step < 1 || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) || !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) ||
      !(hp->eps >= 0.0f) || !isfinite(hp->eps))
    return FLOD_ERR_INVALID_ARG;
  const float lrs[6] = {hp->lr_means, hp->lr_log_scales, hp->lr_quats, hp->lr_opacity, hp->lr_sh_dc, hp->lr_sh_rest};
  for (float r : lrs)
    if (!isfinite(r)) return FLOD_ERR_INVALID_ARG;
  float *P5[5] = {params->means, params->log_scales, params->quats, params->opacity_logits, params->sh};
  const float *G5[5] = {grads->d_means, grads->d_log_scales, grads->d_quats, grads->d_opacity_logits, grads->d_sh};
  float *M5[5] = {m->means, m->log_scales, m->quats, m->opacity_logits, m->sh};
  float *V5[5] = {v->means, v->log_scales, v->quats, v->opacity_logits, v->sh};
  const int64_t width[5] = {3, 3, 4, 1, FLOD_SH_COEFFS * 3};
  if (n > 0)
    for (int k = 0; k < 5; ++k)
      if (!P5[k] || !G5[k] || !M5[k] || !V5[k] || !aligned(P5[k], 4) || !aligned(G5[k], 4) || !aligned(M5[k], 4) ||
          !aligned(V5[k], 4))
        return FLOD_ERR_INVALID_ARG;
  if (n > ((int64_t)1 << 40)) return FLOD_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  AdamArgs a;
  memset(&a, 0, sizeof(a));
  int64_t slot = 0;
  for (int k = 0; k < 5; ++k) {
    AdamSeg &S = a.seg[k];
    S.p = P5[k]; S.g = G5[k]; S.m = M5[k]; S.v = V5[k];
    S.len = n * width[k];
    S.first4 = slot;
    S.lr = lrs[k];
    S.vec = aligned(S.p, 16) && aligned(S.g, 16) && aligned(S.m, 16) && aligned(S.v, 16);
    slot += (S.len + 3) / 4;
  }
  a.total4 = slot;
  a.lr_sh_rest = hp->lr_sh_rest;
  a.b1 = hp->beta1;
  a.b2 = hp->beta2;
  a.omb1 = (float)(1.0 - (double)hp->beta1);
  a.omb2 = (float)(1.0 - (double)hp->beta2);
  a.inv_bc1 = (float)(1.0 / (1.0 - pow((double)hp->beta1, (double)hp->step)));
  a.inv_bc2 = (float)(1.0 / (1.0 - pow((double)hp->beta2, (double)hp->step)));
  a.eps = hp->eps;
  return dev(launch_adam(a, (hipStream_t)stream));
}

flod_status flod_level_transition(flod_ctx *ctx, const flod_level *in, float s_min_next, flod_level *out,
                                  void *stream) {
  if (!ctx || !in || !out) return FLOD_ERR_INVALID_ARG;
  flod_status st = check_level(in);
  if (st != FLOD_OK) return st;
  if (!(s_min_next >= 0.0f) || !(s_min_next <= in->s_min)) return FLOD_ERR_INVALID_ARG;
  if (!level_arrays_ok(*out) || out->n < in->n) return FLOD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if ((st = begin_level_op(ctx, s)) != FLOD_OK) return st;
  flod_level o = *out;
  o.n = in->n;
  if (launch_level_transition(*in, s_min_next, o, s) != hipSuccess) return FLOD_ERR_DEVICE;
  out->n = in->n;
  out->s_min = s_min_next;
  return FLOD_OK;
}

flod_status flod_render_backward(flod_ctx *ctx, const float *dL_dimage, flod_grads *grads, void *stream) {
  if (!ctx || !dL_dimage || !grads) return FLOD_ERR_INVALID_ARG;
  const Saved &sv = ctx->saved;
  if (!sv.valid || !sv.is_level || !sv.has_blended) return FLOD_ERR_UNSUPPORTED;
  const int64_t N = sv.level.n;
  if (N > 0 && (!grads->d_means || !grads->d_log_scales || !grads->d_quats || !grads->d_opacity_logits ||
                !grads->d_sh || !aligned(grads->d_quats, 16) || !aligned(grads->d_sh, 16)))
    return FLOD_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
  hipStream_t s = (hipStream_t)stream;
  if (use_stream(ctx, s) != hipSuccess) return FLOD_ERR_DEVICE;
  ctx->required = 0;
  timing_flush(ctx);
  StageTimer tm(ctx, s);
  if (N == 0) return FLOD_OK;
  size_t extra = 0;
  const int n_tiles = sv.cam.tiles_x * sv.cam.tiles_y;
  if (ensure(ctx, B_G2D, 9 * 4 * (size_t)N, s, &extra) != FLOD_OK ||
      ensure(ctx, B_TILE_ORDER, 4 * ((size_t)n_tiles + 2), s, &extra) != FLOD_OK) {
    ctx->required = ws_bytes(ctx) + extra;
    return FLOD_ERR_WORKSPACE;
  }
  float *g2d = P<float>(ctx, B_G2D);
  uint32_t *order = P<uint32_t>(ctx, B_TILE_ORDER);
  hipEvent_t ev_a, ev_b;
  tm.dispatch(FLOD_STAGE_BLEND_BWD, &ev_a, &ev_b);
  if (launch_blend_bwd(P<uint2>(ctx, B_RANGES), P<float4>(ctx, B_XYAB), P<float4>(ctx, B_COP),
                       P<float2>(ctx, B_BLUE), sv.cam, sv.bg, sv.final_T, sv.n_contrib, dL_dimage, g2d, 9 * N,
                       P<uint2>(ctx, B_BLENDED), P<uint32_t>(ctx, B_TILE_BLENDED), order, s, ev_a, ev_b) !=
          hipSuccess)
    return FLOD_ERR_DEVICE;
  tm.begin(FLOD_STAGE_PREPROCESS_BWD);
  PreParams p = base_params(sv.cam, sv.sh_degree);
  p.n_levels = 1;
  DevLevel &L = p.lv[0];
  L.means = sv.level.means; L.log_scales = sv.level.log_scales; L.quats = sv.level.quats;
  L.logits = sv.level.opacity_logits; L.sh = sv.level.sh;
  L.offset = 0; L.n = N; L.s_min = sv.level.s_min;
  p.n_total = N;
  if (launch_preprocess_bwd(p, P<uint32_t>(ctx, B_TILES), g2d, P<float4>(ctx, B_SHJAC), *grads, s) != hipSuccess)
    return FLOD_ERR_DEVICE;
  tm.end();
  ctx->saved.has_grad2d = true;
  ctx->saved.grad2d_moments = true;
  return FLOD_OK;
}

flod_status flod_ctx_stats(const flod_ctx *ctx, flod_stats *out) {
  if (!ctx || !out) return FLOD_ERR_INVALID_ARG;
  *out = ctx->stats;
  return FLOD_OK;
}

flod_status flod_ctx_view(const flod_ctx *ctx, flod_view *out) {
  if (!ctx || !out) return FLOD_ERR_INVALID_ARG;
  flod_ctx *c = const_cast<flod_ctx *>(ctx);
  const Saved &sv = ctx->saved;
  memset(out, 0, sizeof(*out));
  if (!sv.valid) return FLOD_ERR_UNSUPPORTED;
  out->tile_ids = sv.sorted_keys ? P<uint32_t>(c, B_TKEY1) : P<uint32_t>(c, B_TKEY0);
  out->values = sv.sorted_vals ? P<uint32_t>(c, B_TVAL1) : P<uint32_t>(c, B_TVAL0);
  out->ranges = P<uint32_t>(c, B_RANGES);
  out->depth_bits = P<uint32_t>(c, B_DEPTH);
  out->bin = P<float>(c, B_BIN);
  out->tiles_touched = P<uint32_t>(c, B_TILES);
  out->xy_conic = P<float>(c, B_XYAB);
  out->conic_c_opacity_rg = P<float>(c, B_COP);
  out->blue = P<float>(c, B_BLUE);
  if (sv.has_grad2d && sv.grad2d_moments) {
    // the first view after a backward turns its moment sums into the gradient, in place
    if (hipSetDevice(ctx->device) != hipSuccess ||
        launch_g2d_from_moments(sv.level.n, P<uint32_t>(c, B_TILES), P<float4>(c, B_XYAB), P<float4>(c, B_COP),
                                P<float>(c, B_G2D), c->last_stream) != hipSuccess ||
        hipStreamSynchronize(c->last_stream) != hipSuccess)
      return FLOD_ERR_DEVICE;
    c->saved.grad2d_moments = false;
  }
  out->grad2d = sv.has_grad2d ? P<float>(c, B_G2D) : nullptr;
  out->blended = P<uint32_t>(c, B_BLENDED);
  out->tile_blended = P<uint32_t>(c, B_TILE_BLENDED);
  return FLOD_OK;
}

flod_status flod_ctx_keep_backward_state(flod_ctx *ctx, int keep) {
  if (!ctx) return FLOD_ERR_INVALID_ARG;
  ctx->keep_backward = keep != 0;
  return FLOD_OK;
}

flod_status flod_ctx_set_timing(flod_ctx *ctx, int enable) {
  return flod_ctx_set_timing_stages(ctx, enable ? ((1u << FLOD_NUM_STAGES) - 1u) : 0u);
}

flod_status flod_ctx_set_timing_stages(flod_ctx *ctx, unsigned int stage_mask) {
  if (!ctx) return FLOD_ERR_INVALID_ARG;
  const int enable = stage_mask != 0u;
  if (enable && !ctx->events_made) {
    if (hipSetDevice(ctx->device) != hipSuccess) return FLOD_ERR_DEVICE;
    for (int k = 0; k < FLOD_NUM_STAGES; ++k) {
      if (hipEventCreate(&ctx->ev[k][0]) != hipSuccess || hipEventCreate(&ctx->ev[k][1]) != hipSuccess)
        return FLOD_ERR_DEVICE;
    }
    ctx->events_made = true;
  }
  ctx->timing = enable != 0;
  ctx->timing_mask = stage_mask;
  return FLOD_OK;
}

flod_status flod_ctx_stage_times(flod_ctx *ctx, double *ms, int64_t *calls, int reset) {
  if (!ctx) return FLOD_ERR_INVALID_ARG;
  timing_flush(ctx);
  for (int k = 0; k < FLOD_NUM_STAGES; ++k) {
    if (ms) ms[k] = ctx->ms[k];
    if (calls) calls[k] = ctx->calls[k];
    if (reset) { ctx->ms[k] = 0.0; ctx->calls[k] = 0; }
  }
  return FLOD_OK;
}

const char *flod_stage_name(int stage) {
  static const char *names[FLOD_NUM_STAGES] = {"preprocess", "depth_sort", "offsets", "emit",
                                               "tile_sort", "ranges", "blend", "blend_bwd", "preprocess_bwd"};
  return (stage >= 0 && stage < FLOD_NUM_STAGES) ? names[stage] : "unknown";
}

float flod_smin(int l, int l_max, float lambda, float rho) {
  if (l >= l_max) return 0.0f;
  return (float)((double)lambda * pow((double)rho, (double)(1 - l)));
}

float flod_dproj(float s_min, float f, float gamma) {
  return (float)((double)s_min / (double)gamma * (double)f);
}

const char *flod_status_str(flod_status status) {
  switch (status) {
    case FLOD_OK: return "ok";
    case FLOD_ERR_INVALID_ARG: return "invalid argument";
    case FLOD_ERR_WORKSPACE: return "workspace allocation refused";
    case FLOD_ERR_TOO_LARGE: return "input exceeds the fixed scratch of the allocation-free entry point";
    case FLOD_ERR_OVERFLOW: return "instance count overflow (more than 2^32-1 tile instances)";
    case FLOD_ERR_DEVICE: return "HIP device error";
    case FLOD_ERR_UNSUPPORTED: return "unsupported operation";
  }
  return "unknown status";
}

flod_status flod_copy_to_host(void *dst_host, const void *src_device, size_t bytes) {
  if (bytes == 0) return FLOD_OK;
  if (!dst_host || !src_device) return FLOD_ERR_INVALID_ARG;
  return dev(hipMemcpy(dst_host, src_device, bytes, hipMemcpyDeviceToHost));
}

}  // extern "C"

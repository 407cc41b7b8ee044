/*
 * flod.h - C ABI of the MI355X (gfx950) FLoD-3DGS rasterizer.
 *
 * What it computes (FLoD, "Integrating Flexible Level of Detail into 3D Gaussian Splatting"):
 *   - a level G^(l) of 3D Gaussians with mean mu, opacity o = sigmoid(logit), covariance
 *     Sigma = R S S^T R^T (Preliminary section, eq. 1) where R comes from a quaternion and
 *     S = diag(s) with s = exp(s_opt) + s_min^(l) (section 3D Scale Constraint, eq. 4);
 *   - their projection to the image, the per-pixel opacity of eq. 2 and front-to-back alpha
 *     blending in depth order (Preliminary section);
 *   - single-level rendering (section Single-level Rendering) and selective rendering over a
 *     level range [l_start, l_end] with distance bands d_proj (section Selective Rendering,
 *     eq. 6 and eq. 7);
 *   - the gradient of a loss through the rasterizer with respect to every Gaussian attribute
 *     (the rasterize-and-backpropagate step of the training algorithm, Algorithm 1).
 * The projection, tiling and compositing constants follow the 3DGS framework that the paper
 * builds on; they are listed under "Conventions" below.
 *
 * Memory: every array pointer is a DEVICE pointer to contiguous row-major data on the
 * context's device, owned by the caller, unless the comment says "host". Inputs must stay
 * valid and unmodified until the enqueued work has run; for render_level they must also
 * stay valid until the matching render_backward has run.
 *
 * Streams: `stream` is a hipStream_t (NULL = the legacy default stream). All work is
 * enqueued on it. A render enqueues the whole frame before it waits for anything: the
 * emission, tile sort and blend are sized for the instances the context's buffers hold and
 * read the instance count K on the device, doing nothing when K exceeds that capacity. The
 * host then waits for the counts, which the kernel that computes them writes to coherent
 * pinned host memory tagged with the render's sequence number (or a stream-ordered copy,
 * where coherent pinned memory is not available); they are there once the binning offsets
 * are known, while the rest of the frame is still queued (FLOD_COUNT_COPY=1 in the
 * environment when a context is created selects the copy). It then fills the
 * statistics and, when K exceeded the capacity, grows the buffers and enqueues the frame's
 * tail again. A context's first render, with no buffers yet, waits for K before the tail.
 * A context may be used on different streams from one call to the next: a call on a stream
 * other than the one the context last used first makes its stream wait (an event, no host
 * wait) for the work already enqueued on the previous one, so no buffer is reused, grown or
 * released under an earlier call's kernels.
 *
 * Errors: no function throws or aborts. Arguments are validated before any launch; on
 * FLOD_ERR_INVALID_ARG the outputs are untouched. flod_status_str() describes a code.
 *
 * Threads: a context is used by one host thread at a time; distinct contexts are fully
 * independent and may run concurrently on different streams.
 */
#ifndef FLOD_H
#define FLOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FLOD_OK = 0,
  FLOD_ERR_INVALID_ARG = -1,  /* null pointer, bad size, bad level range, sh_degree outside 0..3 */
  FLOD_ERR_WORKSPACE = -2,    /* the allocator callback refused; see flod_ctx_required_bytes */
  FLOD_ERR_OVERFLOW = -3,     /* more than 2^32 - 1 tile instances */
  FLOD_ERR_DEVICE = -4,       /* a HIP runtime call failed */
  FLOD_ERR_UNSUPPORTED = -5,  /* e.g. backward after a selective render */
  FLOD_ERR_TOO_LARGE = -6     /* input beyond an allocation-free entry point's fixed scratch */
} flod_status;

#define FLOD_MAX_LEVELS 8
#define FLOD_TILE 16
#define FLOD_SH_COEFFS 16

/* One level G^(l) of the multi-level stack (section Single-level Rendering). n may be 0. */
typedef struct {
  const float *means;           /* [n,3]    mu                                           */
  const float *log_scales;      /* [n,3]    s_opt of eq. 4                               */
  const float *quats;           /* [n,4]    (w,x,y,z); any norm > 0, zero norm = culled  */
  const float *opacity_logits;  /* [n]      o = 1 / (1 + exp(-logit))                    */
  const float *sh;              /* [n,16,3] SH coefficients, index l*l+l+m, channel last;
                                   must be 16-byte aligned                               */
  int64_t n;
  float s_min;                  /* s_min^(l) >= 0 of eq. 3 / eq. 4                       */
} flod_level;

/* Pinhole camera, OpenCV axes (x right, y down, z forward): x_cam = R x_world + t.
   eq. 7 uses f := fx. */
typedef struct {
  float R[9];        /* row-major world->camera rotation */
  float t[3];
  float campos[3];   /* eye position in world coordinates (view direction of SH colour) */
  float fx, fy, cx, cy;
  int32_t width, height;
} flod_camera;

/* Outputs of a forward render (all device, caller-allocated). */
typedef struct {
  float *image;        /* [3,H,W] planar RGB: composite + final_T * background, no clamp */
  float *final_T;      /* [H,W]   transmittance left after the last blended Gaussian     */
  int32_t *n_contrib;  /* [H,W]   tile-list position (1-based) of the last blended entry  */
  int32_t *n_blended;  /* [H,W]   number of Gaussians blended into the pixel; may be NULL */
} flod_frame;

/* Gradients of the loss with respect to the level's inputs (device, caller-allocated,
   same shapes as flod_level; every entry is overwritten). */
typedef struct {
  float *d_means;           /* [n,3]    */
  float *d_log_scales;      /* [n,3]    */
  float *d_quats;           /* [n,4]    16-byte aligned */
  float *d_opacity_logits;  /* [n]      */
  float *d_sh;              /* [n,16,3] 16-byte aligned */
} flod_grads;

/* Workspace allocator. alloc returns a device pointer (256-byte aligned) or NULL to refuse;
   release frees a pointer alloc returned. `stream` is the stream the memory is used on.
   Passing NULL callbacks selects hipMallocAsync / hipFreeAsync on that stream. */
typedef void *(*flod_alloc_fn)(void *user, size_t bytes, void *stream);
typedef void (*flod_free_fn)(void *user, void *ptr, size_t bytes, void *stream);

typedef struct flod_ctx flod_ctx;   /* workspace plus the state kept for the backward pass */

/* Create a context bound to HIP device `device`. Returns FLOD_ERR_DEVICE if the device is
   not usable. *ctx is set only on success. */
flod_status flod_ctx_create(flod_ctx **ctx, int device, flod_alloc_fn alloc, flod_free_fn release,
                            void *user);
/* Release the workspace (stream-ordered on the last stream used) and the context. */
void flod_ctx_destroy(flod_ctx *ctx);
/* Bytes the context currently holds. */
size_t flod_ctx_workspace_bytes(const flod_ctx *ctx);
/* After FLOD_ERR_WORKSPACE: the total bytes the failed call needed (else 0). */
size_t flod_ctx_required_bytes(const flod_ctx *ctx);
/* Free all workspace buffers now (stream-ordered); the saved backward state is dropped. */
flod_status flod_ctx_trim(flod_ctx *ctx, void *stream);

/* Render one level (section Single-level Rendering; eq. 1, eq. 2, eq. 4).
   bg: host float[3] background colour. sh_degree in 0..3 (first (d+1)^2 coefficients).
   The state needed by flod_render_backward is kept in ctx until the next render. */
flod_status flod_render_level(flod_ctx *ctx, const flod_level *level, int sh_degree,
                              const flod_camera *cam, const float bg[3], flod_frame *out,
                              void *stream);

/* Selective rendering (section Selective Rendering, eq. 6): from the levels
   l_start..l_end (1-based, 1 <= l_start <= l_end <= n_levels <= FLOD_MAX_LEVELS), keep a
   Gaussian of level l iff d_proj^(l-1) > |mu - centre| >= d_proj^(l), with
   d_proj^(l_end) = 0 and d_proj^(l_start-1) = infinity; the kept Gaussians of all levels
   form one set rendered in one depth order (global index = level offset + local index,
   levels concatenated in ascending order). Distances are compared squared in FP32.
   d_proj: host float[n_levels], d_proj[l-1] = d_proj^(l) (eq. 7 or explicit bands).
   centre: host float[3]; the eye for per-view selection, a fixed point (e.g. the mean
   training-camera position) for a predetermined set.
   n_selected: device int64[n_levels] (may be NULL): per-level count of kept Gaussians. */
flod_status flod_render_selective(flod_ctx *ctx, const flod_level *levels, int n_levels,
                                  int l_start, int l_end, const float *d_proj,
                                  const float centre[3], int sh_degree, const flod_camera *cam,
                                  const float bg[3], flod_frame *out, int64_t *n_selected,
                                  void *stream);

/* Render several levels as one set, every Gaussian of every level included (each level
   with its own s_min), in one depth order; candidate index = position in the concatenation.
   This renders a predetermined selection set made by flod_select_compact. Backward after
   it returns FLOD_ERR_UNSUPPORTED. */
flod_status flod_render_merged(flod_ctx *ctx, const flod_level *levels, int n_levels, int sh_degree,
                               const flod_camera *cam, const float bg[3], flod_frame *out, void *stream);

/* Predetermined selection set (section Selective Rendering, predetermined Gaussian set):
   evaluate the eq. 6 bands of flod_render_selective once around `centre` (host float[3],
   e.g. the mean training-camera position) and compact each level's kept Gaussians, in
   index order. n_out: host int64[n_levels], receives the kept count per level (0 outside
   [l_start, l_end]). out: NULL to count only; else host array of n_levels flod_level whose
   device arrays receive the kept Gaussians of level l in out[l-1] (on input out[l-1].n is
   the arrays' capacity in Gaussians, on output the kept count; s_min is copied). Returns
   FLOD_ERR_WORKSPACE, with flod_ctx_required_bytes() = the bytes of level arrays that the
   level needs (236 per kept Gaussian), when a level's capacity is too small. One host synchronisation per level (the count).
   flod_render_merged(out[l_start-1 .. l_end-1]) then renders the same image as
   flod_render_selective(levels, l_start, l_end, d_proj, centre). */
flod_status flod_select_compact(flod_ctx *ctx, const flod_level *levels, int n_levels, int l_start, int l_end,
                                const float *d_proj, const float centre[3], flod_level *out, int64_t *n_out,
                                void *stream);

/* Overlap pruning (section Overlap Pruning): Gaussian i of `level` is marked for removal
   when the mean of its distances to its three nearest other Gaussians of the level is below
   d_op (the paper uses d_op = s_min^(l) / 2 while training level l; d_op = 0 removes none).
   Distances are FP64 Euclidean distances between the FP32 means; the three are summed in
   ascending order and divided by 3; all Gaussians are evaluated on the same input set (no
   removal changes another's neighbours). A level of fewer than four Gaussians keeps all.
   keep: device uint8[n], 1 = keep, 0 = remove. d_avg: device double[n] or NULL; receives
   d_avg exactly when the three nearest lie within 3 d_op (1 + 1e-9), +inf otherwise (such a
   Gaussian is kept). n_keep: host, the number kept. Workspace about 44 B per Gaussian plus
   8 B per hash bucket (2^ceil(log2 n) buckets). One host synchronisation (the count) and
   one check of the neighbour-search size: when the means are so dense relative to d_op
   that the scan would exceed 2^36 distance evaluations, returns FLOD_ERR_UNSUPPORTED
   without writing keep. n <= 2^30. */
flod_status flod_overlap_prune(flod_ctx *ctx, const flod_level *level, float d_op, uint8_t *keep,
                               double *d_avg, int64_t *n_keep, void *stream);

/* Compact a level by a keep mask (device uint8[n], nonzero = keep), in index order, into
   `out` (host struct of device arrays; on input out->n = capacity in Gaussians, on output
   the kept count; s_min is copied). out = NULL counts only. *n_out = kept count. Returns
   FLOD_ERR_WORKSPACE, with flod_ctx_required_bytes() = 236 B per kept Gaussian, when the
   capacity is too small. Output arrays must not overlap the input's. */
flod_status flod_compact_level(flod_ctx *ctx, const flod_level *in, const uint8_t *keep, flod_level *out,
                               int64_t *n_out, void *stream);

/* Training loss (section Implementation: L1 and SSIM, as in the backbone model):
   loss = (1 - lambda) mean|x - y| + lambda (1 - SSIM(x, y)), SSIM with an 11 x 11 Gaussian
   window (sigma 1.5, normalised), zeros outside the image, C1 = 0.01^2, C2 = 0.03^2, averaged
   over channels and pixels. image, target: device float[channels, height, width]
   (contiguous). loss: device double[1] (written; no host synchronisation). dmaps: device
   float[3, channels, height, width] or NULL; when given, receives the per-pixel derivatives
   of SSIM with respect to the windowed mean, second moment and cross moment of the image,
   which flod_l1_ssim_backward consumes. Moments and sums in FP64; the loss is reduced in a
   fixed order (deterministic). 0 <= lambda <= 1; 1 <= channels <= 64, sizes <= 65536. */
flod_status flod_l1_ssim_forward(flod_ctx *ctx, const float *image, const float *target, int channels, int height,
                                 int width, float lambda, double *loss, float *dmaps, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
   serving or training loops, harnesses that forbid hipMalloc): flod_l1_ssim_forward with
   the same arguments, results and determinism, but its per-workgroup partial sums live in a
   fixed scratch array of 4 MiB inside the library (one per device, held until the process
   ends) instead of the context's workspace, so the call allocates nothing, not even on its
   first use. ctx only names the device; it must have been created on that device (creation
   looks up the scratch's device address). Limit: channels * ceil(height/16) * ceil(width/16)
   <= 262144 workgroups (3 channels: 87381 tiles of 16x16, so 3840x2160 with 32400 tiles
   fits and 7680x4320 with 129600 does not), else FLOD_ERR_TOO_LARGE before any launch. All calls on one device share the
   scratch: calls that overlap in time on one device (different streams, or different host
   threads) race and give wrong losses; calls ordered on one stream are safe. Nothing is
   read from an earlier call's scratch contents, so nothing needs clearing. */
flod_status flod_l1_ssim_forward_noalloc(flod_ctx *ctx, const float *image, const float *target, int channels,
                                         int height, int width, float lambda, double *loss, float *dmaps,
                                         void *stream);

/* Gradient of the loss above with respect to image, times *dloss (device double[1], NULL
   for 1): d_image, device float[channels, height, width]. dmaps from flod_l1_ssim_forward on
   the same image, target and lambda. d|t|/dt is taken as 0 at t = 0. */
flod_status flod_l1_ssim_backward(flod_ctx *ctx, const float *image, const float *target, int channels, int height,
                                  int width, float lambda, const float *dmaps, const double *dloss, float *d_image,
                                  void *stream);

/* Plain L1 image loss, mean |x - y| over `count` elements (image, target: device float[count]);
   loss: device double[1], summed in FP64 in a fixed order (deterministic), no host
   synchronisation. */
flod_status flod_l1_loss_forward(flod_ctx *ctx, const float *image, const float *target, int64_t count,
                                 double *loss, void *stream);

/* d_image = sign(x - y) / count times *dloss (device double[1], NULL for 1); 0 where x = y. */
flod_status flod_l1_loss_backward(flod_ctx *ctx, const float *image, const float *target, int64_t count,
                                  const double *dloss, float *d_image, void *stream);

/* Arrays with a level's shapes (means [n,3], log_scales [n,3], quats [n,4], opacity_logits
   [n], sh [n,16,3]; device, writable): a level's trainable parameters or an optimiser's
   moment estimates. */
typedef struct {
  float *means;
  float *log_scales;
  float *quats;
  float *opacity_logits;
  float *sh;
} flod_level_state;

/* Adam hyper-parameters for one step over a level: a learning rate per attribute group (SH:
   the degree-0 row, i.e. the first 3 floats of each Gaussian's 48, and the other 15 rows),
   the moment decay rates and eps, and the 1-based step count t of the bias corrections. */
typedef struct {
  float lr_means, lr_log_scales, lr_quats, lr_opacity, lr_sh_dc, lr_sh_rest;
  float beta1, beta2, eps;
  int64_t step;
} flod_adam_params;

/* One Adam step over every attribute of an n-Gaussian level, in place (the optimiser of the
   per-level training loop, section Training Method, Algorithm 1; Kingma and Ba's update):
     m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
     p <- p - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
   FP32 arithmetic; the bias corrections are formed in FP64 and rounded once. params, m, v:
   writable device arrays (m = v = 0 before step 1); grads as flod_render_backward writes
   them. No array may overlap another. One launch, no host synchronisation.
   FLOD_ERR_INVALID_ARG for a NULL pointer with n > 0, n < 0, step < 1, a beta outside
   [0, 1), eps < 0 or a non-finite rate. */
flod_status flod_adam_step(flod_ctx *ctx, const flod_level_state *params, const flod_grads *grads,
                           const flod_level_state *m, const flod_level_state *v, int64_t n,
                           const flod_adam_params *hp, void *stream);

/* Level transition (section Training Method, eq. 5): initialise level l+1 from the trained
   level l = *in: every attribute copied, and s_opt' = log(s^(l) - s_min_next) with
   s^(l) = exp(s_opt) + in->s_min formed as the renderer forms it (exp in FP64 rounded once
   to FP32, the sum and the logarithm in FP64, the result rounded to FP32), so that the
   renderer's scale at level l+1 equals s^(l) up to that rounding. out: host struct of
   device arrays of capacity out->n >= in->n; on return out->n = in->n and
   out->s_min = s_min_next. Each output array either is the input's own (in place; not
   copied) or does not overlap it. Requires 0 <= s_min_next <= in->s_min (eq. 3 floors
   decrease with the level). */
flod_status flod_level_transition(flod_ctx *ctx, const flod_level *in, float s_min_next, flod_level *out,
                                  void *stream);

/* Backward of the last flod_render_level on ctx: given dL/dimage [3,H,W] (device), write
   dL/d(inputs) into grads. Per-pixel transmittance is recovered from the saved final_T
   and n_contrib (no per-pixel contributor lists are stored): the forward's output buffers,
   which must still hold its values (the walk of each pixel is clamped to its tile's list, so
   changed n_contrib values give wrong gradients but no access outside the context's
   buffers). Besides them the backward reads the state the forward left in ctx: the tile
   ranges of the sorted list, per tile the list of the entries blended somewhere in the tile,
   the per-tile counts of those entries (flod_view: blended, tile_blended), and per visible
   Gaussian the Jacobian of its SH colour in the unit view direction with its colours before
   the clamp (48 bytes; the backward reads no SH coefficients). Returns
   FLOD_ERR_UNSUPPORTED after a selective render, after a render that kept no backward state
   (flod_ctx_keep_backward_state) or when no render preceded it; FLOD_ERR_INVALID_ARG for
   a NULL array or d_quats / d_sh not 16-byte aligned. FP32
   atomic accumulation: results are deterministic up to summation order. */
flod_status flod_render_backward(flod_ctx *ctx, const float *dL_dimage, flod_grads *grads,
                                 void *stream);

/* Counts of the last render (host). */
typedef struct {
  int64_t n_candidates;   /* Gaussians considered (all levels in range) */
  int64_t n_visible;      /* Gaussians that survived selection and culling */
  int64_t n_instances;    /* K: (tile, Gaussian) pairs */
  int32_t tiles_x, tiles_y;
  int32_t width, height;
} flod_stats;
flod_status flod_ctx_stats(const flod_ctx *ctx, flod_stats *out);

/* Device pointers to the last render's intermediate buffers, owned by ctx, valid until
   the next call on ctx. For inspection and tests. May run one kernel and wait for it (see
   grad2d); FLOD_ERR_DEVICE if that fails. */
typedef struct {
  const uint32_t *tile_ids;     /* [n_instances] tile id of each sorted instance          */
  const uint32_t *values;       /* [n_instances] Gaussian (global) index, sorted by
                                   (tile, depth bits, index)                              */
  const uint32_t *ranges;       /* [tiles,2] [start, end) of each tile in the list          */
  const uint32_t *depth_bits;   /* [n_candidates] bits of the view-space depth (FP32)       */
  const float *bin;             /* [n_candidates,8] binning record of rendered candidates:
                                   mu'x, mu'y, conic a, b, c, support bound Q_g, then (bits)
                                   the tile rectangle x0 | y0<<16 and x1 | y1<<16, inclusive */
  const uint32_t *tiles_touched;/* [n_candidates] 0 = not rendered                          */
  const float *xy_conic;        /* [n_candidates,4] mu'x, mu'y (FP32 rounding of the FP64
                                   projection), conic a, conic b                            */
  const float *conic_c_opacity_rg; /* [n_candidates,4] conic c, opacity, red, green         */
  const float *blue;            /* [n_candidates,2] blue, and (bits) the residual of mu' as
                                   two bf16: x in the low half, y in the high half          */
  const float *grad2d;          /* [n_candidates, 9] after flod_render_backward: per
                                   Gaussian dL/d(mu'x, mu'y, conic a, b, c, opacity, red,
                                   green, blue), with b the off-diagonal conic entry; NULL
                                   before a backward. The backward leaves moment sums there
                                   (the conic and opacity factors are applied per Gaussian
                                   in its last step); the first view after it applies them
                                   in place with the stored FP32 conic and opacity (one
                                   kernel on the stream of the last call, waited for)      */
  const uint32_t *blended;      /* [n_instances][2] per tile, the sorted instances the forward
                                   blended into some pixel of the tile, as (position in the
                                   tile's list, Gaussian) pairs in list order at the start of
                                   the tile's range; the rest of the range is unspecified
                                   (state the backward reads: it walks only these entries)  */
  const uint32_t *tile_blended; /* [tiles] count of such instances per tile (the backward's
                                   tile order)                                             */
} flod_view;
flod_status flod_ctx_view(const flod_ctx *ctx, flod_view *out);

/* Per-stage device timing with HIP events on the render stream (off by default). */
enum {
  FLOD_STAGE_PREPROCESS = 0,  /* selection (eq. 6), activation (eq. 4), projection, SH */
  FLOD_STAGE_DEPTH_SORT,      /* radix sort by depth; its first pass compacts the visible
                                 set, its last writes the tile counts in depth order   */
  FLOD_STAGE_OFFSETS,         /* scan of the tile counts, count readback             */
  FLOD_STAGE_EMIT,            /* (tile, Gaussian) instance emission                  */
  FLOD_STAGE_TILE_SORT,       /* stable radix sort of instances by tile              */
  FLOD_STAGE_RANGES,          /* per-tile [start, end)                               */
  FLOD_STAGE_BLEND,           /* front-to-back compositing (eq. 2)                   */
  FLOD_STAGE_BLEND_BWD,       /* reverse compositing kernel (its tile order excluded) */
  FLOD_STAGE_PREPROCESS_BWD,  /* chain rule to the 3D attributes                     */
  FLOD_NUM_STAGES
};
/* keep != 0 (the default): every render keeps the state flod_render_backward needs, per tile
   the list of the entries blended into some pixel (8 bytes per instance slot of workspace)
   and, for single-level renders, each Gaussian's colour Jacobian (48 bytes per Gaussian).
   keep == 0: renders keep none of it and take no workspace for it; a backward after such a
   render returns FLOD_ERR_UNSUPPORTED. For callers that only render (a server), which then
   need about a third less workspace per instance. Applies from the next render. */
flod_status flod_ctx_keep_backward_state(flod_ctx *ctx, int keep);
/* enable != 0 records every stage. */
flod_status flod_ctx_set_timing(flod_ctx *ctx, int enable);
/* Record only the stages whose bit (1 << FLOD_STAGE_...) is set; 0 turns timing off. Each
   recorded stage adds two event records to the stream, except FLOD_STAGE_BLEND_BWD, which is
   timed from its kernel's own dispatch (no packets between it and its neighbours). */
flod_status flod_ctx_set_timing_stages(flod_ctx *ctx, unsigned int stage_mask);
/* Accumulated milliseconds and call counts per stage since the last reset; synchronises
   on the last recorded events. ms and calls: host arrays of FLOD_NUM_STAGES. */
flod_status flod_ctx_stage_times(flod_ctx *ctx, double *ms, int64_t *calls, int reset);
const char *flod_stage_name(int stage);

/* eq. 3: s_min^(l) = lambda * rho^(1-l) for l < l_max, 0 for l = l_max. */
float flod_smin(int l, int l_max, float lambda, float rho);
/* eq. 7: d_proj = s_min / gamma * f. */
float flod_dproj(float s_min, float f, float gamma);
const char *flod_status_str(flod_status status);
/* Blocking device-to-host copy (for tests reading flod_view buffers). */
flod_status flod_copy_to_host(void *dst_host, const void *src_device, size_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* FLOD_H */

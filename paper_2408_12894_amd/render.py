"""Torch-facing API over libflod: device memory and streams come from PyTorch, every step of
the rasterizer runs in the HIP kernels behind the C ABI (include/flod.h).

    r = Renderer()
    image, final_T, n_contrib = r.render_level(level, cam, bg)
    image, ... = r.render_selective(levels, l_start, l_end, d_proj, centre, cam, bg)
    image = rasterize(means, log_scales, quats, opacity_logits, sh, cam, s_min, bg)   # autograd
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

SH_COEFFS = 16


@dataclass
class GaussianLevel:
    """One level G^(l) resident on the device (FP32, contiguous)."""
    means: torch.Tensor            # [n,3]
    log_scales: torch.Tensor       # [n,3]
    quats: torch.Tensor            # [n,4]
    opacity_logits: torch.Tensor   # [n]
    sh: torch.Tensor               # [n,16,3]
    s_min: float = 0.0

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_arrays(means, log_scales, quats, opacity_logits, sh, s_min=0.0, device="cuda"):
        def t(a):
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(device).contiguous()
        return GaussianLevel(t(means), t(log_scales), t(quats), t(opacity_logits), t(sh), float(s_min))

    @staticmethod
    def from_scene(scene, device="cuda"):
        return GaussianLevel.from_arrays(*scene.arrays(), s_min=scene.s_min, device=device)

    def nbytes(self) -> int:
        return sum(x.numel() * x.element_size() for x in
                   (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh))

    def c_struct(self) -> _lib.Level:
        for x in (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh):
            if x.dtype != torch.float32 or not x.is_contiguous() or not x.is_cuda:
                raise ValueError("level tensors must be contiguous float32 CUDA tensors")
        return _lib.Level(self.means.data_ptr(), self.log_scales.data_ptr(), self.quats.data_ptr(),
                          self.opacity_logits.data_ptr(), self.sh.data_ptr(), self.n, float(self.s_min))


def camera_struct(cam) -> _lib.Camera:
    c = _lib.Camera()
    c.R[:] = [float(v) for v in np.asarray(cam.R, np.float32).ravel()]
    c.t[:] = [float(v) for v in np.asarray(cam.t, np.float32).ravel()]
    c.campos[:] = [float(v) for v in np.asarray(cam.campos, np.float32).ravel()]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _floats(vals, n):
    arr = (C.c_float * n)()
    arr[:] = [float(v) for v in vals]
    return arr


def _stage_index(L, name: str) -> int:
    for k in range(32):
        n = L.flod_stage_name(k).decode()
        if n == "unknown":
            break
        if n == name:
            return k
    raise ValueError(f"unknown stage {name!r}")


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Renderer:
    """Owns one libflod context (workspace plus the state kept for the backward pass).

    A Renderer is used by one host thread at a time; use one Renderer per concurrent stream.
    alloc/release: optional workspace allocator callbacks (see flod_alloc_fn in flod.h).
    """

    def __init__(self, device: int | None = None, alloc=None, release=None):
        self.L = _lib.load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self._alloc_cb = _lib.ALLOC_FN(alloc) if alloc else _lib.ALLOC_FN(0)
        self._free_cb = _lib.FREE_FN(release) if release else _lib.FREE_FN(0)
        h = C.c_void_p()
        _lib.check(self.L.flod_ctx_create(C.byref(h), self.device, self._alloc_cb, self._free_cb, None),
                   "flod_ctx_create")
        self.ctx = h
        self.generation = 0
        self._last_level_forward = None

    def close(self):
        if getattr(self, "ctx", None):
            self.L.flod_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ forward
    def _frame(self, cam, device, n_blended=None, out=None):
        H, W = int(cam.height), int(cam.width)
        if out is not None:
            image, final_T, n_contrib = out
            if (tuple(image.shape) != (3, H, W) or image.dtype != torch.float32 or tuple(final_T.shape) != (H, W)
                    or final_T.dtype != torch.float32 or tuple(n_contrib.shape) != (H, W)
                    or n_contrib.dtype != torch.int32 or not all(t.is_contiguous() for t in out)):
                raise ValueError("out must be contiguous (image f32 [3,H,W], final_T f32 [H,W], n_contrib i32 [H,W])")
        else:
            image = torch.empty((3, H, W), dtype=torch.float32, device=device)
            final_T = torch.empty((H, W), dtype=torch.float32, device=device)
            n_contrib = torch.empty((H, W), dtype=torch.int32, device=device)
        fr = _lib.Frame(image.data_ptr(), final_T.data_ptr(), n_contrib.data_ptr(),
                        n_blended.data_ptr() if n_blended is not None else None)
        return image, final_T, n_contrib, fr

    def render_level(self, level: GaussianLevel, cam, bg=(0.0, 0.0, 0.0), sh_degree: int = 3, stream=None,
                     n_blended: torch.Tensor | None = None, out=None):
        """Single-level render. Returns (image [3,H,W], final_T [H,W], n_contrib [H,W]), written
        into `out` when given; the optional int32 [H,W] tensor n_blended receives the per-pixel
        blended count."""
        image, final_T, n_contrib, fr = self._frame(cam, level.means.device, n_blended, out)
        lv = level.c_struct()
        cs = camera_struct(cam)
        st = self.L.flod_render_level(self.ctx, C.byref(lv), int(sh_degree), C.byref(cs), _floats(bg, 3),
                                      C.byref(fr), C.c_void_p(_stream_ptr(stream)))
        _lib.check(st, "flod_render_level")
        self.generation += 1
        self._last_level_forward = self.generation
        # the library keeps pointers to final_T and n_contrib for the matching backward: hold
        # the tensors until the next render, so a caller that drops them cannot free them
        self._saved_frame = (final_T, n_contrib)
        return image, final_T, n_contrib

    def render_selective(self, levels, l_start: int, l_end: int, d_proj, centre, cam, bg=(0.0, 0.0, 0.0),
                         sh_degree: int = 3, stream=None, with_counts: bool = False, out=None):
        """Selective render over levels l_start..l_end (1-based) with distance bands d_proj
        (d_proj[l-1] = d_proj^(l)) around `centre`. Returns (image, final_T, n_contrib) and,
        with with_counts, the per-level selected counts (int64 tensor on the device)."""
        n_levels = len(levels)
        arr = (_lib.Level * n_levels)()
        for i, lv in enumerate(levels):
            arr[i] = lv.c_struct()
        dev = levels[l_start - 1].means.device
        image, final_T, n_contrib, fr = self._frame(cam, dev, out=out)
        counts = torch.empty(n_levels, dtype=torch.int64, device=dev) if with_counts else None
        cs = camera_struct(cam)
        st = self.L.flod_render_selective(self.ctx, arr, n_levels, int(l_start), int(l_end),
                                          _floats(d_proj, n_levels), _floats(centre, 3), int(sh_degree),
                                          C.byref(cs), _floats(bg, 3), C.byref(fr),
                                          C.c_void_p(counts.data_ptr() if counts is not None else 0),
                                          C.c_void_p(_stream_ptr(stream)))
        _lib.check(st, "flod_render_selective")
        self.generation += 1
        self._last_level_forward = None
        if with_counts:
            return image, final_T, n_contrib, counts
        return image, final_T, n_contrib

    def render_merged(self, levels, cam, bg=(0.0, 0.0, 0.0), sh_degree: int = 3, stream=None):
        """Render every Gaussian of the given levels (each with its own s_min) as one set, in
        one depth order: the way a stored predetermined selection set is drawn."""
        n_levels = len(levels)
        arr = (_lib.Level * n_levels)()
        for i, lv in enumerate(levels):
            arr[i] = lv.c_struct()
        image, final_T, n_contrib, fr = self._frame(cam, levels[0].means.device)
        cs = camera_struct(cam)
        st = self.L.flod_render_merged(self.ctx, arr, n_levels, int(sh_degree), C.byref(cs), _floats(bg, 3),
                                       C.byref(fr), C.c_void_p(_stream_ptr(stream)))
        _lib.check(st, "flod_render_merged")
        self.generation += 1
        self._last_level_forward = None
        return image, final_T, n_contrib

    def select_compact(self, levels, l_start: int, l_end: int, d_proj, centre, stream=None):
        """Predetermined selection set: the Gaussians each level keeps under the eq. 6 bands
        around a fixed `centre`, compacted into new device levels (index order preserved).
        Returns one GaussianLevel per level in [l_start, l_end] (possibly empty)."""
        n_levels = len(levels)
        arr = (_lib.Level * n_levels)()
        for i, lv in enumerate(levels):
            arr[i] = lv.c_struct()
        counts = (C.c_int64 * n_levels)()
        sp = C.c_void_p(_stream_ptr(stream))
        dp, ce = _floats(d_proj, n_levels), _floats(centre, 3)
        _lib.check(self.L.flod_select_compact(self.ctx, arr, n_levels, int(l_start), int(l_end), dp, ce, None,
                                              counts, sp), "flod_select_compact")
        out = (_lib.Level * n_levels)()
        kept = []
        for l in range(1, n_levels + 1):
            dev = levels[l - 1].means.device
            k = int(counts[l - 1])
            g = _empty_level(k, levels[l - 1].s_min, dev)
            kept.append(g)
            out[l - 1] = _lib.Level(g.means.data_ptr(), g.log_scales.data_ptr(), g.quats.data_ptr(),
                                    g.opacity_logits.data_ptr(), g.sh.data_ptr(), k, float(g.s_min))
        _lib.check(self.L.flod_select_compact(self.ctx, arr, n_levels, int(l_start), int(l_end), dp, ce, out,
                                              counts, sp), "flod_select_compact")
        return kept[l_start - 1: l_end]

    def overlap_prune(self, level: GaussianLevel, d_op: float, with_d_avg: bool = False, stream=None):
        """Overlap pruning decision for every Gaussian of `level` (removed iff the mean
        distance to its three nearest others is below d_op). Returns (keep uint8 tensor,
        kept count) and, with with_d_avg, the float64 d_avg tensor (+inf where the three
        nearest are not all within 3 d_op)."""
        dev = level.means.device
        keep = torch.empty((level.n,), dtype=torch.uint8, device=dev)
        davg = torch.empty((level.n,), dtype=torch.float64, device=dev) if with_d_avg else None
        cs = level.c_struct()
        n_keep = C.c_int64(0)
        _lib.check(self.L.flod_overlap_prune(self.ctx, C.byref(cs), float(d_op), C.c_void_p(keep.data_ptr()),
                                             C.c_void_p(davg.data_ptr() if davg is not None else 0),
                                             C.byref(n_keep), C.c_void_p(_stream_ptr(stream))), "flod_overlap_prune")
        self._last_level_forward = None
        return (keep, int(n_keep.value), davg) if with_d_avg else (keep, int(n_keep.value))

    def compact(self, level: GaussianLevel, keep: torch.Tensor, stream=None) -> GaussianLevel:
        """The Gaussians of `level` whose keep byte is nonzero, in index order, as a new level."""
        if keep.dtype != torch.uint8 or keep.numel() != level.n or not keep.is_contiguous():
            raise ValueError("keep must be a contiguous uint8 tensor with one entry per Gaussian")
        cs = level.c_struct()
        n_out = C.c_int64(0)
        sp = C.c_void_p(_stream_ptr(stream))
        _lib.check(self.L.flod_compact_level(self.ctx, C.byref(cs), C.c_void_p(keep.data_ptr()), None,
                                             C.byref(n_out), sp), "flod_compact_level")
        g = _empty_level(int(n_out.value), level.s_min, level.means.device)
        out = g.c_struct()
        _lib.check(self.L.flod_compact_level(self.ctx, C.byref(cs), C.c_void_p(keep.data_ptr()), C.byref(out),
                                             C.byref(n_out), sp), "flod_compact_level")
        self._last_level_forward = None
        return g

    def level_transition(self, level: GaussianLevel, s_min_next: float, in_place: bool = False,
                         stream=None) -> GaussianLevel:
        """eq. 5: the initial state of the next level (same Gaussians, scale parameters
        re-expressed so that the scale under s_min_next equals the scale under level.s_min)."""
        cs = level.c_struct()
        g = level if in_place else _empty_level(level.n, level.s_min, level.means.device)
        out = g.c_struct()
        _lib.check(self.L.flod_level_transition(self.ctx, C.byref(cs), float(s_min_next), C.byref(out),
                                                C.c_void_p(_stream_ptr(stream))), "flod_level_transition")
        g.s_min = float(out.s_min)
        self._last_level_forward = None
        return g

    # ------------------------------------------------------------------ backward
    def backward(self, level: GaussianLevel, dL_dimage: torch.Tensor, stream=None):
        """Gradients of the last render_level with respect to the level's tensors."""
        if self._last_level_forward != self.generation:
            raise RuntimeError("backward needs the most recent call on this Renderer to be render_level")
        dL = dL_dimage.contiguous().float()
        n = level.n
        dev = level.means.device
        g = dict(means=torch.empty((n, 3), device=dev), log_scales=torch.empty((n, 3), device=dev),
                 quats=torch.empty((n, 4), device=dev), opacity_logits=torch.empty((n,), device=dev),
                 sh=torch.empty((n, SH_COEFFS, 3), device=dev))
        gs = _lib.Grads(g["means"].data_ptr(), g["log_scales"].data_ptr(), g["quats"].data_ptr(),
                        g["opacity_logits"].data_ptr(), g["sh"].data_ptr())
        st = self.L.flod_render_backward(self.ctx, C.c_void_p(dL.data_ptr()), C.byref(gs),
                                         C.c_void_p(_stream_ptr(stream)))
        _lib.check(st, "flod_render_backward")
        return g

    # ------------------------------------------------------------------ introspection
    def stats(self) -> dict:
        s = _lib.Stats()
        _lib.check(self.L.flod_ctx_stats(self.ctx, C.byref(s)), "flod_ctx_stats")
        return {f: getattr(s, f) for f, _ in _lib.Stats._fields_}

    def workspace_bytes(self) -> int:
        return int(self.L.flod_ctx_workspace_bytes(self.ctx))

    def required_bytes(self) -> int:
        return int(self.L.flod_ctx_required_bytes(self.ctx))

    def trim(self, stream=None):
        _lib.check(self.L.flod_ctx_trim(self.ctx, C.c_void_p(_stream_ptr(stream))), "flod_ctx_trim")

    def keep_backward_state(self, keep: bool):
        """Whether renders keep what backward() needs (default True; a renderer that only
        renders saves 8 bytes of workspace per instance slot with False)."""
        _lib.check(self.L.flod_ctx_keep_backward_state(self.ctx, int(bool(keep))), "flod_ctx_keep_backward_state")

    def set_timing(self, on: bool, stages=None):
        """Per-stage device timing; `stages` (names) restricts it to those stages."""
        if stages is None:
            _lib.check(self.L.flod_ctx_set_timing(self.ctx, int(bool(on))), "flod_ctx_set_timing")
            return
        mask = 0
        if on:
            for name in stages:
                mask |= 1 << _stage_index(self.L, name)
        _lib.check(self.L.flod_ctx_set_timing_stages(self.ctx, mask), "flod_ctx_set_timing_stages")

    def stage_times(self, reset: bool = False) -> dict:
        ms = (C.c_double * _lib.NUM_STAGES)()
        calls = (C.c_int64 * _lib.NUM_STAGES)()
        _lib.check(self.L.flod_ctx_stage_times(self.ctx, ms, calls, int(reset)), "flod_ctx_stage_times")
        return {_lib.STAGES[k]: (float(ms[k]), int(calls[k])) for k in range(_lib.NUM_STAGES)}

    def view(self) -> dict:
        """Copy the last render's intermediate buffers to host numpy arrays."""
        torch.cuda.synchronize()
        v = _lib.View()
        _lib.check(self.L.flod_ctx_view(self.ctx, C.byref(v)), "flod_ctx_view")
        s = self.stats()
        N, K = s["n_candidates"], s["n_instances"]
        tiles = s["tiles_x"] * s["tiles_y"]

        def get(ptr, count, dtype):
            out = np.empty(count if ptr else 0, dtype=dtype)
            if out.size:
                _lib.check(self.L.flod_copy_to_host(out.ctypes.data_as(C.c_void_p), C.c_void_p(ptr),
                                                    out.nbytes), "flod_copy_to_host")
            return out

        return dict(tile_ids=get(v.tile_ids, K, np.uint32), values=get(v.values, K, np.uint32),
                    ranges=get(v.ranges, 2 * tiles, np.uint32).reshape(tiles, 2),
                    depth_bits=get(v.depth_bits, N, np.uint32),
                    rect=get(v.bin, 8 * N, np.uint32).reshape(N, 8)[:, 6:8].copy(),
                    bin=get(v.bin, 8 * N, np.float32).reshape(N, 8),
                    tiles_touched=get(v.tiles_touched, N, np.uint32),
                    xy_conic=get(v.xy_conic, 4 * N, np.float32).reshape(N, 4),
                    cop=get(v.conic_c_opacity_rg, 4 * N, np.float32).reshape(N, 4),
                    blue=get(v.blue, 2 * N, np.float32).reshape(N, 2)[:, 0].copy(),
                    mu_lo_bits=get(v.blue, 2 * N, np.float32).reshape(N, 2)[:, 1].copy().view(np.uint32), stats=s,
                    grad2d=get(v.grad2d, 9 * N, np.float32).reshape(N, 9).T.copy() if v.grad2d else None,
                    blended=get(v.blended, 2 * K, np.uint32).reshape(K, 2),
                    tile_blended=get(v.tile_blended, tiles, np.uint32))


def _empty_level(n: int, s_min: float, device) -> GaussianLevel:
    return GaussianLevel(torch.empty((n, 3), device=device), torch.empty((n, 3), device=device),
                         torch.empty((n, 4), device=device), torch.empty((n,), device=device),
                         torch.empty((n, SH_COEFFS, 3), device=device), float(s_min))


def save_levels(path: str, levels) -> None:
    """Store a level stack (or a compacted selection set): one .npz per level plus a JSON
    level table (index, count, s_min)."""
    import json
    import os
    os.makedirs(path, exist_ok=True)
    table = []
    for i, lv in enumerate(levels):
        np.savez(os.path.join(path, f"level_{i}.npz"), means=lv.means.cpu().numpy(),
                 log_scales=lv.log_scales.cpu().numpy(), quats=lv.quats.cpu().numpy(),
                 opacity_logits=lv.opacity_logits.cpu().numpy(), sh=lv.sh.cpu().numpy())
        table.append({"index": i, "n": lv.n, "s_min": lv.s_min, "file": f"level_{i}.npz"})
    with open(os.path.join(path, "levels.json"), "w") as f:
        json.dump({"levels": table}, f, indent=1)


def load_levels(path: str, device="cuda"):
    """Load a stack written by save_levels onto the device (no pickled objects are read)."""
    import json
    import os
    with open(os.path.join(path, "levels.json")) as f:
        table = json.load(f)["levels"]
    out = []
    for e in table:
        z = np.load(os.path.join(path, e["file"]), allow_pickle=False)
        out.append(GaussianLevel.from_arrays(z["means"], z["log_scales"], z["quats"], z["opacity_logits"], z["sh"],
                                             s_min=e["s_min"], device=device))
    return out


def smin_schedule(l: int, l_max: int, lam: float = 0.2, rho: float = 4.0) -> float:
    """eq. 3 via the library's host helper."""
    return float(_lib.load().flod_smin(int(l), int(l_max), float(lam), float(rho)))


def dproj(s_min: float, f: float, gamma: float = 1.0) -> float:
    """eq. 7 via the library's host helper."""
    return float(_lib.load().flod_dproj(float(s_min), float(f), float(gamma)))


# ---------------------------------------------------------------------------------------
# Differentiable rasterization
# ---------------------------------------------------------------------------------------

class FLoDRasterize(torch.autograd.Function):
    """image = rasterize(level tensors); backward through the hand-written HIP kernels."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, renderer, cam, s_min, bg, sh_degree):
        level = GaussianLevel(means.detach().contiguous(), log_scales.detach().contiguous(),
                              quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                              sh.detach().contiguous(), float(s_min))
        image, final_T, n_contrib = renderer.render_level(level, cam, bg, sh_degree)
        ctx.renderer = renderer
        ctx.level = level
        ctx.gen = renderer.generation
        ctx.frame = (final_T, n_contrib)
        return image

    @staticmethod
    def backward(ctx, grad_image):
        r = ctx.renderer
        if r.generation != ctx.gen:
            raise RuntimeError("the Renderer rendered again between this forward and its backward; "
                               "use one Renderer per differentiable render in flight")
        g = r.backward(ctx.level, grad_image)
        return g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], None, None, None, None, None


def rasterize(means, log_scales, quats, opacity_logits, sh, cam, s_min=0.0, bg=(0.0, 0.0, 0.0), sh_degree=3,
              renderer: Renderer | None = None):
    if renderer is None:
        renderer = _default_renderer()
    return FLoDRasterize.apply(means, log_scales, quats, opacity_logits, sh, renderer, cam, s_min, bg, sh_degree)


_DEFAULT = {}


def _default_renderer() -> Renderer:
    dev = torch.cuda.current_device()
    if dev not in _DEFAULT:
        _DEFAULT[dev] = Renderer(dev)
    return _DEFAULT[dev]


# ---------------------------------------------------------------------------------------
# Training loss: (1 - lam) L1 + lam (1 - SSIM)
# ---------------------------------------------------------------------------------------

class L1SsimLoss(torch.autograd.Function):
    """Scalar FP64 loss of image [C,H,W] against target; forward and backward in HIP."""

    @staticmethod
    def forward(ctx, image, target, renderer, lam):
        image = image.detach().contiguous()
        target = target.detach().contiguous()
        if image.dtype != torch.float32 or target.dtype != torch.float32 or image.shape != target.shape \
                or image.dim() != 3 or not image.is_cuda:
            raise ValueError("image and target must be float32 CUDA tensors of the same [C,H,W] shape")
        C_, H, W = image.shape
        loss = torch.empty((), dtype=torch.float64, device=image.device)
        dmaps = torch.empty((3, C_, H, W), dtype=torch.float32, device=image.device) \
            if ctx.needs_input_grad[0] else None
        _lib.check(renderer.L.flod_l1_ssim_forward(
            renderer.ctx, C.c_void_p(image.data_ptr()), C.c_void_p(target.data_ptr()), C_, H, W, float(lam),
            C.c_void_p(loss.data_ptr()), C.c_void_p(dmaps.data_ptr() if dmaps is not None else 0),
            C.c_void_p(_stream_ptr(None))), "flod_l1_ssim_forward")
        ctx.save_for_backward(image, target, dmaps)
        ctx.renderer, ctx.lam = renderer, float(lam)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        image, target, dmaps = ctx.saved_tensors
        r = ctx.renderer
        C_, H, W = image.shape
        g = grad_loss.to(torch.float64).contiguous()
        d = torch.empty_like(image)
        _lib.check(r.L.flod_l1_ssim_backward(
            r.ctx, C.c_void_p(image.data_ptr()), C.c_void_p(target.data_ptr()), C_, H, W, ctx.lam,
            C.c_void_p(dmaps.data_ptr()), C.c_void_p(g.data_ptr()), C.c_void_p(d.data_ptr()),
            C.c_void_p(_stream_ptr(None))), "flod_l1_ssim_backward")
        return d, None, None, None


def l1_ssim_loss(image, target, lam: float = 0.2, renderer: Renderer | None = None):
    """(1 - lam) mean|image - target| + lam (1 - SSIM(image, target)); FP64 scalar."""
    if renderer is None:
        renderer = _default_renderer()
    return L1SsimLoss.apply(image, target, renderer, lam)


class L1Loss(torch.autograd.Function):
    """mean|image - target| as an FP64 scalar; forward and backward in HIP."""

    @staticmethod
    def forward(ctx, image, target, renderer):
        image = image.detach().contiguous()
        target = target.detach().contiguous()
        if image.dtype != torch.float32 or target.dtype != torch.float32 or image.shape != target.shape \
                or not image.is_cuda:
            raise ValueError("image and target must be float32 CUDA tensors of the same shape")
        loss = torch.empty((), dtype=torch.float64, device=image.device)
        _lib.check(renderer.L.flod_l1_loss_forward(renderer.ctx, C.c_void_p(image.data_ptr()),
                                                   C.c_void_p(target.data_ptr()), image.numel(),
                                                   C.c_void_p(loss.data_ptr()), C.c_void_p(_stream_ptr(None))),
                   "flod_l1_loss_forward")
        ctx.save_for_backward(image, target)
        ctx.renderer = renderer
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        image, target = ctx.saved_tensors
        r = ctx.renderer
        g = grad_loss.to(torch.float64).contiguous()
        d = torch.empty_like(image)
        _lib.check(r.L.flod_l1_loss_backward(r.ctx, C.c_void_p(image.data_ptr()), C.c_void_p(target.data_ptr()),
                                             image.numel(), C.c_void_p(g.data_ptr()), C.c_void_p(d.data_ptr()),
                                             C.c_void_p(_stream_ptr(None))), "flod_l1_loss_backward")
        return d, None, None


def l1_loss(image, target, renderer: Renderer | None = None):
    """mean|image - target| (FP64 scalar) through the library's fused kernels."""
    if renderer is None:
        renderer = _default_renderer()
    return L1Loss.apply(image, target, renderer)

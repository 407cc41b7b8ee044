"""Level-by-level training of a FLoD stack (section Training Method, Algorithm 1) over the
library's kernels: per iteration one view is rasterized (eq. 4 scales under the level's
s_min), the L1 + SSIM loss and its image gradient are taken, the rasterizer's backward gives
the attribute gradients and one fused Adam step updates the level in place. Overlap pruning
(section Overlap Pruning, d_OP = s_min / 2) runs at a fixed interval during the density-control
window of every level but the last, compacting the Adam moments with the Gaussians. After a
level is trained it is kept as that level's final Gaussians and its clone, re-parametrised by
eq. 5, starts the next level with fresh Adam moments.

Densification and opacity reset (the backbone's density control) are not part of this loop.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from .render import GaussianLevel, Renderer, _stream_ptr, l1_ssim_loss, smin_schedule

_ARRAYS = ("means", "log_scales", "quats", "opacity_logits", "sh")


@dataclass
class AdamConfig:
    """Per-group learning rates and Adam constants (the backbone's defaults; the means' rate is
    for a scene of unit extent)."""
    lr_means: float = 1.6e-4
    lr_log_scales: float = 5e-3
    lr_quats: float = 1e-3
    lr_opacity: float = 5e-2
    lr_sh_dc: float = 2.5e-3
    lr_sh_rest: float = 2.5e-3 / 20.0
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15

    def c_struct(self, step: int) -> _lib.AdamParams:
        return _lib.AdamParams(self.lr_means, self.lr_log_scales, self.lr_quats, self.lr_opacity, self.lr_sh_dc,
                               self.lr_sh_rest, self.beta1, self.beta2, self.eps, int(step))


def _state(arrays) -> _lib.LevelState:
    return _lib.LevelState(*(a.data_ptr() for a in arrays))


def _zeros_like_level(level: GaussianLevel):
    return [torch.zeros_like(getattr(level, k)) for k in _ARRAYS]


class LevelAdam:
    """Adam moments of one level and its step count; step() updates the level's tensors in place."""

    def __init__(self, level: GaussianLevel, cfg: AdamConfig | None = None):
        self.cfg = cfg or AdamConfig()
        self.m = _zeros_like_level(level)
        self.v = _zeros_like_level(level)
        self.t = 0

    def step(self, renderer: Renderer, level: GaussianLevel, grads: dict, stream=None) -> None:
        params = [getattr(level, k) for k in _ARRAYS]
        g = [grads[k] for k in _ARRAYS]
        for a in params + g + self.m + self.v:
            if a.dtype != torch.float32 or not a.is_contiguous() or not a.is_cuda:
                raise ValueError("Adam arrays must be contiguous float32 CUDA tensors")
        self.t += 1
        gs = _lib.Grads(*(x.data_ptr() for x in g))
        hp = self.cfg.c_struct(self.t)
        _lib.check(renderer.L.flod_adam_step(renderer.ctx, C.byref(_state(params)), C.byref(gs),
                                             C.byref(_state(self.m)), C.byref(_state(self.v)), level.n,
                                             C.byref(hp), C.c_void_p(_stream_ptr(stream))), "flod_adam_step")

    def compact(self, renderer: Renderer, keep: torch.Tensor) -> None:
        """Keep the moments of the Gaussians whose keep byte is nonzero (index order)."""
        for name in ("m", "v"):
            arrs = getattr(self, name)
            g = renderer.compact(GaussianLevel(*arrs), keep)
            setattr(self, name, [getattr(g, k) for k in _ARRAYS])


def clone_level(level: GaussianLevel) -> GaussianLevel:
    return GaussianLevel(*(getattr(level, k).clone() for k in _ARRAYS), s_min=level.s_min)


@dataclass
class LevelLog:
    level: int
    s_min: float
    losses: list = field(default_factory=list)
    n_start: int = 0
    n_end: int = 0
    pruned: int = 0


def train_level(renderer: Renderer, level: GaussianLevel, cams, targets, iters: int, opt: LevelAdam,
                rng: np.random.Generator, prune_every: int = 0, prune_until: int = 0, bg=(0.0, 0.0, 0.0),
                sh_degree: int = 3, ssim_lambda: float = 0.2, log: LevelLog | None = None) -> GaussianLevel:
    """`iters` iterations of Algorithm 1's inner loop on one level; returns the (possibly
    pruned) level. The views are visited in a fresh random order on every pass."""
    order = []
    for i in range(iters):
        if not order:
            order = list(rng.permutation(len(cams)))
        k = order.pop()
        image, _, _ = renderer.render_level(level, cams[k], bg, sh_degree)
        x = image.detach().requires_grad_(True)
        loss = l1_ssim_loss(x, targets[k], ssim_lambda, renderer=renderer)
        loss.backward()
        grads = renderer.backward(level, x.grad)
        opt.step(renderer, level, grads)
        if log is not None:
            log.losses.append(loss.detach())
        if prune_every and i < prune_until and (i + 1) % prune_every == 0 and level.s_min > 0:
            keep, n_keep = renderer.overlap_prune(level, 0.5 * level.s_min)
            if n_keep < level.n:
                if log is not None:
                    log.pruned += level.n - n_keep
                level = renderer.compact(level, keep)
                opt.compact(renderer, keep)
    return level


def fit_levels(renderer: Renderer, init: GaussianLevel, cams, targets, l_max: int, iters, lam: float = 0.2,
               rho: float = 4.0, prune_every: int = 0, prune_until=None, bg=(0.0, 0.0, 0.0), sh_degree: int = 3,
               ssim_lambda: float = 0.2, adam: AdamConfig | None = None, seed: int = 0):
    """Train levels 1..l_max one after another (Algorithm 1 without densification).

    s_min^(l) follows eq. 3 (0 at the max level). Level 1 starts from `init` (its log_scales
    are taken as s_opt); level l+1 starts from the trained level l re-parametrised by eq. 5.
    iters / prune_until: per-level counts. Returns (levels, logs): the trained level of every
    l (each kept as trained) and a LevelLog per level (losses as device scalars)."""
    rng = np.random.default_rng(seed)
    levels, logs = [], []
    level = None
    for l in range(1, l_max + 1):
        s_min = smin_schedule(l, l_max, lam, rho)
        if level is None:
            level = clone_level(init)
            level.s_min = s_min
        else:
            level = renderer.level_transition(level, s_min)
        log = LevelLog(level=l, s_min=s_min, n_start=level.n)
        opt = LevelAdam(level, adam)
        pu = 0 if (prune_until is None or l == l_max) else int(prune_until[l - 1])
        level = train_level(renderer, level, cams, targets, int(iters[l - 1]), opt, rng,
                            prune_every=prune_every if l < l_max else 0, prune_until=pu, bg=bg,
                            sh_degree=sh_degree, ssim_lambda=ssim_lambda, log=log)
        log.n_end = level.n
        levels.append(level)
        logs.append(log)
    return levels, logs

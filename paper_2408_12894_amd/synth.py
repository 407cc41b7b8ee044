"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random scenes, cameras and request traces. It holds none of the
rasterizer's arithmetic (no activation, projection, selection or compositing): every
array it returns is a raw input that both the oracle and the HIP path consume.

Gaussian attributes follow the parametrisation of the Preliminary section (position,
opacity, covariance through a log-scale vector and a quaternion, spherical-harmonic
colour coefficients). Layout, one Gaussian per row, float32, C-contiguous:

    means           [n, 3]
    log_scales      [n, 3]      s_opt of eq. 4
    quats           [n, 4]      (w, x, y, z), unit norm as drawn
    opacity_logits  [n]         opacity = sigmoid(logit)
    sh              [n, 16, 3]  coefficient k = l*l + l + m, colour channel last

Cameras use OpenCV axes (x right, y down, z forward) with world->camera x_c = R x + t.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SH_COEFFS = 16


@dataclass
class Camera:
    R: np.ndarray          # [3,3] float32, rows are the camera axes in world coordinates
    t: np.ndarray          # [3] float32
    campos: np.ndarray     # [3] float32, the eye point in world coordinates
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


@dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    s_min: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh)

    def copy(self) -> "Scene":
        return Scene(*(a.copy() for a in self.arrays()), s_min=self.s_min, meta=dict(self.meta))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def focal_for_width(width: int, hfov_deg: float = 60.0) -> float:
    """Pinhole focal length (pixels) for a horizontal field of view."""
    return float(np.float32(width / (2.0 * math.tan(math.radians(hfov_deg) / 2.0))))


def look_at_camera(eye, target, width: int, height: int, hfov_deg: float = 60.0,
                   down=(0.0, 1.0, 0.0)) -> Camera:
    """Camera at `eye` looking at `target`; world `down` maps to image +y."""
    eye = np.asarray(eye, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    z = target - eye
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(down, dtype=np.float64), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z], axis=0)
    t = -R @ eye
    f = focal_for_width(width, hfov_deg)
    return Camera(R=_f32(R), t=_f32(t), campos=_f32(eye), fx=f, fy=f,
                  cx=float(width) / 2.0, cy=float(height) / 2.0, width=int(width), height=int(height))


def orbit_cameras(seed: int, count: int, radius: float, width: int, height: int,
                  hfov_deg: float = 60.0):
    """`count` eyes at radius*(sin th, 0, cos th), th ~ U[0, 2 pi), looking at the origin."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, 2.0 * math.pi, size=count)
    return [look_at_camera((radius * math.sin(a), 0.0, radius * math.cos(a)), (0.0, 0.0, 0.0),
                           width, height, hfov_deg) for a in th]


def _attributes(rng, n, s_mu, s_sigma, a_sigma, sh_sigma=0.3):
    log_scales = rng.normal(s_mu, s_sigma, size=(n, 3))
    g = rng.normal(0.0, 1.0, size=(n, 4))
    quats = g / np.linalg.norm(g, axis=1, keepdims=True)
    opacity_logits = rng.normal(0.0, a_sigma, size=n)
    sh = rng.normal(0.0, sh_sigma, size=(n, SH_COEFFS, 3))
    return _f32(log_scales), _f32(quats), _f32(opacity_logits), _f32(sh)


def uniform_scene(n: int, seed: int, s_mu=-4.0, s_sigma=0.5, a_sigma=1.0, extent=1.0,
                  s_min=0.0, sh_sigma=0.3) -> Scene:
    """Means ~ U[-extent, extent]^3 with the attribute distributions given."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-extent, extent, size=(n, 3))
    ls, q, a, sh = _attributes(rng, n, s_mu, s_sigma, a_sigma, sh_sigma)
    return Scene(_f32(means), ls, q, a, sh, s_min=float(s_min), meta={"kind": "uniform", "seed": seed})


def cluster_layout(layout_seed: int = 1, n_clusters: int = 64):
    """Cluster centres ~ U[-1,1]^3, per-axis std ~ U[0.05, 0.3], random orientation."""
    rng = np.random.default_rng(layout_seed)
    centres = rng.uniform(-1.0, 1.0, size=(n_clusters, 3))
    stds = rng.uniform(0.05, 0.3, size=(n_clusters, 3))
    rots = []
    for _ in range(n_clusters):
        a = rng.normal(size=(3, 3))
        qm, r = np.linalg.qr(a)
        qm = qm * np.sign(np.diag(r))
        rots.append(qm)
    return centres, stds, np.stack(rots)


def cluster_scene(n: int, seed: int, layout_seed: int = 1, shell_frac=0.15, shell_radius=10.0,
                  s_mu=-4.5, s_sigma=0.7, a_sigma=1.5, s_min=0.0, sh_sigma=0.3) -> Scene:
    """Mixture of 64 anisotropic clusters plus a thin background shell at `shell_radius`."""
    centres, stds, rots = cluster_layout(layout_seed)
    rng = np.random.default_rng(seed)
    n_shell = int(round(n * shell_frac))
    n_cl = n - n_shell
    which = rng.integers(0, centres.shape[0], size=n_cl)
    local = rng.normal(size=(n_cl, 3)) * stds[which]
    pts = centres[which] + np.einsum("nij,nj->ni", rots[which], local)
    u = rng.normal(size=(n_shell, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    means = np.concatenate([pts, shell_radius * u], axis=0)
    perm = rng.permutation(n)
    means = means[perm]
    ls, q, a, sh = _attributes(rng, n, s_mu, s_sigma, a_sigma, sh_sigma)
    return Scene(_f32(means), ls, q, a, sh, s_min=float(s_min),
                 meta={"kind": "cluster", "seed": seed, "layout_seed": layout_seed})


# ---------------------------------------------------------------------------------------
# Named workloads (sizes and distributions of the paper-shaped synthetic benchmarks)
# ---------------------------------------------------------------------------------------

def small_forward_case():
    """2,000 uniform Gaussians, one camera at distance 4, 128x128, black background."""
    scene = uniform_scene(2000, seed=0, s_mu=-4.0, s_sigma=0.5, a_sigma=1.0)
    cam = look_at_camera((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), 128, 128)
    return scene, cam, np.zeros(3, dtype=np.float32)


def hd_forward_case(n: int = 1_000_000, n_cams: int = 8):
    """Cluster scene at 1920x1080 with 8 seeded orbit cameras of radius 4."""
    scene = cluster_scene(n, seed=1, layout_seed=1)
    cams = orbit_cameras(2, n_cams, 4.0, 1920, 1080)
    return scene, cams, np.zeros(3, dtype=np.float32)


LEVEL_SIZES = (40_000, 150_000, 500_000, 1_200_000, 2_500_000)
LEVEL_SMIN = tuple(0.2 * 2.0 ** (1 - l) for l in range(1, 6))     # 0.2, 0.1, 0.05, 0.025, 0.0125
LEVEL_BANDS = (16.0, 8.0, 4.0, 2.0, 0.0)                           # d_proj^(1..5): explicit bands


def level_stack(sizes=LEVEL_SIZES, s_mins=LEVEL_SMIN):
    """Independent levels drawn from the same cluster layout, seeds 10+l."""
    return [cluster_scene(n, seed=10 + l, layout_seed=1, s_min=s)
            for l, (n, s) in enumerate(zip(sizes, s_mins), start=1)]


def training_case(n: int = 500_000, width: int = 1280, height: int = 720):
    """Single level (s_min = 0.0125) and its perturbed copy for the target image."""
    scene = cluster_scene(n, seed=20, layout_seed=1, s_min=0.0125)
    target = scene.copy()
    rng = np.random.default_rng(21)
    target.means = _f32(scene.means + rng.normal(0.0, 0.01, size=scene.means.shape))
    target.opacity_logits = _f32(scene.opacity_logits + rng.normal(0.0, 0.2, size=scene.n))
    cam = orbit_cameras(2, 1, 4.0, width, height)[0]
    return scene, target, cam, np.zeros(3, dtype=np.float32)


def fd_case(seed: int = 22, n: int = 64, size: int = 32):
    """Tiny instance whose Gaussians span several pixels, for finite differences."""
    scene = uniform_scene(n, seed=seed, s_mu=-1.5, s_sigma=0.3, a_sigma=1.0, s_min=0.05)
    cam = look_at_camera((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), size, size)
    return scene, cam, np.zeros(3, dtype=np.float32)


RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080), (3840, 2160))
SELECTIVE_RANGES = ((1, 2), (2, 3), (3, 4), (4, 5), (1, 3), (2, 4), (3, 5))


@dataclass
class Request:
    rid: int
    arrival_s: float
    camera: Camera
    l_start: int
    l_end: int


def serving_trace(seed: int = 30, count: int = 512, mean_gap_s: float = 0.002, radius: float = 4.0,
                  resolutions=RESOLUTIONS, n_levels: int = 5):
    """Poisson arrivals; each request draws an orbit camera, a resolution and a level spec.

    With probability 1/2 the level spec is a single level (l, l); otherwise one of the
    contiguous two- or three-level ranges.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_gap_s, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        th = rng.uniform(0.0, 2.0 * math.pi)
        w, h = resolutions[rng.integers(0, len(resolutions))]
        if rng.uniform() < 0.5:
            l = int(rng.integers(1, n_levels + 1))
            ls, le = l, l
        else:
            ls, le = SELECTIVE_RANGES[rng.integers(0, len(SELECTIVE_RANGES))]
        cam = look_at_camera((radius * math.sin(th), 0.0, radius * math.cos(th)), (0.0, 0.0, 0.0), w, h)
        out.append(Request(i, float(arrivals[i]), cam, int(ls), int(le)))
    return out


def random_dl_dimage(seed: int, width: int, height: int) -> np.ndarray:
    """Upstream image gradient [3, H, W] for parity of the backward pass."""
    rng = np.random.default_rng(seed)
    return _f32(rng.normal(0.0, 1.0, size=(3, height, width)))

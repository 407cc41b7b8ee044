"""CPU oracle for the FLoD-3DGS rasterizer hot path (ctypes wrapper around liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's
CPU-baseline leg. The product package never imports this module, and this module never
imports the product package (it only receives the same seeded numpy inputs).

Parts (see oracle.cpp for the arithmetic):
  keys()          O1 key mirror per Gaussian (culls, depth bits, tile footprint and its
                  bounding rectangle, stored FP32 mu' with its bf16 residual and conic)
  instances()     O1 instance list sorted by (tile, depth bits, index) and tile ranges
  depth_order()   surviving ids in (depth bits, index) order: the compositing order
  image()         O2 FP64 brute-force image at chosen pixels, with ambiguity flags (bit 1: a
                  decision that changes the image is near its threshold; bit 2: the alpha clamp's
                  kink, which changes only the gradient)
  grad()          O3 FP64 gradient of sum(dL_dimage * image) over chosen pixels
  select()        eq. 6 band selection over a level range, FP32 squared distances
  ssim, adam      the training loss (L1 + SSIM) and the optimiser step (numpy modules)
Host helpers for eq. 3, eq. 5 and eq. 7 are plain formulas on scalars.

Pins (tests/test_oracle_pins.py): eq. 3/5/7 closed forms and identities; eq. 6 band
partition and special cases; eq. 1 covariance against scipy's quaternion rotation; the
projected covariance against a numerical Jacobian of the pinhole map; single-Gaussian and
two-Gaussian closed-form images; the weights-plus-transmittance invariant; SH against
scipy's complex harmonics and quadrature orthonormality; the sorted instance list against
brute-force enumeration plus numpy lexsort; the gradient against FP64 central differences.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TILE = 16


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (strict IEEE: no contraction, no fast-math).

    FLOD_ORACLE_LIB in the environment names another build of oracle.cpp to load instead
    (the mutation test builds deliberately broken copies); nothing is compiled then."""
    alt = os.environ.get("FLOD_ORACLE_LIB")
    if alt:
        return alt
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class CamIn(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("campos", C.c_float * 3),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("W", C.c_int32), ("H", C.c_int32)]


def _cam(cam) -> CamIn:
    c = CamIn()
    c.R[:] = [float(v) for v in np.asarray(cam.R, np.float32).ravel()]
    c.t[:] = [float(v) for v in np.asarray(cam.t, np.float32).ravel()]
    c.campos[:] = [float(v) for v in np.asarray(cam.campos, np.float32).ravel()]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.W, c.H = int(cam.width), int(cam.height)
    return c


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        vp, i64, i32, f32 = C.c_void_p, C.c_int64, C.c_int32, C.c_float
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        L.or_sh_basis.argtypes = [C.c_int, vp, vp]
        L.or_select_level.argtypes = [i64, vp, vp, f32, f32, vp]
        L.or_overlap_prune.argtypes = [i64, vp, C.c_double, i64, vp, vp, vp]
        L.or_level_transition.argtypes = [i64, vp, C.c_double, C.c_double, vp]
        L.or_keys.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.or_instances.argtypes = [i64, vp, vp, vp, vp, vp, i32, i32, i64, vp, vp, vp]
        L.or_instances.restype = i64
        L.or_project64.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, C.c_int, vp, vp]
        L.or_image.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, C.c_int, vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.or_grad.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, vp, C.c_int, vp, vp, i64, vp, vp,
                              vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


# ----------------------------------------------------------------------------------
# Scalar helpers: eq. 3, eq. 5, eq. 7
# ----------------------------------------------------------------------------------

def smin_schedule(l: int, l_max: int, lam: float = 0.2, rho: float = 4.0) -> float:
    """eq. 3: s_min^(l) = lam * rho^(1-l) below the top level, 0 at l = l_max."""
    return 0.0 if l == l_max else lam * rho ** (1 - l)


def reparam_next_level(s_level: np.ndarray, s_min_next: float) -> np.ndarray:
    """eq. 5: s_opt for level l+1 from the trained level-l scales, log(s^(l) - s_min^(l+1))."""
    return np.log(np.asarray(s_level, np.float64) - s_min_next)


def overlap_prune(means, d_op: float, ids=None):
    """Overlap pruning: (keep uint8, d_avg float64); removed iff the mean distance to the three
    nearest other Gaussians is below d_op. ids: evaluate only these Gaussians (against all)."""
    m = np.ascontiguousarray(np.asarray(means, np.float32).reshape(-1, 3))
    n = m.shape[0]
    idx = None if ids is None else np.ascontiguousarray(np.asarray(ids, np.int64))
    count = n if idx is None else idx.shape[0]
    keep = np.zeros(count, np.uint8)
    davg = np.zeros(count, np.float64)
    if count:
        lib().or_overlap_prune(n, _p(m), float(d_op), 0 if idx is None else count,
                               None if idx is None else _p(idx), _p(keep), _p(davg))
    return keep, davg


def level_transition(log_scales, s_min_l: float, s_min_next: float) -> np.ndarray:
    """eq. 5 from level-l scale parameters: log(exp(s_opt) + s_min^(l) - s_min^(l+1)) in FP64,
    exp rounded once to FP32 as the rasterizer forms s^(l)."""
    ls = np.ascontiguousarray(np.asarray(log_scales, np.float32))
    out = np.zeros(ls.shape, np.float64)
    if ls.size:
        lib().or_level_transition(ls.size // 3, _p(ls), float(np.float32(s_min_l)), float(np.float32(s_min_next)),
                                  _p(out))
    return out


def dproj(s_min: float, f: float, gamma: float) -> float:
    """eq. 7: distance at which s_min projects to gamma pixels, d = s_min / gamma * f."""
    return float(np.float32(float(s_min) / float(gamma) * float(f)))


def band_edges(l: int, l_start: int, l_end: int, d_proj) -> tuple[float, float]:
    """eq. 6 band of level l: (lo, hi) = (d_proj^(l), d_proj^(l-1)), with
    d_proj^(l_end) = 0 and d_proj^(l_start - 1) = infinity."""
    hi = math.inf if l == l_start else float(d_proj[l - 2])
    lo = 0.0 if l == l_end else float(d_proj[l - 1])
    return lo, hi


def _sq32(d: float) -> float:
    return math.inf if math.isinf(d) else float(np.float32(float(d) * float(d)))


def select(levels_means, centre, l_start: int, l_end: int, d_proj) -> np.ndarray:
    """eq. 6 over concatenated levels: uint8 keep mask, one entry per candidate."""
    L = lib()
    cen = np.ascontiguousarray(np.asarray(centre, np.float32))
    out = []
    for l, means in enumerate(levels_means, start=1):
        means = np.ascontiguousarray(means, np.float32)
        keep = np.zeros(means.shape[0], np.uint8)
        if l_start <= l <= l_end:
            lo, hi = band_edges(l, l_start, l_end, d_proj)
            L.or_select_level(means.shape[0], _p(means), _p(cen), _sq32(lo), _sq32(hi), _p(keep))
        out.append(keep)
    return np.concatenate(out) if out else np.zeros(0, np.uint8)


# ----------------------------------------------------------------------------------
# O1: key mirror
# ----------------------------------------------------------------------------------

def _arrays(means, log_scales, quats, logits, smin, dt=np.float32):
    n = int(np.asarray(means).shape[0])
    a = [np.ascontiguousarray(np.asarray(x, dt)) for x in (means, log_scales, quats, logits)]
    sm = np.ascontiguousarray(np.broadcast_to(np.asarray(smin, dt), (n,)).copy())
    return n, a, sm


def keys(means, log_scales, quats, logits, smin, cam, keep=None) -> dict:
    n, (m, ls, q, lg), sm = _arrays(means, log_scales, quats, logits, smin)
    kp = None if keep is None else np.ascontiguousarray(np.asarray(keep, np.uint8))
    out = dict(visible=np.zeros(n, np.uint8), depth_bits=np.zeros(n, np.uint32),
               rect=np.zeros((n, 4), np.int32), tiles=np.zeros(n, np.uint32),
               radius=np.zeros(n, np.float32), mxy=np.zeros((n, 2), np.float32),
               conic=np.zeros((n, 3), np.float32), mu_lo=np.zeros(n, np.uint32), qsup=np.zeros(n, np.float32))
    c = _cam(cam)
    lib().or_keys(n, _p(m), _p(ls), _p(q), _p(lg), _p(sm), None if kp is None else _p(kp), C.byref(c),
                  _p(out["visible"]), _p(out["depth_bits"]), _p(out["rect"]), _p(out["tiles"]),
                  _p(out["radius"]), _p(out["mxy"]), _p(out["conic"]), _p(out["mu_lo"]), _p(out["qsup"]))
    out["tiles_x"] = (int(cam.width) + TILE - 1) // TILE
    out["tiles_y"] = (int(cam.height) + TILE - 1) // TILE
    return out


def instances(k: dict):
    """Sorted (tile, value) lists and per-tile [start, end) ranges from keys() output."""
    n = k["visible"].shape[0]
    n_tiles = k["tiles_x"] * k["tiles_y"]
    K = int(k["tiles"].astype(np.int64).sum())
    tile = np.zeros(max(K, 1), np.uint32)
    val = np.zeros(max(K, 1), np.uint32)
    ranges = np.zeros((n_tiles, 2), np.uint32)
    got = lib().or_instances(n, _p(k["visible"]), _p(k["depth_bits"]), _p(k["mxy"]), _p(k["conic"]),
                             _p(k["qsup"]), k["tiles_x"], k["tiles_y"], K, _p(tile), _p(val), _p(ranges))
    assert got == K
    return tile[:K], val[:K], ranges


def depth_order(k: dict) -> np.ndarray:
    """Visible ids ordered by (depth bits, index): the front-to-back compositing order."""
    ids = np.nonzero(k["visible"])[0].astype(np.int64)
    o = np.lexsort((ids, k["depth_bits"][ids]))
    return np.ascontiguousarray(ids[o])


# ----------------------------------------------------------------------------------
# O2 / O3: FP64
# ----------------------------------------------------------------------------------

def project64(ids, means, log_scales, quats, logits, smin, sh, deg, cam) -> np.ndarray:
    """[len(ids), 9]: mu'x, mu'y, conic a, b, c, opacity, r, g, b in FP64."""
    n, (m, ls, q, lg), sm = _arrays(means, log_scales, quats, logits, smin, np.float64)
    shc = np.ascontiguousarray(np.asarray(sh, np.float64))
    ids = np.ascontiguousarray(np.asarray(ids, np.int64))
    out = np.zeros((ids.shape[0], 9), np.float64)
    c = _cam(cam)
    lib().or_project64(ids.shape[0], _p(ids), _p(m), _p(ls), _p(q), _p(lg), _p(sm), _p(shc), int(deg),
                       C.byref(c), _p(out))
    return out


def all_pixels(width: int, height: int) -> np.ndarray:
    ys, xs = np.mgrid[0:height, 0:width]
    return np.ascontiguousarray(np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32))


def image(order, means, log_scales, quats, logits, smin, sh, deg, cam, bg, pix=None) -> dict:
    n, (m, ls, q, lg), sm = _arrays(means, log_scales, quats, logits, smin, np.float64)
    shc = np.ascontiguousarray(np.asarray(sh, np.float64))
    order = np.ascontiguousarray(np.asarray(order, np.int64))
    if pix is None:
        pix = all_pixels(cam.width, cam.height)
    pix = np.ascontiguousarray(np.asarray(pix, np.int32))
    P = pix.shape[0]
    bgv = np.ascontiguousarray(np.asarray(bg, np.float32))
    out = dict(rgb=np.zeros((P, 3), np.float64), T=np.zeros(P, np.float64), last=np.zeros(P, np.int64),
               flag=np.zeros(P, np.uint8), nblend=np.zeros(P, np.int32), pix=pix)
    c = _cam(cam)
    lib().or_image(order.shape[0], _p(order), _p(m), _p(ls), _p(q), _p(lg), _p(sm), _p(shc), int(deg),
                   C.byref(c), _p(bgv), P, _p(pix), _p(out["rgb"]), _p(out["T"]), _p(out["last"]),
                   _p(out["flag"]), _p(out["nblend"]))
    return out


def grad(order, means, log_scales, quats, logits, smin, sh, deg, cam, bg, pix, dL_dpix, with_scale=False) -> dict:
    """O3. With with_scale, out['scale'][name] holds each entry's summation scale (the
    magnitudes of the per-pixel terms it sums, through the absolute Jacobian)."""
    n, (m, ls, q, lg), sm = _arrays(means, log_scales, quats, logits, smin, np.float64)
    shc = np.ascontiguousarray(np.asarray(sh, np.float64))
    order = np.ascontiguousarray(np.asarray(order, np.int64))
    pix = np.ascontiguousarray(np.asarray(pix, np.int32))
    dl = np.ascontiguousarray(np.asarray(dL_dpix, np.float64).reshape(-1, 3))
    assert dl.shape[0] == pix.shape[0]
    bgv = np.ascontiguousarray(np.asarray(bg, np.float32))
    out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), sh=np.zeros((n, 16, 3)))
    sc = None
    if with_scale:
        sc = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
                  opacity_logits=np.zeros(n), sh=np.zeros((n, 16, 3)))
    sp = [None] * 5 if sc is None else [_p(sc[k]) for k in ("means", "log_scales", "quats", "opacity_logits", "sh")]
    out["g2d"] = np.zeros((n, 9))
    s2d = np.zeros((n, 9)) if with_scale else None
    sp += [_p(out["g2d"]), None if s2d is None else _p(s2d)]
    c = _cam(cam)
    lib().or_grad(n, order.shape[0], _p(order), _p(m), _p(ls), _p(q), _p(lg), _p(sm), _p(shc), int(deg),
                  C.byref(c), _p(bgv), pix.shape[0], _p(pix), _p(dl), _p(out["means"]), _p(out["log_scales"]),
                  _p(out["quats"]), _p(out["opacity_logits"]), _p(out["sh"]), *sp)
    if sc is not None:
        sc["g2d"] = s2d
        out["scale"] = sc
    return out


def sh_basis(deg: int, direction) -> np.ndarray:
    d = np.ascontiguousarray(np.asarray(direction, np.float64))
    out = np.zeros(16, np.float64)
    lib().or_sh_basis(int(deg), _p(d), _p(out))
    return out


def render(scene_arrays, smin, cam, bg, deg=3, keep=None, pix=None) -> dict:
    """O1 + O2 convenience: keys, order and FP64 image at `pix` (default: every pixel)."""
    means, log_scales, quats, logits, sh = scene_arrays
    k = keys(means, log_scales, quats, logits, smin, cam, keep)
    order = depth_order(k)
    img = image(order, means, log_scales, quats, logits, smin, sh, deg, cam, bg, pix)
    img["keys"] = k
    img["order"] = order
    return img


from . import ssim  # noqa: E402  (L1 + SSIM training loss, numpy FP64)
from . import adam  # noqa: E402  (the training loop's Adam step, numpy FP64)

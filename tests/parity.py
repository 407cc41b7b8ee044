"""Helpers for GPU-versus-oracle parity tests (imported by tests only).

Tolerances (floating point, the bar stated for this hot path):
  image and final_T     1e-4 absolute on every pixel the oracle does not flag. A flagged pixel
                        has a decision that changes the image (support cut, alpha floor, stop)
                        within a relative 1e-4 of its threshold, where FP32 and FP64 may decide
                        apart; flagged pixels are compared too, against the largest change one
                        flipped decision can make (FLIP_TOL), and the pixels that differ by more
                        than 1e-4 anywhere must stay below 0.1% of those compared (MISMATCH_MAX).
  key path              bit-exact: visibility, depth bits, tile rectangle, tiles touched, stored
                        mu' (FP32 and bf16 residual), conic; sorted (tile, Gaussian) list and
                        tile ranges
"""
from __future__ import annotations

import numpy as np

import oracle

IMG_TOL = 1e-4
# One flipped decision changes a pixel by the flipped Gaussian's share: alpha T |c - behind|
# with alpha at most o e^{-9/2} < 0.0112 at the support cut, about 1/255 at the alpha floor and
# T < 1e-4 at the stop; with colours below 2 in magnitude that is under 0.023.
FLIP_TOL = 0.05
MISMATCH_MAX = 1e-3
# The flag rate grows with the pairs a pixel evaluates (about 2e-4 per evaluated pair): 0.09% at
# 128x128 / 2k, 0.5-0.9% at 1M Gaussians; a rate far above that would mean the flags hide errors.
FLAG_FRAC_MAX = 2e-2


def sample_pixels(width, height, n, seed, ranges=None, n_long=0, tiles_x=None):
    """n uniform pixels, plus n_long pixels drawn uniformly inside the 1% of tiles with the
    longest lists (ranges: the oracle's per-tile [start, end)), unique."""
    rng = np.random.default_rng(seed)
    pix = [np.stack([rng.integers(0, width, n), rng.integers(0, height, n)], 1)]
    if n_long and ranges is not None:
        lens = ranges[:, 1].astype(np.int64) - ranges[:, 0]
        top = np.argsort(-lens, kind="stable")[:max(1, len(lens) // 100)]
        t = top[rng.integers(0, len(top), n_long)]
        tx, ty = t % tiles_x, t // tiles_x
        x = np.minimum(tx * 16 + rng.integers(0, 16, n_long), width - 1)
        y = np.minimum(ty * 16 + rng.integers(0, 16, n_long), height - 1)
        pix.append(np.stack([x, y], 1))
    return np.unique(np.concatenate(pix).astype(np.int32), axis=0)


def unpack_rect(r):
    r = np.asarray(r, np.uint32)
    return np.stack([r[:, 0] & 0xFFFF, r[:, 0] >> 16, r[:, 1] & 0xFFFF, r[:, 1] >> 16], axis=1).astype(np.int32)


def check_keys(view, k, idx=None):
    """Per-candidate key fields and the sorted instance list against O1 (bit-exact).
    idx: oracle indices of the GPU candidates (default: the identity)."""
    vis = k["visible"].astype(bool)
    if idx is not None:
        vis = vis[idx]
        sub = {n: k[n][idx] for n in ("depth_bits", "rect", "tiles", "mxy", "conic", "mu_lo", "qsup")}
    else:
        sub = k
    g_vis = view["tiles_touched"] > 0
    np.testing.assert_array_equal(g_vis, vis, err_msg="visibility")
    np.testing.assert_array_equal(view["tiles_touched"][vis], sub["tiles"][vis], err_msg="tiles touched")
    np.testing.assert_array_equal(view["depth_bits"][vis], sub["depth_bits"][vis], err_msg="depth bits")
    np.testing.assert_array_equal(unpack_rect(view["rect"][vis]), sub["rect"][vis], err_msg="tile rect")
    np.testing.assert_array_equal(view["xy_conic"][vis, :2].view(np.uint32), sub["mxy"][vis].view(np.uint32),
                                  err_msg="mu' bits")
    g_conic = np.stack([view["xy_conic"][vis, 2], view["xy_conic"][vis, 3], view["cop"][vis, 0]], 1)
    np.testing.assert_array_equal(g_conic.view(np.uint32), sub["conic"][vis].view(np.uint32), err_msg="conic bits")
    np.testing.assert_array_equal(view["mu_lo_bits"][vis], sub["mu_lo"][vis], err_msg="mu' residual bits")
    # the binning record repeats mu' and the conic, and carries the support bound Q_g
    rec = view["bin"][vis]
    np.testing.assert_array_equal(rec[:, :4].view(np.uint32), view["xy_conic"][vis].view(np.uint32),
                                  err_msg="record mu', conic a, b")
    np.testing.assert_array_equal(rec[:, 4].view(np.uint32), view["cop"][vis, 0].view(np.uint32),
                                  err_msg="record conic c")
    np.testing.assert_array_equal(rec[:, 5].view(np.uint32), np.asarray(sub["qsup"], np.float32)[vis].view(np.uint32),
                                  err_msg="record support bound")


def check_instances(view, k, index_offset=0):
    tile, val, ranges = oracle.instances(k)
    assert view["stats"]["n_instances"] == tile.shape[0], (view["stats"]["n_instances"], tile.shape[0])
    np.testing.assert_array_equal(view["tile_ids"], tile, err_msg="sorted tile ids")
    np.testing.assert_array_equal(view["values"].astype(np.int64) + index_offset, val.astype(np.int64),
                                  err_msg="sorted values")
    # ranges of empty tiles are [0, 0) on the GPU; compare lengths there
    gl = view["ranges"][:, 1].astype(np.int64) - view["ranges"][:, 0]
    ol = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    np.testing.assert_array_equal(gl, ol, err_msg="range lengths")
    ne = ol > 0
    np.testing.assert_array_equal(view["ranges"][ne], ranges[ne], err_msg="ranges")
    return tile, val, ranges


def check_image(image, final_T, n_contrib, ref, view, cam, index_offset=0, tol=IMG_TOL, frac_max=FLAG_FRAC_MAX,
                n_blended=None, label=""):
    """Compare GPU outputs with O2 at ref['pix']; returns (max error on unflagged pixels,
    flagged fraction). Prints the flagged fraction and how many pixels differ by more than tol."""
    pix = ref["pix"]
    xs, ys = pix[:, 0], pix[:, 1]
    img = np.asarray(image)
    got = img[:, ys, xs].T.astype(np.float64)
    gT = np.asarray(final_T)[ys, xs].astype(np.float64)
    gn = np.asarray(n_contrib)[ys, xs].astype(np.int64)
    flagged = (ref["flag"] & 1) != 0
    ok = ~flagged
    frac = float(flagged.mean())
    e_pix = np.maximum(np.abs(got - ref["rgb"]).max(axis=1), np.abs(gT - ref["T"]))
    err = float(e_pix[ok].max()) if ok.any() else 0.0
    err_f = float(e_pix[flagged].max()) if flagged.any() else 0.0
    n_over = int((e_pix > tol).sum())
    print(f"[parity] {label} {pix.shape[0]} pixels: flagged {frac:.3%}; max |diff| {err:.2e} unflagged, "
          f"{err_f:.2e} flagged; pixels over {tol:g}: {n_over} ({n_over / pix.shape[0]:.3%})", flush=True)
    assert frac <= frac_max, f"flagged fraction {frac}"
    assert err <= tol, f"image / final_T max abs error {err} on an unflagged pixel"
    assert err_f <= FLIP_TOL, f"flagged pixel off by {err_f}, more than one flipped decision can make"
    assert n_over <= MISMATCH_MAX * pix.shape[0], f"{n_over} pixels differ by more than {tol}"
    # the last blended Gaussian, read through the tile list position n_contrib
    tiles_x = (cam.width + 15) // 16
    tile = (ys // 16) * tiles_x + xs // 16
    start = view["ranges"][tile, 0].astype(np.int64)
    has = gn > 0
    assert np.all((ref["last"] >= 0)[ok] == has[ok]), "pixels with / without a blended Gaussian"
    sel = ok & has
    last_gpu = view["values"][start[sel] + gn[sel] - 1].astype(np.int64) + index_offset
    np.testing.assert_array_equal(last_gpu, ref["last"][sel], err_msg="last blended Gaussian")
    if n_blended is not None:
        gb = np.asarray(n_blended)[ys, xs].astype(np.int64)
        np.testing.assert_array_equal(gb[ok], ref["nblend"][ok].astype(np.int64), err_msg="blended count")
    return err, frac


def unpack_mu_lo(bits):
    bits = np.asarray(bits, np.uint32)
    lx = (bits << np.uint32(16)).view(np.float32).astype(np.float64)
    ly = (bits & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    return lx, ly


def check_fp64_fields(view, p64, vis_ids, rtol_conic=1e-6):
    """Continuous per-Gaussian fields against the oracle's FP64 projection (tolerance): mu'
    as hi + lo to 1e-6 px, the conic to FP32 rounding, opacity and colour to FP32 evaluation."""
    g = view["xy_conic"][vis_ids].astype(np.float64)
    c = view["cop"][vis_ids].astype(np.float64)
    lx, ly = unpack_mu_lo(view["mu_lo_bits"][vis_ids])
    for hi, lo, ref in ((g[:, 0], lx, p64[:, 0]), (g[:, 1], ly, p64[:, 1])):
        err = np.abs(hi + lo - ref)
        assert np.all(err <= 1e-6 + 1e-9 * np.abs(ref)), f"mu' off by {err.max():.3g} px"
    scale = np.abs(p64[:, 2:5]).max(axis=1, keepdims=True)
    conic = np.stack([g[:, 2], g[:, 3], c[:, 0]], 1)
    assert np.all(np.abs(conic - p64[:, 2:5]) <= rtol_conic * scale + 1e-9), "conic"
    np.testing.assert_allclose(c[:, 1], p64[:, 5], atol=2e-6)          # opacity
    rgb = np.stack([c[:, 2], c[:, 3], view["blue"][vis_ids]], 1)
    np.testing.assert_allclose(rgb, p64[:, 6:9], atol=2e-5)

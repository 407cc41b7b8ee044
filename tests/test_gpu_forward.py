"""GPU forward parity: the HIP path (through the C ABI) against the CPU oracle.

Key path bit-exact against the FP32 mirror, images within 1e-4 of the FP64 brute-force
splatter on unflagged pixels (tolerances in tests/parity.py).
"""
import numpy as np
import pytest

import oracle
from paper_2408_12894_amd import synth
from parity import FLAG_FRAC_MAX, check_fp64_fields, check_image, check_instances, check_keys, sample_pixels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer():
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return render.Renderer(0)


def _say(msg):
    print(f"[case] {msg}", flush=True)


def gpu_render(renderer, scene, cam, bg, deg=3):
    from paper_2408_12894_amd import render
    level = render.GaussianLevel.from_scene(scene)
    nbl = torch.empty((cam.height, cam.width), dtype=torch.int32, device="cuda")
    image, final_T, n_contrib = renderer.render_level(level, cam, bg, deg, n_blended=nbl)
    torch.cuda.synchronize()
    view = renderer.view()
    view["n_blended"] = nbl.cpu().numpy()
    return image.cpu().numpy(), final_T.cpu().numpy(), n_contrib.cpu().numpy(), view


def full_parity(renderer, scene, cam, bg, deg=3, pix=None, frac_max=FLAG_FRAC_MAX, sample=None, label=""):
    """sample = (n uniform pixels, n pixels in the 1% longest tile lists of the oracle's own
    list, seed) replaces pix."""
    image, T, nc, view = gpu_render(renderer, scene, cam, bg, deg)
    k = oracle.keys(*scene.arrays()[:4], scene.s_min, cam)
    check_keys(view, k)
    _, _, oranges = check_instances(view, k)
    if sample is not None:
        pix = sample_pixels(cam.width, cam.height, sample[0], sample[2], oranges, sample[1], (cam.width + 15) // 16)
    order = oracle.depth_order(k)
    ref = oracle.image(order, *scene.arrays()[:4], scene.s_min, scene.sh, deg, cam, bg, pix)
    err, frac = check_image(image, T, nc, ref, view, cam, frac_max=frac_max, n_blended=view["n_blended"],
                            label=label or f"{scene.n} Gaussians {cam.width}x{cam.height}")
    vis = np.nonzero(k["visible"])[0]
    if vis.size:
        p64 = oracle.project64(vis, *scene.arrays()[:4], scene.s_min, scene.sh, deg, cam)
        check_fp64_fields(view, p64, vis)
    return err, frac, view


def test_small_case_parity(renderer):
    _say("2k Gaussians, 128x128")
    scene, cam, bg = synth.small_forward_case()
    err, frac, view = full_parity(renderer, scene, cam, bg)
    assert view["stats"]["n_instances"] > 1000
    print(f"max err {err:.2e}, flagged {frac:.4%}, K={view['stats']['n_instances']}")


def test_small_case_background(renderer):
    _say("2k Gaussians, 128x128, coloured background")
    scene, cam, _ = synth.small_forward_case()
    full_parity(renderer, scene, cam, np.array([0.3, 0.6, 0.9], np.float32))


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_sh_degrees(renderer, deg):
    _say(f"sh degree {deg}")
    scene, cam, bg = synth.small_forward_case()
    full_parity(renderer, scene, cam, bg, deg=deg)


@pytest.mark.parametrize("W,H", [(100, 75), (17, 33), (1, 1), (255, 129)])
def test_ragged_frames(renderer, W, H):
    _say(f"ragged frame {W}x{H}")
    scene = synth.uniform_scene(3000, seed=40, s_mu=-3.5, s_sigma=0.6)
    cam = synth.look_at_camera((0.7, -0.4, -3.6), (0, 0, 0), W, H)
    full_parity(renderer, scene, cam, np.array([0.05, 0.1, 0.2], np.float32))


def test_large_footprints_near_camera(renderer):
    _say("large footprints near the camera")
    scene = synth.uniform_scene(1500, seed=41, s_mu=-2.0, s_sigma=0.8, extent=2.5)
    cam = synth.look_at_camera((0.0, 0.0, -2.0), (0, 0, 0), 160, 120)
    err, frac, view = full_parity(renderer, scene, cam, np.zeros(3, np.float32))
    k = view["tiles_touched"]
    assert k.max() >= 40   # some Gaussians cover half of the 10x8 tile grid or more


def test_level_scale_floor(renderer):
    _say("s_min = 0.05")
    scene = synth.uniform_scene(1500, seed=42, s_mu=-5.0, s_sigma=0.5, s_min=0.05)
    cam = synth.look_at_camera((0.0, 0.3, -4.0), (0, 0, 0), 96, 96)
    full_parity(renderer, scene, cam, np.zeros(3, np.float32))


def test_empty_level(renderer):
    _say("empty level")
    scene = synth.uniform_scene(0, seed=1)
    cam = synth.look_at_camera((0.0, 0.0, -4.0), (0, 0, 0), 40, 24)
    bg = np.array([0.25, 0.5, 0.75], np.float32)
    image, T, nc, view = gpu_render(renderer, scene, cam, bg)
    assert view["stats"]["n_instances"] == 0
    np.testing.assert_array_equal(image, np.broadcast_to(bg[:, None, None], image.shape))
    assert np.all(T == 1.0) and np.all(nc == 0)


def test_everything_culled(renderer):
    _say("all Gaussians behind the camera")
    scene = synth.uniform_scene(500, seed=43)
    scene.means[:, 2] = -10.0      # camera at z = -4 looks at +z
    cam = synth.look_at_camera((0.0, 0.0, -4.0), (0, 0, 0), 64, 48)
    bg = np.array([0.1, 0.2, 0.3], np.float32)
    image, T, nc, view = gpu_render(renderer, scene, cam, bg)
    assert view["stats"]["n_visible"] == 0 and view["stats"]["n_instances"] == 0
    np.testing.assert_array_equal(image, np.broadcast_to(bg[:, None, None], image.shape))
    assert np.all(T == 1.0) and np.all(nc == 0)


def test_equal_depth_ties(renderer):
    _say("equal-depth ties")
    base = synth.uniform_scene(200, seed=44, s_mu=-2.5)
    rep = synth.Scene(*(np.repeat(a, 3, axis=0) for a in base.arrays()))
    rng = np.random.default_rng(45)
    perm = rng.permutation(rep.n)
    rep = synth.Scene(*(a[perm] for a in rep.arrays()))
    rep.opacity_logits[:] = rng.normal(0, 1, rep.n).astype(np.float32)   # same depth, different looks
    cam = synth.look_at_camera((0.0, 0.0, -4.0), (0, 0, 0), 80, 80)
    full_parity(renderer, rep, cam, np.zeros(3, np.float32))


def test_repeat_bit_identical(renderer):
    _say("10 repeats bit-identical")
    scene, cam, bg = synth.small_forward_case()
    first = gpu_render(renderer, scene, cam, bg)
    for _ in range(9):
        again = gpu_render(renderer, scene, cam, bg)
        for a, b in zip(first[:3], again[:3]):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(first[3]["values"], again[3]["values"])


def test_hd_full_size_sampled(renderer):
    """1M cluster Gaussians at 1920x1080 (the benchmark configuration): the whole key path
    and instance list bit-exact, the image on 4096 uniform pixels plus 512 in the 1% of tiles
    with the longest lists."""
    _say("1M Gaussians, 1920x1080, camera 0")
    scene, cams, bg = synth.hd_forward_case()
    cam = cams[0]
    err, frac, view = full_parity(renderer, scene, cam, bg, sample=(4096, 512, 50), label="1080p / 1M")
    print(f"K={view['stats']['n_instances']} visible={view['stats']['n_visible']} err={err:.2e}")


def test_instance_capacity_growth():
    """A context's frame tail is enqueued before the instance count is read back, sized for the
    instances its buffers hold: a frame with more instances than that grows the buffers and
    runs the tail again. Every frame of a small -> large -> small -> large sequence on one
    context is bit-identical to the same frame on a fresh context, and matches the oracle."""
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    small = synth.uniform_scene(300, seed=60, s_mu=-3.5, s_sigma=0.5)
    large = synth.uniform_scene(4000, seed=61, s_mu=-2.5, s_sigma=0.7)
    cam = synth.look_at_camera((0.3, -0.2, -3.8), (0, 0, 0), 144, 112)
    bg = np.array([0.1, 0.3, 0.5], np.float32)
    shared = render.Renderer(0)
    k_seen = []
    for step, scene in enumerate([small, large, small, large]):
        _say(f"capacity growth frame {step} (n={scene.n})")
        got = gpu_render(shared, scene, cam, bg)
        ref = gpu_render(render.Renderer(0), scene, cam, bg)
        for a, b in zip(got[:3], ref[:3]):
            np.testing.assert_array_equal(a, b)
        K = got[3]["stats"]["n_instances"]
        assert K == ref[3]["stats"]["n_instances"]
        np.testing.assert_array_equal(got[3]["values"], ref[3]["values"])
        np.testing.assert_array_equal(got[3]["tile_ids"], ref[3]["tile_ids"])
        k_seen.append(K)
        if step < 2:
            full_parity(shared, scene, cam, bg)
    assert k_seen[1] > 2 * k_seen[0]   # the second frame outgrows the first frame's buffers


def test_small_frame_after_large_frame():
    """A context keeps the instance capacity of its largest frame, and the sort, emission and
    range kernels launch grids sized for that capacity: after a 1080p / 1M frame (about 8.5M
    instances, so the tile sort takes its large-workgroup path), a 128x128 frame of 2k
    Gaussians on the same context runs with almost every workgroup past the frame's counts.
    It is bit-identical to the same frame on a fresh context and matches the oracle."""
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    shared = render.Renderer(0)
    big, cams, bg_big = synth.hd_forward_case()
    _say("capacity set by 1M Gaussians, 1920x1080")
    k_big = gpu_render(shared, big, cams[0], bg_big)[3]["stats"]["n_instances"]
    assert k_big > 4 << 20
    scene, cam, bg = synth.small_forward_case()
    _say("2k Gaussians, 128x128 on the grown context")
    got = gpu_render(shared, scene, cam, bg)
    ref = gpu_render(render.Renderer(0), scene, cam, bg)
    for a, b in zip(got[:3], ref[:3]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(got[3]["values"], ref[3]["values"])
    np.testing.assert_array_equal(got[3]["tile_ids"], ref[3]["tile_ids"])
    assert got[3]["stats"]["n_instances"] * 1000 < k_big
    full_parity(shared, scene, cam, bg)


def test_count_copy_fallback(monkeypatch):
    """The instance counts reach the host through coherent pinned memory the scan kernel writes,
    or, where that memory is unavailable, through a copy (forced here by FLOD_COUNT_COPY=1 at
    context creation). A small -> large -> small sequence gives bit-identical frames and
    counts both ways."""
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    small = synth.uniform_scene(300, seed=70, s_mu=-3.5, s_sigma=0.5)
    large = synth.uniform_scene(4000, seed=71, s_mu=-2.5, s_sigma=0.7)
    cam = synth.look_at_camera((0.3, -0.2, -3.8), (0, 0, 0), 144, 112)
    bg = np.array([0.2, 0.1, 0.3], np.float32)
    direct = render.Renderer(0)
    monkeypatch.setenv("FLOD_COUNT_COPY", "1")
    copied = render.Renderer(0)
    for step, scene in enumerate([small, large, small]):
        _say(f"count read-back both ways, frame {step} (n={scene.n})")
        a = gpu_render(direct, scene, cam, bg)
        b = gpu_render(copied, scene, cam, bg)
        for x, y in zip(a[:3], b[:3]):
            np.testing.assert_array_equal(x, y)
        for key in ("n_instances", "n_visible"):
            assert a[3]["stats"][key] == b[3]["stats"][key]
        np.testing.assert_array_equal(a[3]["values"], b[3]["values"])


def test_4k_full_size_sampled(renderer):
    """The same 1M cluster scene at 3840x2160, the largest serving resolution (32,400 tiles,
    15-bit tile ids, about four times the 1080p instance count): the whole key path and
    instance list bit-exact, the image on 4096 uniform pixels plus 512 in the 1% of tiles with
    the longest lists."""
    _say("1M Gaussians, 3840x2160")
    scene, _, bg = synth.hd_forward_case()
    cam = synth.orbit_cameras(2, 1, 4.0, 3840, 2160)[0]
    err, frac, view = full_parity(renderer, scene, cam, bg, sample=(4096, 512, 51), label="4K / 1M")
    assert view["stats"]["tiles_x"] * view["stats"]["tiles_y"] == 32400
    print(f"K={view['stats']['n_instances']} visible={view['stats']['n_visible']} err={err:.2e}")


def test_huge_footprints_many_windows(renderer):
    """Coarse-level Gaussians (scale floor 0.2, as level 1 of the stack) at 3840x2160: single
    footprints of thousands of tiles, so one emission workgroup fills hundreds of 4096-instance
    windows. Key path and instance list bit-exact, image on 4096 uniform pixels plus 512 in the
    longest lists."""
    _say("3k level-1 Gaussians, 3840x2160")
    scene = synth.cluster_scene(3000, seed=11, layout_seed=1, s_min=0.2)
    cam = synth.orbit_cameras(2, 1, 4.0, 3840, 2160)[0]
    err, frac, view = full_parity(renderer, scene, cam, np.zeros(3, np.float32), sample=(4096, 512, 52),
                                  label="4K / 3k level-1")
    tt = view["tiles_touched"].astype(np.int64)
    n_wg = -(-int((tt > 0).sum()) // 256)  # emission workgroups (256 Gaussians each)
    assert tt.max() > 4096                 # one footprint alone spans more than one window
    assert tt.sum() / n_wg > 50 * 4096     # a workgroup fills over 50 windows on average
    print(f"K={view['stats']['n_instances']} max footprint {tt.max()} tiles, err={err:.2e}")


def test_max_frame_16384(renderer):
    """The largest frame the API accepts, 16384 x 16384: 1,048,576 tiles, so tile ids take 20
    bits (a third radix pass) and the tile-order kernel spans a million tiles. Key path and
    instance list bit-exact, the image on 4096 uniform pixels plus 512 in the longest lists."""
    _say("2k Gaussians, 16384x16384")
    scene = synth.uniform_scene(2000, seed=53, s_mu=-4.0, s_sigma=0.5)
    cam = synth.look_at_camera((0.4, -0.3, -3.8), (0, 0, 0), 16384, 16384)
    err, frac, view = full_parity(renderer, scene, cam, np.array([0.2, 0.1, 0.4], np.float32),
                                  sample=(4096, 512, 54), label="16384^2 / 2k")
    assert view["stats"]["tiles_x"] * view["stats"]["tiles_y"] == 1 << 20
    assert int(view["tile_ids"].max()) >= 1 << 16       # ids beyond two radix digits
    print(f"K={view['stats']['n_instances']} err={err:.2e}")


def test_context_used_on_two_streams():
    """A context's render on a second stream waits for the first render's frame, still queued on
    the first stream when the call returns, before reusing the buffers: both frames equal the
    same frames rendered on one stream."""
    from paper_2408_12894_amd import render
    _say("one context, two streams back to back")
    scene = synth.cluster_scene(200_000, seed=41, layout_seed=1)
    cams = synth.orbit_cameras(2, 2, 4.0, 1280, 720)
    lv = render.GaussianLevel.from_scene(scene)
    ref_r = render.Renderer(0)
    ref = [ref_r.render_level(lv, c)[0].cpu().numpy() for c in cams]
    r = render.Renderer(0)
    r.render_level(lv, cams[0])          # buffers sized for this frame
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    a = r.render_level(lv, cams[0], stream=sa)[0]
    b = r.render_level(lv, cams[1], stream=sb)[0]
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.cpu().numpy(), ref[0])
    np.testing.assert_array_equal(b.cpu().numpy(), ref[1])



def _min_q_over_boxes(dxa, dxb, dya, dyb, a, b, c):
    """Smallest q = a dx^2 + 2 b dx dy + c dy^2 (positive definite) over the boxes
    [dxa, dxb] x [dya, dyb] of offsets from the mean, FP64, elementwise."""
    def edge_x(dx, lo, hi):      # dx fixed, dy free in [lo, hi]
        dy = np.clip(-b * dx / c, lo, hi)
        return a * dx * dx + 2 * b * dx * dy + c * dy * dy

    def edge_y(dy, lo, hi):
        dx = np.clip(-b * dy / a, lo, hi)
        return a * dx * dx + 2 * b * dx * dy + c * dy * dy

    q = np.minimum(np.minimum(edge_x(dxa, dya, dyb), edge_x(dxb, dya, dyb)),
                   np.minimum(edge_y(dya, dxa, dxb), edge_y(dyb, dxa, dxb)))
    inside = (dxa <= 0) & (dxb >= 0) & (dya <= 0) & (dyb >= 0)
    return np.where(inside, 0.0, q)


@pytest.mark.parametrize("case", ["small", "cluster"])
def test_instance_list_against_fp64_geometry(renderer, case):
    """The GPU's tile lists checked against the FP64 projection directly, not against the FP32
    key mirror. Completeness: for every Gaussian in front of the near plane, every tile holding
    a pixel centre where it blends with a margin (q <= 9 (1 - 1e-4) and o e^{-q/2} >=
    (1 + 1e-4) / 255) lists it. Soundness: a listed tile meets the support, i.e. its band of
    pixel-centre rows (columns over the whole tile) holds a point with q <= Q_g (1 + 1e-2) +
    1e-2, Q_g = min(9, 2 ln(255 o)). Order: along each tile's list the FP64 view depth never
    falls by more than FP32 rounding of it."""
    _say(f"instance list against FP64 geometry ({case})")
    if case == "small":
        scene, cam, bg = synth.small_forward_case()
    else:
        scene = synth.cluster_scene(20_000, seed=44, layout_seed=1)
        cam = synth.orbit_cameras(2, 1, 4.0, 480, 272)[0]
        bg = np.zeros(3, np.float32)
    image, T, nc, view = gpu_render(renderer, scene, cam, bg)
    W, H = cam.width, cam.height
    tx_n = (W + 15) // 16
    tiles, vals = view["tile_ids"].astype(np.int64), view["values"].astype(np.int64)
    assert tiles.size == view["stats"]["n_instances"] > 0
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    tz = scene.means.astype(np.float64) @ R[2] + float(np.asarray(cam.t, np.float64)[2])
    front = np.nonzero(tz > 0.2 * (1 + 1e-6))[0]
    p64 = oracle.project64(front, *scene.arrays()[:4], scene.s_min, scene.sh, 3, cam)
    row = np.full(scene.n, -1, np.int64)
    row[front] = np.arange(front.size)
    listed = {}
    for t, v in zip(tiles.tolist(), vals.tolist()):
        listed.setdefault(v, set()).add(t)
    # completeness over each Gaussian's q <= 9 window of pixel centres
    n_need = 0
    for j, i in enumerate(front):
        mx, my, a, b, c, o = p64[j, :6]
        det = a * c - b * b
        if not (det > 0) or o * 255.0 < 1 + 1e-4:
            continue
        hx, hy = np.sqrt(9 * c / det), np.sqrt(9 * a / det)
        x0, x1 = max(0, int(np.floor(mx - hx - 1))), min(W, int(np.ceil(mx + hx + 1)))
        y0, y1 = max(0, int(np.floor(my - hy - 1))), min(H, int(np.ceil(my + hy + 1)))
        if x0 >= x1 or y0 >= y1:
            continue
        ys, xs = np.mgrid[y0:y1, x0:x1]
        dx, dy = xs + 0.5 - mx, ys + 0.5 - my
        q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        must = (q <= 9.0 * (1 - 1e-4)) & (o * np.exp(-0.5 * q) >= (1 + 1e-4) / 255.0)
        if not must.any():
            continue
        need = set(((ys[must] // 16) * tx_n + xs[must] // 16).tolist())
        n_need += len(need)
        have = listed.get(int(i), set())
        assert need <= have, f"Gaussian {i}: tiles {sorted(need - have)[:5]} missing from its list"
    # soundness of every listed (tile, Gaussian) pair
    j = row[vals]
    assert (j >= 0).all(), "a Gaussian behind the near plane is listed"
    mx, my, a, b, c, o = (p64[j, k] for k in range(6))
    txs, tys = tiles % tx_n, tiles // tx_n
    qmin = _min_q_over_boxes(16.0 * txs - mx, 16.0 * txs + 16 - mx, 16.0 * tys + 0.5 - my,
                             16.0 * tys + 15.5 - my, a, b, c)
    qg = np.minimum(9.0, 2 * np.log(255.0 * o))
    far = qmin > qg * (1 + 1e-2) + 1e-2
    assert not far.any(), f"{int(far.sum())} listed pairs away from the support, e.g. value {vals[far][:3]}"
    # depth order inside every tile
    same = tiles[1:] == tiles[:-1]
    da, db = tz[vals[:-1][same]], tz[vals[1:][same]]
    bad = da > db + 2e-7 * np.abs(db)
    assert not bad.any(), f"{int(bad.sum())} adjacent entries out of depth order"
    print(f"K={tiles.size}, front {front.size}, required pairs {n_need}", flush=True)


def check_blended_lists(view, n_contrib, cam, ref=None):
    """The forward lists, per tile, the entries it blended into some pixel of the tile (the only
    entries the backward walks): (position in the tile's list, Gaussian) pairs in list order at
    the start of the tile's range. Positions rise strictly inside the list, each pair carries the
    list's Gaussian, and every pixel's last blended entry (n_contrib - 1) is listed. With the
    oracle's per-pixel results (ref, all pixels): every unflagged pixel's last blended Gaussian
    is listed, and a tile lists at least as many entries as any one of its unflagged pixels
    blended and at most as many as all its pixels blended together (plus one per flagged pixel,
    whose decisions may flip)."""
    tiles_x, tiles_y = (cam.width + 15) // 16, (cam.height + 15) // 16
    n_tiles = tiles_x * tiles_y
    rg = view["ranges"].astype(np.int64)
    vals = view["values"].astype(np.int64)
    bl = view["blended"].astype(np.int64)
    m = view["tile_blended"].astype(np.int64)
    length = rg[:, 1] - rg[:, 0]
    assert m.shape == (n_tiles,)
    assert np.all(m <= length), "listed count beyond the tile's list"
    # every listed entry, with its tile and its index in the tile's range
    tile_e = np.repeat(np.arange(n_tiles), m)
    k = np.arange(int(m.sum())) - np.repeat(np.cumsum(m) - m, m)
    pos, ids = bl[rg[tile_e, 0] + k, 0], bl[rg[tile_e, 0] + k, 1]
    assert np.all(pos >= 0) and np.all(pos < length[tile_e]), "a position outside its tile's list"
    same = tile_e[1:] == tile_e[:-1]
    assert np.all(np.diff(pos)[same] > 0), "positions not rising within a tile"
    np.testing.assert_array_equal(ids, vals[rg[tile_e, 0] + pos], err_msg="listed Gaussians")
    listed = rg[tile_e, 0] + pos                       # absolute list index of every listed entry
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    tile_px = ((ys // 16) * tiles_x + xs // 16).ravel()
    nc = np.asarray(n_contrib).astype(np.int64).ravel()
    has = nc > 0
    assert np.isin(rg[tile_px[has], 0] + nc[has] - 1, listed).all(), "a pixel's last blended entry is not listed"
    if ref is not None:
        ok = (ref["flag"] & 1) == 0
        ref_tile = (ref["pix"][:, 1] // 16) * tiles_x + ref["pix"][:, 0] // 16
        big = int(max(vals.max(initial=0), ref["last"].max(initial=0))) + 1
        lasts = ok & (ref["last"] >= 0)
        assert np.isin(ref_tile[lasts] * big + ref["last"][lasts], tile_e * big + ids).all(), \
            "the oracle's last blended Gaussian of a pixel is not listed"
        most = np.zeros(n_tiles, np.int64)
        np.maximum.at(most, ref_tile[ok], ref["nblend"][ok].astype(np.int64))
        total = np.zeros(n_tiles, np.int64)
        np.add.at(total, ref_tile, ref["nblend"].astype(np.int64) + (~ok))
        assert np.all(m >= most), "a tile lists fewer entries than one of its pixels blended"
        assert np.all(m <= total), "a tile lists more entries than its pixels blended"


def test_blended_entry_lists(renderer):
    _say("2k Gaussians, 128x128: lists of the blended entries against the oracle")
    scene, cam, bg = synth.small_forward_case()
    _, _, nc, view = gpu_render(renderer, scene, cam, bg)
    k = oracle.keys(*scene.arrays()[:4], scene.s_min, cam)
    ref = oracle.image(oracle.depth_order(k), *scene.arrays()[:4], scene.s_min, scene.sh, 3, cam, bg,
                       oracle.all_pixels(cam.width, cam.height))
    check_blended_lists(view, nc, cam, ref)
    print(f"listed {int(view['tile_blended'].sum())} of K={view['stats']['n_instances']}")


def test_blended_entry_lists_hd(renderer):
    """1080p / 1M: lists spanning several 256-entry batches of the forward."""
    _say("1M Gaussians, 1920x1080, camera 0: lists of the blended entries")
    scene, cams, bg = synth.hd_forward_case()
    _, _, nc, view = gpu_render(renderer, scene, cams[0], bg)
    n = view["ranges"][:, 1].astype(np.int64) - view["ranges"][:, 0]
    assert n.max() > 1024
    check_blended_lists(view, nc, cams[0])
    print(f"listed {int(view['tile_blended'].sum())} of K={view['stats']['n_instances']}, longest list {n.max()}")

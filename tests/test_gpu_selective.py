"""GPU selective rendering (eq. 6 / eq. 7 bands over a multi-level stack) against the oracle.

The GPU indexes candidates over the concatenation of levels l_start..l_end; the oracle's
selection mask covers all levels, so the comparison restricts it to the in-range slice.
"""
import numpy as np
import pytest

import oracle
from paper_2408_12894_amd import synth
from parity import FLAG_FRAC_MAX, check_image, check_instances, check_keys, sample_pixels

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


def small_stack(sizes=(300, 700, 1500, 3000, 5000), seed0=70):
    return [synth.cluster_scene(n, seed=seed0 + l, layout_seed=1, s_mu=-3.0, s_sigma=0.5, a_sigma=1.0,
                                s_min=synth.LEVEL_SMIN[l - 1], shell_radius=3.0)
            for l, n in enumerate(sizes, start=1)]


def concat(levels):
    arrs = [np.concatenate([lv.arrays()[i] for lv in levels]) for i in range(5)]
    smin = np.concatenate([np.full(lv.n, lv.s_min, np.float32) for lv in levels])
    return arrs, smin


def selective_parity(renderer, levels, l_start, l_end, d_proj, centre, cam, bg, pix=None, frac_max=FLAG_FRAC_MAX,
                     sample=None, label=""):
    """sample = (n uniform pixels, n in the 1% longest tile lists of the oracle's list, seed)."""
    from paper_2408_12894_amd import render
    dev = [render.GaussianLevel.from_scene(lv) for lv in levels]
    image, T, nc, counts = renderer.render_selective(dev, l_start, l_end, d_proj, centre, cam, bg, with_counts=True)
    torch.cuda.synchronize()
    view = renderer.view()
    keep_all = oracle.select([lv.means for lv in levels], centre, l_start, l_end, d_proj)
    sizes = [lv.n for lv in levels]
    off = int(sum(sizes[: l_start - 1]))
    in_range = levels[l_start - 1: l_end]
    n_range = int(sum(lv.n for lv in in_range))
    keep = keep_all[off: off + n_range]
    # per-level selected counts
    got_counts = counts.cpu().numpy()
    for l in range(1, len(levels) + 1):
        o = int(sum(sizes[: l - 1]))
        assert got_counts[l - 1] == int(keep_all[o: o + sizes[l - 1]].sum()), l
    arrs, smin = concat(in_range)
    k = oracle.keys(*arrs[:4], smin, cam, keep=keep)
    check_keys(view, k)
    _, _, oranges = check_instances(view, k)
    if sample is not None:
        pix = sample_pixels(cam.width, cam.height, sample[0], sample[2], oranges, sample[1], (cam.width + 15) // 16)
    order = oracle.depth_order(k)
    ref = oracle.image(order, *arrs[:4], smin, arrs[4], 3, cam, bg, pix)
    check_image(image.cpu().numpy(), T.cpu().numpy(), nc.cpu().numpy(), ref, view, cam, frac_max=frac_max,
                label=label or f"selective [{l_start},{l_end}] {cam.width}x{cam.height}")
    return view, got_counts


def test_single_level_range_equals_level_render(renderer):
    from paper_2408_12894_amd import render
    _say("selective [l, l] == render_level(l)")
    levels = small_stack()
    cam = synth.look_at_camera((0.3, -0.2, -3.0), (0, 0, 0), 96, 80)
    dev = [render.GaussianLevel.from_scene(lv) for lv in levels]
    bg = (0.1, 0.0, 0.2)
    for l in (1, 3, 5):
        a = [t.cpu().numpy() for t in renderer.render_level(dev[l - 1], cam, bg)]
        va = renderer.view()
        b = [t.cpu().numpy() for t in renderer.render_selective(dev, l, l, synth.LEVEL_BANDS, cam.campos, cam, bg)]
        vb = renderer.view()
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(va["values"], vb["values"])


@pytest.mark.parametrize("rng_range", [(1, 5), (2, 4), (3, 5), (1, 2), (4, 5)])
def test_per_view_bands(renderer, rng_range):
    _say(f"per-view selective {rng_range}")
    levels = small_stack()
    cam = synth.look_at_camera((0.5, -0.3, -2.5), (0, 0, 0), 128, 96)
    bands = [3.0, 2.5, 2.0, 1.5, 0.0]          # crossing the stack's extent
    view, counts = selective_parity(renderer, levels, *rng_range, bands, cam.campos, cam,
                                    np.array([0.05, 0.05, 0.1], np.float32))
    ls, le = rng_range
    assert counts[ls - 1: le].sum() > 0


def test_predetermined_centre(renderer):
    _say("predetermined centre (mean of camera positions)")
    levels = small_stack()
    cams = [synth.look_at_camera((2.5 * np.sin(t), 0.2, 2.5 * np.cos(t)), (0, 0, 0), 112, 64)
            for t in (0.3, 1.4, 2.9)]
    centre = np.mean([c.campos for c in cams], axis=0).astype(np.float32)
    for cam in cams:
        selective_parity(renderer, levels, 1, 5, [2.0, 1.5, 1.0, 0.6, 0.0], centre, cam, np.zeros(3, np.float32))


def test_eq7_bands_from_focal_length(renderer):
    from paper_2408_12894_amd import render
    _say("eq. 7 bands")
    levels = small_stack()
    cam = synth.look_at_camera((0.0, 0.0, -2.5), (0, 0, 0), 64, 64)
    gamma = 8.0
    d_proj = [render.dproj(lv.s_min, cam.fx, gamma) for lv in levels]
    for l, lv in enumerate(levels):
        assert abs(d_proj[l] - oracle.dproj(lv.s_min, cam.fx, gamma)) <= 1e-6 * d_proj[l]
    selective_parity(renderer, levels, 1, 5, d_proj, cam.campos, cam, np.zeros(3, np.float32))


def test_empty_level_in_range(renderer):
    _say("empty level inside the range")
    levels = small_stack(sizes=(300, 0, 1500, 0, 2000))
    cam = synth.look_at_camera((0.4, 0.1, -2.8), (0, 0, 0), 80, 80)
    selective_parity(renderer, levels, 1, 5, [2.5, 2.0, 1.5, 1.0, 0.0], cam.campos, cam, np.zeros(3, np.float32))


def test_invalid_ranges_rejected(renderer):
    from paper_2408_12894_amd import _lib, render
    _say("invalid level ranges")
    levels = [render.GaussianLevel.from_scene(lv) for lv in small_stack(sizes=(10, 10))]
    cam = synth.look_at_camera((0.0, 0.0, -3.0), (0, 0, 0), 32, 32)
    for ls, le in ((0, 1), (2, 1), (1, 3)):
        with pytest.raises(_lib.FlodError) as e:
            renderer.render_selective(levels, ls, le, [1.0, 0.0], cam.campos, cam)
        assert e.value.status == _lib.FLOD_ERR_INVALID_ARG
    with pytest.raises(_lib.FlodError) as e:
        renderer.render_selective(levels, 1, 2, [-1.0, 0.0], cam.campos, cam)
    assert e.value.status == _lib.FLOD_ERR_INVALID_ARG


def test_full_stack_1080p(renderer):
    """The 5-level stack (40k..2.5M, 4.39M resident) at 1920x1080: selective [1,5] with the
    2/4/8/16 bands around the eye, and the top level alone; key path and instance list
    bit-exact over every candidate, image on 4096 uniform pixels plus 512 in the 1% of tiles
    with the longest lists."""
    _say("5-level stack, 1920x1080, selective [1,5] and level 5 alone")
    levels = synth.level_stack()
    cam = synth.orbit_cameras(2, 1, 4.0, 1920, 1080)[0]
    bg = np.zeros(3, np.float32)
    view, counts = selective_parity(renderer, levels, 1, 5, synth.LEVEL_BANDS, cam.campos, cam, bg,
                                    sample=(4096, 512, 71), label="stack selective [1,5] 1080p")
    print(f"selected per level {counts.tolist()}, K={view['stats']['n_instances']}")
    view, counts = selective_parity(renderer, levels, 5, 5, synth.LEVEL_BANDS, cam.campos, cam, bg,
                                    sample=(4096, 512, 72), label="stack level 5 1080p")
    print(f"level 5 alone: K={view['stats']['n_instances']}")

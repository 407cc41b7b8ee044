"""Predetermined selection set (section Selective Rendering): compacting the eq. 6 selection
around a fixed centre keeps exactly the Gaussians the oracle's band predicate keeps, in
index order, and rendering the stored subset gives the same frames, bit for bit, as
selective rendering of the whole stack around that centre."""
import numpy as np
import pytest

import oracle
from paper_2408_12894_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    scenes = [synth.cluster_scene(n, seed=80 + l, layout_seed=1, s_mu=-3.0, s_sigma=0.5, a_sigma=1.0,
                                  s_min=synth.LEVEL_SMIN[l - 1], shell_radius=3.0)
              for l, n in enumerate((400, 900, 2000, 4000, 6000), start=1)]
    levels = [render.GaussianLevel.from_scene(s) for s in scenes]
    cams = [synth.look_at_camera((2.5 * np.sin(t), 0.3, 2.5 * np.cos(t)), (0, 0, 0), 160, 120)
            for t in (0.2, 1.1, 2.4, 4.0)]
    centre = np.mean([c.campos for c in cams], axis=0).astype(np.float32)
    return render.Renderer(0), scenes, levels, cams, centre


BANDS = [2.0, 1.6, 1.2, 0.8, 0.0]


@pytest.mark.parametrize("rng_range", [(1, 5), (2, 4), (3, 3)])
def test_compaction_matches_band_predicate(setup, rng_range):
    r, scenes, levels, cams, centre = setup
    print(f"[case] compaction {rng_range}", flush=True)
    ls, le = rng_range
    kept = r.select_compact(levels, ls, le, BANDS, centre)
    keep = oracle.select([s.means for s in scenes], centre, ls, le, BANDS)
    off = 0
    for l, s in enumerate(scenes, start=1):
        m = keep[off: off + s.n].astype(bool)
        off += s.n
        if not (ls <= l <= le):
            assert m.sum() == 0
            continue
        g = kept[l - ls]
        assert g.n == int(m.sum()) and g.s_min == s.s_min
        for name, arr in zip(("means", "log_scales", "quats", "opacity_logits", "sh"), s.arrays()):
            np.testing.assert_array_equal(getattr(g, name).cpu().numpy(), arr[m], err_msg=name)


def test_stored_subset_renders_like_selective(setup, tmp_path):
    from paper_2408_12894_amd import render
    r, scenes, levels, cams, centre = setup
    print("[case] stored subset == selective around the same centre", flush=True)
    kept = r.select_compact(levels, 1, 5, BANDS, centre)
    render.save_levels(str(tmp_path / "gsel"), kept)
    stored = render.load_levels(str(tmp_path / "gsel"))
    resident = sum(lv.nbytes() for lv in stored)
    assert resident < sum(lv.nbytes() for lv in levels)
    bg = (0.1, 0.05, 0.0)
    for cam in cams:
        a = [t.cpu().numpy() for t in r.render_selective(levels, 1, 5, BANDS, centre, cam, bg)]
        va = r.view()["values"]
        b = [t.cpu().numpy() for t in r.render_merged(stored, cam, bg)]
        vb = r.view()["values"]
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
        assert va.shape == vb.shape


def test_capacity_and_count_only(setup):
    import ctypes as C
    from paper_2408_12894_amd import _lib
    r, scenes, levels, cams, centre = setup
    print("[case] count-only call and too-small capacity", flush=True)
    arr = (_lib.Level * 5)()
    for i, lv in enumerate(levels):
        arr[i] = lv.c_struct()
    counts = (C.c_int64 * 5)()
    dp = (C.c_float * 5)(*BANDS)
    ce = (C.c_float * 3)(*[float(v) for v in centre])
    st = r.L.flod_select_compact(r.ctx, arr, 5, 1, 5, dp, ce, None, counts, None)
    assert st == _lib.FLOD_OK and sum(counts) > 0
    out = (_lib.Level * 5)()
    small = [torch.empty((1, k), device="cuda") for k in (3, 3, 4, 1, 48)]
    for i in range(5):
        out[i] = _lib.Level(*(t.data_ptr() for t in small), 0, 0.0)   # capacity 0
    st = r.L.flod_select_compact(r.ctx, arr, 5, 1, 5, dp, ce, out, counts, None)
    assert st == _lib.FLOD_ERR_WORKSPACE
    assert r.required_bytes() > 0

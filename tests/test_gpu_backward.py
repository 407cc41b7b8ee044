"""GPU backward parity: hand-written HIP gradients against the oracle's FP64 analytic
gradient (itself pinned by FP64 central differences in test_oracle_pins.py).

Loss: L = sum_p sum_ch w[p,ch] * image[p,ch] with fixed random w (w = 0 on pixels the oracle
flags, on both sides). Tolerance per entry:
    |g_gpu - g_oracle| <= 1e-4 * max(1, |g_oracle|) + 3e-5 * scale
where `scale` (from the oracle) is the sum of the magnitudes of the per-pixel terms that the
entry adds up, carried through the absolute projection Jacobian. The first term is the
1e-4 bar; the second is FP32 summation: each per-pixel term carries the rounding of a
transmittance chain through up to a few hundred contributors (~500 eps = 3e-5), so an entry
that is a small sum of large opposite-signed terms cannot be closer than that. A genuine
error (a wrong sign, a missing term, a wrong clamp) is of the order of the terms themselves.
"""
import numpy as np
import pytest

import oracle
from paper_2408_12894_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4
SUM_TOL = 3e-5
NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


@pytest.fixture(scope="module")
def renderer():
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return render.Renderer(0)


def _say(msg):
    print(f"[case] {msg}", flush=True)


def grad_parity(renderer, scene, cam, bg, deg=3, pix=None, seed=0):
    from paper_2408_12894_amd import render
    level = render.GaussianLevel.from_scene(scene)
    image, final_T, n_contrib = renderer.render_level(level, cam, bg, deg)
    k = oracle.keys(*scene.arrays()[:4], scene.s_min, cam)
    order = oracle.depth_order(k)
    if pix is None:
        pix = oracle.all_pixels(cam.width, cam.height)
    ref = oracle.image(order, *scene.arrays()[:4], scene.s_min, scene.sh, deg, cam, bg, pix)
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(pix.shape[0], 3))
    w[ref["flag"] != 0] = 0.0
    dimg = np.zeros((3, cam.height, cam.width), np.float32)
    dimg[:, pix[:, 1], pix[:, 0]] = w.T.astype(np.float32)
    w64 = dimg[:, pix[:, 1], pix[:, 0]].T.astype(np.float64)      # exactly what the GPU sees
    g = renderer.backward(level, torch.from_numpy(dimg).cuda())
    torch.cuda.synchronize()
    go = oracle.grad(order, *scene.arrays()[:4], scene.s_min, scene.sh, deg, cam, bg, pix, w64, with_scale=True)
    worst = {}
    report = []
    g2d = renderer.view()["grad2d"].T.astype(np.float64)        # [n, 9]
    g2d_names = ("mu_x", "mu_y", "conic_a", "conic_b", "conic_c", "opacity", "red", "green", "blue")
    allowed = GRAD_TOL * np.maximum(1.0, np.abs(go["g2d"])) + SUM_TOL * go["scale"]["g2d"]
    ratio = np.abs(g2d - go["g2d"]) / allowed
    worst["2d"] = float(ratio.max())
    d = np.abs(g2d - go["g2d"])
    report.append(f"2d: max |diff| {d.max():.2e} (max |g| {np.abs(go['g2d']).max():.2e}), "
                  f"over 1e-4: {int((d > GRAD_TOL).sum())}/{d.size}, worst/allowed {ratio.max():.3f}")
    if ratio.max() > 1.0:
        i = np.unravel_index(ratio.argmax(), ratio.shape)
        raise AssertionError(f"2D gradient {g2d_names[i[1]]} of Gaussian {i[0]}: gpu {g2d[i]:.6g} oracle "
                             f"{go['g2d'][i]:.6g} allowed {allowed[i]:.3g}; entries over {(ratio > 1).sum()}")
    for name in NAMES:
        a = g[name].cpu().numpy().astype(np.float64).reshape(scene.n, -1)
        b = go[name].reshape(scene.n, -1)
        sc = go["scale"][name].reshape(scene.n, -1)
        if name == "sh":
            nk = (deg + 1) ** 2
            a = a.reshape(scene.n, 16, 3)[:, :nk].reshape(scene.n, -1)
            b = b.reshape(scene.n, 16, 3)[:, :nk].reshape(scene.n, -1)
            sc = sc.reshape(scene.n, 16, 3)[:, :nk].reshape(scene.n, -1)
            assert np.all(g["sh"].cpu().numpy()[:, nk:] == 0)
        allowed = GRAD_TOL * np.maximum(1.0, np.abs(b)) + SUM_TOL * sc
        ratio = np.abs(a - b) / allowed
        worst[name] = float(ratio.max()) if ratio.size else 0.0
        d = np.abs(a - b)
        if d.size:
            report.append(f"{name}: max |diff| {d.max():.2e} (max |g| {np.abs(b).max():.2e}), "
                          f"over 1e-4: {int((d > GRAD_TOL).sum())}/{d.size}, worst/allowed {ratio.max():.3f}")
        if ratio.size and ratio.max() > 1.0:
            i = np.unravel_index(ratio.argmax(), ratio.shape)
            raise AssertionError(f"{name}{i}: gpu {a[i]:.6g} oracle {b[i]:.6g} |diff| {abs(a[i] - b[i]):.3g} "
                                 f"allowed {allowed[i]:.3g} (scale {sc[i]:.3g}); tensor max |g| "
                                 f"{np.abs(b).max():.3g}; entries over {(ratio > 1).sum()} of {ratio.size}")
    nz = sum(int((np.abs(go[n]) > 1e-6).sum()) for n in NAMES)
    print(f"[grad] {scene.n} Gaussians {cam.width}x{cam.height}, {pix.shape[0]} pixels (flagged "
          f"{(ref['flag'] != 0).mean():.3%}, masked):", flush=True)
    for line in report:
        print(f"[grad]   {line}", flush=True)
    return worst, nz


def test_fd_instance(renderer):
    _say("64 Gaussians, 32x32 (the finite-difference instance)")
    scene, cam, _ = synth.fd_case()
    worst, nz = grad_parity(renderer, scene, cam, np.array([0.2, 0.1, 0.3], np.float32))
    assert nz > 1000
    print(worst)


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_small_scene(renderer, deg):
    _say(f"2k Gaussians, 128x128, sh degree {deg}")
    scene, cam, _ = synth.small_forward_case()
    worst, nz = grad_parity(renderer, scene, cam, np.array([0.1, 0.2, 0.3], np.float32), deg=deg, seed=1)
    print(worst)


def test_ragged_with_scale_floor(renderer):
    _say("3k Gaussians, 100x75, s_min = 0.02")
    scene = synth.uniform_scene(3000, seed=60, s_mu=-4.0, s_sigma=0.6, s_min=0.02)
    cam = synth.look_at_camera((0.6, 0.3, -3.5), (0, 0, 0), 100, 75)
    grad_parity(renderer, scene, cam, np.zeros(3, np.float32), seed=2)


def test_opaque_scene_with_active_clamp(renderer):
    """Opacities from 0.88 to 0.9999 (logits U[2, 9.2]): entries above opacity 0.98 take the
    decision with the 0.99 alpha clamp, and near the centres of those above 0.99 the clamp is
    active (no opacity or q gradient there); the rest take the decision without it."""
    _say("300 opaque Gaussians, 96x80")
    scene = synth.uniform_scene(300, seed=62, s_mu=-1.0, s_sigma=0.3)
    rng = np.random.default_rng(62)
    scene.opacity_logits[:] = rng.uniform(2.0, 9.2, scene.n).astype(np.float32)
    o = 1.0 / (1.0 + np.exp(-scene.opacity_logits.astype(np.float64)))
    assert (o > 0.99).mean() > 0.3 and (o < 0.98).mean() > 0.2
    cam = synth.look_at_camera((0.2, -0.1, -3.8), (0, 0, 0), 96, 80)
    worst, nz = grad_parity(renderer, scene, cam, np.array([0.3, 0.2, 0.1], np.float32), seed=5)
    assert nz > 1000
    print(worst)


def test_training_size_sampled(renderer):
    """500k Gaussians at 1280x720 (the training-step configuration) with the loss restricted
    to 1024 sampled pixels, so the oracle's FP64 gradient stays cheap."""
    _say("500k Gaussians, 1280x720, 1024 sampled pixels")
    scene, _, cam, bg = synth.training_case()
    rng = np.random.default_rng(61)
    pix = np.stack([rng.integers(0, 1280, 1024), rng.integers(0, 720, 1024)], 1).astype(np.int32)
    pix = np.unique(pix, axis=0)
    worst, nz = grad_parity(renderer, scene, cam, bg, pix=pix, seed=3)
    print(worst, nz)


def test_hd_sampled(renderer):
    """The benchmark configuration, 1M cluster Gaussians at 1920x1080 (camera 0), with the loss
    on 1024 sampled pixels."""
    _say("1M Gaussians, 1920x1080, 1024 sampled pixels")
    scene, cams, bg = synth.hd_forward_case()
    rng = np.random.default_rng(64)
    pix = np.stack([rng.integers(0, 1920, 1024), rng.integers(0, 1080, 1024)], 1).astype(np.int32)
    pix = np.unique(pix, axis=0)
    worst, nz = grad_parity(renderer, scene, cams[0], bg, pix=pix, seed=6)
    print(worst, nz)


def test_4k_sampled(renderer):
    """The 1M cluster scene at 3840x2160 (the largest serving resolution) with the loss on 1024
    sampled pixels: the backward's tile order, ranges and atomics at 32,400 tiles."""
    _say("1M Gaussians, 3840x2160, 1024 sampled pixels")
    scene, _, bg = synth.hd_forward_case()
    cam = synth.orbit_cameras(2, 1, 4.0, 3840, 2160)[0]
    rng = np.random.default_rng(62)
    pix = np.stack([rng.integers(0, 3840, 1024), rng.integers(0, 2160, 1024)], 1).astype(np.int32)
    pix = np.unique(pix, axis=0)
    worst, nz = grad_parity(renderer, scene, cam, bg, pix=pix, seed=4)
    print(worst, nz)


def test_max_frame_16384(renderer):
    """The largest frame the API accepts (16384 x 16384, 2^20 tiles) with the loss on 128
    sampled pixels: the backward's million-tile order and its atomics."""
    _say("2k Gaussians, 16384x16384, 128 sampled pixels")
    scene = synth.uniform_scene(2000, seed=53, s_mu=-4.0, s_sigma=0.5)
    cam = synth.look_at_camera((0.4, -0.3, -3.8), (0, 0, 0), 16384, 16384)
    rng = np.random.default_rng(63)
    pix = np.stack([rng.integers(0, 16384, 128), rng.integers(0, 16384, 128)], 1).astype(np.int32)
    pix = np.unique(pix, axis=0)
    worst, nz = grad_parity(renderer, scene, cam, np.array([0.2, 0.1, 0.4], np.float32), pix=pix, seed=5)
    print(worst, nz)


def test_autograd_l1_step(renderer):
    """rasterize() under an L1 loss: torch autograd reaches the HIP backward, and its
    gradients equal Renderer.backward with dL/dimage = sign(I - I_target) / P."""
    from paper_2408_12894_amd import render
    _say("autograd L1 step")
    scene, cam, _ = synth.small_forward_case()
    target = scene.copy()
    target.means = target.means + np.float32(0.01)
    bg = (0.0, 0.0, 0.0)
    tl = render.GaussianLevel.from_scene(target)
    tgt, _, _ = renderer.render_level(tl, cam, bg)
    lv = render.GaussianLevel.from_scene(scene)
    params = [t.clone().requires_grad_(True) for t in (lv.means, lv.log_scales, lv.quats, lv.opacity_logits, lv.sh)]
    img = render.rasterize(*params, cam, scene.s_min, bg, renderer=renderer)
    loss = (img - tgt).abs().mean()
    loss.backward()
    dimg = torch.sign(img.detach() - tgt) / img.numel()
    renderer.render_level(lv, cam, bg)
    g = renderer.backward(lv, dimg)
    for p, name in zip(params, NAMES):
        torch.testing.assert_close(p.grad, g[name], rtol=1e-5, atol=1e-7)
    assert float(params[0].grad.abs().sum()) > 0


def test_backward_after_dropping_the_frame(renderer):
    """The library reads the forward's final_T and n_contrib in the backward. The Renderer holds
    those tensors until its next render, so a caller that drops the frame and allocates and fills
    device memory before the backward gets the same gradients as one that keeps the frame."""
    from paper_2408_12894_amd import render
    _say("backward after the caller dropped the forward's outputs")
    scene, cam, _ = synth.small_forward_case()
    bg = (0.1, 0.2, 0.3)
    lv = render.GaussianLevel.from_scene(scene)
    rng = np.random.default_rng(91)
    dimg = torch.from_numpy(rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)).cuda()
    frame = renderer.render_level(lv, cam, bg)
    ref = {k: v.cpu().numpy() for k, v in renderer.backward(lv, dimg).items()}
    del frame
    renderer.render_level(lv, cam, bg)
    junk = [torch.full((cam.height, cam.width), 1 << 30, dtype=torch.int32, device="cuda") for _ in range(8)]
    got = renderer.backward(lv, dimg)
    torch.cuda.synchronize()
    del junk
    for k in NAMES:
        np.testing.assert_allclose(got[k].cpu().numpy(), ref[k], rtol=1e-4, atol=1e-6, err_msg=k)


def test_backward_after_selective_is_unsupported(renderer):
    from paper_2408_12894_amd import _lib, render
    _say("backward after a selective render")
    scene, cam, _ = synth.small_forward_case()
    lv = render.GaussianLevel.from_scene(scene)
    renderer.render_selective([lv], 1, 1, [0.0], cam.campos, cam)
    renderer._last_level_forward = renderer.generation     # bypass the Python-side guard
    with pytest.raises(_lib.FlodError) as e:
        renderer.backward(lv, torch.zeros((3, cam.height, cam.width), device="cuda"))
    assert e.value.status == _lib.FLOD_ERR_UNSUPPORTED


def test_stage_timing_records_and_changes_nothing():
    """Per-stage device timing (HIP events; the backward blend timed from its own kernel
    dispatch): with every stage timed, a first forward and backward on a context record each
    stage once with a positive time; with only the backward blend timed, only it is recorded.
    Images are bit-identical with and without timing, gradients equal up to the order of the
    atomic sums."""
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _say("stage timing on a forward and backward")
    scene, cam, _ = synth.small_forward_case()
    bg = (0.1, 0.2, 0.3)
    lv = render.GaussianLevel.from_scene(scene)
    rng = np.random.default_rng(90)
    dimg = torch.from_numpy(rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)).cuda()

    def run(r):
        img, T, nc = r.render_level(lv, cam, bg)
        g = r.backward(lv, dimg)
        torch.cuda.synchronize()
        return [img.cpu().numpy(), T.cpu().numpy(), nc.cpu().numpy()], [g[k].cpu().numpy() for k in NAMES]

    plain = run(render.Renderer(0))
    r = render.Renderer(0)
    r.set_timing(True)
    r.stage_times(reset=True)
    timed = run(r)
    st = r.stage_times(reset=True)
    for name, (ms, calls) in st.items():
        assert calls == 1 and ms > 0.0, (name, ms, calls)
    r.set_timing(True, stages=["blend_bwd"])
    only = run(r)
    st = r.stage_times(reset=True)
    for name, (ms, calls) in st.items():
        assert calls == (1 if name == "blend_bwd" else 0), (name, calls)
    assert st["blend_bwd"][0] > 0.0
    for other in (timed, only):
        for a, b in zip(plain[0], other[0]):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(plain[1], other[1]):
            np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-6)


def test_render_without_backward_state():
    """A renderer told not to keep backward state (a server's) renders the same image in less
    workspace, refuses a backward after such a render, and after it is told to keep the state
    again backs the next render with the same gradient as a renderer that always kept it."""
    from paper_2408_12894_amd import _lib, render
    _say("128x128: render without backward state")
    scene, cam, bg = synth.small_forward_case()
    level = render.GaussianLevel.from_scene(scene)
    keep, lean = render.Renderer(0), render.Renderer(0)
    lean.keep_backward_state(False)
    img_k = keep.render_level(level, cam, bg)[0].clone()
    img_l = lean.render_level(level, cam, bg)[0].clone()
    torch.cuda.synchronize()
    assert torch.equal(img_k, img_l)
    assert lean.workspace_bytes() < keep.workspace_bytes()
    dimg = torch.ones((3, cam.height, cam.width), device="cuda") / (3 * cam.height * cam.width)
    with pytest.raises(_lib.FlodError) as e:
        lean.backward(level, dimg)
    assert e.value.status == _lib.FLOD_ERR_UNSUPPORTED
    lean.keep_backward_state(True)
    lean.render_level(level, cam, bg)
    g_l = {k: v.clone() for k, v in lean.backward(level, dimg).items()}
    g_k = keep.backward(level, dimg)
    torch.cuda.synchronize()
    for name in NAMES:
        a, b = g_l[name].cpu().numpy(), g_k[name].cpu().numpy()
        # the same arithmetic; only the order of the FP32 atomic sums may differ
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-5 * max(1e-30, float(np.abs(b).max())), err_msg=name)

"""GPU: the Adam step (C ABI) against the FP64 oracle, and the level-by-level training loop
(Algorithm 1 without densification) on a synthetic target set."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2408_12894_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HP = dict(lr_means=1.6e-4, lr_log_scales=5e-3, lr_quats=1e-3, lr_opacity=5e-2, lr_sh_dc=2.5e-3,
          lr_sh_rest=1.25e-4, beta1=0.9, beta2=0.999, eps=1e-8)
SHAPES = dict(means=(3,), log_scales=(3,), quats=(4,), opacity_logits=(), sh=(16, 3))
NAMES = tuple(SHAPES)


@pytest.fixture(scope="module")
def r():
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return render.Renderer(0)


def _rand_state(n, seed):
    rng = np.random.default_rng(seed)
    p = {k: rng.normal(0, 1, (n,) + s).astype(np.float32) for k, s in SHAPES.items()}
    g = {k: rng.normal(0, 1e-2, (n,) + s).astype(np.float32) for k, s in SHAPES.items()}
    m = {k: rng.normal(0, 1e-2, (n,) + s).astype(np.float32) for k, s in SHAPES.items()}
    v = {k: np.abs(rng.normal(0, 1e-4, (n,) + s)).astype(np.float32) for k, s in SHAPES.items()}
    return p, g, m, v


def _gpu_adam(r, p, g, m, v, n, t, hp, offset=0):
    """Run flod_adam_step on device copies; offset > 0 places every array `offset` floats into
    its buffer (not 16-byte aligned: the scalar path)."""
    from paper_2408_12894_amd import _lib

    def dev(a):
        flat = np.ascontiguousarray(a, np.float32).ravel()
        buf = torch.zeros(flat.size + offset, dtype=torch.float32, device="cuda")
        buf[offset:] = torch.from_numpy(flat).cuda()
        return buf, buf[offset:]

    keep, views = [], {}
    for name, d in (("p", p), ("g", g), ("m", m), ("v", v)):
        views[name] = {}
        for k in NAMES:
            buf, view = dev(d[k])
            keep.append(buf)
            views[name][k] = view
    st = {x: _lib.LevelState(*(views[x][k].data_ptr() for k in NAMES)) for x in ("p", "m", "v")}
    gs = _lib.Grads(*(views["g"][k].data_ptr() for k in NAMES))
    hpc = _lib.AdamParams(hp["lr_means"], hp["lr_log_scales"], hp["lr_quats"], hp["lr_opacity"], hp["lr_sh_dc"],
                          hp["lr_sh_rest"], hp["beta1"], hp["beta2"], hp["eps"], int(t))
    _lib.check(r.L.flod_adam_step(r.ctx, C.byref(st["p"]), C.byref(gs), C.byref(st["m"]), C.byref(st["v"]), n,
                                  C.byref(hpc), None), "flod_adam_step")
    torch.cuda.synchronize()
    out = {x: {k: views[x][k].cpu().numpy().reshape((n,) + SHAPES[k]) for k in NAMES} for x in ("p", "m", "v")}
    return out["p"], out["m"], out["v"]


def _check(p, g, m, v, gp, gm, gv, t, hp):
    """FP32 kernel vs FP64 oracle: moments within a few FP32 roundings of their two terms; the
    parameter within 2 ulp plus a 1e-5 relative error of its update, where the update's error
    bound carries the moments' rounding through m / sqrt(v)."""
    n = p["means"].shape[0]
    hp = {k: float(np.float32(x)) for k, x in hp.items()}   # the FP32 values the kernel receives
    op, om, ov = oracle.adam.level_step(p, g, m, v, t, hp)
    lr = oracle.adam.group_rates(n, hp)
    b1, b2 = hp["beta1"], hp["beta2"]
    for k in NAMES:
        m_scale = b1 * np.abs(m[k].astype(np.float64)) + (1 - b1) * np.abs(g[k].astype(np.float64))
        v_scale = b2 * np.abs(v[k].astype(np.float64)) + (1 - b2) * g[k].astype(np.float64) ** 2
        assert np.all(np.abs(gm[k] - om[k]) <= 4e-7 * m_scale + 1e-45), k
        assert np.all(np.abs(gv[k] - ov[k]) <= 4e-7 * v_scale + 1e-45), k
        mh = om[k] / (1 - b1 ** t)
        den = np.sqrt(ov[k] / (1 - b2 ** t)) + hp["eps"]
        upd_err = np.asarray(lr[k]) * (1e-5 * np.abs(mh) + 1e-6 * m_scale / (1 - b1 ** t)) / den
        ulp = np.spacing(np.abs(op[k]).astype(np.float32)).astype(np.float64)
        err = np.abs(gp[k].astype(np.float64) - op[k])
        assert np.all(err <= 2 * ulp + upd_err), (k, float((err - 2 * ulp - upd_err).max()))


@pytest.mark.parametrize("n", [1, 5, 1003, 65537])
def test_adam_step_parity(r, n):
    print(f"[case] adam step n={n}", flush=True)
    p, g, m, v = _rand_state(n, seed=n)
    gp, gm, gv = _gpu_adam(r, p, g, m, v, n, 7, HP)
    _check(p, g, m, v, gp, gm, gv, 7, HP)


def test_adam_step_unaligned_arrays(r):
    print("[case] adam step, arrays offset by one float (scalar path)", flush=True)
    n = 777
    p, g, m, v = _rand_state(n, seed=3)
    gp, gm, gv = _gpu_adam(r, p, g, m, v, n, 3, HP, offset=1)
    _check(p, g, m, v, gp, gm, gv, 3, HP)
    ap, am, av = _gpu_adam(r, p, g, m, v, n, 3, HP, offset=0)
    for k in NAMES:   # the vector and scalar paths compute the same expressions
        np.testing.assert_array_equal(gp[k], ap[k])
        np.testing.assert_array_equal(gm[k], am[k])
        np.testing.assert_array_equal(gv[k], av[k])


def test_adam_first_step_group_rates(r):
    # unit gradients from rest at t = 1: every element moves by its group's rate (eps tiny)
    print("[case] adam group rates", flush=True)
    n = 9
    hp = dict(HP, eps=1e-20)
    p = {k: np.zeros((n,) + s, np.float32) for k, s in SHAPES.items()}
    g = {k: -np.ones((n,) + s, np.float32) for k, s in SHAPES.items()}
    gp, _, _ = _gpu_adam(r, p, g, p, p, n, 1, hp)
    lr = oracle.adam.group_rates(n, {k: float(np.float32(x)) for k, x in hp.items()})
    for k in NAMES:
        np.testing.assert_allclose(gp[k], np.broadcast_to(lr[k], gp[k].shape), rtol=3e-7, err_msg=k)


def test_adam_step_empty_and_bad_args(r):
    from paper_2408_12894_amd import _lib
    print("[case] adam step n=0 and argument checks", flush=True)
    st, gs = _lib.LevelState(), _lib.Grads()
    hp = _lib.AdamParams(1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 0.9, 0.999, 1e-15, 1)
    assert r.L.flod_adam_step(r.ctx, C.byref(st), C.byref(gs), C.byref(st), C.byref(st), 0, C.byref(hp),
                              None) == _lib.FLOD_OK
    assert r.L.flod_adam_step(r.ctx, C.byref(st), C.byref(gs), C.byref(st), C.byref(st), 4, C.byref(hp),
                              None) == _lib.FLOD_ERR_INVALID_ARG
    for field, val in (("step", 0), ("beta1", 1.0), ("beta2", -0.1), ("eps", -1.0), ("lr_quats", float("nan"))):
        bad = _lib.AdamParams(1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 0.9, 0.999, 1e-15, 1)
        setattr(bad, field, val)
        assert r.L.flod_adam_step(r.ctx, C.byref(st), C.byref(gs), C.byref(st), C.byref(st), 0, C.byref(bad),
                                  None) == _lib.FLOD_ERR_INVALID_ARG, field


def test_level_by_level_training(r):
    """Three levels (eq. 3 floors 0.2, 0.05, 0) fitted to renders of a synthetic scene from six
    views: the loss falls within every level, the last level fits better than the first,
    overlap pruning removes Gaussians at level 1, and each eq. 5 hand-over renders as the
    trained level did."""
    from paper_2408_12894_amd import fit, render
    print("[case] level-by-level training, 3 levels, 1500 Gaussians, 6 views 128x128", flush=True)
    gt = synth.uniform_scene(1500, seed=70, s_mu=-3.8, s_sigma=0.5, a_sigma=1.0)
    cams = synth.orbit_cameras(71, 6, 4.0, 128, 128)
    gt_level = render.GaussianLevel.from_scene(gt)
    targets = [r.render_level(gt_level, c)[0].clone() for c in cams]
    rng = np.random.default_rng(72)
    init = render.GaussianLevel.from_arrays(
        gt.means + rng.normal(0, 0.03, gt.means.shape), gt.log_scales + rng.normal(0, 0.3, gt.log_scales.shape),
        gt.quats, np.zeros(gt.n), gt.sh + rng.normal(0, 0.1, gt.sh.shape))
    levels, logs = fit.fit_levels(r, init, cams, targets, l_max=3, iters=[60, 60, 80], prune_every=20,
                                  prune_until=[40, 40, 0], seed=73)
    assert [lv.s_min for lv in levels] == [np.float32(0.2), np.float32(0.05), 0.0]
    first_last = []
    for lg in logs:
        loss = torch.stack(lg.losses).cpu().numpy()
        assert np.all(np.isfinite(loss))
        first_last.append((loss[:10].mean(), loss[-10:].mean()))
        print(f"level {lg.level}: s_min {lg.s_min:.4f} n {lg.n_start}->{lg.n_end} pruned {lg.pruned} "
              f"loss {loss[:10].mean():.4f} -> {loss[-10:].mean():.4f}", flush=True)
        assert loss[-10:].mean() < loss[:10].mean()
    assert first_last[-1][1] < first_last[0][1]
    assert logs[0].pruned > 0 and levels[0].n == gt.n - logs[0].pruned
    assert logs[2].pruned == 0     # no overlap pruning at the max level
    for lv in levels:
        for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            assert torch.isfinite(getattr(lv, k)).all()
    # eq. 5 hand-over: the next level's first render equals the trained level's render
    for l in (0, 1):
        nxt = r.level_transition(levels[l], levels[l + 1].s_min)
        a = r.render_level(levels[l], cams[0])[0].cpu().numpy()
        b = r.render_level(nxt, cams[0])[0].cpu().numpy()
        diff = np.abs(a - b).max(axis=0)
        print(f"[hand-over] level {l + 1} -> {l + 2}: pixels over 1e-4 {(diff > 1e-4).mean():.3%}, "
              f"max {diff.max():.2e}, mean {diff.mean():.2e}", flush=True)
        assert (diff > 1e-4).mean() <= 1e-3 and diff.max() <= 0.05

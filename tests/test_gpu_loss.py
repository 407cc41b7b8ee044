"""L1 + SSIM loss on the device against the FP64 numpy oracle (values and gradients)."""
import ctypes as C

import numpy as np
import pytest

from oracle import ssim as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def r():
    from paper_2408_12894_amd import render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return render.Renderer(0)


def _pair(shape, seed, close=False):
    rng = np.random.default_rng(seed)
    x = rng.random(shape).astype(np.float32)
    y = (x + rng.normal(0, 0.05, shape)).astype(np.float32) if close else rng.random(shape).astype(np.float32)
    return x, y


def _run(r, x, y, lam=0.2, scale=None):
    from paper_2408_12894_amd import render
    xt = torch.as_tensor(x).cuda().requires_grad_(True)
    yt = torch.as_tensor(y).cuda()
    loss = render.l1_ssim_loss(xt, yt, lam, renderer=r)
    (loss * scale if scale is not None else loss).backward()
    return float(loss.item()), xt.grad.cpu().numpy().astype(np.float64)


def _check(x, y, loss, grad, lam=0.2, scale=1.0):
    lam = float(np.float32(lam))          # the library takes lambda as FP32
    ref = S.loss(x, y, lam)
    assert abs(loss - ref) <= 1e-12 * max(1.0, abs(ref)), (loss, ref)
    g = S.loss_grad(x, y, lam) * scale
    tol = 1e-5 * np.abs(g).max() + 1e-6 * np.abs(g)
    bad = np.abs(grad - g) > tol
    assert not bad.any(), (np.argwhere(bad)[:5], grad[bad][:5], g[bad][:5])


@pytest.mark.parametrize("shape,seed,close", [((3, 40, 53), 0, False), ((3, 67, 45), 1, True),
                                              ((1, 16, 16), 2, True), ((3, 7, 5), 3, False),
                                              ((3, 1, 1), 4, False), ((2, 33, 129), 5, True)])
def test_loss_and_gradient(r, shape, seed, close):
    print(f"[case] l1+ssim {shape} seed={seed}", flush=True)
    x, y = _pair(shape, seed, close)
    loss, grad = _run(r, x, y)
    _check(x, y, loss, grad)


@pytest.mark.parametrize("lam", [0.0, 1.0, 0.5])
def test_weights_and_upstream_scale(r, lam):
    print(f"[case] l1+ssim lam={lam}", flush=True)
    x, y = _pair((3, 50, 61), 9, True)
    loss, grad = _run(r, x, y, lam, scale=3.0)
    _check(x, y, loss, grad, lam, scale=3.0)


def test_identical_images(r):
    print("[case] l1+ssim identical", flush=True)
    x, _ = _pair((3, 48, 64), 11)
    loss, grad = _run(r, x, x.copy())
    assert loss == 0.0
    assert np.abs(grad).max() <= 1e-12


def test_full_hd(r):
    print("[case] l1+ssim 1920x1080", flush=True)
    x, y = _pair((3, 1080, 1920), 12, True)
    loss, grad = _run(r, x, y)
    _check(x, y, loss, grad)


def test_forward_only_and_argument_checks(r):
    from paper_2408_12894_amd import _lib
    print("[case] l1+ssim forward only, argument checks", flush=True)
    x, y = _pair((3, 20, 30), 13)
    xt, yt = torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda()
    loss = torch.empty((), dtype=torch.float64, device="cuda")
    st = r.L.flod_l1_ssim_forward(r.ctx, xt.data_ptr(), yt.data_ptr(), 3, 20, 30, 0.2, loss.data_ptr(), None, None)
    torch.cuda.synchronize()
    assert st == _lib.FLOD_OK and abs(loss.item() - S.loss(x, y, float(np.float32(0.2)))) <= 1e-12
    assert r.L.flod_l1_ssim_forward(r.ctx, xt.data_ptr(), yt.data_ptr(), 3, 20, 30, 1.5, loss.data_ptr(), None,
                                    None) == _lib.FLOD_ERR_INVALID_ARG
    assert r.L.flod_l1_ssim_forward(r.ctx, xt.data_ptr(), yt.data_ptr(), 0, 20, 30, 0.2, loss.data_ptr(), None,
                                    None) == _lib.FLOD_ERR_INVALID_ARG


@pytest.mark.parametrize("n", [1, 7, 4096, 3 * 1080 * 1920 + 3])
def test_plain_l1(r, n):
    from paper_2408_12894_amd import render
    print(f"[case] l1 n={n}", flush=True)
    rng = np.random.default_rng(n)
    x = rng.random(n).astype(np.float32)
    y = rng.random(n).astype(np.float32)
    y[::5] = x[::5]                                   # ties: zero gradient
    xt = torch.as_tensor(x).cuda().requires_grad_(True)
    loss = render.l1_loss(xt, torch.as_tensor(y).cuda(), renderer=r)
    (loss * 2.0).backward()
    d = x.astype(np.float64) - y.astype(np.float64)
    ref = np.abs(x - y).astype(np.float64).mean()
    assert abs(loss.item() - ref) <= 1e-12 * max(ref, 1e-30)
    g = xt.grad.cpu().numpy()
    np.testing.assert_array_equal(g, (np.sign(d) * np.float32(2.0 / n)).astype(np.float32))

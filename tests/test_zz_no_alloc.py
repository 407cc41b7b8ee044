"""The allocation-free L1 + SSIM forward (flod_l1_ssim_forward_noalloc) against the allocating
flod_l1_ssim_forward, through the C ABI: same loss and derivative maps bit for bit (both are
deterministic, fixed-order reductions of the same kernels), on two calls in a row, the second
with a smaller image, with no change in the device's free memory across the calls; inputs
beyond the fixed scratch are refused before any launch."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _vp(t):
    return C.c_void_p(t.data_ptr())


def test_noalloc_forward_matches_allocating_forward():
    from paper_2408_12894_amd import _lib, render
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    r = render.Renderer(0)
    L = r.L
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(41)
    shapes = [(3, 270, 481), (3, 67, 45)]         # the second call is smaller
    bufs = []
    for (ch, h, w) in shapes:
        x = torch.as_tensor(rng.random((ch, h, w), dtype=np.float32)).cuda()
        y = (x + torch.as_tensor(rng.normal(0, 0.05, (ch, h, w)).astype(np.float32)).cuda()).contiguous()
        bufs.append(dict(x=x, y=y,
                         loss_a=torch.zeros(1, dtype=torch.float64, device="cuda"),
                         loss_b=torch.full((1,), -1.0, dtype=torch.float64, device="cuda"),
                         dm_a=torch.zeros((3, ch, h, w), dtype=torch.float32, device="cuda"),
                         dm_b=torch.full((3, ch, h, w), -7.0, dtype=torch.float32, device="cuda")))
    # the allocating entry point first: its workspace and every lazy initialisation exist
    # before the free-memory reading
    for (ch, h, w), b in zip(shapes, bufs):
        print(f"[case] allocating l1+ssim forward {ch}x{h}x{w}", flush=True)
        _lib.check(L.flod_l1_ssim_forward(r.ctx, _vp(b["x"]), _vp(b["y"]), ch, h, w, C.c_float(0.2),
                                          _vp(b["loss_a"]), _vp(b["dm_a"]), stream), "flod_l1_ssim_forward")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for (ch, h, w), b in zip(shapes, bufs):
        print(f"[case] allocation-free l1+ssim forward {ch}x{h}x{w}", flush=True)
        _lib.check(L.flod_l1_ssim_forward_noalloc(r.ctx, _vp(b["x"]), _vp(b["y"]), ch, h, w, C.c_float(0.2),
                                                  _vp(b["loss_b"]), _vp(b["dm_b"]), stream),
                   "flod_l1_ssim_forward_noalloc")
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    for (ch, h, w), b in zip(shapes, bufs):
        la, lb = b["loss_a"].cpu().numpy(), b["loss_b"].cpu().numpy()
        assert la[0] == lb[0], ((ch, h, w), la, lb)
        assert torch.equal(b["dm_a"], b["dm_b"]), (ch, h, w)
        assert 0.0 < la[0] < 1.0
    # without derivative maps (loss only)
    b = bufs[1]
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    _lib.check(L.flod_l1_ssim_forward_noalloc(r.ctx, _vp(b["x"]), _vp(b["y"]), 3, 67, 45, C.c_float(0.2),
                                              _vp(out), None, stream), "flod_l1_ssim_forward_noalloc")
    torch.cuda.synchronize()
    assert out.item() == b["loss_a"].item()
    # beyond the fixed scratch: refused on the host before any launch (3 x 7680 x 4320 is
    # 388,800 workgroups against 262,144); the loss stays untouched
    st = L.flod_l1_ssim_forward_noalloc(r.ctx, _vp(b["x"]), _vp(b["y"]), 3, 4320, 7680, C.c_float(0.2),
                                        _vp(out), None, stream)
    assert st == _lib.FLOD_ERR_TOO_LARGE
    torch.cuda.synchronize()
    assert out.item() == b["loss_a"].item()
    r.close()

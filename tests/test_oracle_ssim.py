"""Pins of the L1 + SSIM loss oracle against independent computations: scipy's Gaussian
filter for the window and padding, closed forms for constant and scaled images, direct
2D summation on a tiny image, and FP64 central differences for the gradient."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle import ssim as S


def _gf(z):
    # scipy's separable Gaussian: radius int(truncate * sigma + 0.5) = 5, normalised, zeros outside
    return ndimage.gaussian_filter(np.asarray(z, np.float64), S.SIGMA, truncate=5.0 / S.SIGMA, mode="constant",
                                   cval=0.0)


def test_window_and_padding_match_scipy():
    x = np.random.default_rng(0).random((37, 29))
    np.testing.assert_allclose(S.filt(x), _gf(x), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(S.window_1d().sum(), 1.0, rtol=1e-15)


def test_identical_images_score_one():
    x = np.random.default_rng(1).random((3, 30, 40))
    np.testing.assert_allclose(S.ssim_map(x, x), 1.0, rtol=1e-13)
    assert abs(S.loss(x, x)) < 1e-13


def test_constant_images_interior_closed_form():
    a, b = 0.3, 0.7
    x = np.full((1, 24, 24), a)
    y = np.full((1, 24, 24), b)
    m = S.ssim_map(x, y)[0, 5:-5, 5:-5]
    np.testing.assert_allclose(m, (2 * a * b + S.C1) / (a * a + b * b + S.C1), rtol=1e-12)


def test_scaled_image_closed_form():
    rng = np.random.default_rng(2)
    x = rng.random((2, 26, 31))
    s = 0.6
    y = s * x
    mu = np.stack([_gf(c) for c in x])
    var = np.stack([_gf(c * c) for c in x]) - mu * mu
    ref = ((2 * s * mu * mu + S.C1) * (2 * s * var + S.C2)) / \
          (((1 + s * s) * mu * mu + S.C1) * ((1 + s * s) * var + S.C2))
    np.testing.assert_allclose(S.ssim_map(x, y), ref, rtol=1e-9, atol=1e-12)


def test_direct_summation_tiny():
    rng = np.random.default_rng(3)
    x, y = rng.random((2, 9, 10)), rng.random((2, 9, 10))
    g = S.window_1d()
    H, W = 9, 10
    out = np.zeros((2, H, W))
    for c in range(2):
        for i in range(H):
            for j in range(W):
                acc = np.zeros(5)
                for di in range(-5, 6):
                    for dj in range(-5, 6):
                        u, v = i + di, j + dj
                        if 0 <= u < H and 0 <= v < W:
                            w = g[di + 5] * g[dj + 5]
                            xv, yv = x[c, u, v], y[c, u, v]
                            acc += w * np.array([xv, yv, xv * xv, yv * yv, xv * yv])
                mx, my, exx, eyy, exy = acc
                vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
                out[c, i, j] = ((2 * mx * my + S.C1) * (2 * cxy + S.C2)) / \
                               ((mx * mx + my * my + S.C1) * (vx + vy + S.C2))
    np.testing.assert_allclose(S.ssim_map(x, y), out, rtol=1e-11)


def test_loss_weighting():
    rng = np.random.default_rng(4)
    x, y = rng.random((3, 12, 13)), rng.random((3, 12, 13))
    np.testing.assert_allclose(S.loss(x, y, lam=0.0), np.abs(x - y).mean(), rtol=1e-14)
    np.testing.assert_allclose(S.loss(x, y, lam=1.0), 1.0 - S.ssim(x, y), rtol=1e-14)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_gradient_central_differences(lam):
    rng = np.random.default_rng(5)
    x, y = rng.random((3, 14, 17)), rng.random((3, 14, 17))
    g = S.loss_grad(x, y, lam)
    h = 1e-6
    for idx in [tuple(rng.integers(0, s) for s in x.shape) for _ in range(40)] + [(0, 0, 0), (2, 13, 16)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (S.loss(xp, y, lam) - S.loss(xm, y, lam)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(g[idx])) + 1e-9, (idx, fd, g[idx])


def test_oracle_package_exports_ssim():
    assert oracle.ssim is S

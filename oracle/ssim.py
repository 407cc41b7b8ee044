"""CPU oracle for the training loss: L1 plus SSIM (section Implementation: the loss follows
the backbone 3DGS model, which combines L1 with the SSIM of Wang et al. 2004).

TEST INFRASTRUCTURE ONLY (same rules as the rest of `oracle/`). Plain numpy in FP64.

Definition (the readings it fixes are the backbone's conventions; the paper only names the
losses):
  window   w = g g^T, g_k = exp(-(k - 5)^2 / (2 * 1.5^2)) / sum, k = 0..10 (11 x 11, sigma 1.5)
  filter   F(z)[p] = sum_q w[q - p + 5] z[q] over the image, zeros outside it ("same" size)
  moments  per channel: mu_x = F(x), mu_y = F(y), s_xx = F(x x) - mu_x^2,
           s_yy = F(y y) - mu_y^2, s_xy = F(x y) - mu_x mu_y
  map      S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)),
           C1 = 0.01^2, C2 = 0.03^2
  SSIM     mean of S over channels and pixels
  loss     (1 - lam) mean|x - y| + lam (1 - SSIM), lam = 0.2; d|t|/dt = sign(t), 0 at t = 0
The gradient with respect to x follows from the chain rule through the five windowed
moments; the filter is its own adjoint (the window is symmetric).
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WINDOW = 11
SIGMA = 1.5
LAMBDA = 0.2


def window_1d(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    k = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def filt(z: np.ndarray, g: np.ndarray | None = None) -> np.ndarray:
    """Separable window over the last two axes, zero outside the image, same size."""
    g = window_1d() if g is None else g
    r = len(g) // 2
    z = np.asarray(z, np.float64)
    H, W = z.shape[-2:]
    p = np.pad(z, [(0, 0)] * (z.ndim - 2) + [(r, r), (r, r)])
    h = sum(g[k] * p[..., :, k:k + W] for k in range(len(g)))
    return sum(g[k] * h[..., k:k + H, :] for k in range(len(g)))


def moments(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = filt(x), filt(y)
    return mx, my, filt(x * x), filt(y * y), filt(x * y)


def ssim_map(x, y) -> np.ndarray:
    mx, my, exx, eyy, exy = moments(x, y)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim(x, y) -> float:
    return float(ssim_map(x, y).mean())


def loss(x, y, lam: float = LAMBDA) -> float:
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return float((1 - lam) * np.abs(x - y).mean() + lam * (1.0 - ssim(x, y)))


def loss_grad(x, y, lam: float = LAMBDA) -> np.ndarray:
    """d loss / d x, same shape as x, FP64."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = x.size
    mx, my, exx, eyy, exy = moments(x, y)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    A = 2 * mx * my + C1
    B = 2 * sxy + C2
    Cc = mx * mx + my * my + C1
    D = sxx + syy + C2
    S = (A * B) / (Cc * D)
    # partials of S with respect to the moments mu_x, E[xx], E[xy] (mu_y, E[yy] are constants)
    d_exx = -S / D
    d_exy = 2 * A / (Cc * D)
    d_mx = 2 * my * B / (Cc * D) - 2 * mx * S / Cc + 2 * mx * S / D - 2 * my * A / (Cc * D)
    c = -lam / n                                     # d loss / d S at every map entry
    g = c * (filt(d_mx) + 2 * x * filt(d_exx) + y * filt(d_exy))
    return g + (1 - lam) * np.sign(x - y) / n

"""CPU oracle for the optimiser step of the per-level training loop (section Training Method,
Algorithm 1: each iteration rasterizes, takes the loss and applies an Adam update to the
means, scale parameters s_opt, rotations, colours and opacities).

TEST INFRASTRUCTURE ONLY (same rules as the rest of `oracle/`). Plain numpy in FP64.

The update is Adam as Kingma and Ba (2015) define it, with the bias-corrected moments:
  m_t = beta1 m_{t-1} + (1 - beta1) g_t
  v_t = beta2 v_{t-1} + (1 - beta2) g_t^2
  p_t = p_{t-1} - lr * (m_t / (1 - beta1^t)) / (sqrt(v_t / (1 - beta2^t)) + eps)
The learning rate is chosen per attribute group: means, log_scales, quats, opacity logits,
SH degree-0 coefficients (row 0 of each Gaussian's [16,3] block) and the other SH rows.
"""
from __future__ import annotations

import numpy as np

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def step(p, g, m, v, t: int, lr, beta1: float, beta2: float, eps: float):
    """One Adam step on arrays of any shape; lr may be a scalar or broadcastable array.
    Returns (p_t, m_t, v_t) in FP64."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return p - np.asarray(lr, np.float64) * m_hat / (np.sqrt(v_hat) + eps), m, v


def group_rates(n: int, hp: dict) -> dict:
    """Per-element learning rates for an n-Gaussian level, shaped like its arrays."""
    sh = np.full((n, 16, 3), hp["lr_sh_rest"], np.float64)
    sh[:, 0, :] = hp["lr_sh_dc"]
    return {"means": hp["lr_means"], "log_scales": hp["lr_log_scales"], "quats": hp["lr_quats"],
            "opacity_logits": hp["lr_opacity"], "sh": sh}


def level_step(params: dict, grads: dict, m: dict, v: dict, t: int, hp: dict):
    """Adam over every attribute array of a level (dicts keyed by GROUPS).
    Returns new (params, m, v) dicts in FP64."""
    n = int(np.asarray(params["means"]).shape[0])
    lr = group_rates(n, hp)
    out_p, out_m, out_v = {}, {}, {}
    for k in GROUPS:
        out_p[k], out_m[k], out_v[k] = step(params[k], grads[k], m[k], v[k], t, lr[k], hp["beta1"],
                                            hp["beta2"], hp["eps"])
    return out_p, out_m, out_v

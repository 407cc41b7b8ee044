"""Pins of the Adam oracle (oracle/adam.py) against closed forms of Kingma and Ba's update.

A dropped (1 - beta) factor, a bias correction with the wrong power, a missing square root or
a group learning rate applied to the wrong SH row fails one of these."""
import numpy as np
import pytest

from oracle import adam

HP = dict(lr_means=1.6e-4, lr_log_scales=5e-3, lr_quats=1e-3, lr_opacity=5e-2, lr_sh_dc=2.5e-3,
          lr_sh_rest=1.25e-4, beta1=0.9, beta2=0.999, eps=1e-15)


def test_first_step_moves_by_lr_times_sign():
    # t = 1 from zero moments: m_hat = g and v_hat = g^2 exactly, so the step is lr g / (|g| + eps)
    g = np.array([3.0, -0.25, 1e-3, -7e5])
    p0 = np.array([1.0, 2.0, -3.0, 0.5])
    p, m, v = adam.step(p0, g, np.zeros(4), np.zeros(4), 1, 0.01, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(p, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-13)


@pytest.mark.parametrize("t_max", [2, 5, 40])
def test_constant_gradient_steps_are_equal(t_max):
    # with g constant from zero moments, m_t = g (1 - b1^t) and v_t = g^2 (1 - b2^t): the bias
    # corrections make every step exactly lr g / (|g| + eps)
    g = np.array([0.5, -2.0])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, t_max + 1):
        p, m, v = adam.step(p, g, m, v, t, 0.1, 0.9, 0.999, 0.0)
        np.testing.assert_allclose(m, g * (1 - 0.9 ** t), rtol=1e-12)
        np.testing.assert_allclose(v, g * g * (1 - 0.999 ** t), rtol=1e-12)
    np.testing.assert_allclose(p, -0.1 * t_max * np.sign(g), rtol=1e-12)


def test_two_step_hand_example():
    # g1 = 1, g2 = -1, beta1 = 0.9, beta2 = 0.999, eps = 0, lr = 1:
    #   m2 = 0.9 * 0.1 - 0.1 = -0.01,   m_hat = -0.01 / (1 - 0.81) = -1/19
    #   v2 = 0.999 * 0.001 + 0.001 = 0.001999,   v_hat = 0.001999 / (1 - 0.998001) = 1
    p, m, v = adam.step(0.0, 1.0, 0.0, 0.0, 1, 1.0, 0.9, 0.999, 0.0)
    assert p == pytest.approx(-1.0, abs=1e-15)
    p, m, v = adam.step(p, -1.0, m, v, 2, 1.0, 0.9, 0.999, 0.0)
    assert m == pytest.approx(-0.01, rel=1e-13)
    assert v == pytest.approx(0.001999, rel=1e-13)
    assert p == pytest.approx(-1.0 + 1.0 / 19.0, rel=1e-12)


def test_zero_gradient_from_rest_is_a_fixed_point():
    p0 = np.array([0.3, -1.2])
    p, m, v = adam.step(p0, np.zeros(2), np.zeros(2), np.zeros(2), 3, 0.1, 0.9, 0.999, 1e-8)
    np.testing.assert_array_equal(p, p0)
    np.testing.assert_array_equal(m, 0)
    np.testing.assert_array_equal(v, 0)


def test_group_rates_on_a_level():
    # unit gradients everywhere at t = 1 (eps tiny): every element moves by exactly its group's
    # rate; SH row 0 (the degree-0 coefficients, 3 floats) takes lr_sh_dc, rows 1..15 lr_sh_rest
    n = 5
    shapes = dict(means=(n, 3), log_scales=(n, 3), quats=(n, 4), opacity_logits=(n,), sh=(n, 16, 3))
    params = {k: np.zeros(s) for k, s in shapes.items()}
    grads = {k: -np.ones(s) for k, s in shapes.items()}
    zeros = {k: np.zeros(s) for k, s in shapes.items()}
    p, m, v = adam.level_step(params, grads, zeros, zeros, 1, HP)
    np.testing.assert_allclose(p["means"], HP["lr_means"], rtol=1e-12)
    np.testing.assert_allclose(p["log_scales"], HP["lr_log_scales"], rtol=1e-12)
    np.testing.assert_allclose(p["quats"], HP["lr_quats"], rtol=1e-12)
    np.testing.assert_allclose(p["opacity_logits"], HP["lr_opacity"], rtol=1e-12)
    np.testing.assert_allclose(p["sh"][:, 0, :], HP["lr_sh_dc"], rtol=1e-12)
    np.testing.assert_allclose(p["sh"][:, 1:, :], HP["lr_sh_rest"], rtol=1e-12)
    assert p["sh"][:, 1:, :].size == n * 45

"""Pins of the FP64 U-Net oracle: central finite differences of the analytic
gradient, primitive identities, and the channel packing round trip."""

import numpy as np
import pytest

from oracle import unet as U


def test_param_count_matches_specs():
    n = U.param_count(8, 32, 4)
    assert 1.8e6 < n < 2.1e6          # the ~1.9 M parameter network of the warm start
    p = U.init_params(8, 32, 4, seed=0)
    assert p.size == n
    W = U.unpack(p, 8, 32, 4)
    assert W["enc0a"][0].shape == (3, 3, 32, 8) and W["up0"][0].shape == (2, 2, 32, 64)
    assert W["final"][0].shape == (1, 1, 8, 32)


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 5, 6, 3))
    W = rng.standard_normal((3, 3, 2, 3))
    b = rng.standard_normal(2)
    out = U.conv(x, W, b, False)
    y, xx, o = 2, 0, 1
    ref = b[o]
    for kh in range(3):
        for kw in range(3):
            yy, xq = y + kh - 1, xx + kw - 1
            if 0 <= yy < 5 and 0 <= xq < 6:
                ref += W[kh, kw, o] @ x[0, yy, xq]
    assert abs(out[0, y, xx, o] - ref) < 1e-12


def test_up_and_pool_direct():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 2, 3, 4))
    W = rng.standard_normal((2, 2, 5, 4))
    b = rng.standard_normal(5)
    u = U.up(x, W, b)
    assert u.shape == (1, 4, 6, 5)
    assert abs(u[0, 3, 2, 1] - (b[1] + W[1, 0, 1] @ x[0, 1, 1])) < 1e-12
    p = U.pool(x.repeat(2, axis=1).repeat(2, axis=2) + 0.0)
    assert np.allclose(p, x)


@pytest.mark.parametrize("levels,base", [(2, 4), (3, 4)])
def test_gradient_central_differences(levels, base):
    rng = np.random.default_rng(levels)
    cin, H = 4, 8
    params = U.init_params(cin, base, levels, seed=3, final_scale=1.0).astype(np.float64)
    params += 0.05 * rng.standard_normal(params.size)            # break symmetric zeros (biases)
    x = rng.standard_normal((2, H, H, cin))
    t = rng.standard_normal((2, H, H, cin))
    loss, g = U.loss_and_grad(params, x, t, base, levels)
    idx = rng.choice(params.size, 40, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(params)
        e[i] = eps
        lp, _ = U.mse(U.forward(params + e, x, base, levels)[0], t)
        lm, _ = U.mse(U.forward(params - e, x, base, levels)[0], t)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_pool_gradient_ties_go_to_first_maximum():
    x = np.zeros((1, 2, 2, 1))
    d = np.ones((1, 1, 1, 1))
    g = U.pool_backward(x, d)
    assert g[0, 0, 0, 0] == 1.0 and g.sum() == 1.0


def test_pack_round_trip():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((4, 6, 8)) + 1j * rng.standard_normal((4, 6, 8))
    x = U.pack(a, 2.5)
    assert x.shape == (6, 8, 8)
    assert np.isclose(x[1, 2, 3], a[1, 1, 2].imag / 2.5) and np.isclose(x[1, 2, 2], a[1, 1, 2].real / 2.5)
    assert np.allclose(U.unpack_channels(x, 2.5), a)


# --- Adam (Kingma & Ba 2015, Algorithm 1) ---------------------------------------------


def test_adam_constant_gradient_moves_every_weight_by_lr():
    """With a constant gradient the bias corrections make m_hat = g and v_hat = g^2 exactly
    at every step, so each step moves w by lr g / (|g| + eps): a wrong decay, a swapped beta,
    a missing correction or a missing square root breaks this."""
    rng = np.random.default_rng(0)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-3, 3, 50)
    w = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    for t in range(1, 8):
        w_new, m, v = U.adam_step(w, g, m, v, t, lr)
        np.testing.assert_allclose(w - w_new, lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
        w = w_new


def test_adam_second_step_after_zero_gradient():
    """Step 1 with g, step 2 with 0: m_hat_2 = beta1 (1 - beta1) g / (1 - beta1^2) = beta1 g / (1 + beta1),
    v_hat_2 = beta2 g^2 / (1 + beta2); the second move is lr m_hat_2 / (sqrt(v_hat_2) + eps)."""
    g = np.array([2.0, -0.5, 3e-3])
    w0 = np.array([1.0, 2.0, 3.0])
    lr = 0.01
    w1, m, v = U.adam_step(w0, g, np.zeros(3), np.zeros(3), 1, lr)
    w2, m, v = U.adam_step(w1, np.zeros(3), m, v, 2, lr)
    m_hat = 0.9 * g / 1.9
    v_hat = 0.999 * g * g / 1.999
    np.testing.assert_allclose(w1 - w2, lr * m_hat / (np.sqrt(v_hat) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.9 * 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.999 * 0.001 * g * g, rtol=1e-12)


def test_adam_descends_a_quadratic():
    """Adam on f(w) = 1/2 ||w - w*||^2 with a decaying rate ends near the minimiser."""
    rng = np.random.default_rng(1)
    target = rng.standard_normal(20)
    w = np.zeros(20)
    m = np.zeros(20)
    v = np.zeros(20)
    for t in range(1, 3001):
        w, m, v = U.adam_step(w, w - target, m, v, t, 0.05 / np.sqrt(t))
    assert np.abs(w - target).max() < 1e-2

"""Pins of the closure network's FP64 reference (oracle/cnn.py).

- The convolution against torch's CPU conv3d with circular padding
  (an independent library implementation of the same operation).
- Backward (data and weight gradients through SiLU) against central
  finite differences of the loss.
- Adam against its closed form on a quadratic after one step.
"""
import numpy as np
import pytest

from oracle import cnn


def test_conv_matches_torch_circular_conv3d():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = rng.normal(size=(5, 6, 7, 8))
    W = rng.normal(size=(4, 5, 3, 3, 3))
    b = rng.normal(size=4)
    y = cnn.conv3d(x, W, b)
    xt = torch.nn.functional.pad(torch.from_numpy(x)[None], (1, 1, 1, 1, 1, 1), mode="circular")
    yt = torch.nn.functional.conv3d(xt, torch.from_numpy(W), torch.from_numpy(b))[0].numpy()
    np.testing.assert_allclose(y, yt, rtol=1e-12, atol=1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    ch = (3, 4, 4, 2)
    layers = cnn.init_params(seed=3, channels=ch)
    for L in layers:
        L["b"] = rng.normal(scale=0.1, size=L["b"].shape)
    x = rng.normal(size=(3, 4, 5, 4))
    t = rng.normal(size=(2, 4, 5, 4))

    def loss_of(layers_, x_):
        y, _ = cnn.forward(layers_, x_)
        return cnn.mse(y, t)[0]

    y, caches = cnn.forward(layers, x)
    _, gy = cnn.mse(y, t)
    grads, gx = cnn.backward(layers, caches, gy)
    h = 1e-6
    for l, key, idx in [(0, "W", (1, 2, 0, 1, 2)), (1, "W", (3, 0, 2, 2, 1)), (2, "W", (1, 3, 1, 0, 0)),
                        (1, "b", (2,)), (2, "b", (0,))]:
        p = layers[l][key]
        old = p[idx]
        p[idx] = old + h
        lp = loss_of(layers, x)
        p[idx] = old - h
        lm = loss_of(layers, x)
        p[idx] = old
        num = (lp - lm) / (2 * h)
        assert abs(num - grads[l][key][idx]) <= 1e-7 * max(1.0, abs(num)), (l, key, num, grads[l][key][idx])
    for idx in [(0, 1, 2, 3), (2, 3, 4, 0)]:
        old = x[idx]
        x[idx] = old + h
        lp = loss_of(layers, x)
        x[idx] = old - h
        lm = loss_of(layers, x)
        x[idx] = old
        assert abs((lp - lm) / (2 * h) - gx[idx]) <= 1e-7


def test_adam_first_step_is_sign_times_lr():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    m, v = np.zeros(3), np.zeros(3)
    cnn.adam_step(p, g, m, v, 1, lr=0.01, eps=0.0)
    # bias-corrected moments equal g and g^2 after one step
    np.testing.assert_allclose(p, np.array([1.0, -2.0, 3.0]) - 0.01 * np.sign(g), rtol=1e-12)

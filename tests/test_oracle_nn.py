"""Pins for the network reference: finite differences for every gradient,
library cross-correlation for the convolution, closed forms for the rest."""
import numpy as np

from oracle import nn


def _fd(f, x, eps=1e-6):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = x[i]
        x[i] = old + eps
        fp = f()
        x[i] = old - eps
        fm = f()
        x[i] = old
        g[i] = (fp - fm) / (2 * eps)
    return g


def test_conv_matches_library_cross_correlation():
    from scipy.signal import correlate
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = nn.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            want = b[o] + sum(correlate(x[n, :, :, c], w[o, :, :, c], mode="same") for c in range(3))
            assert np.allclose(y[n, :, :, o], want, atol=1e-12)


def test_conv_with_a_centre_delta_kernel_is_the_identity():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 5, 6, 2))
    w = np.zeros((2, 3, 3, 2))
    w[0, 1, 1, 0] = w[1, 1, 1, 1] = 1.0
    assert np.array_equal(nn.conv3x3(x, w), x)


def test_conv_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 5, 3))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    gy = rng.standard_normal((2, 4, 5, 2))

    def loss():
        return float(np.sum(gy * nn.conv3x3(x, w, b)))
    assert np.allclose(nn.conv3x3_grad_input(gy, w), _fd(loss, x), rtol=1e-6, atol=1e-7)
    gw, gb = nn.conv3x3_grad_weight(x, gy)
    assert np.allclose(gw, _fd(loss, w), rtol=1e-6, atol=1e-7)
    assert np.allclose(gb, _fd(loss, b), rtol=1e-6, atol=1e-7)


def test_pool_upsample_relu_and_mse_gradients():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 4, 6, 2))
    g = rng.standard_normal((1, 2, 3, 2))
    assert np.allclose(nn.avgpool2_grad(g), _fd(lambda: float(np.sum(g * nn.avgpool2(x))), x), atol=1e-8)
    g2 = rng.standard_normal((1, 8, 12, 2))
    assert np.allclose(nn.upsample2_grad(g2), _fd(lambda: float(np.sum(g2 * nn.upsample2(x))), x), atol=1e-7)
    xr = x + 0.05 * np.sign(x)   # keep away from the kink
    gr = rng.standard_normal(x.shape)
    assert np.allclose(nn.relu_grad(nn.relu(xr), gr),
                       _fd(lambda: float(np.sum(gr * nn.relu(xr))), xr), atol=1e-8)
    t = rng.standard_normal(x.shape)
    loss, gm = nn.mse(x, t)
    assert np.allclose(gm, _fd(lambda: nn.mse(x, t)[0], x), atol=1e-8)
    # pooling of an upsampled map returns it
    assert np.allclose(nn.avgpool2(nn.upsample2(x)), x)


def test_adam_first_step_moves_each_weight_by_lr_against_the_gradient_sign():
    w = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -0.1, 2.0])
    w1, m, v = nn.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(w1, w - 0.01 * np.sign(g), atol=1e-7)

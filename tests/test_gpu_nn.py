"""The learned initialiser's kernels against the FP64 oracle, on the same
BF16-rounded inputs (which isolates the FP32 accumulation): relative error
1e-5 of the largest output for the convolutions and their gradients, exact
or 1e-6 for the data movement.  Then a short training run must lower the
loss (stochastic: parity unpinned beyond that)."""
import numpy as np
import pytest

from gpu_util import banner, to_np
from oracle import nn as ON
from paper_1902_10559_amd import native

pytestmark = pytest.mark.gpu


def _bf16(a):
    """Round FP32 to BF16 (nearest-even); returns (bits as int16, values)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().copy(), t.float().numpy().astype(np.float64)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(got, want):
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-30))


def _weights(rng, O, C):
    import torch
    w = rng.standard_normal((O, 3, 3, C)).astype(np.float32) * 0.3
    wd = _dev(w)
    wf = torch.empty(O * 9 * ((C + 7) // 8 * 8), dtype=torch.int16, device="cuda")
    wb = torch.empty(C * 9 * ((O + 7) // 8 * 8), dtype=torch.int16, device="cuda")
    native.nn_prep_weights(wd, O, C, wf, wb)
    _, wr = _bf16(w)
    return wd, wf, wb, wr


@pytest.mark.parametrize("N,H,W,C,O", [(2, 8, 16, 1, 16), (1, 16, 32, 16, 16), (2, 8, 8, 48, 16),
                                       (1, 8, 16, 192, 64), (1, 4, 8, 64, 128), (2, 16, 16, 16, 1),
                                       (1, 6, 20, 8, 24)])
def test_conv3x3_forward_and_input_gradient(N, H, W, C, O):
    import torch
    banner(f"conv N={N} H={H} W={W} C={C} O={O}")
    rng = np.random.default_rng(C * 7 + O)
    xb, xr = _bf16(rng.standard_normal((N, H, W, C)))
    wd, wf, wb, wr = _weights(rng, O, C)
    bias = rng.standard_normal(O).astype(np.float32)
    for relu in (0, 1):
        y = torch.empty(N * H * W * O, dtype=torch.float32, device="cuda")
        native.nn_conv3x3(_dev(xb), N, H, W, C, wf, _dev(bias), O, relu, y, True)
        want = ON.conv3x3(xr, wr, bias)
        if relu:
            want = ON.relu(want)
        assert _rel(to_np(y).reshape(N, H, W, O), want) <= 1e-5
    # the input gradient through the flipped, transposed weights
    gb16, gr = _bf16(rng.standard_normal((N, H, W, O)))
    gx = torch.empty(N * H * W * C, dtype=torch.float32, device="cuda")
    native.nn_conv3x3(_dev(gb16), N, H, W, O, wb, None, C, 0, gx, True)
    assert _rel(to_np(gx).reshape(N, H, W, C), ON.conv3x3_grad_input(gr, wr)) <= 1e-5


# staged kernel (W a multiple of 32): 16-byte loads (C, O multiples of 8)
# or value by value (C = 1, O = 1), partial channel tiles, many partial
# groups; the element-wise kernel: W not a multiple of 32
@pytest.mark.parametrize("N,H,W,C,O", [(2, 8, 32, 1, 16), (1, 16, 32, 16, 32), (2, 8, 64, 48, 16),
                                       (1, 8, 32, 64, 128), (3, 8, 40, 8, 8), (2, 8, 64, 8, 24),
                                       (4, 32, 128, 16, 16), (2, 8, 32, 16, 1), (2, 12, 20, 3, 5)])
def test_conv3x3_weight_and_bias_gradient(N, H, W, C, O):
    import torch
    banner(f"wgrad N={N} H={H} W={W} C={C} O={O}")
    rng = np.random.default_rng(C * 13 + O)
    xb, xr = _bf16(rng.standard_normal((N, H, W, C)))
    gb16, gr = _bf16(rng.standard_normal((N, H, W, O)))
    gw = torch.zeros(O * 9 * C, dtype=torch.float32, device="cuda")
    gbias = torch.zeros(O, dtype=torch.float32, device="cuda")
    native.nn_conv3x3_wgrad(_dev(xb), _dev(gb16), N, H, W, C, O, gw, gbias)
    want_w, want_b = ON.conv3x3_grad_weight(xr, gr)
    assert _rel(to_np(gw).reshape(O, 3, 3, C), want_w) <= 1e-5
    assert _rel(to_np(gbias), want_b) <= 1e-5


def test_pool_slices_relu_mask_mse_and_adam():
    import torch
    banner("nn data movement")
    rng = np.random.default_rng(5)
    N, H, W = 2, 8, 12
    xb, xr = _bf16(rng.standard_normal((N, H, W, 6)))
    y = torch.empty(N * H // 2 * W // 2 * 6, dtype=torch.int16, device="cuda")
    native.nn_pool2(_dev(xb), N, H, W, 6, y)
    got = y.view(torch.bfloat16).float().cpu().numpy().reshape(N, H // 2, W // 2, 6)
    _, want = _bf16(ON.avgpool2(xr))
    assert np.array_equal(got, want)
    g = rng.standard_normal((N, H // 2, W // 2, 6)).astype(np.float32)
    gx = torch.full((N * H * W * 6,), 1.0, dtype=torch.float32, device="cuda")
    native.nn_pool2_grad(_dev(g), N, H, W, 6, gx, accumulate=True)
    assert np.allclose(to_np(gx).reshape(N, H, W, 6), 1.0 + ON.avgpool2_grad(g), atol=1e-7)
    # upsampled and plain copies into channel slices, and their gradients
    small_b, small_r = _bf16(rng.standard_normal((N, H // 2, W // 2, 3)))
    cat = torch.zeros(N * H * W * 9, dtype=torch.int16, device="cuda")
    native.nn_to_slice(_dev(small_b), N, H, W, 3, True, cat, 9, 0)
    native.nn_to_slice(_dev(xb), N, H, W, 6, False, cat, 9, 3)
    c = cat.view(torch.bfloat16).float().cpu().numpy().reshape(N, H, W, 9)
    assert np.array_equal(c[..., :3], ON.upsample2(small_r)) and np.array_equal(c[..., 3:], xr)
    gc = rng.standard_normal((N, H, W, 9)).astype(np.float32)
    gs = torch.empty(N * H // 2 * W // 2 * 3, dtype=torch.float32, device="cuda")
    native.nn_from_slice(_dev(gc), N, H // 2, W // 2, 3, True, 9, 0, gs)
    assert np.allclose(to_np(gs).reshape(N, H // 2, W // 2, 3), ON.upsample2_grad(gc[..., :3]), atol=1e-6)
    gp = torch.empty(N * H * W * 6, dtype=torch.float32, device="cuda")
    native.nn_from_slice(_dev(gc), N, H, W, 6, False, 9, 3, gp)
    assert np.array_equal(to_np(gp).reshape(N, H, W, 6), gc[..., 3:])
    # ReLU mask from the layer output
    out = torch.empty(N * H * W * 6, dtype=torch.int16, device="cuda")
    gfull = rng.standard_normal((N, H, W, 6)).astype(np.float32)
    native.nn_relu_mask(_dev(gfull), _dev(xb), out)
    _, want = _bf16(ON.relu_grad(xr, gfull))
    assert np.array_equal(out.view(torch.bfloat16).float().cpu().numpy().reshape(N, H, W, 6), want)
    # residual + squared error
    r = rng.standard_normal(500).astype(np.float32)
    x = rng.standard_normal(500).astype(np.float32)
    t = rng.standard_normal(500).astype(np.float32)
    o = torch.empty(500, dtype=torch.float32, device="cuda")
    gg = torch.empty(500, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    native.nn_residual_mse(_dev(r), _dev(x), _dev(t), o, gg, loss)
    lw, gw_ = ON.mse(x.astype(np.float64) + r, t)
    assert abs(loss.item() - lw) <= 1e-6 * lw and np.allclose(to_np(gg), gw_, rtol=1e-5, atol=1e-9)
    # Adam
    w = rng.standard_normal(300).astype(np.float32)
    g2 = rng.standard_normal(300).astype(np.float32)
    wd, m, v = _dev(w), torch.zeros(300, device="cuda"), torch.zeros(300, device="cuda")
    w64, m64, v64 = w.astype(np.float64), np.zeros(300), np.zeros(300)
    for step in (1, 2, 3):
        native.nn_adam(wd, _dev(g2 * step), m, v, 1e-3, step)
        w64, m64, v64 = ON.adam(w64, g2 * step, m64, v64, step, 1e-3)
    assert np.allclose(to_np(wd), w64, rtol=0, atol=1e-6)


def test_snake_image_round_trip():
    import torch
    from oracle import geometry as G
    banner("snake <-> image")
    rng = np.random.default_rng(6)
    nx, nz = 12, 6
    f = rng.standard_normal((3, nx * nz)).astype(np.float32)
    img = torch.empty(3 * nx * nz, dtype=torch.float32, device="cuda")
    native.nn_snake_image(_dev(f), 3, nx, nz, True, img)
    want = np.stack([G.snake_to_image(f[b], nx, nz) for b in range(3)])
    assert np.array_equal(to_np(img).reshape(3, nz, nx), want)
    back = torch.empty(3 * nx * nz, dtype=torch.float32, device="cuda")
    native.nn_snake_image(img, 3, nx, nz, False, back)
    assert np.array_equal(to_np(back).reshape(3, -1), f)


def test_network_starts_as_identity_and_training_lowers_the_loss():
    import torch
    from paper_1902_10559_amd import unet
    banner("unet training smoke")
    H = W = 32
    N = 4
    net = unet.UNet(H, W, seed=1)
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 1, (N, H, W, 1)).astype(np.float32)
    t = (x + 0.2 * np.sin(np.arange(W) / 3.0)[None, None, :, None]).astype(np.float32)
    x32, t32 = _dev(x), _dev(t)
    x16 = torch.empty(N * H * W, dtype=torch.int16, device="cuda")
    native.nn_to_bf16(x32, x16)
    out = net.forward(x32, x16, N)
    assert np.array_equal(to_np(out).reshape(x.shape), x)
    losses = [net.train_step(x32, x16, t32, N, 2e-3).item() for _ in range(60)]
    banner(f"loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert losses[-1] < 0.5 * losses[0]

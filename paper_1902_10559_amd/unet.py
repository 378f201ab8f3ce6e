"""The learned SART initialiser's network: a 4-level convolutional
encoder-decoder (channels 16, 32, 64, 128; two 3x3 convolutions per level
and five at the 128-channel bottom, about 0.93 M parameters; 2x2 average
pooling down, nearest 2x upsampling and skip concatenation up) that
predicts a correction to an early split-SART image: out = x + net(x).

Every operation is a call into libssart (BF16 matrix-core convolutions,
FP32 gradients and Adam); this module only allocates buffers and sequences
the calls.  The output layer starts at zero, so the untrained network is the
identity map and a learned start is never worse than its input before
training.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import native

# (name, input channels, output channels, ReLU)
LAYERS = [
    ("e1a", 1, 16, True), ("e1b", 16, 16, True),
    ("e2a", 16, 32, True), ("e2b", 32, 32, True),
    ("e3a", 32, 64, True), ("e3b", 64, 64, True),
    ("ba", 64, 128, True), ("bb", 128, 128, True), ("bc", 128, 128, True), ("bd", 128, 128, True),
    ("be", 128, 128, True),
    ("d3a", 192, 64, True), ("d3b", 64, 64, True),
    ("d2a", 96, 32, True), ("d2b", 32, 32, True),
    ("d1a", 48, 16, True), ("d1b", 16, 16, True),
    ("out", 16, 1, False),
]


# resolution level (0 = full, 3 = 1/8) of each layer
LEVEL = {"e1a": 0, "e1b": 0, "e2a": 1, "e2b": 1, "e3a": 2, "e3b": 2, "ba": 3, "bb": 3, "bc": 3, "bd": 3,
         "be": 3, "d3a": 2, "d3b": 2, "d2a": 1, "d2b": 1, "d1a": 0, "d1b": 0, "out": 0}


def _r8(c):
    return (c + 7) // 8 * 8


@dataclasses.dataclass
class Layer:
    name: str
    C: int
    O: int
    relu: bool
    w: "torch.Tensor"      # FP32 master [O, 3, 3, C] (view of the flat buffer)
    b: "torch.Tensor"      # FP32 [O]
    gw: "torch.Tensor"
    gb: "torch.Tensor"
    wf: "torch.Tensor"     # BF16 bits [O, 9, Cp]
    wb: "torch.Tensor"     # BF16 bits [C, 9, Op]


class UNet:
    def __init__(self, H: int, W: int, device="cuda", seed: int = 0):
        import torch
        assert H % 8 == 0 and W % 8 == 0
        self.H, self.W, self.device = H, W, torch.device(device)
        sizes = [(O * 9 * C, O) for _, C, O, _ in LAYERS]
        self.nparams = sum(a + b for a, b in sizes)
        self.params = torch.zeros(self.nparams, dtype=torch.float32, device=self.device)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_count = 0
        rng = np.random.default_rng(seed)
        init = np.zeros(self.nparams, np.float32)
        self.layers: dict[str, Layer] = {}
        off = 0
        for (name, C, O, relu), (nw, nb) in zip(LAYERS, sizes):
            if name != "out":   # He-normal; the output layer starts at zero
                init[off:off + nw] = rng.standard_normal(nw) * np.sqrt(2.0 / (9 * C))
            w = self.params[off:off + nw].view(O, 3, 3, C)
            gw = self.grads[off:off + nw].view(O, 3, 3, C)
            off += nw
            b = self.params[off:off + nb]
            gb = self.grads[off:off + nb]
            off += nb
            wf = torch.empty(O * 9 * _r8(C), dtype=torch.int16, device=self.device)
            wb = torch.empty(C * 9 * _r8(O), dtype=torch.int16, device=self.device)
            self.layers[name] = Layer(name, C, O, relu, w, b, gw, gb, wf, wb)
        self.params.copy_(torch.from_numpy(init))
        self.prep()
        self._bufs = {}

    # ----------------------------------------------------------- weights
    def prep(self):
        for L in self.layers.values():
            native.nn_prep_weights(L.w, L.O, L.C, L.wf, L.wb)

    def load_params(self, flat):
        import torch
        self.params.copy_(torch.as_tensor(flat, dtype=torch.float32))
        self.prep()

    # ----------------------------------------------------------- buffers
    def _buffers(self, N):
        import torch
        if N in self._bufs:
            return self._bufs[N]
        H, W = self.H, self.W
        dev = self.device
        lv = [(H, W), (H // 2, W // 2), (H // 4, W // 4), (H // 8, W // 8)]

        def a16(level, C):
            h, w = lv[level]
            return torch.empty(N * h * w * C, dtype=torch.int16, device=dev)

        def a32(level, C):
            h, w = lv[level]
            return torch.empty(N * h * w * C, dtype=torch.float32, device=dev)
        B = dict(
            x16=a16(0, 1), e1a=a16(0, 16), e1=a16(0, 16), p1=a16(1, 16),
            e2a=a16(1, 32), e2=a16(1, 32), p2=a16(2, 32),
            e3a=a16(2, 64), e3=a16(2, 64), p3=a16(3, 64),
            ba=a16(3, 128), bb=a16(3, 128), bc=a16(3, 128), bd=a16(3, 128), be=a16(3, 128),
            c3=a16(2, 192), d3a=a16(2, 64), d3=a16(2, 64),
            c2=a16(1, 96), d2a=a16(1, 32), d2=a16(1, 32),
            c1=a16(0, 48), d1a=a16(0, 16), d1=a16(0, 16),
            r=a32(0, 1), out=a32(0, 1), gout=a32(0, 1),
            # gradients (FP32) and the BF16 conv-input gradient scratch
            g_d1=a32(0, 16), g_d1a=a32(0, 16), g_c1=a32(0, 48), g_e1=a32(0, 16), g_e1a=a32(0, 16),
            g_d2=a32(1, 32), g_d2a=a32(1, 32), g_c2=a32(1, 96), g_e2=a32(1, 32), g_e2a=a32(1, 32),
            g_p1=a32(1, 16),
            g_d3=a32(2, 64), g_d3a=a32(2, 64), g_c3=a32(2, 192), g_e3=a32(2, 64), g_e3a=a32(2, 64),
            g_p2=a32(2, 32),
            g_be=a32(3, 128), g_bd=a32(3, 128), g_bc=a32(3, 128),
            g_bb=a32(3, 128), g_ba=a32(3, 128), g_p3=a32(3, 64),
            gy=torch.empty(N * H * W * 48, dtype=torch.int16, device=dev),
            loss=torch.zeros(1, dtype=torch.float64, device=dev),
        )
        # scratch of the fixed-order gradient and loss sums: the largest any
        # layer needs
        need = native.nn_mse_workspace_bytes(N * H * W)
        for name, C, O, _ in LAYERS:
            lvl = LEVEL[name]
            need = max(need, native.nn_wgrad_workspace_bytes(N, H >> lvl, W >> lvl, C, O))
        B["ws"] = torch.empty(need, dtype=torch.uint8, device=dev)
        self._bufs[N] = B
        return B

    def _conv(self, name, x, N, level, y, y_f32=False):
        L = self.layers[name]
        h, w = self.H >> level, self.W >> level
        native.nn_conv3x3(x, N, h, w, L.C, L.wf, L.b, L.O, L.relu, y, y_f32)

    # ----------------------------------------------------------- forward
    def forward(self, x32, x16, N, target=None, want_grad=False):
        """x32, x16: (N, H, W, 1) FP32 and BF16 images; returns out (FP32).
        With a target, also the squared-error loss (on device)."""
        B = self._buffers(N)
        H, W = self.H, self.W
        h2, w2, h3, w3, h4, w4 = H // 2, W // 2, H // 4, W // 4, H // 8, W // 8
        B["x16"] = x16
        self._conv("e1a", x16, N, 0, B["e1a"])
        self._conv("e1b", B["e1a"], N, 0, B["e1"])
        native.nn_pool2(B["e1"], N, H, W, 16, B["p1"])
        self._conv("e2a", B["p1"], N, 1, B["e2a"])
        self._conv("e2b", B["e2a"], N, 1, B["e2"])
        native.nn_pool2(B["e2"], N, h2, w2, 32, B["p2"])
        self._conv("e3a", B["p2"], N, 2, B["e3a"])
        self._conv("e3b", B["e3a"], N, 2, B["e3"])
        native.nn_pool2(B["e3"], N, h3, w3, 64, B["p3"])
        self._conv("ba", B["p3"], N, 3, B["ba"])
        self._conv("bb", B["ba"], N, 3, B["bb"])
        self._conv("bc", B["bb"], N, 3, B["bc"])
        self._conv("bd", B["bc"], N, 3, B["bd"])
        self._conv("be", B["bd"], N, 3, B["be"])
        native.nn_to_slice(B["be"], N, h3, w3, 128, True, B["c3"], 192, 0)
        native.nn_to_slice(B["e3"], N, h3, w3, 64, False, B["c3"], 192, 128)
        self._conv("d3a", B["c3"], N, 2, B["d3a"])
        self._conv("d3b", B["d3a"], N, 2, B["d3"])
        native.nn_to_slice(B["d3"], N, h2, w2, 64, True, B["c2"], 96, 0)
        native.nn_to_slice(B["e2"], N, h2, w2, 32, False, B["c2"], 96, 64)
        self._conv("d2a", B["c2"], N, 1, B["d2a"])
        self._conv("d2b", B["d2a"], N, 1, B["d2"])
        native.nn_to_slice(B["d2"], N, H, W, 32, True, B["c1"], 48, 0)
        native.nn_to_slice(B["e1"], N, H, W, 16, False, B["c1"], 48, 32)
        self._conv("d1a", B["c1"], N, 0, B["d1a"])
        self._conv("d1b", B["d1a"], N, 0, B["d1"])
        self._conv("out", B["d1"], N, 0, B["r"], y_f32=True)
        if target is not None:
            B["loss"].zero_()
        native.nn_residual_mse(B["r"], x32, target, B["out"], B["gout"] if want_grad else None,
                               B["loss"] if target is not None else None, ws=B["ws"])
        return B["out"]

    # ---------------------------------------------------------- backward
    def _back(self, name, x_in, N, level, g_out, y_out, g_in):
        """Gradient through layer `name`: g_out (FP32, dL/d output) and the
        layer's output y_out (for the ReLU mask) -> weight/bias gradients and
        g_in (FP32, dL/d input) when g_in is not None."""
        L = self.layers[name]
        B = self._bufs[N]
        h, w = self.H >> level, self.W >> level
        gy = B["gy"][: N * h * w * L.O]
        native.nn_relu_mask(g_out, y_out if L.relu else None, gy)
        native.nn_conv3x3_wgrad(x_in, gy, N, h, w, L.C, L.O, L.gw, L.gb, ws=B["ws"])
        if g_in is not None:
            native.nn_conv3x3(gy, N, h, w, L.O, L.wb, None, L.C, False, g_in, True)

    def backward(self, N):
        """Gradients of the last forward's loss (forward(..., want_grad=True))."""
        B = self._bufs[N]
        H, W = self.H, self.W
        h2, w2, h3, w3, h4, w4 = H // 2, W // 2, H // 4, W // 4, H // 8, W // 8
        self._back("out", B["d1"], N, 0, B["gout"], None, B["g_d1"])
        self._back("d1b", B["d1a"], N, 0, B["g_d1"], B["d1"], B["g_d1a"])
        self._back("d1a", B["c1"], N, 0, B["g_d1a"], B["d1a"], B["g_c1"])
        native.nn_from_slice(B["g_c1"], N, h2, w2, 32, True, 48, 0, B["g_d2"])
        native.nn_from_slice(B["g_c1"], N, H, W, 16, False, 48, 32, B["g_e1"])
        self._back("d2b", B["d2a"], N, 1, B["g_d2"], B["d2"], B["g_d2a"])
        self._back("d2a", B["c2"], N, 1, B["g_d2a"], B["d2a"], B["g_c2"])
        native.nn_from_slice(B["g_c2"], N, h3, w3, 64, True, 96, 0, B["g_d3"])
        native.nn_from_slice(B["g_c2"], N, h2, w2, 32, False, 96, 64, B["g_e2"])
        self._back("d3b", B["d3a"], N, 2, B["g_d3"], B["d3"], B["g_d3a"])
        self._back("d3a", B["c3"], N, 2, B["g_d3a"], B["d3a"], B["g_c3"])
        native.nn_from_slice(B["g_c3"], N, h4, w4, 128, True, 192, 0, B["g_be"])
        native.nn_from_slice(B["g_c3"], N, h3, w3, 64, False, 192, 128, B["g_e3"])
        self._back("be", B["bd"], N, 3, B["g_be"], B["be"], B["g_bd"])
        self._back("bd", B["bc"], N, 3, B["g_bd"], B["bd"], B["g_bc"])
        self._back("bc", B["bb"], N, 3, B["g_bc"], B["bc"], B["g_bb"])
        self._back("bb", B["ba"], N, 3, B["g_bb"], B["bb"], B["g_ba"])
        self._back("ba", B["p3"], N, 3, B["g_ba"], B["ba"], B["g_p3"])
        native.nn_pool2_grad(B["g_p3"], N, h3, w3, 64, B["g_e3"], accumulate=True)
        self._back("e3b", B["e3a"], N, 2, B["g_e3"], B["e3"], B["g_e3a"])
        self._back("e3a", B["p2"], N, 2, B["g_e3a"], B["e3a"], B["g_p2"])
        native.nn_pool2_grad(B["g_p2"], N, h2, w2, 32, B["g_e2"], accumulate=True)
        self._back("e2b", B["e2a"], N, 1, B["g_e2"], B["e2"], B["g_e2a"])
        self._back("e2a", B["p1"], N, 1, B["g_e2a"], B["e2a"], B["g_p1"])
        native.nn_pool2_grad(B["g_p1"], N, H, W, 16, B["g_e1"], accumulate=True)
        self._back("e1b", B["e1a"], N, 0, B["g_e1"], B["e1"], B["g_e1a"])
        self._back("e1a", B["x16"], N, 0, B["g_e1a"], B["e1a"], None)

    def train_step(self, x32, x16, target, N, lr):
        self.grads.zero_()
        self.forward(x32, x16, N, target, want_grad=True)
        self.backward(N)
        self.step_count += 1
        native.nn_adam(self.params, self.grads, self.m, self.v, lr, self.step_count)
        self.prep()
        return self._bufs[N]["loss"]

"""FP64 reference for the learned SART initialiser's network (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Not part of the
paper's method: the spec workload adds a small convolutional
encoder-decoder that maps an early split-SART image to a later one.  This
module is the plain definition of each layer, checked in
``tests/test_oracle_nn.py`` by finite differences and by library
cross-correlation.

Layout: activations NHWC (batch, height, width, channels); 3x3 weights
w[co, ky, kx, ci]; zero padding of one pixel; stride 1.
"""
from __future__ import annotations

import numpy as np


def conv3x3(x, w, b=None):
    """y[n, i, j, o] = b[o] + sum_{ky, kx, c} w[o, ky, kx, c] x[n, i+ky-1, j+kx-1, c]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    N, H, W, C = x.shape
    O = w.shape[0]
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    y = np.zeros((N, H, W, O))
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("nhwc,oc->nhwo", xp[:, ky:ky + H, kx:kx + W, :], w[:, ky, kx, :])
    if b is not None:
        y += np.asarray(b, np.float64)
    return y


def conv3x3_grad_input(gy, w):
    """d(sum gy * conv3x3(x, w)) / dx."""
    gy = np.asarray(gy, np.float64)
    w = np.asarray(w, np.float64)
    N, H, W, O = gy.shape
    C = w.shape[3]
    gp = np.zeros((N, H + 2, W + 2, O))
    gp[:, 1:H + 1, 1:W + 1, :] = gy
    gx = np.zeros((N, H, W, C))
    # x[i, j] feeds y[i - ky + 1, j - kx + 1] through w[., ky, kx, .]
    for ky in range(3):
        for kx in range(3):
            gx += np.einsum("nhwo,oc->nhwc", gp[:, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W, :],
                            w[:, ky, kx, :])
    return gx


def conv3x3_grad_weight(x, gy):
    """(d/dw, d/db) of sum gy * conv3x3(x, w, b)."""
    x = np.asarray(x, np.float64)
    gy = np.asarray(gy, np.float64)
    N, H, W, C = x.shape
    O = gy.shape[3]
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    gw = np.zeros((O, 3, 3, C))
    for ky in range(3):
        for kx in range(3):
            gw[:, ky, kx, :] = np.einsum("nhwo,nhwc->oc", gy, xp[:, ky:ky + H, kx:kx + W, :])
    return gw, gy.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


def relu_grad(y, gy):
    """Gradient through y = relu(x), given the output y."""
    return np.where(y > 0, gy, 0.0)


def avgpool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_grad(gy):
    return np.repeat(np.repeat(gy, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_grad(gy):
    N, H, W, C = gy.shape
    return gy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def mse(y, t):
    """Mean squared error and its gradient with respect to y."""
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected; returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v

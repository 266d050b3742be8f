"""FP64 reference of the warm-start network: a multilayer perceptron with
ReLU hidden layers, a linear output layer and the mean squared error loss,
with its gradient by reverse-mode differentiation written out layer by
layer.  Used to check the HIP forward/backward kernels (which run with BF16
weights and FP32 accumulation: the same BF16-rounded weights are fed here).

Parameter layout: for each layer l, W_l [out][in] row-major then b_l [out].
Pinned by central finite differences and by the closed form of a single
linear layer (tests/test_learned.py).
"""
from __future__ import annotations

import numpy as np


def unpack(params, widths):
    out, o = [], 0
    for l in range(len(widths) - 1):
        ni, no = widths[l], widths[l + 1]
        W = np.asarray(params[o:o + ni * no], np.float64).reshape(no, ni)
        o += ni * no
        b = np.asarray(params[o:o + no], np.float64)
        o += no
        out.append((W, b))
    return out


def forward(params, widths, X):
    """Returns the output and the list of pre-activations."""
    a = np.asarray(X, np.float64)
    zs = []
    layers = unpack(params, widths)
    for l, (W, b) in enumerate(layers):
        z = a @ W.T + b
        zs.append(z)
        a = np.maximum(z, 0.0) if l < len(layers) - 1 else z
    return a, zs


def loss_grad(params, widths, X, T):
    X = np.asarray(X, np.float64)
    T = np.asarray(T, np.float64)
    y, zs = forward(params, widths, X)
    B, no = y.shape
    loss = float(np.sum((y - T) ** 2) / (B * no))
    d = 2.0 * (y - T) / (B * no)
    layers = unpack(params, widths)
    acts = [X] + [np.maximum(z, 0.0) for z in zs[:-1]]
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        gW = d.T @ acts[l]
        gb = d.sum(axis=0)
        grads[l] = (gW, gb)
        if l > 0:
            d = (d @ W) * (zs[l - 1] > 0)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat

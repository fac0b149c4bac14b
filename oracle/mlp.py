"""FP64 oracle of the learned reduced-step model.  TEST INFRASTRUCTURE ONLY.

Not part of the paper: a multilayer perceptron maps the reduced state (all
bonds' POD coefficients plus the log shear rate) to the coefficient increment
of one time step.  Layers: Linear -> SiLU -> Linear -> SiLU -> Linear.
Loss: mean squared error over every output entry of every sample.
Optimiser: Adam (Kingma and Ba, 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(layers, X: np.ndarray):
    """Returns the output and the cache of pre-activations and activations."""
    acts = [X]
    pres = []
    a = X
    for i, (W, b) in enumerate(layers):
        z = a @ W.T + b
        pres.append(z)
        a = silu(z) if i < len(layers) - 1 else z
        acts.append(a)
    return a, (pres, acts)


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (8 significant bits, FP32's exponent range) to nearest,
    ties to even, from the FP32 value: keep the upper 16 bits of the FP32
    pattern after adding 0x7fff plus the lowest kept bit.  Finite values only."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(layers, X: np.ndarray) -> np.ndarray:
    """The inference arithmetic of the learned step's BF16 form: every layer's
    weights and inputs (the network input, then each hidden activation, as FP32
    values) rounded to bfloat16, the products summed exactly (FP64 here), FP32
    biases, SiLU between layers."""
    a = np.asarray(X, dtype=np.float64)
    for i, (W, b) in enumerate(layers):
        z = bf16_round(a) @ bf16_round(W).T + np.asarray(b, dtype=np.float32).astype(np.float64)
        a = silu(z) if i < len(layers) - 1 else z
    return a


def loss(layers, X, Y) -> float:
    y, _ = forward(layers, X)
    return float(((y - Y) ** 2).mean())


def backward(layers, X: np.ndarray, Y: np.ndarray):
    """Loss and gradients [(dW, db), ...] of the mean squared error by the chain rule."""
    y, (pres, acts) = forward(layers, X)
    n_el = y.size
    dz = 2.0 * (y - Y) / n_el
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        grads[i] = (dz.T @ acts[i], dz.sum(0))
        if i > 0:
            dz = (dz @ W) * silu_grad(pres[i - 1])
    return float(((y - Y) ** 2).mean()), grads


def adam_init(layers):
    return [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers], \
           [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]


def adam_step(layers, grads, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns new (layers, m, v)."""
    out_l, out_m, out_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(layers, grads, m, v):
        new = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = beta1 * mm + (1.0 - beta1) * g
            vv = beta2 * vv + (1.0 - beta2) * g * g
            mh = mm / (1.0 - beta1 ** t)
            vh = vv / (1.0 - beta2 ** t)
            new.append((p - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        out_l.append((new[0][0], new[1][0]))
        out_m.append((new[0][1], new[1][1]))
        out_v.append((new[0][2], new[1][2]))
    return out_l, out_m, out_v

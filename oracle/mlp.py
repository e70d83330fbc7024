"""FP64 reference of the order-prediction network -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may import
this module. It shares nothing with the HIP network kernels.

The network is the plain three-layer perceptron
    h1 = relu(x W1 + b1),  h2 = relu(h1 W2 + b2),  y = h2 W3 + b3
with the weighted mean-squared loss  L = sum(w (y - t)^2) / (n n_out)  and its gradient by the
chain rule (reverse mode), and Adam (Kingma and Ba 2015: beta1 0.9, beta2 0.999, eps 1e-8, bias
corrected moments). The parameter vector is W1, b1, W2, b2, W3, b3, matrices row-major.

``bf16=True`` rounds, to the nearest BF16 value (ties to even), exactly the operands that the
library's matrix products take in BF16: the input, the three weight matrices, both hidden
activations, the output gradient and both pre-activation gradients (the bias gradients sum the
unrounded ones). Everything else stays FP64.
This is the "same precision" comparison point for the kernels; ``bf16=False`` is the exact
network, pinned by finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a) -> np.ndarray:
    """Round to the nearest BF16 value (8 significant bits), ties to even; via FP32 bit patterns.

    The input is first rounded to FP32 (the library rounds FP32 values)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64).reshape(f.shape)


def param_count(n_in: int, n_h: int, n_out: int) -> int:
    return n_in * n_h + n_h + n_h * n_h + n_h + n_h * n_out + n_out


def unpack(p, n_in: int, n_h: int, n_out: int):
    p = np.asarray(p, dtype=np.float64)
    if p.size != param_count(n_in, n_h, n_out):
        raise ValueError("parameter vector has the wrong length")
    shapes = [(n_in, n_h), (n_h,), (n_h, n_h), (n_h,), (n_h, n_out), (n_out,)]
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(p[o:o + k].reshape(s))
        o += k
    return out


def _q(a, bf16):
    return bf16_round(a) if bf16 else a


def forward(p, x, dims, bf16: bool = False):
    """Network output y (n, n_out) and the intermediates the backward pass needs."""
    W1, b1, W2, b2, W3, b3 = unpack(p, *dims)
    x = _q(np.asarray(x, dtype=np.float64), bf16)
    z1 = x @ _q(W1, bf16) + b1
    h1 = _q(np.maximum(z1, 0.0), bf16)
    z2 = h1 @ _q(W2, bf16) + b2
    h2 = _q(np.maximum(z2, 0.0), bf16)
    y = h2 @ _q(W3, bf16) + b3
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t, w, dims, bf16: bool = False) -> float:
    y, _ = forward(p, x, dims, bf16)
    t = np.asarray(t, dtype=np.float64)
    w = np.ones_like(t) if w is None else np.asarray(w, dtype=np.float64)
    return float(np.sum(w * (y - t) ** 2) / y.size)


def loss_and_grad(p, x, t, w, dims, bf16: bool = False):
    """Loss and its gradient with respect to the parameter vector (reverse-mode chain rule)."""
    n_in, n_h, n_out = dims
    W1, b1, W2, b2, W3, b3 = unpack(p, *dims)
    y, (xq, z1, h1, z2, h2) = forward(p, x, dims, bf16)
    t = np.asarray(t, dtype=np.float64)
    w = np.ones_like(t) if w is None else np.asarray(w, dtype=np.float64)
    e = y - t
    L = float(np.sum(w * e * e) / y.size)
    # bias gradients sum the unrounded gradients; the products take the rounded ones
    dy = 2.0 * w * e / y.size
    gb3, dy = dy.sum(0), _q(dy, bf16)
    gW3 = h2.T @ dy
    dz2 = (dy @ _q(W3, bf16).T) * (z2 > 0)
    gb2, dz2 = dz2.sum(0), _q(dz2, bf16)
    gW2 = h1.T @ dz2
    dz1 = (dz2 @ _q(W2, bf16).T) * (z1 > 0)
    gb1, dz1 = dz1.sum(0), _q(dz1, bf16)
    gW1 = xq.T @ dz1
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return L, g


def adam_step(p, g, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns the new (p, m, v)."""
    p, g = np.asarray(p, np.float64), np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

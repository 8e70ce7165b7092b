"""FP64 CPU oracle of the inlet controller's network (test infrastructure).

Only the tests, the smoke entry point and the benchmark's CPU leg use this
module; the library never does.

The network is a 32 -> 128 -> 128 -> 1 multilayer perceptron with tanh
hidden activations, trained on the mean squared error with Adam. The paper
has no learned part: this is the plain textbook definition, written out in
numpy FP64 so that the GPU's matrix-core products (BF16 operands, FP32
accumulation) can be checked against it.

Parameter vector order: W1 [128][32], b1 [128], W2 [128][128], b2 [128],
W3 [1][128], b3 [1].

``bf16=True`` rounds every operand of the three products to BF16 (round to
nearest, ties to even) before an FP64 product: the precision the GPU kernels
fix for their operands, so the remaining difference is accumulation order and
FP32 rounding only.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 32, 128
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (1, N_HID)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    """Split a flat parameter vector into named FP64 arrays (views)."""
    p = np.asarray(p, dtype=np.float64)
    if p.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters")
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def round_bf16(x):
    """Round to the nearest BF16 value, ties to even (FP32 first, as the
    operands are FP32 arrays on the device)."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    keep = (u >> 16) & 1
    r = ((u + 0x7FFF + keep) >> 16) << 16
    nan = ((u & 0x7F800000) == 0x7F800000) & ((u & 0x007FFFFF) != 0)
    r = np.where(nan, u | 0x00400000, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(a, b, bf16):
    if bf16:
        a, b = round_bf16(a), round_bf16(b)
    return np.asarray(a, np.float64) @ np.asarray(b, np.float64)


def forward(p, x, bf16=False):
    """y [batch] and the hidden activations for input x [batch][32]."""
    w = unpack(p)
    x = np.asarray(x, np.float64)
    h1 = np.tanh(_mm(x, w["W1"].T, bf16) + w["b1"])
    h2 = np.tanh(_mm(h1, w["W2"].T, bf16) + w["b2"])
    y = (_mm(h2, w["W3"].T, bf16) + w["b3"])[:, 0]
    return y, h1, h2


def loss(p, x, t, bf16=False):
    y, _, _ = forward(p, x, bf16)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def gradients(p, x, t, bf16=False):
    """Mean squared error and its gradient by the chain rule (backpropagation)."""
    w = unpack(p)
    x = np.asarray(x, np.float64)
    y, h1, h2 = forward(p, x, bf16)
    b = x.shape[0]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / b            # dL/dy
    g = {}
    g["W3"] = _mm(dy[None, :], h2, bf16)                       # [1][128]
    g["b3"] = np.array([dy.sum()])
    dh2 = _mm(dy[:, None], w["W3"], bf16)                      # [b][128]
    dz2 = dh2 * (1.0 - h2 * h2)
    g["W2"] = _mm(dz2.T, h1, bf16)
    g["b2"] = dz2.sum(axis=0)
    dh1 = _mm(dz2, w["W2"], bf16)
    dz1 = dh1 * (1.0 - h1 * h1)
    g["W1"] = _mm(dz1.T, x, bf16)
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2)), pack(g)


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; returns
    the new (p, m, v). ``step`` counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

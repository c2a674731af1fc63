"""FP64 reference of the spectral/budget predictor MLP (oracle side).

TEST INFRASTRUCTURE ONLY (see the package header).

The network maps 8 standardised features of a phi-action instance to 2
standardised targets (log of the scaled spectral bound, log of the Leja
sweep count): 8 -> 64 -> 64 -> 2, ReLU after the two hidden layers, hidden
activations stored in bfloat16 (round to nearest even of the float32
value), weights in float32, loss the mean squared error over the batch and
both outputs, optimiser Adam (Kingma and Ba, 2015) with bias correction.
The paper has no learned component; this follows the benchmark workload's
description of the predictor.  Everything here is float64 except the two
roundings (float32, then bfloat16) that define the stored activations.

Parameter vector layout (shared with the library's C ABI):
    W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [2][64], b3 [2]
"""
from __future__ import annotations

import numpy as np

IN, H, OUT = 8, 64, 2
SHAPES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (OUT, H)), ("b3", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x) -> np.ndarray:
    """Round to float32, then to bfloat16 by round-to-nearest-even on the
    upper 16 bits of the float32 pattern (finite values)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = (b + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, X, round_bf16: bool = True):
    """X: [B, 8] standardised features.  Returns (Y [B, 2], cache)."""
    p = unpack(theta)
    q = bf16 if round_bf16 else (lambda a: a)
    z1 = X @ p["W1"].T + p["b1"]
    a1 = q(np.maximum(z1, 0.0))
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = q(np.maximum(z2, 0.0))
    Y = a2 @ p["W3"].T + p["b3"]
    return Y, (X, z1, a1, z2, a2)


def loss_and_grad(theta, X, T, round_bf16: bool = True):
    """Mean squared error over the batch and both outputs, and its gradient
    with respect to the parameter vector.  The bfloat16 rounding is treated
    as the identity in the backward pass (straight-through)."""
    p = unpack(theta)
    Y, (X, z1, a1, z2, a2) = forward(theta, X, round_bf16)
    B = X.shape[0]
    diff = Y - T
    loss = float(np.mean(diff * diff))
    dY = 2.0 * diff / (B * OUT)
    g = {"W3": dY.T @ a2, "b3": dY.sum(axis=0)}
    da2 = dY @ p["W3"]
    dz2 = da2 * (z2 > 0.0)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(axis=0)
    da1 = dz2 @ p["W2"]
    dz1 = da1 * (z1 > 0.0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1**t)
    vhat = v / (1.0 - beta2**t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v

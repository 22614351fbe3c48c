"""TEST INFRASTRUCTURE: plain numpy oracle of the learned-initialisation
network (not in the paper; it predicts, per back-projected point, the
initial temporal scale and velocity of the 4D Gaussian that the paper's
heuristic initialisation of Sec. 4.1 otherwise fixes).

Network: 16 inputs -> 64 -> 64 -> 64 -> 4 outputs, SiLU between layers,
    h1 = silu(W1 x + b1), h2 = silu(W2 h1 + b2), h3 = silu(W3 h2 + b3),
    y  = W4 h3 + b4,            silu(z) = z / (1 + exp(-z)).
Parameters are held as one flat vector in the order W1, b1, W2, b2, W3, b3,
W4, b4 with each W row-major [out][in]: 9,668 values.  The network computes
with BF16 parameters (each FP32 master value rounded to the nearest BF16,
ties to even) and FP32 accumulation; this oracle evaluates the same BF16
values in FP64.

Only ``tests/`` may import this module.
"""
from __future__ import annotations

import numpy as np

SIZES = (16, 64, 64, 64, 4)
N_PARAMS = sum(SIZES[i] * SIZES[i + 1] + SIZES[i + 1] for i in range(4))   # 9668


def bf16_round(x):
    """FP32 values rounded to the nearest BF16 value (ties to even),
    returned as FP32.  BF16 keeps the upper 16 bits of the FP32 pattern;
    rounding adds 0x7FFF plus the lowest kept bit before truncating."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).copy()
    nan = np.isnan(f)
    out[nan] = f[nan]
    return out


def unpack(theta):
    """Flat parameter vector -> [(W1, b1), ..., (W4, b4)] views."""
    theta = np.asarray(theta)
    assert theta.shape == (N_PARAMS,)
    out, o = [], 0
    for i in range(4):
        fi, fo = SIZES[i], SIZES[i + 1]
        W = theta[o:o + fi * fo].reshape(fo, fi)
        o += fi * fo
        b = theta[o:o + fo]
        o += fo
        out.append((W, b))
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X):
    """y [N, 4] for inputs X [N, 16], in FP64; also the pre-activations and
    activations of every layer for the backward."""
    layers = [(W.astype(np.float64), b.astype(np.float64)) for W, b in unpack(theta)]
    h = np.asarray(X, np.float64)
    acts, pres = [h], []
    for i, (W, b) in enumerate(layers):
        z = h @ W.T + b
        pres.append(z)
        h = silu(z) if i < 3 else z
        acts.append(h)
    return h, dict(acts=acts, pres=pres, layers=layers)


def backward(theta, X, dY):
    """Gradients of sum(dY * y) with respect to the flat parameters [9668]
    and the inputs [N, 16], in FP64 (chain rule through the layers above)."""
    _, c = forward(theta, X)
    acts, pres, layers = c["acts"], c["pres"], c["layers"]
    g = np.asarray(dY, np.float64)
    grads = [None] * 4
    for i in range(3, -1, -1):
        if i < 3:
            g = g * dsilu(pres[i])
        W, _ = layers[i]
        grads[i] = (g.T @ acts[i], g.sum(axis=0))
        g = g @ W
    flat = np.concatenate([np.concatenate([dW.reshape(-1), db]) for dW, db in grads])
    return flat, g

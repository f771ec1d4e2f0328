"""Double-precision oracle of the learned proposal network (test infrastructure only).

Plain numpy: the multilayer perceptron in -> H -> H -> out with exact-erf
GELU, its mean-squared-error gradient by the chain rule, and Adam.  Two
modes: ``bf16=True`` rounds the matrix operands to bfloat16 (round to nearest
even) exactly where the matrix-core kernels do, so that the GPU's fp32
accumulations can be compared against double-precision sums of the same
operands; ``bf16=False`` is the plain network, pinned by finite differences.
Parameter vector layout: W1[in][H], b1[H], W2[H][H], b2[H], W3[H][out], b3[out].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def unpack(theta, n_in, H, n_out):
    sizes = [n_in * H, H, H * H, H, H * n_out, n_out]
    out, k = [], 0
    for s in sizes:
        out.append(np.asarray(theta[k:k + s], dtype=np.float64))
        k += s
    W1, b1, W2, b2, W3, b3 = out
    return W1.reshape(n_in, H), b1, W2.reshape(H, H), b2, W3.reshape(H, n_out), b3


def pack(*parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(theta, X, n_in, H, n_out, bf=True):
    """Returns a dict of intermediates: x, pre1, a1, pre2, a2, out."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, H, n_out)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    x = r(X)
    pre1 = x @ r(W1) + b1
    a1 = r(gelu(pre1))
    pre2 = a1 @ r(W2) + b2
    a2 = r(gelu(pre2))
    out = a2 @ r(W3) + b3
    return dict(x=x, pre1=pre1, a1=a1, pre2=pre2, a2=a2, out=out)


def loss(theta, X, Y, n_in, H, n_out, bf=False):
    f = forward(theta, X, n_in, H, n_out, bf)
    return float(np.mean((f["out"] - Y) ** 2))


def backward(theta, X, Y, n_in, H, n_out, bf=True, given=None):
    """Gradient of the mean squared error (parameter layout).

    given (optional): intermediates from the GPU (keys of forward() plus
    dout, dh2, dh1) used instead of recomputing them, so each layer can be
    checked on the GPU's own inputs.
    """
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, H, n_out)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    f = forward(theta, X, n_in, H, n_out, bf)
    if given:
        f.update({k: np.asarray(v, dtype=np.float64) for k, v in given.items() if k in f})
    M = X.shape[0]
    dout = 2.0 * (f["out"] - Y) / (M * n_out)
    if given and "dout" in given:
        dout = np.asarray(given["dout"], dtype=np.float64)
    gW3 = f["a2"].T @ r(dout)
    gb3 = dout.sum(0)
    dh2 = (r(dout) @ r(W3).T) * gelu_grad(f["pre2"])
    if given and "dh2" in given:
        dh2 = np.asarray(given["dh2"], dtype=np.float64)
    gW2 = f["a1"].T @ r(dh2)
    gb2 = dh2.sum(0)
    dh1 = (r(dh2) @ r(W2).T) * gelu_grad(f["pre1"])
    if given and "dh1" in given:
        dh1 = np.asarray(given["dh1"], dtype=np.float64)
    gW1 = f["x"].T @ r(dh1)
    gb1 = dh1.sum(0)
    return pack(gW1, gb1, gW2, gb2, gW3, gb3), dict(dout=dout, dh2=dh2, dh1=dh1, **f)


def adam(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v

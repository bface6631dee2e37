"""FP64 reference of the surrogate perceptron -- TEST INFRASTRUCTURE ONLY.

Network: 16 -> 256 -> 256 -> 256 -> 256 -> 16, tanh-form GELU
    gelu(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)))
after every layer but the last; y = x W^T + b per layer.  The GPU kernels
store layer inputs and the back-propagated pre-activation gradients in BF16
and accumulate in FP32; ``bf16=True`` applies the same BF16 roundings here (at
the same places) so that the comparison only sees the accumulation order.
Loss (per row, averaged over rows):
    (o0 - label)^2 + lam (o1 - log10(|o0 - label| + 1e-6))^2,
with the second target held fixed (no gradient flows through it).
"""
from __future__ import annotations

import numpy as np

C = np.sqrt(2.0 / np.pi)
A = 0.044715


def bf16_round(x):
    """Round float64 values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C * (z + A * z ** 3)))


def gelu_grad(z):
    t = np.tanh(C * (z + A * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C * (1.0 + 3.0 * A * z * z)


def forward(Ws, bs, X, bf16=False):
    """Returns (out, cache); Ws[l] is [N_l][K_l], bs[l] [N_l], X [B][16]."""
    r = bf16_round if bf16 else (lambda a: a)
    xs, zs = [r(X)], []
    x = xs[0]
    L = len(Ws)
    for l in range(L):
        z = x @ r(Ws[l]).T + bs[l]
        if l < L - 1:
            zs.append(z)
            x = r(gelu(z))
            xs.append(x)
        else:
            out = z
    return out, (xs, zs)


def loss_and_grad(out, label, lam):
    o0, o1 = out[:, 0], out[:, 1]
    res = o0 - label
    tgt = np.log10(np.abs(res) + 1e-6)
    r1 = o1 - tgt
    n = out.shape[0]
    loss = float(np.mean(res ** 2 + lam * r1 ** 2))
    dout = np.zeros_like(out)
    dout[:, 0] = 2.0 * res / n
    dout[:, 1] = 2.0 * lam * r1 / n
    return loss, dout


def backward(Ws, bs, cache, dout, bf16=False):
    """Gradients (dWs, dbs, dX) for dL/dout = dout."""
    r = bf16_round if bf16 else (lambda a: a)
    xs, _ = cache
    dzs = backward_dz(Ws, cache, dout, bf16)
    dWs = [dz.T @ x for dz, x in zip(dzs, xs)]
    dbs = [dz.sum(0) for dz in dzs]
    return dWs, dbs, dzs[0] @ r(Ws[0])


def backward_dz(Ws, cache, dout, bf16=False):
    """The back-propagated pre-activation gradients dZ_l of every layer (as
    stored: BF16-rounded when bf16), for dL/dout = dout."""
    r = bf16_round if bf16 else (lambda a: a)
    xs, zs = cache
    L = len(Ws)
    dzs = [None] * L
    dy = dout
    for l in range(L - 1, -1, -1):
        dz = dy if l == L - 1 else dy * gelu_grad(zs[l])
        dz = r(dz)
        dzs[l] = dz
        dy = dz @ r(Ws[l])
    return dzs

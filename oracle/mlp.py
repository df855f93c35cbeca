"""FP64 CPU oracle of the MLP surrogate (TEST INFRASTRUCTURE: only tests/,
the smoke check and the benchmark's CPU-baseline leg use it; it shares no
code with the GPU library).

The surrogate is not part of the paper; its definition here follows the
hot-path reading of the surrogate row:
  * 4 linear layers d -> w -> w -> w -> m, GELU with the exact error
    function after the first three, linear output;
  * targets standardised per output, mean-squared-error loss over the
    (batch, output) entries;
  * Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights, cosine
    learning-rate decay from lr0 to 0 over the run.

``storage='bf16'`` reproduces where the GPU kernels store BF16 values: the
network input, the BF16 copies of the weights, the post-GELU activations, the
output gradient and the pre-activation gradients (GEMM operands), each
rounded to BF16 (round to nearest even).  Products and sums are FP64 here
(FP32 accumulation on the GPU).  ``storage='exact'`` is the plain FP64
network, used by the finite-difference pins.
"""
from __future__ import annotations

import math

import numpy as np

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)
_erf = np.vectorize(math.erf, otypes=[np.float64])


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), via FP32, as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    """0.5 z (1 + erf(z / sqrt 2))."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / SQRT2))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z)."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def unpack(params, d, width, m):
    dims = [d, width, width, width, m]
    out, o = [], 0
    for l in range(4):
        W = np.asarray(params[o:o + dims[l + 1] * dims[l]], np.float64).reshape(dims[l + 1], dims[l])
        o += dims[l + 1] * dims[l]
        b = np.asarray(params[o:o + dims[l + 1]], np.float64)
        o += dims[l + 1]
        out.append((W, b))
    assert o == len(params)
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def _r(x, storage):
    return bf16_round(x) if storage == "bf16" else np.asarray(x, np.float64)


def forward(params, X, d, width, m, storage="bf16"):
    """Network output (standardised space) and the cache of the backward pass."""
    layers = unpack(params, d, width, m)
    H = _r(X, storage)
    cache = []
    for l, (W, b) in enumerate(layers):
        Z = H @ _r(W, storage).T + b
        cache.append((H, Z))
        if l < 3:
            H = _r(gelu(Z), storage)
    return Z, cache


def loss_and_grads(params, X, Ystd, d, width, m, storage="bf16"):
    """MSE over all (batch, output) entries and its gradient (packed like params)."""
    layers = unpack(params, d, width, m)
    out, cache = forward(params, X, d, width, m, storage)
    B = X.shape[0]
    diff = out - Ystd
    loss = float(np.mean(diff * diff))
    G = _r(2.0 * diff / (B * m), storage)
    grads = [None] * 4
    for l in range(3, -1, -1):
        H, Z = cache[l]
        W, _ = layers[l]
        grads[l] = (G.T @ H, G.sum(axis=0))
        if l > 0:
            dH = G @ _r(W, storage)
            Zp = cache[l - 1][1]
            G = _r(dH * gelu_grad(Zp), storage)
    return loss, pack(grads)


def adam_step(p, g, mom, vel, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Alg. 1), t counted from 1; returns new
    (p, mom, vel)."""
    mom = beta1 * mom + (1.0 - beta1) * g
    vel = beta2 * vel + (1.0 - beta2) * g * g
    mhat = mom / (1.0 - beta1 ** t)
    vhat = vel / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), mom, vel


def cosine_lr(step, total, lr0):
    """lr0 * (1 + cos(pi * step / total)) / 2 for step in [0, total]."""
    return lr0 * 0.5 * (1.0 + math.cos(math.pi * step / total))

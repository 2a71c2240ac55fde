"""FP64 reference of the learned-proposal MLP -- TEST INFRASTRUCTURE ONLY.

Network 64 -> 256 -> 256 -> 256 -> 256 with GELU (x * Phi(x), erf form) after
the three hidden layers, trained with a mean-squared-error loss.  With
``bf16=True`` the reference rounds to bfloat16 (round to nearest even) at the
same points as the GPU kernels: the input rows, the weights, every hidden
activation after GELU, and every pre-activation gradient before it enters a
matrix product.  Everything else is FP64.  With ``bf16=False`` it is the plain
FP64 network, whose backward pass the finite-difference pin checks.

Parameter packing (row-major, output-major weights):
W1[256,64] b1[256] W2[256,256] b2[256] W3[256,256] b3[256] W4[256,256] b4[256]
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SIZES = [(256, 64), (256, 256), (256, 256), (256, 256)]
N_PARAMS = sum(o * i + o for o, i in SIZES)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, at = [], 0
    for o, i in SIZES:
        W = theta[at:at + o * i].reshape(o, i)
        at += o * i
        b = theta[at:at + o]
        at += o
        out.append((W, b))
    return out


def pack(grads):
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def forward(theta, x, bf16=True):
    """Returns (y, cache).  y is the FP64 output of the last layer."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, np.float64))
    layers = unpack(theta)
    a = rnd(x)
    acts, zs = [a], []
    for li, (W, b) in enumerate(layers):
        z = a @ rnd(W).T + b
        zs.append(z)
        if li < 3:
            a = rnd(gelu(z))
            acts.append(a)
    return zs[-1], (acts, zs)


def loss_and_grad(theta, x, t, bf16=True):
    """Mean squared error over all outputs and its gradient w.r.t. theta."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, np.float64))
    layers = unpack(theta)
    t = rnd(t)
    y, (acts, zs) = forward(theta, x, bf16)
    M = y.shape[0]
    diff = y - t
    loss = float((diff * diff).sum() / (M * y.shape[1]))
    dz = rnd(2.0 * diff / (M * y.shape[1]))
    grads = [None] * 4
    for li in range(3, -1, -1):
        W, _ = layers[li]
        dW = dz.T @ acts[li]
        db = dz.sum(0)
        grads[li] = (dW, db)
        if li > 0:
            da = dz @ rnd(W)
            dz = rnd(da * gelu_grad(zs[li - 1]))
    return loss, pack(grads)


def init_params(seed=0):
    """Uniform(+-1/sqrt(fan_in)) weights, zero biases (seeded numpy)."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in SIZES:
        bound = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-bound, bound, o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def adam_step(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) in FP64; step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v

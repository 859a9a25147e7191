"""TEST INFRASTRUCTURE ONLY: FP64 numpy oracle of the ensemble MLP surrogate.

Members map (a, omega, F, D, gamma) to <v> through 5 -> 256 -> 256 -> 256 -> 1 with
the tanh form of GELU (Hendrycks & Gimpel) between layers.  Written from those
definitions: input normalisation, affine layers, GELU, mean squared error,
back-propagation by the chain rule, and the Adam update (Kingma & Ba).
Only the tests and the benchmark's CPU leg import it.

Parameter vector of one member (133377 values, row-major [out][in] weights):
W1[256][5] | b1[256] | W2[256][256] | b2[256] | W3[256][256] | b3[256] | W4[256] | b4.
"""
from __future__ import annotations

import math

import numpy as np

IN, H = 5, 256
SIZES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
         ("W4", (H,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
C_GELU = math.sqrt(2.0 / math.pi)


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to BF16 (nearest, ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def normalise(x: np.ndarray) -> np.ndarray:
    """Map a in [0,8], omega in [1,10], F in [-0.5,0.5], log10 D in [-4,-1], gamma in [0.5,2]
    linearly onto [-1, 1]."""
    x = np.asarray(x, dtype=np.float64)
    u = np.empty_like(x)
    u[:, 0] = x[:, 0] / 4.0 - 1.0
    u[:, 1] = (x[:, 1] - 5.5) / 4.5
    u[:, 2] = 2.0 * x[:, 2]
    u[:, 3] = (np.log10(x[:, 3]) + 2.5) / 1.5
    u[:, 4] = (x[:, 4] - 1.25) / 0.75
    return u


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    t = np.tanh(C_GELU * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C_GELU * (1.0 + 3.0 * 0.044715 * z * z)


def forward(p: np.ndarray, x: np.ndarray, bf16_weights: bool = False):
    """Prediction y[B] of one member and the cache needed by backward."""
    q = unpack(p)
    W = {k: (bf16_round(q[k]) if bf16_weights and k.startswith("W") else q[k]) for k in q}
    u = normalise(x)
    z1 = u @ W["W1"].T + W["b1"]
    a1 = gelu(z1)
    z2 = a1 @ W["W2"].T + W["b2"]
    a2 = gelu(z2)
    z3 = a2 @ W["W3"].T + W["b3"]
    a3 = gelu(z3)
    y = a3 @ W["W4"] + W["b4"][0]
    return y, dict(u=u, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, W=W)


def loss(p: np.ndarray, x: np.ndarray, t: np.ndarray, bf16_weights: bool = False) -> float:
    y, _ = forward(p, x, bf16_weights)
    return float(np.mean((y - t) ** 2))


def backward(p: np.ndarray, x: np.ndarray, t: np.ndarray, bf16_weights: bool = False):
    """(loss, gradient of the mean squared error w.r.t. the parameter vector)."""
    y, c = forward(p, x, bf16_weights)
    W = c["W"]
    B = len(t)
    dy = 2.0 * (y - t) / B
    g = {}
    g["W4"] = c["a3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = np.outer(dy, W["W4"]) * gelu_grad(c["z3"])
    g["W3"] = dz3.T @ c["a2"]
    g["b3"] = dz3.sum(axis=0)
    dz2 = (dz3 @ W["W3"]) * gelu_grad(c["z2"])
    g["W2"] = dz2.T @ c["a1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ W["W2"]) * gelu_grad(c["z1"])
    g["W1"] = dz1.T @ c["u"]
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), pack(g)


def adam(p, g, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def ensemble_stats(preds: np.ndarray):
    """Mean and population standard deviation over members (axis 0)."""
    return preds.mean(axis=0), preds.std(axis=0)


def route(std: np.ndarray, threshold: float) -> np.ndarray:
    """Indices (increasing) of the queries whose ensemble std exceeds the threshold."""
    return np.nonzero(std > threshold)[0].astype(np.uint32)

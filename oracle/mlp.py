"""FP64 oracle for the learned rewrite policy's network (test infrastructure).

The paper does not define a learned policy; this network is this library's
addition, a replacement for the thin-level test of the naive strategy (Sec. III).
Architecture: 20 inputs -> 64 -> 64 -> 1, ReLU after the hidden layers, sigmoid
on the output, mean binary cross-entropy loss, Adam. Written plainly with numpy
matrix products so it can be read against the definitions; used to check the
GPU's FP32 forward/backward/Adam kernels.

Flat parameter layout (5569 values):
  W1[64,20] | b1[64] | W2[64,64] | b2[64] | W3[64] | b3[1]   (row-major)
"""
from __future__ import annotations

import numpy as np

F_IN, H = 20, 64
SIZES = [("W1", (H, F_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], np.float64).reshape(shp)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in SIZES])


def init(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases (float64; cast for the GPU)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SIZES:
        if name.startswith("W"):
            fan_in = shp[-1] if len(shp) == 2 else H
            lim = np.sqrt(6.0 / fan_in)
            p[name] = rng.uniform(-lim, lim, size=shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p)


def forward(theta: np.ndarray, feat: np.ndarray):
    """Returns (probabilities [B], cache for backward)."""
    p = unpack(theta)
    x = np.asarray(feat, np.float64)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"] + p["b3"][0]
    prob = 1.0 / (1.0 + np.exp(-z))
    return prob, (x, a1, h1, a2, h2, z)


def loss(theta: np.ndarray, feat: np.ndarray, label: np.ndarray) -> float:
    """Mean binary cross-entropy, written on the logit for stability:
    max(z,0) - z*y + log(1 + exp(-|z|))."""
    _, (_, _, _, _, _, z) = forward(theta, feat)
    y = np.asarray(label, np.float64)
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(theta: np.ndarray, feat: np.ndarray, label: np.ndarray):
    """Gradient of the mean BCE with respect to every parameter (flat), and the loss."""
    p = unpack(theta)
    prob, (x, a1, h1, a2, h2, z) = forward(theta, feat)
    y = np.asarray(label, np.float64)
    B = x.shape[0]
    dz = (prob - y) / B
    g = {}
    g["W3"] = h2.T @ dz
    g["b3"] = np.array([dz.sum()])
    dh2 = np.outer(dz, p["W3"])
    da2 = dh2 * (a2 > 0.0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0.0)
    g["W1"] = da1.T @ x
    g["b1"] = da1.sum(axis=0)
    lval = float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))
    return pack(g), lval


def adam(theta, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected; step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v

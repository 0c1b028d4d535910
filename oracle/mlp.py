"""FP64 oracle of the spectrum surrogate MLP (TEST INFRASTRUCTURE ONLY).

Network: the 2 normalised inputs -> 24 fixed features -> 256 -> 256 -> 256
-> 64, three hidden layers with the exact (erf) GELU, a linear output,
mean-squared-error loss, Adam.  The features are the inputs themselves and a
Fourier encoding of each (sine and cosine of 2^k w_c u_c, octaves k = 0..5 of
input 0 and 0..4 of input 1).  The computation
is done in FP64; with ``bf16=True`` values are rounded to bfloat16
(round-to-nearest-even) at the points where the GPU kernels store them in
BF16:
  - the weights W1..W4 (the GPU keeps FP32 master weights and feeds BF16
    copies to the matrix cores),
  - the hidden activations h1, h2, h3 (inputs of the next product),
  - the output gradient dL/dy and the pre-activation gradients dL/da3,
    dL/da2 (inputs of the backward products).
Biases, pre-activations, the features, the layer-1 product (K = 24) and the
gradients of W1, b1 stay in full precision.

The network is not a step of the paper's method; it is the learned add-on
whose targets are the lattice spectra of Sec. 3.1 / 4.4.2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_FREQ = (6, 5)
SIZES = (2 + 2 * sum(N_FREQ), 256, 256, 256, 64)


def features(u: np.ndarray, enc_freq=(0.0, 0.0)) -> np.ndarray:
    """(B, 2) normalised inputs u -> (B, 24): u_0, u_1, then for input 0 and
    k = 0..5 the pair sin(2^k w_0 u_0), cos(2^k w_0 u_0), then the same for
    input 1 and k = 0..4 (w = enc_freq)."""
    u = np.asarray(u, dtype=np.float64)
    cols = [u[:, 0], u[:, 1]]
    for c, K in enumerate(N_FREQ):
        for k in range(K):
            a = (2.0 ** k) * float(enc_freq[c]) * u[:, c]
            cols += [np.sin(a), np.cos(a)]
    return np.stack(cols, 1)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    Values are first rounded to float32 (the GPU holds them in FP32 before the
    conversion), then the low 16 bits of the float32 pattern are rounded away.
    """
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    """Exact GELU, x Phi(x) = x (1 + erf(x/sqrt 2)) / 2."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx GELU = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(p: dict, u: np.ndarray, bf16: bool = False, enc_freq=(0.0, 0.0)) -> tuple:
    """u: (B, 2) normalised inputs -> y: (B, 64); returns y and the cache for
    backward."""
    r = bf16_round if bf16 else (lambda v: v)
    W = [r(p[f"W{l}"]) for l in range(1, 5)]
    x = features(u, enc_freq)
    c = {"x": x, "W": W}
    a1 = x @ W[0].T + p["b1"]
    h1 = r(gelu(a1))
    a2 = h1 @ W[1].T + p["b2"]
    h2 = r(gelu(a2))
    a3 = h2 @ W[2].T + p["b3"]
    h3 = r(gelu(a3))
    y = h3 @ W[3].T + p["b4"]
    c.update(a1=a1, h1=h1, a2=a2, h2=h2, a3=a3, h3=h3)
    return y, c


def loss_and_grads(p: dict, u: np.ndarray, t: np.ndarray, bf16: bool = False, enc_freq=(0.0, 0.0)) -> tuple:
    """Mean over batch and outputs of (y - t)^2 and its gradients."""
    r = bf16_round if bf16 else (lambda v: v)
    y, c = forward(p, u, bf16, enc_freq)
    B = u.shape[0]
    L = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / (B * y.shape[1])
    W = c["W"]
    g = {}
    dyb = r(dy)
    g["W4"] = dyb.T @ c["h3"]
    g["b4"] = dy.sum(0)
    da3 = (dyb @ W[3]) * gelu_grad(c["a3"])
    da3b = r(da3)
    g["W3"] = da3b.T @ c["h2"]
    g["b3"] = da3.sum(0)
    da2 = (da3b @ W[2]) * gelu_grad(c["a2"])
    da2b = r(da2)
    g["W2"] = da2b.T @ c["h1"]
    g["b2"] = da2.sum(0)
    da1 = (da2b @ W[1]) * gelu_grad(c["a1"])
    g["W1"] = da1.T @ c["x"]
    g["b1"] = da1.sum(0)
    return L, g


def adam_step(p: dict, g: dict, state: dict, lr: float, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
    """Adam (Kingma & Ba 2015) with bias correction, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m" + k, np.zeros_like(p[k]))
        v = state.setdefault("v" + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)

"""Reference multilayer perceptron of the growth-rate surrogate (float64 numpy).

TEST INFRASTRUCTURE ONLY (part of the oracle; see oracle/oracle.py).

Forward: hidden layers z = a W^T + b, a' = SiLU(z) = z / (1 + exp(-z)); the last layer is linear,
its output split into a mean head mu and a log-variance head s. Loss: the Gaussian negative
log-likelihood (1/(B D)) sum 0.5 (exp(-s)(t - mu)^2 + s), s clamped to [-12, 12]. Backward by the
chain rule, written out layer by layer; Adam with bias correction.

With bf16=True the reference rounds to bfloat16 (round to nearest even) exactly where the GPU
path does: GEMM inputs (input rows, weights, activations, back-propagated gradients); everything
else stays float64 here (float32 on the GPU).
"""
from __future__ import annotations

import numpy as np


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), via float32: keep the upper 16 bits."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(widths, flat):
    """Packed parameters -> [(W (out x in), b (out))] per layer."""
    out, o = [], 0
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        W = np.asarray(flat[o:o + n_in * n_out], dtype=np.float64).reshape(n_out, n_in)
        o += n_in * n_out
        b = np.asarray(flat[o:o + n_out], dtype=np.float64)
        o += n_out
        out.append((W, b))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(layers, x, bf16: bool = False):
    """Returns (y, cache) with cache = (a_l inputs of every layer, z_l of the hidden layers)."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    a = [rnd(x)]
    zs = []
    for i, (W, b) in enumerate(layers):
        z = a[-1] @ rnd(W).T + b
        if i + 1 < len(layers):
            zs.append(z)
            a.append(rnd(silu(z)))
        else:
            return z, (a, zs)


def nll(y, t):
    """Loss and dL/dy for the mean / log-variance heads."""
    B, D = t.shape
    mu, s_raw = y[:, :D], y[:, D:]
    s = np.clip(s_raw, -12.0, 12.0)
    e = np.exp(-s)
    r = t - mu
    loss = (0.5 * (e * r * r + s)).sum() / (B * D)
    dmu = -e * r / (B * D)
    ds = np.where((s_raw > -12.0) & (s_raw < 12.0), 0.5 * (1.0 - e * r * r) / (B * D), 0.0)
    return loss, np.concatenate([dmu, ds], axis=1)


def loss_and_grads(layers, x, t, bf16: bool = False):
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    y, (a, zs) = forward(layers, x, bf16)
    loss, dy = nll(y, t)
    dz = rnd(dy)
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        gW = dz.T @ a[i]
        gb = dz.sum(axis=0)
        grads[i] = (gW, gb)
        if i > 0:
            dz = rnd((dz @ rnd(W)) * dsilu(zs[i - 1]))
    return loss, grads


class Adam:
    """Adam with bias correction on a packed parameter vector."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, w, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return w - self.lr * mh / (np.sqrt(vh) + self.eps)

"""Oracle MLP for the learned initial interface traces.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy in FP64:
Linear -> GELU (erf form) repeated, then a final Linear; mean-squared-error
loss; Adam.  With skip=True the final Linear reads the last hidden
activations followed by the network input (concatenated in that order), so
the network is a GELU trunk plus a linear map of its input.  An optional
mode rounds every matrix-product operand to bfloat16 (round to nearest, ties
to even) before the product, mirroring a network that keeps BF16 weights and
BF16 activations and accumulates in higher precision.

Weights are stored as W[out][in] (y = x W^T + b).
"""
from __future__ import annotations

import math

import numpy as np

_ERF = np.vectorize(math.erf, otypes=[np.float64])


def bf16_round(x):
    """Round FP64/FP32 values to the nearest bfloat16 (ties to even), returned
    as FP64.  Goes through FP32 first (as a device would hold it)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + _ERF(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _ERF(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


class MLP:
    """params: list of (W [out][in], b [out]) in FP64."""

    def __init__(self, params, bf16=False, skip=False):
        self.params = [(np.array(W, dtype=np.float64), np.array(b, dtype=np.float64))
                       for W, b in params]
        self.bf16 = bf16
        self.skip = skip and len(self.params) > 1

    def _r(self, a):
        return bf16_round(a) if self.bf16 else a

    def forward(self, x):
        """Returns output y and the cache of (input, pre-activation) per layer."""
        x = np.asarray(x, dtype=np.float64)
        a = x
        cache = []
        L = len(self.params)
        for l, (W, b) in enumerate(self.params):
            if self.skip and l == L - 1:
                a = np.concatenate([a, x], axis=1)
            ar = self._r(a)
            z = ar @ self._r(W).T + b
            cache.append((ar, z))
            a = gelu(z) if l < L - 1 else z
        return a, cache

    def loss(self, x, t):
        y, _ = self.forward(x)
        return float(np.mean((y - t) ** 2))

    def backward(self, x, t):
        """Loss and gradients [(dW, db)] of the mean-squared error."""
        y, cache = self.forward(x)
        t = np.asarray(t, dtype=np.float64)
        n = y.size
        loss = float(np.mean((y - t) ** 2))
        d = 2.0 * (y - t) / n  # dL/dz of the last layer
        grads = [None] * len(self.params)
        for l in range(len(self.params) - 1, -1, -1):
            W, b = self.params[l]
            ar, z = cache[l]
            if l < len(self.params) - 1:
                d = d * gelu_grad(z)
            dr = self._r(d)
            grads[l] = (dr.T @ ar, d.sum(axis=0))
            if l > 0:
                d = dr @ self._r(W)
                if self.skip and l == len(self.params) - 1:
                    d = d[:, : self.params[l - 1][0].shape[0]]  # the input part ends here
        return loss, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected) on FP64 masters; state = dict(t, m, v)."""
    t = state.get("t", 0) + 1
    state["t"] = t
    if "m" not in state:
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    out = []
    for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for i, (p, g) in enumerate(((W, gW), (b, gb))):
            m = beta1 * state["m"][l][i] + (1 - beta1) * g
            v = beta2 * state["v"][l][i] + (1 - beta2) * g * g
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
            ms = list(state["m"][l])
            vs = list(state["v"][l])
            ms[i], vs[i] = m, v
            state["m"][l] = tuple(ms)
            state["v"][l] = tuple(vs)
        out.append(tuple(new))
    return out

"""Reference MLP of the learned Newton initial guess (oracle; test infrastructure only).

Not part of the paper: the per-element network is a build addition.  The oracle mirrors
the arithmetic contract of the GPU kernels, not their code:
  * operands of every dense product are rounded to BF16 (round to nearest, ties to even);
  * products are accumulated exactly (FP64 here, FP32 on the GPU);
  * hidden layers apply GELU in its erf form; the last layer is linear;
  * loss 0.5/B sum (y - t)^2 over the valid output columns; backward rounds dZ and the
    layer inputs to BF16 where they enter a product;
  * Adam with bias-corrected moments on FP32 master weights.
`rounding=False` switches the BF16 rounding off (used to pin the oracle to autograd).
"""
import math

import numpy as np


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).reshape(x.shape)


_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def pad32(w):
    return (w + 31) // 32 * 32


class MLP:
    """Widths w[0..L]; W[l] has shape (P(w_{l+1}), P(w_l)), b[l] shape (P(w_{l+1}),)."""

    def __init__(self, widths, W, b, rounding=True):
        self.widths = list(widths)
        self.W = [np.asarray(x, dtype=np.float64) for x in W]
        self.b = [np.asarray(x, dtype=np.float64) for x in b]
        self.rounding = rounding

    def _r(self, x):
        return bf16_round(x).astype(np.float64) if self.rounding else np.asarray(x, dtype=np.float64)

    def forward(self, x):
        """Returns (zs, acts) per layer; x has shape (B, P(w_0))."""
        a = np.asarray(x, dtype=np.float64)
        zs, acts = [], []
        L = len(self.W)
        for l in range(L):
            z = self._r(a) @ self._r(self.W[l]).T + self.b[l]
            a = gelu(z) if l < L - 1 else z
            zs.append(z)
            acts.append(a)
        return zs, acts

    def backward(self, x, zs, acts, t):
        """Gradients (dW, db) and loss of 0.5/B sum_{valid cols} (y - t)^2."""
        B = x.shape[0]
        L = len(self.W)
        nvalid = self.widths[-1]
        d = acts[-1] - t
        d[:, nvalid:] = 0.0
        loss = 0.5 * float(np.sum(d * d)) / B
        dZ = d / B
        dW, db = [None] * L, [None] * L
        for l in range(L - 1, -1, -1):
            xin = x if l == 0 else acts[l - 1]
            dW[l] = self._r(dZ).T @ self._r(xin)
            db[l] = dZ.sum(axis=0)
            if l > 0:
                dX = self._r(dZ) @ self._r(self.W[l])
                dZ = dX * gelu_d(zs[l - 1])
        return dW, db, loss


def adam_step(p, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step: p -= lr mhat / (sqrt(vhat) + eps), bias-corrected moments."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mhat = m1 / (1 - b1 ** step)
    vhat = m2 / (1 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m1, m2

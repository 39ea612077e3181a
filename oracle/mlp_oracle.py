"""FP64 reference of the learned surrogate (test infrastructure only).

The surrogate is not in the paper: it is a coordinate MLP trained on fields computed
by the RSI model.  This module spells out its forward pass, its gradients and the Adam
update in plain numpy FP64, optionally rounding to bfloat16 at exactly the points where
the GPU kernels hold bfloat16 operands, so that GPU results can be compared element
by element.  A finite-difference test (pure FP64, no rounding) pins the gradients of
this reference itself.

Network (all matrices row-major, out x in):
    v      in [-1, 1]^5, the affine image of (x, z, f, depth, tilt) on their box
    u      = B v                     B: [m, 5] fixed (not trained)
    h0     = [sin(2 pi u), cos(2 pi u)]                         -> bf16
    z_l    = W_l h_{l-1} + b_l,  h_l = silu(z_l)  (l = 1..L)    W_l, h_l -> bf16
    y      = Wo h_L + bo                          (FP32 head, 2 outputs)
    loss   = sum_b |y_b - t_b|^2 / (2 n_batch)
"""
from __future__ import annotations

import numpy as np


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), via float32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    bias = np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))
    r = ((u + bias) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def normalise(raw: np.ndarray, lo, hi) -> np.ndarray:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return 2.0 * (np.asarray(raw, dtype=np.float64) - lo) / (hi - lo) - 1.0


class MLPOracle:
    """noise = (rng, rel): multiply every value by (1 + rel N(0,1)) before it is rounded to
    bfloat16.  With rel at the FP32 accumulation error this estimates how far two correct
    implementations drift apart through bfloat16 roundings taken on opposite sides of a
    rounding boundary (used to size the GPU parity tolerance of deep networks)."""

    def __init__(self, Bff, Ws, bs, Wo, bo, emulate_bf16: bool = True, noise=None):
        self.B = np.asarray(Bff, dtype=np.float64)
        self.Ws = [np.asarray(W, dtype=np.float64) for W in Ws]
        self.bs = [np.asarray(b, dtype=np.float64) for b in bs]
        self.Wo = np.asarray(Wo, dtype=np.float64)
        self.bo = np.asarray(bo, dtype=np.float64)
        # weights are stored values: both sides round them identically, never perturbed
        self.rw = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
        if not emulate_bf16:
            self.r = lambda a: np.asarray(a, dtype=np.float64)
        elif noise is None:
            self.r = bf16
        else:
            rng, rel = noise
            self.r = lambda a: bf16(np.asarray(a) * (1.0 + rel * rng.standard_normal(np.shape(a))))

    def forward(self, v):
        r = self.r
        u = v @ self.B.T
        h = r(np.concatenate([np.sin(2 * np.pi * u), np.cos(2 * np.pi * u)], axis=1))
        hs, zs = [h], []
        for W, b in zip(self.Ws, self.bs):
            z = h @ self.rw(W).T + b
            h = r(silu(z))
            zs.append(z)
            hs.append(h)
        y = h @ self.Wo.T + self.bo
        return y, (hs, zs)

    def loss_and_grads(self, v, t):
        r = self.r
        y, (hs, zs) = self.forward(v)
        n = v.shape[0]
        diff = y - t
        loss = 0.5 * np.sum(diff * diff) / n
        dy = diff / n
        gWo = dy.T @ hs[-1]
        gbo = dy.sum(0)
        dz = r((dy @ self.Wo) * silu_grad(zs[-1]))
        gWs, gbs = [None] * len(self.Ws), [None] * len(self.Ws)
        for l in range(len(self.Ws) - 1, -1, -1):
            gWs[l] = dz.T @ hs[l]
            gbs[l] = dz.sum(0)
            if l > 0:
                dz = r((dz @ self.rw(self.Ws[l])) * silu_grad(zs[l - 1]))
        return loss, y, {"Ws": gWs, "bs": gbs, "Wo": gWo, "bo": gbo}

    # flat parameter order shared with the GPU: W_1, b_1, ..., W_L, b_L, Wo, bo
    def flat(self):
        parts = []
        for W, b in zip(self.Ws, self.bs):
            parts += [W.ravel(), b.ravel()]
        parts += [self.Wo.ravel(), self.bo.ravel()]
        return np.concatenate(parts)

    @staticmethod
    def flat_grads(g):
        parts = []
        for W, b in zip(g["Ws"], g["bs"]):
            parts += [W.ravel(), b.ravel()]
        parts += [g["Wo"].ravel(), g["bo"].ravel()]
        return np.concatenate(parts)

    def set_flat(self, p):
        o = 0
        for l in range(len(self.Ws)):
            n = self.Ws[l].size
            self.Ws[l] = p[o:o + n].reshape(self.Ws[l].shape)
            o += n
            n = self.bs[l].size
            self.bs[l] = p[o:o + n].copy()
            o += n
        n = self.Wo.size
        self.Wo = p[o:o + n].reshape(self.Wo.shape)
        o += n
        self.bo = p[o:o + self.bo.size].copy()


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), bias-corrected; returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

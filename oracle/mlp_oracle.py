"""FP64 NumPy reference of the MLP surrogate (forward, loss, backward, Adam).

TEST INFRASTRUCTURE ONLY: used by the tests; the GPU product path never
imports it.

The network: z-scored inputs (padded with zeros to a multiple of 32), hidden
layers Z = X W + b, A = GELU(Z) with GELU(x) = x Phi(x), a linear output
layer, and the mean squared error on z-scored targets.  With `rounded=True`
the operands are rounded to BF16 (round to nearest even) exactly where the
GPU stores BF16: the inputs X0, the weights, the activations A, the output
gradient and the hidden-layer gradients dZ.  Everything else is FP64.
With `rounded=False` the same function is smooth, and its gradients are
pinned by central finite differences.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + ((u >> 16) & 1) + 0x7FFF) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


class MLPOracle:
    def __init__(self, Ws, bs, x_mean, x_std, y_mean, y_std, n_in):
        self.Ws = [np.asarray(W, np.float64) for W in Ws]
        self.bs = [np.asarray(b, np.float64) for b in bs]
        self.x_mean, self.x_std = np.asarray(x_mean, np.float32), np.asarray(x_std, np.float32)
        self.y_mean, self.y_std = np.asarray(y_mean, np.float32), np.asarray(y_std, np.float32)
        self.n_in = n_in
        self.K0p = self.Ws[0].shape[0]

    def _r(self, x, rounded):
        return bf16(x) if rounded else np.asarray(x, np.float64)

    def forward(self, x_raw, rounded=True):
        x32 = np.asarray(x_raw, np.float32)
        xn = ((x32 - self.x_mean) / self.x_std).astype(np.float64)
        X = np.zeros((x32.shape[0], self.K0p))
        X[:, :self.n_in] = xn
        X = self._r(X, rounded)
        acts, pre = [X], []
        W = [self._r(w, rounded) for w in self.Ws]
        for l in range(len(W) - 1):
            Z = acts[-1] @ W[l] + self.bs[l]
            pre.append(Z)
            acts.append(self._r(gelu(Z), rounded))
        pred = acts[-1] @ W[-1] + self.bs[-1]
        return pred, dict(acts=acts, pre=pre, W=W)

    def loss_and_grads(self, x_raw, y_raw, rounded=True):
        pred, c = self.forward(x_raw, rounded)
        y32 = np.asarray(y_raw, np.float32)
        t = ((y32 - self.y_mean) / self.y_std).astype(np.float64)
        d = pred - t
        n = d.size
        loss = float(np.mean(d * d))
        dZ = self._r(2.0 * d / n, rounded)
        L = len(c["W"])
        dWs, dbs = [None] * L, [None] * L
        for l in range(L - 1, -1, -1):
            dWs[l] = c["acts"][l].T @ dZ
            dbs[l] = dZ.sum(axis=0)
            if l > 0:
                dZ = self._r((dZ @ c["W"][l].T) * gelu_grad(c["pre"][l - 1]), rounded)
        return loss, dWs, dbs, pred


def adam_step(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One bias-corrected Adam step (Kingma & Ba) with decoupled weight decay
    wd (Loshchilov & Hutter; wd = 0 is plain Adam), returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    w = w - lr * ((m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps) + wd * w)
    return w, m, v


# ---------------------------------------------------------------------------
# Predict-or-Monte-Carlo decision (the surrogate's answer for the thermal side
# of the hybrid iteration, coupling paragraph).  The network's outputs are the
# encoding [heat shape (ncell), density shape (ncell), log heat norm, log
# density norm]; definitions as documented for the library's entry point.
# ---------------------------------------------------------------------------
def ensemble_mean_spread(preds):
    """Mean and sample standard deviation (divisor members - 1) over the
    first axis (members) of de-normalised predictions [E, batch, n_out]."""
    p = np.asarray(preds, np.float64)
    if p.shape[0] < 2:
        return p.mean(0), np.zeros(p.shape[1:])
    return p.mean(0), p.std(0, ddof=1)


def decode_maps(mean, ncell):
    """Per-subcell heat and density maps [batch, 2 ncell] from the mean
    encoding: each map is its shape times exp(its log-norm)."""
    m = np.atleast_2d(np.asarray(mean, np.float64))
    out = np.empty((m.shape[0], 2 * ncell))
    for k in range(2):
        out[:, k * ncell:(k + 1) * ncell] = m[:, k * ncell:(k + 1) * ncell] * np.exp(m[:, 2 * ncell + k])[:, None]
    return out


def predicted_error(mean, spread, ncell, calib):
    """calib x the larger over the two maps of hypot(|spread of the shape| /
    |mean shape|, spread of the log-norm), norms over the subcells."""
    m = np.atleast_2d(np.asarray(mean, np.float64))
    s = np.atleast_2d(np.asarray(spread, np.float64))
    err = np.zeros(m.shape[0])
    for k in range(2):
        sl = slice(k * ncell, (k + 1) * ncell)
        rel = np.linalg.norm(s[:, sl], axis=1) / np.maximum(np.linalg.norm(m[:, sl], axis=1), 1e-300)
        err = np.maximum(err, np.hypot(rel, s[:, 2 * ncell + k]))
    return calib * err


def inside_box(x, lo, hi):
    """Every feature within [lo, hi] widened by 1e-6 max(1, hi - lo)."""
    x, lo, hi = (np.asarray(a, np.float64) for a in (x, lo, hi))
    pad = 1e-6 * np.maximum(1.0, np.abs(hi - lo))
    return bool(np.all((x >= lo - pad) & (x <= hi + pad)))

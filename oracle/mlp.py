"""Learned coefficient predictor: a small MLP trained with Adam (not in the paper).

Test infrastructure only (see oracle/__init__.py).

Shape: inputs (the last H coefficient vectors of the method, lag order, and sin t,
cos t) -> L hidden layers of width W with SiLU -> M outputs; weights kept in float32
(held here in float64) and used in bfloat16, every product accumulated in float32 on
the device (float64 here).  The rounding points, which the HIP kernels share:

* forward, layer l:  z_l = bf16(a_l) bf16(W_l)^T + b_l;  a_{l+1} = silu(z_l) for hidden
  layers, the output y = z_L;
* loss: mean over the batch and outputs of (y - target)^2;
* backward: dz_L = 2 (y - target) / (B M); dW_l = bf16(dz_l)^T bf16(a_l);
  db_l = sum over the batch of dz_l; da_l = bf16(dz_l) bf16(W_l);
  dz_{l-1} = da_l * silu'(z_{l-1});
* Adam (Kingma and Ba, 2015) on the float32 master weights.

``rounding=False`` drops every bf16 rounding (plain FP64), for the derivative checks.
Parity: pinned by finite differences, torch autograd and torch's Adam (tests).
"""

from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) through float32, as float64."""
    a = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


class MLP:
    """Parameters: list of (W_l (out x in), b_l (out,)) in float64."""

    def __init__(self, params, rounding: bool = True):
        self.params = [(np.array(W, dtype=np.float64), np.array(b, dtype=np.float64)) for W, b in params]
        self.rounding = rounding

    def _r(self, x):
        return bf16(x) if self.rounding else x

    def forward(self, X):
        """Returns (y, cache) for a batch X (B x n_in)."""
        a = np.asarray(X, dtype=np.float64)
        acts, zs = [a], []
        L = len(self.params)
        for l, (W, b) in enumerate(self.params):
            z = self._r(a) @ self._r(W).T + b
            zs.append(z)
            a = silu(z) if l < L - 1 else z
            acts.append(a)
        return a, (acts, zs)

    def loss_and_grads(self, X, T):
        """Mean squared error and its gradients [(dW_l, db_l)]."""
        y, (acts, zs) = self.forward(X)
        B, m = y.shape
        diff = y - T
        loss = float(np.mean(diff * diff))
        dz = 2.0 * diff / (B * m)
        grads = [None] * len(self.params)
        for l in range(len(self.params) - 1, -1, -1):
            W, _ = self.params[l]
            dzr = self._r(dz)
            grads[l] = (dzr.T @ self._r(acts[l]), dz.sum(0))
            if l > 0:
                da = dzr @ self._r(W)
                dz = da * silu_grad(zs[l - 1])
        return loss, grads


class Adam:
    """Adam with bias correction; one (m, v) pair per parameter array."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        self.v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, (pair, gpair) in enumerate(zip(params, grads)):
            new = []
            for j in range(2):
                g = gpair[j]
                self.m[i][j] = self.b1 * self.m[i][j] + (1.0 - self.b1) * g
                self.v[i][j] = self.b2 * self.v[i][j] + (1.0 - self.b2) * g * g
                new.append(pair[j] - self.lr * (self.m[i][j] / c1) / (np.sqrt(self.v[i][j] / c2) + self.eps))
            out.append((new[0], new[1]))
        return out


def train(model: MLP, X, T, epochs: int, batch: int, lr: float, order):
    """Minibatch Adam over the samples in the given order (one permutation per epoch,
    rows of `order`); returns the per-step losses."""
    opt = Adam(model.params, lr=lr)
    losses = []
    n = X.shape[0]
    for e in range(epochs):
        perm = order[e]
        for s0 in range(0, n - batch + 1, batch):
            idx = perm[s0:s0 + batch]
            loss, g = model.loss_and_grads(X[idx], T[idx])
            model.params = opt.step(model.params, g)
            losses.append(loss)
    return losses

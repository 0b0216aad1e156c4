"""Learned initial guess on top of Alg. 1 (not in the paper).

Test infrastructure only (see oracle/__init__.py).

* Target of step i (recorded when its solution x_i is pushed): the coefficients, in lag
  order (oldest history column first), of the sketched least-squares fit of x_i by the
  history X_i that step used, restricted to the basis the sketched QR kept:
  c_i = T1 T1^T (S X_i)^T (S x_i)  (S X_i T1 has orthonormal columns, R3).
* Guess of step i, once n_hist targets exist: the MLP (oracle.mlp) maps the targets of
  steps i - n_hist .. i - 1 and sin t_i, cos t_i, standardised, to standardised
  coefficients; x_pred = X_i c with c mapped back; the guess is x_pred when
  ||b - A x_pred|| < ||b - A x0_projection|| (finite), else the projection's x0.
"""

from __future__ import annotations

import numpy as np

from . import basis as bs
from .mlp import MLP
from .sequence import Sequence


def sketched_ls_target(X, SX, Sx, tau_s=1e-12, tau_c=1e-12):
    """c = T1 T1^T SX^T Sx with T1 from the sketched QR of SX (columns in X's order)."""
    M = X.shape[1]
    if M == 0:
        return np.zeros(0)
    if not np.all(np.isfinite(SX)):
        return np.zeros(M)
    B = bs.sketched_basis(X, SX, None, tau_s, tau_c)
    return B.T1 @ (B.T1.T @ (SX.T @ Sx))


class LearnedSequence(Sequence):
    def attach(self, model: MLP, mu_in, sd_in, mu_out, sd_out, n_hist: int = 8):
        self.model = model
        self.mu_in, self.sd_in = np.asarray(mu_in, float), np.asarray(sd_in, float)
        self.mu_out, self.sd_out = np.asarray(mu_out, float), np.asarray(sd_out, float)
        self.n_hist = n_hist
        self.targets: list[np.ndarray] = []
        self.t_now = 0.0
        self.last_used = False

    def push(self, x):
        X, SX = self.history()
        xs = np.array(x, dtype=np.float64)
        if self.store is not None:
            xs = self.store(xs)
        c = np.zeros(self.M)
        if X.shape[1] > 0:
            c[: X.shape[1]] = sketched_ls_target(X, SX, self.S.apply(xs), self.tau_s, self.tau_c)
        self.targets.append(c)
        super().push(x)

    def features(self, t):
        f = np.concatenate(self.targets[-self.n_hist:] + [np.array([np.sin(t), np.cos(t)])])
        return (f - self.mu_in) / self.sd_in

    def initial_guess(self, A, b):
        g = super().initial_guess(A, b)
        self.last_used = False
        X, _ = self.history()
        if self.guess != "projection" or X.shape[1] == 0 or len(self.targets) < self.n_hist:
            return g
        y, _ = self.model.forward(self.features(self.t_now)[None, :])
        c = y[0] * self.sd_out + self.mu_out
        xp = X @ c[: X.shape[1]]
        r0 = np.linalg.norm(b - A @ g.x0)
        rp = np.linalg.norm(b - A @ xp)
        if np.isfinite(rp) and rp < r0:
            self.last_used = True
            return bs.Guess(xp, g.k, g.k2, g.c, c[: X.shape[1]], False)
        return g

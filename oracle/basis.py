"""Basis generation and the reduced problem (Alg. 1 (basis and reduced problem), Algs. 2 and 3).

The step of Alg. 1 that this module implements, for a history X = [x(t_{i-M}) | ... |
x(t_{i-1})] (Section 2), is

1. basis Q of a subspace S of span(X) (Alg. 1 (basis)):
   * randomized range finder (Section 2.2, Alg. 3): Omega = X Z with Z Gaussian
     (M x m); Z = I when m = M, which spans the same space;
   * orthonormalisation by a sketched QR: QR with column pivoting of the small matrix
     Y = S Omega = (S X) Z gives R11 and the numerical rank k (|R_jj| > tau_s |R_11|);
     Q1 = Omega P R11^-1 is then nearly orthonormal, and a pivoted Cholesky factor of
     G = Q1^T Q1 (threshold tau_c relative to the largest diagonal entry) finishes it,
     Q = Q1 P2 R2^-1 with k' columns;
2. reduced problem (Alg. 1 (reduced problem)): with W = A Q,
   * minimum residual (the paper's choice, Section 2): min_z || W z - b ||_2, solved
     through the normal equations W^T W z = W^T b;
   * Galerkin: Q^T A Q y = Q^T b (Cholesky for the SPD / CG path, LU with partial
     pivoting otherwise);
   and x0 = Q y.

Also here: the plain definitions the method reaches when span(X) is numerically full
rank (used as pins), POD (Alg. 2, eq. (optpod)) and the literal progressive update of
Alg. 3 (rank-one updates of Omega) with periodic refresh (Section 2.2, last paragraph).
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import philox as px


# ---------------------------------------------------------------------------- factors

def qr_pivoted(Y: np.ndarray):
    """Householder QR with column pivoting (Businger-Golub) of Y: Y[:, perm] = Q R.

    LAPACK's geqp3 is the step; the sign convention diag(R) >= 0 is applied after.
    """
    Q, R, perm = sla.qr(Y, mode="economic", pivoting=True)
    sgn = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * sgn[None, :], R * sgn[:, None], perm


def numerical_rank_qr(R: np.ndarray, tau: float) -> int:
    """Leading count of |R_jj| > tau |R_00| (strict); 0 when R_00 is 0."""
    d = np.abs(np.diag(R))
    if d.size == 0 or not d[0] > 0.0:
        return 0
    k = 0
    while k < d.size and d[k] > tau * d[0]:
        k += 1
    return k


def pivoted_cholesky(G: np.ndarray, tau: float):
    """Outer-product Cholesky with diagonal pivoting of a symmetric PSD matrix.

    Returns (R, perm, k) with G[perm[:k]][:, perm[:k]] = R^T R, R upper triangular k x k.
    Stops when the largest remaining Schur-complement diagonal is <= tau * max(diag G);
    ties pick the lowest index.
    """
    A = np.array(G, dtype=np.float64, copy=True)
    n = A.shape[0]
    perm = np.arange(n)
    R = np.zeros((n, n))
    dmax = float(np.max(np.diag(A))) if n else 0.0
    if not dmax > 0.0:
        return R[:0, :0], perm, 0
    k = 0
    for j in range(n):
        d = np.diag(A)[j:]
        p = j + int(np.argmax(d))
        if not A[p, p] > tau * dmax:
            break
        if p != j:
            A[[j, p], :] = A[[p, j], :]
            A[:, [j, p]] = A[:, [p, j]]
            perm[[j, p]] = perm[[p, j]]
            R[:j, [j, p]] = R[:j, [p, j]]
        R[j, j] = np.sqrt(A[j, j])
        R[j, j + 1:] = A[j, j + 1:] / R[j, j]
        A[j + 1:, j + 1:] -= np.outer(R[j, j + 1:], R[j, j + 1:])
        k = j + 1
    return R[:k, :k], perm, k


# ---------------------------------------------------------------------------- the basis

@dataclasses.dataclass
class Basis:
    """Q1 = X T1 (n x k) with the Cholesky finish (R2, perm2, k2); Q = Q1[:, perm2[:k2]] R2^-1."""

    T1: np.ndarray        # M x k
    Q1: np.ndarray        # n x k
    k: int               # rank kept by the sketched QRCP
    R2: np.ndarray        # k2 x k2
    perm2: np.ndarray     # permutation of 0..k-1
    k2: int              # rank kept by the pivoted Cholesky

    def Q(self) -> np.ndarray:
        """The orthonormal basis itself (materialised only by tests)."""
        if self.k2 == 0:
            return np.zeros((self.Q1.shape[0], 0))
        Qp = self.Q1[:, self.perm2[: self.k2]]
        return sla.solve_triangular(self.R2, Qp.T, trans="T").T


def sketched_basis(X: np.ndarray, SX: np.ndarray, Z: np.ndarray | None = None,
                   tau_s: float = 1e-12, tau_c: float = 1e-12, store=None) -> Basis:
    """Alg. 1 (basis) with the randomized range finder and a sketched QR.

    X is the n x M history, SX = S X its sketch (s x M), Z the M x m range-finder
    matrix (None means Z = I).  ``store`` rounds Q1 where it is written to memory (the
    identity in FP64; float32 in the mixed mode), before its Gram matrix is formed.
    Parity: pinned by the plain-definition, orthonormality and basis-invariance tests.
    """
    M = X.shape[1]
    Y = SX if Z is None else SX @ Z
    Zm = np.eye(M) if Z is None else Z
    if Y.shape[1] == 0:
        k = 0
    else:
        _, R, perm = qr_pivoted(Y)
        k = numerical_rank_qr(R, tau_s)
    if k == 0:
        T1 = np.zeros((M, 0))
    else:
        R11inv = sla.solve_triangular(R[:k, :k], np.eye(k))
        T1 = Zm[:, perm[:k]] @ R11inv
    Q1 = X @ T1
    if store is not None:
        Q1 = store(Q1)
    G = Q1.T @ Q1
    R2, perm2, k2 = pivoted_cholesky(G, tau_c)
    return Basis(T1, Q1, k, R2, perm2, k2)


@dataclasses.dataclass
class Guess:
    x0: np.ndarray
    k: int               # columns kept by the QRCP
    k2: int              # columns kept by the Cholesky finish
    c: np.ndarray        # x0 = Q1 c
    cX: np.ndarray       # x0 = X cX (history coordinates)
    used_fallback: bool


def reduced_solve(A, b: np.ndarray, B: Basis, projection: str = "galerkin",
                  spd: bool = True):
    """Alg. 1 (reduced problem): the reduced system on span(Q) and its coefficients c (x0 = Q1 c).

    Galerkin: (Q^T A Q) y = Q^T b; minimum residual: (W^T W) y = W^T b with W = A Q.
    """
    if B.k2 == 0:
        return np.zeros(B.k)
    W1 = np.asarray(A @ B.Q1)                  # A Q1, n x k
    idx = B.perm2[: B.k2]
    Rinv = sla.solve_triangular(B.R2, np.eye(B.k2))
    if projection == "galerkin":
        Ht = B.Q1[:, idx].T @ W1[:, idx]
        gt = B.Q1[:, idx].T @ b
        H = Rinv.T @ Ht @ Rinv
        g = Rinv.T @ gt
        if spd:
            y = sla.cho_solve(sla.cho_factor(0.5 * (H + H.T)), g)
        else:
            y = sla.lu_solve(sla.lu_factor(H), g)
    elif projection == "minres":
        Kt = W1[:, idx].T @ W1[:, idx]
        ht = W1[:, idx].T @ b
        K = Rinv.T @ Kt @ Rinv
        h = Rinv.T @ ht
        y = sla.cho_solve(sla.cho_factor(0.5 * (K + K.T)), h)
    else:
        raise ValueError(projection)
    c = np.zeros(B.k)
    c[idx] = Rinv @ y
    return c


def initial_guess(A, b, X, SX, Z=None, projection="galerkin", spd=True,
                  tau_s=1e-12, tau_c=1e-12, store=None, pod_m: int | None = None) -> Guess:
    """x0 of Alg. 1 from a history X (n x M, any column order) and its sketch SX.

    Empty or rank-zero history gives x0 = 0.  A non-finite sketch or reduced solution
    falls back to the newest history column (the paper's "Baseline" guess, Section 4),
    which the caller passes as the last column of X, or to 0 if that column is not
    finite either.  ``store`` as in ``sketched_basis``.
    """
    n, M = X.shape
    if M == 0:
        return Guess(np.zeros(n), 0, 0, np.zeros(0), np.zeros(0), False)
    if np.all(np.isfinite(SX)):
        B = (pod_basis_from_gram(X, pod_m, tau_c, store) if pod_m is not None
             else sketched_basis(X, SX, Z, tau_s, tau_c, store))
        c = reduced_solve(A, b, B, projection, spd) if np.all(np.isfinite(B.Q1)) else None
        x0 = B.Q1 @ c if c is not None else None
        if x0 is not None and np.all(np.isfinite(x0)):
            return Guess(x0, B.k, B.k2, c, B.T1 @ c, False)
        k, k2 = B.k, B.k2
    else:
        k = k2 = 0
    cX = np.zeros(M)
    if np.all(np.isfinite(X[:, -1])):
        cX[-1] = 1.0
        return Guess(X[:, -1].copy(), k, k2, np.zeros(0), cX, True)
    return Guess(np.zeros(n), k, k2, np.zeros(0), cX, True)


# ---------------------------------------------------------------------------- plain definitions

def galerkin_plain(A, b, X, rtol=1e-12):
    """x0 in span(X) with X^T (b - A x0) = 0: dense SVD of X, Galerkin on its range.

    The definition the method reaches when span(X) is numerically full rank.
    """
    U, sv, _ = np.linalg.svd(X, full_matrices=False)
    r = int(np.sum(sv > rtol * sv[0])) if sv.size and sv[0] > 0 else 0
    U = U[:, :r]
    H = U.T @ np.asarray(A @ U)
    y = np.linalg.solve(H, U.T @ b)
    return U @ y


def minres_plain(A, b, X):
    """argmin over s in span(X) of ||A s - b||_2 (Section 2): least squares on A X."""
    AX = np.asarray(A @ X)
    z, *_ = np.linalg.lstsq(AX, b, rcond=None)
    return X @ z


# ---------------------------------------------------------------------------- POD (Alg. 2)

def pod_basis(X: np.ndarray, m: int) -> np.ndarray:
    """First m left singular vectors of X (Alg. 2)."""
    U, _, _ = np.linalg.svd(X, full_matrices=False)
    return U[:, :m]


POD_TAU = 1e-14  # eigenvalues of X^T X kept above POD_TAU times the largest (sigma ratio 1e-7)


def pod_gram_factor(X: np.ndarray, m: int, tau: float = POD_TAU):
    """Alg. 2 through the Gram matrix: X^T X = V diag(lam) V^T (eigenvalues descending),
    the POD basis U_m = X V_m diag(lam_m)^(-1/2) = X T1.  Returns (T1, k) with
    k = min(m, #{lam_j > tau lam_1}); the squared singular values below tau lam_1 are
    not resolved in FP64 and are dropped.  Pinned against the SVD definition."""
    M = X.shape[1]
    if M == 0:
        return np.zeros((0, 0)), 0
    G = X.T @ X
    lam, V = np.linalg.eigh(0.5 * (G + G.T))
    order = np.argsort(-lam, kind="stable")
    lam, V = lam[order], V[:, order]
    if not lam[0] > 0.0:
        return np.zeros((M, 0)), 0
    k = int(min(m, np.sum(lam > tau * lam[0])))
    return V[:, :k] / np.sqrt(lam[:k]), k


def pod_basis_from_gram(X: np.ndarray, m: int, tau_c: float = 1e-12, store=None) -> "Basis":
    """The POD basis (Alg. 2) in the form the guess uses: Q1 = X T1 with T1 from
    ``pod_gram_factor``, then the same pivoted-Cholesky finish as the sketched basis."""
    M = X.shape[1]
    T1, k = pod_gram_factor(X, m)
    if k == 0:
        T1 = np.zeros((M, 0))
    Q1 = X @ T1
    if store is not None:
        Q1 = store(Q1)
    G = Q1.T @ Q1
    R2, perm2, k2 = pivoted_cholesky(G, tau_c)
    return Basis(T1, Q1, k, R2, perm2, k2)


# ---------------------------------------------------------------------------- Alg. 3 literal

def range_finder_z(M: int, m: int, seed: int, epoch: int, row0: int = 0) -> np.ndarray:
    """Rows row0..row0+M-1 of the Gaussian range-finder stream (M x m), epoch-keyed.

    Row r of the stream, entry c, is normal lane (c & 3) of Philox block
    (r, (epoch << 16) | (c >> 2), STREAM_RANGE_Z) under key seed.
    """
    r = np.arange(row0, row0 + M, dtype=np.uint64)
    q = np.arange((m + 3) // 4, dtype=np.uint64)
    g = px.normals4(r[:, None], (np.uint64(epoch) << np.uint64(16)) | q[None, :],
                    px.STREAM_RANGE_Z, seed)          # (M, nq, 4)
    return g.reshape(M, -1)[:, :m]


def range_finder_rows(rows, m: int, seed: int, epoch: int) -> np.ndarray:
    """The stream rows `rows` (any order) of epoch `epoch`, as a len(rows) x m matrix."""
    rows = np.asarray(rows, dtype=np.uint64)
    q = np.arange((m + 3) // 4, dtype=np.uint64)
    g = px.normals4(rows[:, None], (np.uint64(epoch) << np.uint64(16)) | q[None, :],
                    px.STREAM_RANGE_Z, seed)          # (len, nq, 4)
    return g.reshape(len(rows), -1)[:, :m]


class RangeFinderRows:
    """Which row of the Gaussian range-finder stream each history column carries
    (Alg. 3): the first full window and every `refresh` pushes after it draw a new epoch
    and give the window's columns rows 0..M-1 in lag order (lines 2-4); otherwise the
    oldest column leaves with its row and the new column takes the next unused row of
    the epoch (lines 6-9).  While the window fills, every push starts a new epoch."""

    def __init__(self, M: int, refresh: int = 50):
        self.M, self.refresh = M, refresh
        self.rows: list[int] = []
        self.epoch = 0
        self.since = 0
        self.drawn = 0

    def _scratch(self, cnt: int):
        self.epoch += 1
        self.rows = list(range(cnt))
        self.drawn = cnt
        self.since = 0

    def push(self):
        if len(self.rows) < self.M:
            self._scratch(len(self.rows) + 1)
            return
        self.rows.pop(0)
        self.since += 1
        if self.since >= self.refresh:
            self._scratch(self.M)
            return
        self.rows.append(self.drawn)
        self.drawn += 1


class ProgressiveSketch:
    """Omega = X Z kept up to date by rank-one updates (Alg. 3 (rank-one updates of Omega)).

    Every ``refresh`` pushes (and at the first full window) Z is redrawn and Omega is
    recomputed from scratch (Alg. 3 (initialisation of Omega); Section 2.2 last paragraph and the
    50-step refresh of Section 4).  Between refreshes: Omega -= x_old z_1^T; the rows of
    Z shift up by one; a new row z_M is drawn; Omega += x_new z_M^T.  Parity: the
    mathematical equivalence with the from-scratch sketch (Section 2.2) is the pin.
    """

    def __init__(self, n: int, M: int, m: int, seed: int, refresh: int = 50):
        self.n, self.M, self.m, self.seed, self.refresh = n, M, m, seed, refresh
        self.cols: list[np.ndarray] = []
        self.Omega = None
        self.Z = None
        self.epoch = 0
        self.since = 0
        self.drawn = 0

    def _from_scratch(self):
        self.epoch += 1
        self.Z = range_finder_z(len(self.cols), self.m, self.seed, self.epoch)
        self.drawn = len(self.cols)
        X = np.stack(self.cols, 1)
        self.Omega = X @ self.Z
        self.since = 0

    def push(self, x: np.ndarray):
        x = np.asarray(x, dtype=np.float64).copy()
        if len(self.cols) < self.M:
            self.cols.append(x)
            self._from_scratch()
            return
        old = self.cols.pop(0)
        self.cols.append(x)
        self.since += 1
        if self.since >= self.refresh:
            self._from_scratch()
            return
        self.Omega -= np.outer(old, self.Z[0])
        znew = range_finder_z(1, self.m, self.seed, self.epoch, row0=self.drawn)[0]
        self.drawn += 1
        self.Z = np.vstack([self.Z[1:], znew[None, :]])
        self.Omega += np.outer(x, self.Z[-1])

    def X(self) -> np.ndarray:
        return np.stack(self.cols, 1)

    def basis(self) -> np.ndarray:
        """Reduced QR of Omega (Alg. 3 (reduced QR of Omega))."""
        Q, _ = np.linalg.qr(self.Omega)
        return Q

"""Left sketch S (s x n) applied to history columns.

The paper sketches the history from the right, Omega = X Z (Section 2.2, eq.
(currenttimestep)), and orthonormalises Omega with a reduced QR (Alg. 3 (reduced QR of Omega)).
This project keeps that randomized range finder for m < M and, for the
orthonormalisation itself, uses a left subspace embedding S: the R factor of the
small matrix S X (Z) is computed and X is preconditioned by it (randomized
Cholesky-QR).  S is one of

* Gaussian: S[r, j] = g(r, j) / sqrt(s), g standard normal drawn from Philox with
  counter (j, r >> 2, STREAM_GAUSS_SKETCH), lane r & 3 of the four normals;
* SRHT (n a power of two): S = (1 / sqrt(s)) R H D with D = diag(d_j), d_j = +-1 from
  bit (j & 255) of the 256-bit Philox block (j >> 8, 0, STREAM_SRHT_SIGNS), H the
  Sylvester-Hadamard matrix H[i, j] = (-1)^popcount(i & j), and R the first s
  entries of a partial Fisher-Yates shuffle of 0..n-1 (step i swaps i with
  i + index(word0 of block (i, 0, STREAM_SRHT_ROWS), n - i)).

With ``bf16=True`` (the Gaussian sketch of the mixed-precision mode) the sketch
matrix is BF16: S = BF16(G) / sqrt(s), every normal g(r, j) rounded to FP32 and then
to BF16 (round to nearest, ties to even, on the FP32 bit pattern).  It is applied to
the FP32 column fl32(x) exactly (S x is the exact sum of the products, scaled by
1 / sqrt(s)): on the GPU the FP32 column is split exactly into three BF16 terms
(hi + mid + lo, 8 significant bits each) that the matrix cores multiply in one
instruction, accumulating in FP32 over short runs and the runs in FP64.

Pins: the Gaussian entries' moments, H^T H = n I, S's embedding distortion, the
oracle-independent numpy Philox (via ``philox``), and the BF16 rounding against
hand-worked bit patterns and torch's own float32 -> bfloat16 conversion.
"""

from __future__ import annotations

import numpy as np

from . import philox as px


def to_bf16(v) -> np.ndarray:
    """Round to FP32, then to BF16 (nearest, ties to even), returned as float64."""
    u = np.asarray(v, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gaussian_normals(s: int, j0: int, j1: int, seed: int) -> np.ndarray:
    """The standard normals g(r, j) behind columns j0..j1-1 of the Gaussian sketch."""
    j = np.arange(j0, j1, dtype=np.uint64)
    q = np.arange((s + 3) // 4, dtype=np.uint64)
    g = px.normals4(j[None, :], q[:, None], px.STREAM_GAUSS_SKETCH, seed)  # (nq, nj, 4)
    return np.transpose(g, (0, 2, 1)).reshape(-1, j1 - j0)[:s]


def gaussian_block(s: int, j0: int, j1: int, seed: int) -> np.ndarray:
    """Columns j0..j1-1 of the Gaussian sketch S (s x (j1 - j0))."""
    return gaussian_normals(s, j0, j1, seed) / np.sqrt(s)


def srht_signs(n: int, seed: int) -> np.ndarray:
    """d_j in {+1, -1} for j = 0..n-1."""
    j = np.arange(n, dtype=np.uint64)
    words = px.philox4x64(j >> np.uint64(8), 0, px.STREAM_SRHT_SIGNS, 0, seed, 0)
    lane = (j & np.uint64(255)) >> np.uint64(6)
    w = np.choose(lane.astype(np.int64), words)
    bit = (w >> (j & np.uint64(63))) & np.uint64(1)
    return 1.0 - 2.0 * bit.astype(np.float64)


def srht_rows(n: int, s: int, seed: int) -> np.ndarray:
    """The s sampled Hadamard rows: partial Fisher-Yates over 0..n-1."""
    if s > n:
        raise ValueError("SRHT needs s <= n")
    perm = {}
    out = np.empty(s, dtype=np.int64)
    for i in range(s):
        w0 = px.philox4x64(i, 0, px.STREAM_SRHT_ROWS, 0, seed, 0)[0]
        j = i + int(px.uniform_index(w0, n - i))
        vi = perm.get(i, i)
        vj = perm.get(j, j)
        perm[i], perm[j] = vj, vi
        out[i] = perm[i]
    return out


def hadamard_entries(rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """(-1)^popcount(r & c) for every pair (broadcast)."""
    v = np.bitwise_and(np.asarray(rows, dtype=np.uint64), np.asarray(cols, dtype=np.uint64))
    par = np.bitwise_count(v) & np.uint8(1)
    return 1.0 - 2.0 * par.astype(np.float64)


class Sketch:
    """The sketch S of one sequence; ``apply(x)`` returns S x (length s, float64)."""

    def __init__(self, kind: str, n: int, s: int, seed: int, chunk: int = 1 << 15, bf16: bool = False):
        self.kind, self.n, self.s, self.seed, self.chunk = kind, n, s, seed, chunk
        if bf16 and kind != "gaussian":
            raise ValueError("the BF16 sketch is the Gaussian one")
        self.bf16 = bf16
        if kind == "srht":
            if n & (n - 1):
                raise ValueError("SRHT sketch needs n to be a power of two")
            self.d = srht_signs(n, seed)
            self.rows = srht_rows(n, s, seed)
        elif kind != "gaussian":
            raise ValueError(kind)

    def block(self, j0: int, j1: int) -> np.ndarray:
        if self.kind == "gaussian":
            if self.bf16:  # S = BF16(G) / sqrt(s): the normals are rounded, the scale is not
                return to_bf16(gaussian_normals(self.s, j0, j1, self.seed)) / np.sqrt(self.s)
            return gaussian_block(self.s, j0, j1, self.seed)
        cols = np.arange(j0, j1)
        h = hadamard_entries(self.rows[:, None], cols[None, :])
        return h * self.d[None, j0:j1] / np.sqrt(self.s)

    def dense(self) -> np.ndarray:
        return self.block(0, self.n)

    def apply(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        if self.bf16:
            x = x.astype(np.float32).astype(np.float64)
        out = np.zeros(self.s if x.ndim == 1 else (self.s, x.shape[1]))
        for j0 in range(0, self.n, self.chunk):
            j1 = min(self.n, j0 + self.chunk)
            out += self.block(j0, j1) @ x[j0:j1]
        return out

"""Finite-difference operator and right-hand-side generators.

Every workload is a sequence of sparse systems A(t_i) x = b(t_i), t_i = i * dt, as in
eq. (seq) of Section 1.  The operators are variable-coefficient diffusion
-div(k grad) + c(t) I on the unit square (5-point) or cube (7-point) with zero
Dirichlet data eliminated, optionally plus first-order upwind advection v(t).grad.
Coefficients and sources are analytic in t, the setting of Assumption 1 (Section 3).

Conventions (fixed here so that the oracle and the HIP path read identical inputs):

* N interior nodes per side, h = 1 / (N + 1), node (ix, iy[, iz]) sits at
  ((ix + 1) h, (iy + 1) h[, (iz + 1) h]) and has index ix + N iy [+ N^2 iz].
* Diffusion coefficients are evaluated at face midpoints, so the diffusion part is
  symmetric.  A face on the boundary still contributes k_face / h^2 to the diagonal.
* Upwind advection: v_x >= 0 uses the backward difference (f_P - f_W) / h, v_x < 0 the
  forward one (f_E - f_P) / h; same per axis.  Boundary neighbours are Dirichlet zero.
* Each CSR row lists its columns in ascending order; the pattern never changes with t.
* b(t) is a sum of Gaussian bumps exp(-|x - c(t)|^2 / (2 sigma^2)) with moving centres.

Randomness of the inputs (bump phases and widths, the lognormal field, batch sizes)
comes from numpy's default_rng seeded per workload.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class CSR:
    """Compressed sparse row matrix: int32 row pointers and columns, float values."""

    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix(
            (self.val, self.col.astype(np.int64), self.rowptr.astype(np.int64)),
            shape=(self.n, self.n),
        )

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n), dtype=np.float64)
        for i in range(self.n):
            lo, hi = self.rowptr[i], self.rowptr[i + 1]
            a[i, self.col[lo:hi]] += self.val[lo:hi]
        return a

    def astype(self, dtype) -> "CSR":
        return CSR(self.n, self.rowptr, self.col, self.val.astype(dtype))


@dataclasses.dataclass
class SeqProblem:
    """One sequence of systems.  ``matrix(i)`` / ``rhs(i)`` give step i (t = i dt)."""

    name: str
    dim: int                      # 2 or 3
    N: int                        # interior nodes per side
    dt: float
    steps: int
    seed: int
    advection: float = 0.0        # |v|; 0 disables the advection term
    bump_phase: tuple = (0.0,)    # phi_k of each bump centre
    bump_sigma: tuple = (0.1,)    # sigma_k of each bump
    coef_phase: tuple = (0.0, 0.0, 0.0, 0.0)  # phases (phi1..phi4) of k, k(t), c(t)
    lognormal: float = 0.0        # scale of the seeded lognormal coefficient term (3-D)
    fp32_values: bool = False     # hand out float32 CSR values (A32 = fl32(A))

    def __post_init__(self):
        self.h = 1.0 / (self.N + 1)
        self.n = self.N ** self.dim
        self._pattern = None
        self._lnfield = None

    # ---------------------------------------------------------------- time
    def t(self, i: int) -> float:
        return i * self.dt

    # ---------------------------------------------------------------- coefficients
    def kcoef(self, x, y, z, t):
        """Diffusion coefficient k at points (x, y[, z]) and time t (without lognormal)."""
        p1, p2, p3, _ = self.coef_phase
        if self.dim == 2:
            return 1.0 + 0.5 * np.sin(TWO_PI * x + p1) * np.cos(TWO_PI * y + p2) * math.cos(t + p3)
        return 1.0 + 0.5 * np.sin(TWO_PI * x + t) * np.sin(TWO_PI * y) * np.sin(TWO_PI * z)

    def ccoef(self, t: float) -> float:
        return 1.0 + 0.1 * math.sin(t + self.coef_phase[3])

    def velocity(self, t: float):
        if self.advection == 0.0:
            return (0.0, 0.0)
        p3 = self.coef_phase[2]
        return (self.advection * math.cos(t + p3), self.advection * math.sin(t + p3))

    def _ln_nodes(self):
        """exp(G) on the (N+2)^3 node grid including boundary nodes, G ~ N(0, 1) i.i.d."""
        if self._lnfield is None:
            rng = np.random.default_rng([self.seed, 7])
            m = self.N + 2
            self._lnfield = np.exp(rng.standard_normal((m, m, m)))
        return self._lnfield

    # ---------------------------------------------------------------- pattern
    def _offsets(self):
        N = self.N
        if self.dim == 2:
            return [(-N, (0, -1)), (-1, (-1, 0)), (0, None), (1, (1, 0)), (N, (0, 1))]
        return [(-N * N, (0, 0, -1)), (-N, (0, -1, 0)), (-1, (-1, 0, 0)), (0, None),
                (1, (1, 0, 0)), (N, (0, 1, 0)), (N * N, (0, 0, 1))]

    def _masks(self):
        """Validity mask (n, nstencil) of each stencil entry, in ascending column order."""
        N = self.N
        idx = np.arange(self.n)
        ix = idx % N
        iy = (idx // N) % N
        iz = idx // (N * N) if self.dim == 3 else None
        cols, masks = [], []
        for off, d in self._offsets():
            cols.append(idx + off)
            if d is None:
                masks.append(np.ones(self.n, dtype=bool))
                continue
            ok = np.ones(self.n, dtype=bool)
            for coord, step in zip((ix, iy, iz), d):
                if step < 0:
                    ok &= coord > 0
                elif step > 0:
                    ok &= coord < N - 1
            masks.append(ok)
        return np.stack(cols, 1), np.stack(masks, 1)

    def pattern(self):
        """(rowptr, col) int32 arrays of the fixed sparsity pattern."""
        if self._pattern is None:
            cols, mask = self._masks()
            counts = mask.sum(1)
            rowptr = np.zeros(self.n + 1, dtype=np.int64)
            np.cumsum(counts, out=rowptr[1:])
            self._pattern = (rowptr.astype(np.int32), cols[mask].astype(np.int32), mask)
        return self._pattern[0], self._pattern[1]

    # ---------------------------------------------------------------- assembly
    def _node_index_coords(self):
        """Integer coordinates (ix + 1, iy + 1[, iz + 1]) of every node, as float64."""
        N = self.N
        idx = np.arange(self.n)
        gx = ((idx % N) + 1).astype(np.float64)
        gy = (((idx // N) % N) + 1).astype(np.float64)
        gz = ((idx // (N * N)) + 1).astype(np.float64) if self.dim == 3 else None
        return gx, gy, gz

    def _node_coords(self):
        gx, gy, gz = self._node_index_coords()
        h = self.h
        return gx * h, gy * h, (gz * h if gz is not None else None)

    def _face_k(self, t):
        """k at the 2*dim faces of every node, ordered like the stencil minus the centre.

        Face coordinates are formed as (integer + 0.5 d) * h, so the two nodes sharing a
        face see bit-identical coordinates and the diffusion part is exactly symmetric.
        """
        h = self.h
        gx, gy, gz = self._node_index_coords()
        faces = []
        if self.dim == 2:
            for d in [(0, -1), (-1, 0), (1, 0), (0, 1)]:
                faces.append(self.kcoef((gx + 0.5 * d[0]) * h, (gy + 0.5 * d[1]) * h, None, t))
            return faces
        # lognormal node values live on the padded grid, index order [iz, iy, ix]
        ln = self._ln_nodes() if self.lognormal != 0.0 else None
        g1 = np.arange(1, self.N + 1, dtype=np.float64)
        for d in [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]:
            # the 3-D k is a product of one factor per axis: evaluate the factors on the
            # 1-D face coordinates and broadcast (same values and operation order as
            # kcoef on the full grid)
            sa = np.sin(TWO_PI * ((g1 + 0.5 * d[0]) * h) + t)
            sb = np.sin(TWO_PI * ((g1 + 0.5 * d[1]) * h))
            sc = np.sin(TWO_PI * ((g1 + 0.5 * d[2]) * h))
            kf = (1.0 + ((0.5 * sa[None, None, :]) * sb[None, :, None]) * sc[:, None, None]).reshape(-1)
            if ln is not None:
                centre = ln[1:-1, 1:-1, 1:-1]
                nb = ln[1 + d[2]:ln.shape[0] - 1 + d[2], 1 + d[1]:ln.shape[1] - 1 + d[1],
                        1 + d[0]:ln.shape[2] - 1 + d[0]]
                kf = kf + self.lognormal * 0.5 * (centre + nb).reshape(-1)
            faces.append(kf)
        return faces

    def matrix(self, i: int, fp32: Optional[bool] = None) -> CSR:
        """A(t_i) in CSR (float64, or float32 values when the workload says so)."""
        t = self.t(i)
        rowptr, col = self.pattern()
        mask = self._pattern[2]
        inv_h2 = 1.0 / (self.h * self.h)
        faces = self._face_k(t)
        nst = 2 * self.dim + 1
        vals = np.zeros((self.n, nst), dtype=np.float64)
        centre = self.dim  # index of the centre entry in the stencil order
        diag = np.full(self.n, self.ccoef(t))
        off_slots = [j for j in range(nst) if j != centre]
        for slot, kf in zip(off_slots, faces):
            vals[:, slot] = -kf * inv_h2
            diag += kf * inv_h2
        if self.advection != 0.0:
            assert self.dim == 2, "advection is defined for the 2-D workloads"
            vx, vy = self.velocity(t)
            # 2-D only: slots are S=0, W=1, P=2, E=3, N=4
            for v, back, fwd in ((vx, 1, 3), (vy, 0, 4)):
                if v >= 0.0:
                    diag += v / self.h
                    vals[:, back] -= v / self.h
                else:
                    diag -= v / self.h
                    vals[:, fwd] += v / self.h
        vals[:, centre] = diag
        val = vals[mask]
        want32 = self.fp32_values if fp32 is None else fp32
        return CSR(self.n, rowptr, col, val.astype(np.float32) if want32 else val)

    def value_basis(self):
        """CSR values of A(t) as sum_k coef_k(t) B[k]; 3-D: see ``_value_basis_3d``.

        2-D workloads (B: 7 x nnz):

        A(t) = D0 + cos(t + phi3) D1 + c(t) I + |v_x| / h I + v_x+ / h (-W) + v_x- / h E
        + |v_y| / h I + v_y+ / h (-S) + v_y- / h N, with D0, D1 the diffusion part split by
        k = 1 + cos(t + phi3) K(x, y) and W, E, S, N the indicator of each stencil slot;
        `value_coefs(i)` gives the 7 coefficients.  Equal to `matrix(i)` up to rounding.
        """
        if self.dim == 3:
            return self._value_basis_3d()
        self.pattern()
        mask = self._pattern[2]
        h = self.h
        inv_h2 = 1.0 / (h * h)
        gx, gy, _ = self._node_index_coords()
        p1, p2, _, _ = self.coef_phase
        n, nst = self.n, 5
        D0 = np.zeros((n, nst))
        D1 = np.zeros((n, nst))
        slots = [0, 1, 3, 4]  # S, W, E, N
        for slot, d in zip(slots, [(0, -1), (-1, 0), (1, 0), (0, 1)]):
            x = (gx + 0.5 * d[0]) * h
            y = (gy + 0.5 * d[1]) * h
            K = 0.5 * np.sin(TWO_PI * x + p1) * np.cos(TWO_PI * y + p2)
            D0[:, slot] = -inv_h2
            D1[:, slot] = -K * inv_h2
            D0[:, 2] += inv_h2
            D1[:, 2] += K * inv_h2
        E = [np.zeros((n, nst)) for _ in range(5)]   # I, -W, E, -S, N
        E[0][:, 2] = 1.0
        E[1][:, 1] = -1.0
        E[2][:, 3] = 1.0
        E[3][:, 0] = -1.0
        E[4][:, 4] = 1.0
        return np.stack([D0[mask], D1[mask], E[0][mask], E[1][mask], E[2][mask], E[3][mask], E[4][mask]])

    def _value_basis_3d(self):
        """3-D workload (B: 4 x nnz): with sin(2 pi x + t) = sin(2 pi x) cos t + cos(2 pi x) sin t
        the face coefficients are K0 + cos t K1 + sin t K2, so
        A(t) = D(K0) + cos t D(K1) + sin t D(K2) + c(t) I, D(K) the diffusion part of K."""
        assert self.advection == 0.0, "the 3-D workloads carry no advection"
        self.pattern()
        mask = self._pattern[2]
        h = self.h
        inv_h2 = 1.0 / (h * h)
        ln = self._ln_nodes() if self.lognormal != 0.0 else None
        g1 = np.arange(1, self.N + 1, dtype=np.float64)
        n, nst, centre = self.n, 7, 3
        D = [np.zeros((n, nst)) for _ in range(3)]
        off_slots = [0, 1, 2, 4, 5, 6]
        for slot, d in zip(off_slots, [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            xa = TWO_PI * ((g1 + 0.5 * d[0]) * h)
            sb = np.sin(TWO_PI * ((g1 + 0.5 * d[1]) * h))
            sc = np.sin(TWO_PI * ((g1 + 0.5 * d[2]) * h))
            yz = (sb[None, :, None] * sc[:, None, None])
            K1 = (0.5 * np.sin(xa)[None, None, :] * yz).reshape(-1)
            K2 = (0.5 * np.cos(xa)[None, None, :] * yz).reshape(-1)
            K0 = np.ones(n)
            if ln is not None:
                cen = ln[1:-1, 1:-1, 1:-1]
                nb = ln[1 + d[2]:ln.shape[0] - 1 + d[2], 1 + d[1]:ln.shape[1] - 1 + d[1],
                        1 + d[0]:ln.shape[2] - 1 + d[0]]
                K0 = K0 + self.lognormal * 0.5 * (cen + nb).reshape(-1)
            for Dk, K in zip(D, (K0, K1, K2)):
                Dk[:, slot] = -K * inv_h2
                Dk[:, centre] += K * inv_h2
        E = np.zeros((n, nst))
        E[:, centre] = 1.0
        return np.stack([D[0][mask], D[1][mask], D[2][mask], E[mask]])

    def value_coefs(self, i: int) -> np.ndarray:
        """Coefficients of `value_basis` at t_i."""
        t = self.t(i)
        if self.dim == 3:
            return np.array([1.0, math.cos(t), math.sin(t), self.ccoef(t)])
        h = self.h
        vx, vy = self.velocity(t)
        diag = self.ccoef(t) + (abs(vx) + abs(vy)) / h
        return np.array([1.0, math.cos(t + self.coef_phase[2]), diag, max(vx, 0.0) / h, min(vx, 0.0) / h,
                         max(vy, 0.0) / h, min(vy, 0.0) / h])

    def rhs(self, i: int) -> np.ndarray:
        """b(t_i): sum of Gaussian bumps with centres moving on a circle of radius 0.25."""
        t = self.t(i)
        x, y, z = self._node_coords()
        b = np.zeros(self.n, dtype=np.float64)
        for phi, sig in zip(self.bump_phase, self.bump_sigma):
            cx = 0.5 + 0.25 * math.cos(t + phi)
            cy = 0.5 + 0.25 * math.sin(t + phi)
            r2 = (x - cx) ** 2 + (y - cy) ** 2
            if self.dim == 3:
                r2 = r2 + (z - 0.5) ** 2
            b += np.exp(-r2 / (2.0 * sig * sig))
        return b


# -------------------------------------------------------------------- workloads

def _cfg0(N=64):
    return SeqProblem("poisson2d-spd", 2, N, dt=0.01, steps=50, seed=0)


def _cfg1(N=512, steps=200):
    rng = np.random.default_rng(1)
    phases = tuple(rng.uniform(0.0, TWO_PI, 4))
    sigmas = tuple(rng.uniform(0.05, 0.15, 4))
    return SeqProblem("advdiff2d", 2, N, dt=0.005, steps=steps, seed=1, advection=20.0,
                      bump_phase=phases, bump_sigma=sigmas)


def _cfg2(N=128):
    return SeqProblem("lognormal3d-fp32", 3, N, dt=0.005, steps=300, seed=2,
                      lognormal=1e-2, fp32_values=True)


# Method settings of each workload.  Sketch sizes follow the workload descriptions
# (Gaussian 2M, SRHT 4M); where a setting is unstated the value is a documented choice.
_METHODS = {
    0: dict(M=10, sketch="gaussian", s=20, solver="cg", restart=30, tol=1e-10,
            prec="fp64", method_seed=0),
    1: dict(M=20, sketch="srht", s=80, solver="gmres", restart=30, tol=1e-8,
            prec="fp64", method_seed=1),
    2: dict(M=30, sketch="gaussian", s=60, solver="cg", restart=30, tol=1e-8,
            prec="mixed", method_seed=2),
    3: dict(M=20, sketch="srht", s=80, solver="gmres", restart=30, tol=1e-8,
            prec="fp64", method_seed=1, train_steps=2000, eval_steps=500),
}


def config(k: int, N: Optional[int] = None, steps: Optional[int] = None):
    """Workload k (0..3) as (SeqProblem, method dict); N/steps shrink it for tests."""
    if k == 0:
        p = _cfg0(N or 64)
    elif k in (1, 3):
        p = _cfg1(N or 512, 200 if k == 1 else 2500)
    elif k == 2:
        p = _cfg2(N or 128)
    else:
        raise ValueError("config index must be 0..3 (4 is batch_problems)")
    if steps is not None:
        p.steps = steps
    return p, dict(_METHODS[k])


def make_problem(k: int, N: Optional[int] = None):
    return config(k, N)[0]


def batch_problems(seed: int = 4, nseq: int = 64, lo: int = 96, hi: int = 768,
                   steps: int = 100):
    """64 independent 2-D sequences of uneven sizes (the batched workload).

    Side lengths L_j ~ U{lo..hi}, history lengths M_j in {8, 16, 24}, half of the
    sequences advective (GMRES(30)), the rest SPD (CG).  Per-sequence phases come from
    default_rng([seed, j]).  Returns a list of (SeqProblem, method dict).
    """
    rng = np.random.default_rng(seed)
    sides = rng.integers(lo, hi + 1, size=nseq)
    Ms = rng.choice(np.array([8, 16, 24]), size=nseq)
    adv = np.zeros(nseq, dtype=bool)
    adv[rng.permutation(nseq)[: nseq // 2]] = True
    out = []
    for j in range(nseq):
        r = np.random.default_rng([seed, j])
        ph = tuple(r.uniform(0.0, TWO_PI, 5))
        p = SeqProblem(f"batch{j}", 2, int(sides[j]), dt=0.005, steps=steps,
                       seed=seed * 1000 + j, advection=20.0 if adv[j] else 0.0,
                       bump_phase=(ph[4],), bump_sigma=(0.1,), coef_phase=ph[:4],
                       fp32_values=True)
        M = int(Ms[j])
        # unpreconditioned GMRES(30) needs up to ~7000 iterations per step on the largest
        # advective grids: with inner solves capped at 10 cycles the refinement sweeps
        # must allow that many iterations
        m = dict(M=M, sketch="gaussian", s=2 * M, solver="gmres" if adv[j] else "cg",
                 restart=30, tol=1e-8, prec="mixed_krylov", max_refine=100, method_seed=seed * 1000 + j)
        out.append((p, m))
    return out

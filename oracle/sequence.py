"""Per-step driver of Alg. 1 over a stream of systems A(t_i) x = b(t_i) (eq. (seq)).

Step i: build X from the min(i, M) most recent solutions (Section 2; the window drops
its oldest column and appends the newest, Section 2.1), compute the initial guess
(``basis.initial_guess``), run the Krylov solver from it (``krylov``), then push the
solution.  The sketch S x of every pushed solution is kept next to it, so the small
sketched matrix S X never needs a pass over X.

Guess kinds: "projection" (the method), "zero" (x0 = 0) and "previous" (x0 = x(t_{i-1}),
the paper's Baseline of Sections 4 and 5).

Precision "fp64" (the paper's setting) or "mixed" (not in the paper): the history and
the basis Q1 are stored in float32 (the sketch is taken of the stored column), the
matrix carries float32 values, and each system is solved by FP64 iterative refinement
around float32-stored inner Krylov solves (``mixed.solve_ir``).  Precision "mixed_krylov"
keeps the history and basis in float64 and otherwise equals "mixed".
"""

from __future__ import annotations

import time

import numpy as np

from . import basis as bs
from . import krylov as kr
from . import mixed as mx
from .sketch import Sketch


class Sequence:
    def __init__(self, n: int, M: int, sketch: str = "gaussian", s: int | None = None,
                 seed: int = 0, solver: str = "cg", restart: int = 30, tol: float = 1e-8,
                 maxit: int = 200000, projection: str = "galerkin", tau_s: float = 1e-12,
                 tau_c: float = 1e-12, m: int | None = None, guess: str = "projection",
                 precision: str = "fp64", inner_tol: float = 1e-4, max_refine: int = 10,
                 refresh: int = 50, basis: str = "sketched_qr", precond: str = "none"):
        self.n, self.M = n, M
        self.m = M if m is None else m
        self.s = 2 * M if s is None else s
        self.solver, self.restart, self.tol, self.maxit = solver, restart, tol, maxit
        self.projection, self.tau_s, self.tau_c, self.guess = projection, tau_s, tau_c, guess
        self.seed = seed
        if precision not in ("fp64", "mixed", "mixed_krylov"):
            raise ValueError(precision)
        self.precision, self.inner_tol, self.max_refine = precision, inner_tol, max_refine
        self.store = mx.fl32 if precision == "mixed" else None
        # the mixed mode applies the Gaussian sketch in BF16 (its history is FP32)
        self.S = Sketch(sketch, n, self.s, seed, bf16=precision == "mixed" and sketch == "gaussian")
        self.cols: list[np.ndarray] = []
        self.scols: list[np.ndarray] = []
        # m < M: the range finder's Z follows Alg. 3 (each column keeps the Gaussian row it
        # was given, a new Z every `refresh` pushes); Omega = X Z is never formed (its span
        # is folded into the small factor of the sketched QR)
        if basis not in ("sketched_qr", "pod"):
            raise ValueError(basis)
        self.basis = basis   # "pod": Alg. 2's basis (m leading left singular vectors of X)
        if precond not in ("none", "jacobi"):
            raise ValueError(precond)
        self.precond = precond
        self.zrows = bs.RangeFinderRows(M, refresh) if (self.m < self.M and basis == "sketched_qr") else None

    # ------------------------------------------------------------------ history
    def push(self, x: np.ndarray):
        x = np.array(x, dtype=np.float64, copy=True)
        if self.store is not None:
            x = self.store(x)
        self.cols.append(x)
        self.scols.append(self.S.apply(x))
        if len(self.cols) > self.M:
            self.cols.pop(0)
            self.scols.pop(0)
        if self.zrows is not None:
            self.zrows.push()

    def history(self):
        """(X, SX) with columns oldest first."""
        if not self.cols:
            return np.zeros((self.n, 0)), np.zeros((self.s, 0))
        return np.stack(self.cols, 1), np.stack(self.scols, 1)

    # ------------------------------------------------------------------ one step
    def initial_guess(self, A, b) -> bs.Guess:
        X, SX = self.history()
        k_h = X.shape[1]
        if self.guess == "zero" or k_h == 0:
            return bs.Guess(np.zeros(self.n), 0, 0, np.zeros(0), np.zeros(k_h), False)
        if self.guess == "previous":
            cX = np.zeros(k_h)
            cX[-1] = 1.0
            return bs.Guess(X[:, -1].copy(), 0, 0, np.zeros(0), cX, False)
        Z = None
        if self.zrows is not None:
            Z = bs.range_finder_rows(self.zrows.rows, self.m, self.seed, self.zrows.epoch)
        return bs.initial_guess(A, b, X, SX, Z, self.projection, self.solver == "cg",
                                self.tau_s, self.tau_c, self.store,
                                pod_m=self.m if self.basis == "pod" else None)

    def solve(self, A, b, x0):
        """Krylov solve from x0; in the mixed mode A must carry float32 values."""
        if self.precision != "fp64":
            return mx.solve_ir(A, b, x0, self.tol, self.solver, self.restart, self.inner_tol,
                               self.max_refine, self.maxit, precond=self.precond)
        dinv = kr.jacobi_dinv(A) if self.precond == "jacobi" else None
        if self.solver == "cg":
            return kr.cg(A, b, x0, self.tol, self.maxit, dinv=dinv)
        return kr.gmres(A, b, x0, self.tol, self.restart, self.maxit, dinv=dinv)

    def step(self, A, b):
        t0 = time.perf_counter()
        g = self.initial_guess(A, b)
        t1 = time.perf_counter()
        x, info = self.solve(A, b, g.x0)
        t2 = time.perf_counter()
        self.push(x)
        info = dict(info, k=g.k, k2=g.k2, used_fallback=g.used_fallback,
                    s_guess=t1 - t0, s_solve=t2 - t1)
        return x, g, info


def make_sequence(problem, method: dict, **over) -> Sequence:
    """A Sequence for a workload from ``gen.config``."""
    kw = dict(n=problem.n, M=method["M"], sketch=method["sketch"], s=method["s"],
              seed=method["method_seed"], solver=method["solver"],
              restart=method["restart"], tol=method["tol"])
    kw.update(over)
    return Sequence(**kw)


def run(problem, method: dict, steps: int | None = None, **over):
    """Run the whole sequence; returns the list of per-step info dicts."""
    seq = make_sequence(problem, method, **over)
    out = []
    for i in range(problem.steps if steps is None else steps):
        A = problem.matrix(i).to_scipy()
        b = problem.rhs(i)
        _, _, info = seq.step(A, b)
        out.append(info)
    return out

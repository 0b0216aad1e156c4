"""Mixed-precision solve: FP64 iterative refinement around FP32-stored inner solves.

Not in the paper.  The system solved is A32 = fl32(A) (the FP32 matrix values are
exact in FP64).  Each sweep forms the true residual r = b - A32 x in FP64 and stops when
||r|| <= tol ||b||; otherwise it solves A32 d = fl32(r) with CG or GMRES whose vectors
are stored in FP32 (``fl32`` at every store, FP64 arithmetic between stores) to the
inner tolerance relative to ||fl32(r)|| as judged by the solver's own recursive
estimate (no true-residual confirmation: the next sweep's FP64 residual is the check),
or at most ``inner_maxit`` iterations (default 10 GMRES cycles or 1000 CG iterations,
since float32 storage can keep the inner residual above the inner tolerance), and
updates x += d in FP64.  The iteration count is the sum of the inner iterations; the
refinement count is the number of sweeps that ran an inner solve.

Parity: the rounding points follow the description above; the GPU tests compare the
iteration counts with the HIP path's under the bar stated in tests/test_gpu_mixed.py and
check the final residual against the tolerance.
"""

from __future__ import annotations

import numpy as np

from . import krylov as kr


def fl32(v) -> np.ndarray:
    """Round to float32 and return as float64 (a store to FP32 memory)."""
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def inner_cap(solver: str, restart: int, inner_maxit: int = 0) -> int:
    if inner_maxit > 0:
        return inner_maxit
    return 10 * restart if solver == "gmres" else 1000


def solve_ir(A32, b, x0, tol: float, solver: str = "cg", restart: int = 30,
             inner_tol: float = 1e-4, max_refine: int = 10, maxit: int = 100000,
             inner_maxit: int = 0, precond: str = "none"):
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    dinv = kr.jacobi_dinv(A32) if precond == "jacobi" else None
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, restarts=0, refinements=0, relres=0.0, relres0=0.0,
                                      status=kr.CONVERGED)
    iters = restarts = sweeps = 0
    relres0 = None
    status = kr.NOTCONV
    rel = np.inf
    for sweep in range(max_refine + 1):
        r = b - A32 @ x
        nr = float(np.linalg.norm(r))
        rel = nr / bnorm
        if relres0 is None:
            relres0 = rel
        if nr <= tol * bnorm:
            status = kr.CONVERGED
            break
        if not np.isfinite(nr):
            status = kr.BREAKDOWN
            break
        if sweep == max_refine or iters >= maxit:
            break
        r32 = fl32(r)
        cap = min(maxit - iters, inner_cap(solver, restart, inner_maxit))
        if solver == "cg":
            d, info = kr.cg(A32, r32, np.zeros_like(b), inner_tol, cap, store=fl32, confirm=False, dinv=dinv)
        else:
            d, info = kr.gmres(A32, r32, np.zeros_like(b), inner_tol, restart, cap, store=fl32,
                               confirm=False, dinv=dinv)
        iters += info["iters"]
        restarts += info["restarts"]
        if info["status"] == kr.BREAKDOWN:
            status = kr.BREAKDOWN
            break
        x = x + d
        sweeps = sweep + 1
    return x, dict(iters=iters, restarts=restarts, refinements=sweeps, relres=rel, relres0=relres0,
                   status=status)

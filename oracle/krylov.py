"""Krylov solvers seeded by the initial guess (Alg. 1 (Krylov solve); Section 1).

Stopping rule (the paper states none): ||b - A x||_2 <= tol ||b||_2, checked before the
first iteration, so a good enough initial guess costs zero iterations (the paper
reports iterations that "vanish" for that reason in Sections 4 and 5).  A recursive
estimate that meets the tolerance is confirmed with the true residual; if the
confirmation fails the solver continues from the true residual.

* CG: Hestenes-Stiefel.  One iteration = one product A p.  Continuing after a failed
  confirmation restarts the direction (p = r).
* GMRES(m): Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
  matrix, |g_{j+1}| as the residual estimate, restart from the true residual.  One
  iteration = one Arnoldi step; the count sums over restarts.

``confirm=False`` (inner solves of the mixed mode) accepts the recursive estimate:
CG stops on its recursive residual and GMRES after the cycle whose estimate met the
tolerance, without the true-residual check.

``store`` models where a vector is written to memory: every vector the solver keeps
(x, r, p, q; the Arnoldi vectors) passes through it.  It is the identity for FP64 runs
and a round trip through float32 for the inner solves of the mixed mode (all
arithmetic stays in float64 between stores).

``dinv`` (optional) applies the Jacobi preconditioner M^-1 = diag(dinv), dinv = 1 / diag(A)
(``jacobi_dinv``): CG becomes preconditioned CG (z = M^-1 r, beta = r^T z / r_old^T z_old,
the stopping rule still on ||r||); GMRES is right-preconditioned (Arnoldi on A M^-1, the
cycle's correction M^-1 V y), so its residual estimate is the true residual's.  The
paper preconditions every solve (ILU in Section 4, algebraic multigrid in Section 5);
the diagonal is the simplest such M.  In the mixed mode dinv is stored in float32 like
the other vectors.

Both return (x, info) with info = dict(iters, restarts, relres, relres0, status),
status 0 converged, 1 not converged within maxit, -5 breakdown (CG p^T A p <= 0 or
not finite).  A zero right-hand side returns x = 0 with zero iterations.
"""

from __future__ import annotations

import numpy as np

CONVERGED, NOTCONV, BREAKDOWN = 0, 1, -5


def _norm(v):
    return float(np.sqrt(np.dot(v, v)))


def _identity(v):
    return v


def jacobi_dinv(A) -> np.ndarray:
    """1 / diag(A) (an entry 1 where the diagonal is zero or missing)."""
    d = np.asarray(A.diagonal(), dtype=np.float64)
    out = np.ones_like(d)
    nz = d != 0.0
    out[nz] = 1.0 / d[nz]
    return out


def cg(A, b, x0, tol: float, maxit: int = 100000, store=None, confirm: bool = True, dinv=None):
    """Hestenes-Stiefel conjugate gradients from x0 (preconditioned with diag(dinv))."""
    st = _identity if store is None else store
    b = np.asarray(b, dtype=np.float64)
    x = st(np.array(x0, dtype=np.float64, copy=True))
    bnorm = _norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, restarts=0, relres=0.0, relres0=0.0, status=CONVERGED)
    thresh = tol * bnorm
    pre = (lambda v: v) if dinv is None else (lambda v: st(dinv) * v)
    r = st(b - A @ x)
    rr = float(np.dot(r, r))
    relres0 = np.sqrt(rr) / bnorm
    it = 0
    restarts = 0
    if np.sqrt(rr) <= thresh:
        return x, dict(iters=0, restarts=0, relres=relres0, relres0=relres0, status=CONVERGED)
    p = st(pre(r))
    rho = float(np.dot(r, pre(r)))
    status = NOTCONV
    while it < maxit:
        q = st(A @ p)
        pq = float(np.dot(p, q))
        if not (pq > 0.0) or not np.isfinite(pq):
            status = BREAKDOWN
            break
        alpha = rho / pq
        x = st(x + alpha * p)
        r = st(r - alpha * q)
        rr_new = float(np.dot(r, r))
        it += 1
        if np.sqrt(rr_new) <= thresh:
            if not confirm:
                status = CONVERGED
                break
            r = st(b - A @ x)
            rr = float(np.dot(r, r))
            if np.sqrt(rr) <= thresh:
                status = CONVERGED
                break
            restarts += 1
            p = st(pre(r))
            rho = float(np.dot(r, pre(r)))
            continue
        rho_new = float(np.dot(r, pre(r)))
        beta = rho_new / rho
        rho = rho_new
        p = st(pre(r) + beta * p)
    rt = b - A @ x
    return x, dict(iters=it, restarts=restarts, relres=_norm(rt) / bnorm, relres0=relres0,
                   status=status)


def givens(a: float, b: float):
    """(c, s, rho) with [c s; -s c] [a; b] = [rho; 0]."""
    rho = float(np.hypot(a, b))
    if rho == 0.0:
        return 1.0, 0.0, 0.0
    return a / rho, b / rho, rho


def gmres(A, b, x0, tol: float, restart: int = 30, maxit: int = 100000, store=None,
          confirm: bool = True, dinv=None):
    """Restarted GMRES(restart) with modified Gram-Schmidt Arnoldi and Givens rotations
    (right-preconditioned with diag(dinv): Arnoldi on A diag(dinv))."""
    st = _identity if store is None else store
    pre = (lambda v: v) if dinv is None else (lambda v: st(dinv) * v)
    b = np.asarray(b, dtype=np.float64)
    x = st(np.array(x0, dtype=np.float64, copy=True))
    n = b.shape[0]
    bnorm = _norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, restarts=0, relres=0.0, relres0=0.0, status=CONVERGED)
    thresh = tol * bnorm
    r = st(b - A @ x)
    beta = _norm(r)
    relres0 = beta / bnorm
    total = 0
    cycles = 0
    status = NOTCONV if beta > thresh else CONVERGED
    while status == NOTCONV and total < maxit:
        m = restart
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[:, 0] = st(r / beta)
        g[0] = beta
        jend = 0
        for j in range(m):
            w = st(A @ pre(V[:, j]))
            for l in range(j + 1):
                H[l, j] = float(np.dot(V[:, l], w))
                w -= H[l, j] * V[:, l]
            w = st(w)
            H[j + 1, j] = _norm(w)
            for l in range(j):
                t = cs[l] * H[l, j] + sn[l] * H[l + 1, j]
                H[l + 1, j] = -sn[l] * H[l, j] + cs[l] * H[l + 1, j]
                H[l, j] = t
            hnext = H[j + 1, j]
            cs[j], sn[j], H[j, j] = givens(H[j, j], hnext)
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            jend = j + 1
            if abs(g[j + 1]) <= thresh or hnext == 0.0 or total >= maxit:
                break
            V[:, j + 1] = st(w / hnext)
        y = np.zeros(jend)
        for i in range(jend - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:jend], y[i + 1:jend])) / H[i, i]
        x = st(x + pre(V[:, :jend] @ y))
        r = st(b - A @ x)
        beta = _norm(r)
        cycles += 1
        if beta <= thresh or (not confirm and abs(g[jend]) <= thresh and np.isfinite(beta)):
            status = CONVERGED
        elif not np.isfinite(beta):
            status = BREAKDOWN
    return x, dict(iters=total, restarts=max(cycles - 1, 0), relres=beta / bnorm,
                   relres0=relres0, status=status)

"""Pins of the oracle's Krylov solvers (CG, GMRES(m)) against textbook facts and SciPy."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import krylov as kr


def _spd(n, rng, cond=50.0):
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (U * np.geomspace(1.0, cond, n)) @ U.T


def test_cg_finite_termination_small():
    """CG on an SPD n x n system reaches the solution in about n steps."""
    rng = np.random.default_rng(0)
    n = 24
    A = _spd(n, rng, cond=4.0)
    xs = rng.standard_normal(n)
    b = A @ xs
    # in exact arithmetic n steps give the solution; in floating point n steps leave
    # a residual far below the starting one
    x, info = kr.cg(A, b, np.zeros(n), tol=1e-13, maxit=n)
    assert info["iters"] <= n and info["relres"] <= 1e-12
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


def test_cg_few_distinct_eigenvalues():
    """With k distinct eigenvalues CG terminates after k iterations (exact arithmetic)."""
    rng = np.random.default_rng(1)
    n = 60
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.repeat([1.0, 3.0, 7.0, 20.0], n // 4)
    A = (U * ev) @ U.T
    b = rng.standard_normal(n)
    x, info = kr.cg(A, b, np.zeros(n), tol=1e-10)
    assert info["iters"] == 4
    assert np.allclose(A @ x, b, atol=1e-9)


def test_gmres_full_finite_termination():
    rng = np.random.default_rng(2)
    n = 30
    A = np.eye(n) * 4 + rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, info = kr.gmres(A, b, np.zeros(n), tol=1e-12, restart=n + 5)
    assert info["status"] == kr.CONVERGED and info["iters"] <= n
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-10)


def test_gmres_first_step_is_minimal_residual():
    """After one Arnoldi step, x1 minimises ||b - A x|| over x0 + span{r0}."""
    rng = np.random.default_rng(3)
    n = 40
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    x, info = kr.gmres(A, b, np.zeros(n), tol=1e-14, restart=1, maxit=1)
    Ab = A @ b
    xref = b * (Ab @ b) / (Ab @ Ab)
    assert info["iters"] == 1 and info["status"] == kr.NOTCONV
    assert np.allclose(x, xref, rtol=1e-12)


def test_gmres_restart_residuals_non_increasing():
    rng = np.random.default_rng(4)
    n = 200
    A = sp.diags([-1.0, 2.3, -1.2], [-1, 0, 1], shape=(n, n)).tocsr()
    b = rng.standard_normal(n)
    x = np.zeros(n)
    prev = np.linalg.norm(b)
    for _ in range(8):
        x, info = kr.gmres(A, b, x, tol=1e-14, restart=10, maxit=10)
        cur = np.linalg.norm(b - A @ x)
        assert cur <= prev * (1 + 1e-12)
        prev = cur


@pytest.mark.parametrize("solver", ["cg", "gmres"])
def test_solutions_match_scipy(solver):
    rng = np.random.default_rng(5)
    n = 400
    main = 2.0 + rng.uniform(0, 1, n)
    A = sp.diags([-np.ones(n - 1), main, -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    if solver == "gmres":
        A = A + sp.diags([0.4 * np.ones(n - 1)], [1])
    b = rng.standard_normal(n)
    if solver == "cg":
        x, info = kr.cg(A, b, np.zeros(n), tol=1e-12)
        xr, _ = spla.cg(A, b, rtol=1e-13, maxiter=5000)
    else:
        x, info = kr.gmres(A, b, np.zeros(n), tol=1e-12, restart=30)
        xr, _ = spla.gmres(A, b, rtol=1e-13, restart=30, maxiter=5000)
    xs = spla.spsolve(A.tocsc(), b)
    assert info["status"] == kr.CONVERGED and info["relres"] <= 1e-12
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert np.linalg.norm(xr - xs) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("solver", ["cg", "gmres"])
def test_zero_iterations_when_guess_is_good(solver):
    rng = np.random.default_rng(6)
    n = 50
    A = _spd(n, rng)
    b = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)
    f = kr.cg if solver == "cg" else kr.gmres
    x, info = f(A, b, xs, 1e-8)
    assert info["iters"] == 0 and info["status"] == kr.CONVERGED and np.array_equal(x, xs)
    x, info = f(A, np.zeros(n), np.ones(n), 1e-8)
    assert info["iters"] == 0 and np.all(x == 0)


def test_cg_breakdown_on_indefinite():
    A = np.diag([1.0, -1.0, 2.0])
    b = np.array([1.0, 1.0, 0.0])
    _, info = kr.cg(A, b, np.zeros(3), 1e-10)
    assert info["status"] == kr.BREAKDOWN


@pytest.mark.parametrize("solver", ["cg", "gmres"])
def test_maxit_reports_not_converged(solver):
    rng = np.random.default_rng(7)
    n = 100
    A = _spd(n, rng, 1e4)
    b = rng.standard_normal(n)
    f = kr.cg if solver == "cg" else kr.gmres
    _, info = f(A, b, np.zeros(n), 1e-12, maxit=1)
    assert info["status"] == kr.NOTCONV and info["iters"] == 1


def test_givens_rotation():
    c, s, r = kr.givens(3.0, 4.0)
    assert np.isclose(r, 5.0) and np.allclose([c * 3 + s * 4, -s * 3 + c * 4], [5.0, 0.0])


def test_jacobi_preconditioned_solvers():
    """Diagonal preconditioning: PCG equals CG on the symmetrically scaled system
    D^-1/2 A D^-1/2 (the same iterates mapped back, x = D^-1/2 y); right-preconditioned
    GMRES's first step minimises ||b - A D^-1 (c b)|| over c (closed form); both reach
    the tolerance; with an identity diagonal they reduce to the plain solvers."""
    import scipy.sparse as sp

    from oracle import krylov as kr

    rng = np.random.default_rng(51)
    n = 120
    d = rng.uniform(1.0, 50.0, n)
    off = -np.ones(n - 1)
    A = sp.diags([off, d + 2.5, off], [-1, 0, 1]).tocsr()
    b = rng.standard_normal(n)
    dinv = kr.jacobi_dinv(A)
    assert np.allclose(dinv, 1.0 / (d + 2.5))
    for it in (1, 3, 7):
        xp, ip = kr.cg(A, b, np.zeros(n), 1e-14, maxit=it, dinv=dinv)
        s = np.sqrt(dinv)
        As = sp.diags(s) @ A @ sp.diags(s)
        ys, _ = kr.cg(As, s * b, np.zeros(n), 1e-14, maxit=it)
        assert ip["iters"] == it
        assert np.linalg.norm(xp - s * ys) <= 1e-12 * np.linalg.norm(xp)
    x, info = kr.cg(A, b, np.zeros(n), 1e-10, dinv=dinv)
    assert info["status"] == 0 and np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    x0, i0 = kr.cg(A, b, np.zeros(n), 1e-10)
    assert info["iters"] < i0["iters"]     # the diagonal spread 1..50 is what Jacobi removes
    N = sp.diags([off * 1.4, d + 2.5, off * 0.6], [-1, 0, 1]).tocsr()
    x1, i1 = kr.gmres(N, b, np.zeros(n), 1e-14, 30, maxit=1, dinv=dinv)
    w = N @ (dinv * b)
    c = (w @ b) / (w @ w)
    assert np.linalg.norm(x1 - c * dinv * b) <= 1e-12 * np.linalg.norm(x1)
    x2, i2 = kr.gmres(N, b, np.zeros(n), 1e-10, 30, dinv=dinv)
    assert i2["status"] == 0 and np.linalg.norm(b - N @ x2) <= 1e-10 * np.linalg.norm(b)
    for f in (kr.cg, kr.gmres):
        xa, _ = f(A, b, np.zeros(n), 1e-14, maxit=5, dinv=np.ones(n)) if f is kr.cg else \
            f(A, b, np.zeros(n), 1e-14, 30, maxit=5, dinv=np.ones(n))
        xb, _ = f(A, b, np.zeros(n), 1e-14, maxit=5) if f is kr.cg else f(A, b, np.zeros(n), 1e-14, 30, maxit=5)
        assert np.array_equal(xa, xb)

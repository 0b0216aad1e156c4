"""Pins of the oracle's mixed-precision mode (float32 storage, FP64 iterative refinement).

The mode is not in the paper; what fixes its results is the algebra of iterative
refinement (each sweep solves the residual equation, so x + d is closer to the solution
by the inner solve's relative accuracy) and the Galerkin conditions of Section 2 on the
span of the float32-stored basis.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import config
from oracle import basis as bs
from oracle import krylov as kr
from oracle import mixed as mx
from oracle.sequence import Sequence
from oracle.sketch import Sketch


def _system(k, N, seed=7):
    p, meth = config(k, N=N)
    A = p.matrix(3, fp32=True).to_scipy().astype(np.float64)
    b = p.rhs(3)
    return A, b, meth


def test_fl32_is_a_store():
    v = np.array([1.0 + 2.0 ** -30, 1.0 / 3.0, 1e-50, -2.5, 0.0])
    w = mx.fl32(v)
    assert w.dtype == np.float64
    assert w[0] == 1.0 and w[3] == -2.5 and w[4] == 0.0 and w[2] == 0.0
    assert abs(w[1] - 1.0 / 3.0) <= 2.0 ** -25
    assert np.array_equal(mx.fl32(w), w)          # idempotent


@pytest.mark.parametrize("k,solver", [(0, "cg"), (1, "gmres")])
def test_ir_reaches_tolerance(k, solver):
    """The refined solution meets the FP64 tolerance and equals the direct solution."""
    A, b, meth = _system(k, 24)
    tol = 1e-11
    x, info = mx.solve_ir(A, b, np.zeros_like(b), tol, solver, 30, inner_tol=1e-4, max_refine=20)
    assert info["status"] == kr.CONVERGED
    rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert rel <= tol and abs(rel - info["relres"]) <= 1e-3 * tol
    xd = spla.spsolve(A.tocsc(), b)
    cond_est = 1e4
    assert np.linalg.norm(x - xd) <= cond_est * tol * np.linalg.norm(xd)
    # float32 storage alone cannot reach 1e-11: more than one sweep was needed
    assert info["refinements"] >= 2


@pytest.mark.parametrize("solver", ["cg", "gmres"])
def test_ir_contracts_per_sweep(solver):
    """Sweep j leaves relres <= (3 inner_tol)^j relres0 until the FP64 floor."""
    A, b, _ = _system(0 if solver == "cg" else 1, 24)
    inner = 1e-3
    prev = None
    for sweeps in (1, 2, 3):
        x, info = mx.solve_ir(A, b, np.zeros_like(b), 1e-300, solver, 30, inner_tol=inner,
                              max_refine=sweeps)
        rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert info["refinements"] == sweeps and info["status"] == kr.NOTCONV
        assert rel <= (3.0 * inner) ** sweeps
        if prev is not None:
            assert rel <= 3.0 * inner * prev
        prev = rel


def test_ir_single_sweep_is_one_inner_solve():
    """With one sweep from x0 = 0 the answer is the inner solve of A d = fl32(b): its
    true relative residual is at the inner tolerance up to float32 rounding of b and
    the float32 drift of the recursive residual the inner solve stops on."""
    A, b, _ = _system(0, 24)
    inner = 1e-4
    x, info = mx.solve_ir(A, b, np.zeros_like(b), 1e-300, "cg", inner_tol=inner, max_refine=1)
    rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert rel <= inner * 1.5
    assert info["iters"] > 0 and info["refinements"] == 1


def test_ir_zero_rhs_and_exact_start():
    A, b, _ = _system(0, 16)
    x, info = mx.solve_ir(A, np.zeros_like(b), np.ones_like(b), 1e-8, "cg")
    assert np.all(x == 0) and info["iters"] == 0
    xd = spla.spsolve(A.tocsc(), b)
    x, info = mx.solve_ir(A, b, xd, 1e-8, "gmres")
    assert info["iters"] == 0 and info["refinements"] == 0 and info["status"] == kr.CONVERGED


def test_mixed_basis_is_galerkin_on_stored_span():
    """Galerkin conditions (Section 2) hold on the span of the float32-stored basis, and
    the guess is within float32 accuracy of the FP64 one."""
    A, b, meth = _system(0, 32)
    rng = np.random.default_rng(5)
    n, M = A.shape[0], 8
    X = mx.fl32(spla.spsolve(A.tocsc(), b)[:, None] + 0.1 * rng.standard_normal((n, M)))
    S = Sketch("gaussian", n, 2 * M, 11)
    SX = S.apply(X)
    g32 = bs.initial_guess(A, b, X, SX, store=mx.fl32)
    B = bs.sketched_basis(X, SX, store=mx.fl32)
    assert np.array_equal(mx.fl32(B.Q1), B.Q1)         # stored values are float32
    Q = B.Q1
    # x0 lies in span(Q1) ...
    z, *_ = np.linalg.lstsq(Q, g32.x0, rcond=None)
    assert np.linalg.norm(Q @ z - g32.x0) <= 1e-10 * np.linalg.norm(g32.x0)
    # ... and its residual is orthogonal to span(Q1)
    r = b - A @ g32.x0
    assert np.linalg.norm(Q.T @ r) <= 1e-9 * np.linalg.norm(Q, 2) * np.linalg.norm(b)
    g64 = bs.initial_guess(A, b, X, SX)
    assert np.linalg.norm(g32.x0 - g64.x0) <= 1e-4 * np.linalg.norm(g64.x0)


def test_mixed_sequence_stores_float32_history():
    p, meth = config(0, N=16)
    seq = Sequence(p.n, 4, "gaussian", 8, seed=3, solver="cg", tol=1e-10, precision="mixed")
    for i in range(6):
        A = p.matrix(i, fp32=True).to_scipy().astype(np.float64)
        b = p.rhs(i)
        x, g, info = seq.step(A, b)
        assert info["status"] == kr.CONVERGED
        assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    X, SX = seq.history()
    assert np.array_equal(mx.fl32(X), X)
    assert np.allclose(SX, seq.S.apply(X), rtol=0, atol=1e-13 * np.abs(SX).max())
    with pytest.raises(ValueError):
        Sequence(p.n, 4, precision="bf16")

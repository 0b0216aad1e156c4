"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances (derived in DESIGN.md, "Parity bar"):
* SpMV and sketches: summation-order differences only, relative 1e-13 of the
  absolute-value sum.
* Initial guess: the two guesses are Galerkin projections on the same span computed
  with different rounding; their difference must stay two orders of magnitude below
  the solve tolerance: ||A (x0_gpu - x0_oracle)|| <= 1e-2 tol ||b||, and the kept ranks
  agree.
* Solves (same injected history on both sides): both reach ||b - A x|| <= tol ||b||
  and the iteration counts agree within 1.
* Free-running sequences: each side pushes its own solutions, which differ at the
  tolerance level; the oracle alone changes its per-step counts by tens of iterations
  when its pushed solutions are perturbed by 1e-15 (chaotic dependence on the history
  noise), so those runs are compared by their totals and by the tolerance being met.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from gen import config
from oracle import basis as obs
from oracle import krylov as okr
from oracle.sequence import Sequence as OSeq
from oracle.sketch import Sketch
from tests.gpu_helpers import dev, host, method_kwargs, print_case, reversed_order, rounding_spread

pytestmark = pytest.mark.gpu

# Fixed element-wise bars (max |gpu - oracle| / max |oracle|), spread-independent:
# x0 from the same history: 1e-12 (at least 70x the oracle's own change when its inputs X
# and S X are perturbed by 1e-16 relative: 1.5e-14 on the 64 x 64 grids, 2.8e-15 on the
# 512 x 512 one); Krylov iterates after at most two steps: 1e-13 (oracle change under a
# reversed summation order of A x: <= 6.6e-15), after at most eight steps: 2e-11 for
# GMRES (<= 1.9e-12) and 3e-10 for CG (<= 3.2e-11).  Longer solves amplify rounding
# further and keep the bars scaled by the oracle's own spread.
X0_ELEMENTWISE = 1e-12


def iterate_bar(solver: str, steps: int):
    if steps <= 2:
        return 1e-13
    if steps <= 8:
        return 2e-11 if solver == "gmres" else 3e-10
    return None


@pytest.fixture(scope="module")
def sacc():
    import torch

    assert torch.cuda.is_available()
    import paper_2309_02156_amd as pkg

    return pkg


# ---------------------------------------------------------------------------- SpMV

def _random_csr(n, rng, maxrow=7, longrow=None):
    rows = []
    for i in range(n):
        k = rng.integers(0, maxrow + 1)
        if longrow is not None and i == longrow:
            k = min(n, 300)
        cols = np.sort(rng.choice(n, size=k, replace=False))
        rows.append(cols)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum([len(c) for c in rows])
    col = np.concatenate(rows).astype(np.int32) if rowptr[-1] else np.zeros(0, np.int32)
    val = rng.standard_normal(len(col))
    return rowptr, col, val


@pytest.mark.parametrize("case", ["cfg0", "cfg1-64", "cfg1-512", "cfg2-16-fp32", "ragged"])
def test_spmv_parity(sacc, case):
    print_case("spmv", case)
    rng = np.random.default_rng(0)
    if case == "ragged":
        rowptr, col, val = _random_csr(1000, rng, longrow=17)
    else:
        k, N = {"cfg0": (0, 64), "cfg1-64": (1, 64), "cfg1-512": (1, 512), "cfg2-16-fp32": (2, 16)}[case]
        A = config(k, N)[0].matrix(7)
        rowptr, col, val = A.rowptr, A.col, A.val
    n = len(rowptr) - 1
    x = rng.standard_normal(n)
    Ad = sacc.DeviceCSR(rowptr, col, val)
    y = host(sacc.spmv(Ad, dev(x)))
    S = sp.csr_matrix((val.astype(np.float64), col, rowptr), shape=(n, n))
    ref = S @ x
    scale = abs(S) @ abs(x) + 1e-300
    assert np.all(np.abs(y - ref) <= 1e-13 * scale)


# ---------------------------------------------------------------------------- sketch

@pytest.mark.parametrize("kind,n,s", [("gaussian", 4096, 20), ("gaussian", 1000, 24), ("srht", 4096, 40),
                                      ("srht", 262144, 80)])
def test_push_sketch_parity(sacc, kind, n, s):
    print_case("sketch", kind, n, s)
    rng = np.random.default_rng(1)
    M = s // 4 if kind == "srht" else s // 2
    seq = sacc.Sequence(n, M, s=s, sketch=kind, seed=7)
    S = Sketch(kind, n, s, 7)
    xs = [rng.standard_normal(n) for _ in range(M + 3)]
    for x in xs:
        seq.push(dev(x))
    SX = seq.copy_state("SX")
    order = seq.copy_state("order")
    X = seq.copy_state("X")
    for lag, slot in enumerate(order):
        x = xs[len(xs) - M + lag]
        ref = S.apply(x)
        if kind == "srht":       # every |S_rj| = 1 / sqrt(s)
            scale = np.abs(x).sum() / np.sqrt(s) * np.ones(s)
        else:
            scale = np.abs(S.dense()) @ np.abs(x)
        assert np.array_equal(X[:, slot], x)
        assert np.all(np.abs(SX[:, slot] - ref) <= 1e-13 * scale)


@pytest.mark.parametrize("n,s", [(4096, 20), (1000, 24), (300000, 60), (1, 16)])
def test_push_sketch_parity_bf16(sacc, n, s):
    """Mixed mode, Gaussian sketch: S = BF16(G) / sqrt(s) applied to the FP32 column on
    the matrix cores (split exactly into three BF16 terms).  The products are exact on
    both sides; the GPU adds each chunk's 64 products of a term in FP32 (error at most
    63 u of their absolute sum, u = 2^-24) and chunks and terms in FP64; the terms'
    absolute values add up to at most (1 + 2^-7) |x|, so every entry is within
    65 u sum_j |S_rj x_j| of the oracle's exact sum."""
    print_case("sketch bf16", n, s)
    rng = np.random.default_rng(3)
    M = 6
    seq = sacc.Sequence(n, M, s=s, sketch="gaussian", seed=11, precision="mixed")
    S = Sketch("gaussian", n, s, 11, bf16=True)
    xs = [rng.standard_normal(n) * 10.0 ** rng.integers(-3, 3) for _ in range(M + 2)]
    for x in xs:
        seq.push(dev(x))
    SX = seq.copy_state("SX")
    order = seq.copy_state("order")
    X = seq.copy_state("X")
    X32 = np.stack([xs[len(xs) - M + lag].astype(np.float32) for lag in range(M)], 1)
    Xb = X32.astype(np.float64)
    ref, absum = np.zeros((s, M)), np.zeros((s, M))
    for j0 in range(0, n, S.chunk):
        B = S.block(j0, min(n, j0 + S.chunk))
        ref += B @ Xb[j0:j0 + B.shape[1]]
        absum += np.abs(B) @ np.abs(Xb[j0:j0 + B.shape[1]])
    bound = 65 * 2.0 ** -24 * absum
    for lag, slot in enumerate(order):
        assert np.array_equal(X[:, slot], X32[:, lag])
        err = np.abs(SX[:, slot] - ref[:, lag])
        print_case("max err / bound", float(np.max(err / np.maximum(bound[:, lag], 1e-300))))
        assert np.all(err <= bound[:, lag])


# ---------------------------------------------------------------------------- initial guess

def _oracle_history(problem, method, steps):
    """Oracle trajectory: its solutions become the injected history of both sides."""
    seq = OSeq(problem.n, method["M"], method["sketch"], method["s"], method["method_seed"],
               method["solver"], method["restart"], method["tol"])
    sols = []
    for i in range(steps):
        A = problem.matrix(i).to_scipy()
        x, _, _ = seq.step(A, problem.rhs(i))
        sols.append(x)
    return sols


@pytest.mark.parametrize("k,N,steps", [(0, 64, 16), (1, 64, 24)])
def test_stepwise_guess_and_solve(sacc, k, N, steps):
    """Same injected history on both sides: x0, rank and iteration counts per step."""
    print_case("stepwise", k, N, steps)
    p, m = config(k, N)
    sols = _oracle_history(p, m, steps)
    gseq = sacc.Sequence(p.n, **method_kwargs(m))
    oseq = OSeq(p.n, m["M"], m["sketch"], m["s"], m["method_seed"], m["solver"], m["restart"], m["tol"])
    worst, worst_ew = 0.0, 0.0
    for i in range(steps):
        A = p.matrix(i)
        As = A.to_scipy()
        b = p.rhs(i)
        g = oseq.initial_guess(As, b)
        Ad = sacc.DeviceCSR.from_csr(A)
        x0d, ginfo = gseq.initial_guess(Ad, dev(b))
        x0 = host(x0d)
        dres = np.linalg.norm(As @ (x0 - g.x0)) / np.linalg.norm(b)
        worst = max(worst, dres)
        assert ginfo["k_sketch"] == g.k and ginfo["k_eff"] == g.k2, (i, ginfo, g.k, g.k2)
        assert dres <= 1e-2 * m["tol"], (i, dres)
        # element by element: a fixed bar, 1e-12 of the largest entry (the oracle's own
        # guess moves by at most 1.5e-14 of it when X and S X are perturbed by 1e-16
        # relative, measured over these steps)
        if i > 0:
            ew = float(np.max(np.abs(x0 - g.x0)) / np.max(np.abs(g.x0)))
            worst_ew = max(worst_ew, ew)
            assert ew <= X0_ELEMENTWISE, (i, ew)
        # the solve from the oracle's own x0 isolates the Krylov kernels
        xo, oinfo = oseq.solve(As, b, g.x0)
        xd, sinfo = gseq.solve(Ad, dev(b), dev(g.x0))
        assert abs(sinfo["iters"] - oinfo["iters"]) <= 1, (i, sinfo["iters"], oinfo["iters"])
        assert sinfo["relres"] <= m["tol"] and oinfo["relres"] <= m["tol"]
        true = np.linalg.norm(b - As @ host(xd)) / np.linalg.norm(b)
        assert true <= m["tol"] * (1 + 1e-6)
        assert abs(sinfo["relres0"] - oinfo["relres0"]) <= 1e-6 * oinfo["relres0"] + 1e-15
        # inject the oracle's solution into both histories
        oseq.push(sols[i])
        gseq.push(dev(sols[i]))
    print_case("worst ||A dx0||/||b||, max |dx0| / max |x0|", worst, worst_ew)


@pytest.mark.parametrize("k,N,steps", [(0, 64, 50), (1, 64, 30)])
def test_trajectory(sacc, k, N, steps):
    """Free-running sequences on both sides: tolerances met, totals agree."""
    print_case("trajectory", k, N, steps)
    p, m = config(k, N)
    gseq = sacc.Sequence(p.n, **method_kwargs(m))
    oseq = OSeq(p.n, m["M"], m["sketch"], m["s"], m["method_seed"], m["solver"], m["restart"], m["tol"])
    diffs = []
    for i in range(steps):
        A = p.matrix(i)
        As = A.to_scipy()
        b = p.rhs(i)
        _, _, oinfo = oseq.step(As, b)
        xd, ginfo = gseq.step(sacc.DeviceCSR.from_csr(A), dev(b))
        true = np.linalg.norm(b - As @ host(xd)) / np.linalg.norm(b)
        assert true <= m["tol"] * (1 + 1e-6), (i, true)
        diffs.append((ginfo["iters"], oinfo["iters"]))
    print_case("iterations (gpu, oracle)", diffs)
    g_tot = sum(d[0] for d in diffs)
    o_tot = sum(d[1] for d in diffs)
    # identical up to the first history-noise divergence, then statistically equal
    assert abs(diffs[0][0] - diffs[0][1]) <= 1 and abs(diffs[1][0] - diffs[1][1]) <= 1
    assert abs(g_tot - o_tot) <= 0.1 * o_tot, (g_tot, o_tot)


# ---------------------------------------------------------------------------- full size

def _smooth_history(p, M, rng):
    """Synthetic full-size history: M independent combinations of 3 M smooth modes
    (numerically full rank, so the projection is well determined)."""
    x, y, _ = p._node_coords()
    modes = rng.integers(1, 12, size=(3 * M, 2))
    F = np.stack([np.sin(a * np.pi * x) * np.sin(b * np.pi * y) for a, b in modes], 1)
    return [0.01 * (F @ rng.standard_normal(3 * M)) for _ in range(M)]


def test_full_size_guess_and_one_cycle(sacc):
    """The bench workload's shape (512 x 512, M = 20, SRHT s = 80, GMRES(30))."""
    print_case("full-size cfg1")
    p, m = config(1)
    rng = np.random.default_rng(3)
    hist = _smooth_history(p, m["M"], rng)
    A = p.matrix(40)
    As = A.to_scipy()
    b = p.rhs(40)
    gseq = sacc.Sequence(p.n, **method_kwargs(m, maxit=30))
    S = Sketch("srht", p.n, m["s"], m["method_seed"])
    for h in hist:
        gseq.push(dev(h))
    X = np.stack(hist, 1)
    SX = S.apply(X)
    g = obs.initial_guess(As, b, X, SX, spd=False)
    Ad = sacc.DeviceCSR.from_csr(A)
    x0d, ginfo = gseq.initial_guess(Ad, dev(b))
    x0 = host(x0d)
    assert ginfo["k_sketch"] == g.k == m["M"] and ginfo["k_eff"] == g.k2
    assert np.linalg.norm(As @ (x0 - g.x0)) <= 1e-2 * m["tol"] * np.linalg.norm(b)
    ew = float(np.max(np.abs(x0 - g.x0)) / np.max(np.abs(g.x0)))
    print_case("full-size x0: max |dx0| / max |x0|", ew)
    assert ew <= X0_ELEMENTWISE
    # Galerkin orthogonality of the GPU guess against the history span
    B = obs.sketched_basis(X, SX)
    Q = B.Q()
    r = b - As @ x0
    assert np.linalg.norm(Q.T @ r) <= 1e-10 * np.linalg.norm(b)
    # one GMRES(30) cycle from the same start on both sides; the bound is 10x the
    # oracle's own rounding sensitivity (reversed summation order in A x)
    xo, oinfo, spread = rounding_spread(okr.gmres, As, b, g.x0, m["tol"], 30, maxit=30)
    xd, sinfo = gseq.solve(Ad, dev(b), dev(g.x0))
    assert sinfo["iters"] == oinfo["iters"] == 30 and sinfo["rc"] == 1
    xg = host(xd)
    print_case("one cycle: diff / spread / |x|", np.linalg.norm(xg - xo), spread, np.linalg.norm(xo))
    assert np.linalg.norm(xg - xo) <= 10 * max(spread, 1e-12 * np.linalg.norm(xo))
    # the residual after the cycle (about 0.91: the synthetic history does not contain
    # the solution): reported = true, and equal to the oracle's within 1e-5 relative (15x
    # the oracle's own change, 6.6e-7, under a reversed summation order of A x)
    bn = np.linalg.norm(b)
    rg = np.linalg.norm(b - As @ xg) / bn
    print_case("one cycle: relres gpu / reported / oracle", rg, sinfo["relres"], oinfo["relres"])
    assert abs(sinfo["relres"] - rg) <= 1e-9 * rg
    assert abs(rg - oinfo["relres"]) <= 1e-5 * oinfo["relres"]


# ---------------------------------------------------------------------------- edge cases

def _spd_small(n, rng):
    main = 4.0 + rng.uniform(0, 1, n)
    off = -np.ones(n - 1)
    return sp.diags([off, main, off], [-1, 0, 1]).tocsr()


def _dcsr(sacc, S):
    S = S.tocsr()
    return sacc.DeviceCSR(S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))


@pytest.mark.parametrize("n", [1, 5, 63, 65, 257, 1000])
def test_ragged_sizes_cg_and_gmres(sacc, n):
    print_case("ragged", n)
    rng = np.random.default_rng(n)
    S = _spd_small(n, rng)
    b = rng.standard_normal(n)
    for solver in ("cg", "gmres"):
        seq = sacc.Sequence(n, 1, s=2, solver=solver, tol=1e-12, restart=min(30, max(1, n)))
        xd, info = seq.solve(_dcsr(sacc, S), dev(b), dev(np.zeros(n)))
        f = okr.cg if solver == "cg" else okr.gmres
        xo, oinfo = f(S, b, np.zeros(n), 1e-12) if solver == "cg" else f(S, b, np.zeros(n), 1e-12, min(30, n))
        assert info["rc"] == 0 and info["relres"] <= 1e-12
        assert abs(info["iters"] - oinfo["iters"]) <= 1
        assert np.allclose(host(xd), xo, rtol=1e-9, atol=1e-12)


def test_zero_rhs_maxit_breakdown(sacc):
    rng = np.random.default_rng(5)
    n = 300
    S = _spd_small(n, rng)
    Ad = _dcsr(sacc, S)
    seq = sacc.Sequence(n, 2, s=4, solver="cg", tol=1e-10)
    xd, info = seq.solve(Ad, dev(np.zeros(n)), dev(np.ones(n)))
    assert info["rc"] == 0 and info["iters"] == 0 and np.all(host(xd) == 0)
    seq1 = sacc.Sequence(n, 2, s=4, solver="cg", tol=1e-14, maxit=1)
    _, info = seq1.solve(Ad, dev(rng.standard_normal(n)), dev(np.zeros(n)))
    assert info["rc"] == 1 and info["iters"] == 1
    seq2 = sacc.Sequence(n, 2, s=4, solver="gmres", tol=1e-14, maxit=3, restart=2)
    _, info = seq2.solve(Ad, dev(rng.standard_normal(n)), dev(np.zeros(n)))
    assert info["rc"] == 1 and info["iters"] == 3
    Ind = sp.diags([np.r_[np.ones(n // 2), -np.ones(n - n // 2)]], [0]).tocsr()
    _, info = seq.solve(_dcsr(sacc, Ind), dev(np.ones(n)), dev(np.zeros(n)))
    assert info["rc"] == -5


def test_step_gmres_zero_rhs_pushes_zero(sacc):
    """sa_step with GMRES enqueues the push before it reads the final state: a step with
    b = 0 still returns x = 0 and pushes a zero column (slot = pushes mod M).  The guess
    is the previous solution, so the iterate the solve starts from is not zero."""
    rng = np.random.default_rng(9)
    n = 300
    S = _spd_small(n, rng)
    Ad = _dcsr(sacc, S)
    seq = sacc.Sequence(n, 3, s=6, solver="gmres", tol=1e-10, restart=20, guess="previous")
    for _ in range(2):
        _, info = seq.step(Ad, dev(rng.standard_normal(n)))
        assert info["rc"] == 0 and info["relres"] <= 1e-10
    x, info = seq.step(Ad, dev(np.zeros(n)), dev(np.ones(n)))
    assert info["rc"] == 0 and info["iters"] == 0 and info["relres"] == 0.0
    assert np.all(host(x) == 0)
    X, SX = seq.copy_state("X"), seq.copy_state("SX")
    assert np.all(X[:, 2] == 0) and np.all(SX[:, 2] == 0)
    assert np.all(np.any(X[:, :2] != 0, axis=0))
    b = rng.standard_normal(n)
    x, info = seq.step(Ad, dev(b))
    assert info["rc"] == 0 and info["relres"] <= 1e-10
    assert np.linalg.norm(b - S @ host(x)) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)


def test_history_edge_cases(sacc):
    rng = np.random.default_rng(6)
    n = 500
    S = _spd_small(n, rng)
    Ad = _dcsr(sacc, S)
    b = rng.standard_normal(n)
    seq = sacc.Sequence(n, 4, s=8, solver="cg", tol=1e-10)
    x0, info = seq.initial_guess(Ad, dev(b))
    assert info["history"] == 0 and np.all(host(x0) == 0)
    u = rng.standard_normal(n)
    for c in (1.0, 2.0, -1.0):
        seq.push(dev(c * u))
    x0, info = seq.initial_guess(Ad, dev(b))
    assert info["k_sketch"] == 1 and info["k_eff"] == 1
    ref = u * (u @ b) / (u @ (S @ u))
    assert np.allclose(host(x0), ref, rtol=1e-10, atol=1e-14)
    bad = u.copy()
    bad[3] = np.nan
    seq.push(dev(bad))
    x0, info = seq.initial_guess(Ad, dev(b))
    assert info["used_fallback"] == 1 and np.all(host(x0) == 0)   # newest column not finite
    seq.push(dev(2 * u))
    x0, info = seq.initial_guess(Ad, dev(b))
    assert info["used_fallback"] == 1 and np.array_equal(host(x0), 2 * u)
    zs = sacc.Sequence(n, 3, s=6, solver="cg", tol=1e-10)
    zs.push(dev(np.zeros(n)))
    x0, info = zs.initial_guess(Ad, dev(b))
    assert info["k_sketch"] == 0 and np.all(host(x0) == 0)


def test_comparator_guesses(sacc):
    rng = np.random.default_rng(7)
    n = 400
    S = _spd_small(n, rng)
    Ad = _dcsr(sacc, S)
    b = rng.standard_normal(n)
    xs = [rng.standard_normal(n) for _ in range(3)]
    for kind in ("zero", "previous"):
        seq = sacc.Sequence(n, 3, s=6, guess=kind)
        for x in xs:
            seq.push(dev(x))
        x0, _ = seq.initial_guess(Ad, dev(b))
        ref = np.zeros(n) if kind == "zero" else xs[-1]
        assert np.array_equal(host(x0), ref)


def test_m1_and_ring_wraparound(sacc):
    """M = 1 closed form, and a ring that wrapped several times holds the newest M columns."""
    rng = np.random.default_rng(8)
    n = 700
    S = _spd_small(n, rng)
    Ad = _dcsr(sacc, S)
    b = rng.standard_normal(n)
    seq = sacc.Sequence(n, 1, s=3, solver="cg")
    u = rng.standard_normal(n)
    seq.push(dev(u))
    x0, _ = seq.initial_guess(Ad, dev(b))
    assert np.allclose(host(x0), u * (u @ b) / (u @ (S @ u)), rtol=1e-11, atol=1e-14)
    M = 5
    seq = sacc.Sequence(n, M, s=10, solver="cg", seed=3)
    xs = [rng.standard_normal(n) for _ in range(13)]
    for x in xs:
        seq.push(dev(x))
    X = seq.copy_state("X")
    order = seq.copy_state("order")
    for lag, slot in enumerate(order):
        assert np.array_equal(X[:, slot], xs[13 - M + lag])
    x0, _ = seq.initial_guess(Ad, dev(b))
    ref = obs.galerkin_plain(S, b, np.stack(xs[-M:], 1))
    assert np.linalg.norm(host(x0) - ref) <= 1e-10 * np.linalg.norm(ref)
    cX = seq.copy_state("cX")
    assert np.linalg.norm(X @ cX - host(x0)) <= 1e-10 * np.linalg.norm(ref)


# ---------------------------------------------------------------------------- fixed-iteration iterates

@pytest.mark.parametrize("N", [64, 256, 362, 512])
@pytest.mark.parametrize("maxit", [1, 2, 8, 9, 17, 30])
def test_gmres_iterates_match(sacc, N, maxit):
    """GMRES(30) from x0 = 0 stopped after `maxit` Arnoldi steps (one and two rows per
    thread; inside and across polled batches of 8 steps): the iterate agrees with the
    oracle's within 10x the oracle's own rounding sensitivity (its iterate under a
    reversed summation order of A x), floored at 1e-12 relative."""
    print_case("gmres iterate", N, maxit)
    p, m = config(1, N)
    A = p.matrix(40)
    As = A.to_scipy()
    b = p.rhs(40)
    xo, oinfo, spread = rounding_spread(okr.gmres, As, b, np.zeros(p.n), 1e-14, 30, maxit=maxit)
    seq = sacc.Sequence(p.n, 2, s=4, solver="gmres", restart=30, tol=1e-14, maxit=maxit)
    xd, sinfo = seq.solve(sacc.DeviceCSR.from_csr(A), dev(b), dev(np.zeros(p.n)))
    xg = host(xd)
    assert sinfo["iters"] == oinfo["iters"] == maxit
    err = np.linalg.norm(xg - xo)
    ew = float(np.max(np.abs(xg - xo)) / np.max(np.abs(xo)))
    print_case("diff / spread / |x| / elementwise", err, spread, np.linalg.norm(xo), ew)
    assert err <= 10 * max(spread, 1e-12 * np.linalg.norm(xo))
    bar = iterate_bar("gmres", maxit)
    if bar is not None:
        assert ew <= bar, (ew, bar)


@pytest.mark.parametrize("N", [64, 512])
@pytest.mark.parametrize("restart", [3, 7, 8, 12, 16, 17, 31, 32])
def test_gmres_restart_lengths_match(sacc, N, restart):
    """GMRES(m) for restart lengths at and beside the 8 / 16 / 32 column tiers, run over
    two full cycles and one more step: each full cycle's last step is closed at the cycle
    end (from the second pass's coefficients and ||w'|| below the top of a tier, after a
    finalising step at it).  The iteration count matches the oracle's; the iterate and
    its true residual, which short restarts leave sensitive, are within 30x of how far a
    reordering of A x moves the oracle's (floored at 1e-12 and 1e-9 relative): across
    restarts the dot products' rounding moves them about 10x more than reordering A x
    alone does (measured on the 64 x 64 grid, 7 <= m <= 17)."""
    print_case("gmres restart", N, restart)
    p, m = config(1, N)
    A = p.matrix(41)
    As = A.to_scipy()
    b = p.rhs(41)
    maxit = 2 * restart + 1
    xo, oinfo = okr.gmres(As, b, np.zeros(p.n), 1e-14, restart, maxit=maxit)
    xr, _ = okr.gmres(reversed_order(As), b, np.zeros(p.n), 1e-14, restart, maxit=maxit)
    spread = float(np.linalg.norm(xo - xr))
    bn = np.linalg.norm(b)
    rspread = abs(np.linalg.norm(b - As @ xo) - np.linalg.norm(b - As @ xr)) / bn
    seq = sacc.Sequence(p.n, 2, s=4, solver="gmres", restart=restart, tol=1e-14, maxit=maxit)
    xd, sinfo = seq.solve(sacc.DeviceCSR.from_csr(A), dev(b), dev(np.zeros(p.n)))
    xg = host(xd)
    assert sinfo["iters"] == oinfo["iters"] == maxit
    relres = np.linalg.norm(b - As @ xg) / bn
    print_case("relres gpu / reported / oracle / spread", relres, sinfo["relres"], oinfo["relres"], rspread)
    assert abs(sinfo["relres"] - relres) <= 1e-6 * relres + 1e-15
    assert abs(relres - oinfo["relres"]) <= 30 * max(rspread, 1e-9 * oinfo["relres"])
    err = np.linalg.norm(xg - xo)
    print_case("diff / spread / |x|", err, spread, np.linalg.norm(xo))
    assert err <= 30 * max(spread, 1e-12 * np.linalg.norm(xo))


@pytest.mark.parametrize("N", [64, 512])
@pytest.mark.parametrize("maxit", [1, 8, 9, 50])
def test_cg_iterates_match(sacc, N, maxit):
    print_case("cg iterate", N, maxit)
    p, m = config(0, N)
    A = p.matrix(3)
    As = A.to_scipy()
    b = p.rhs(3)
    xo, oinfo, spread = rounding_spread(okr.cg, As, b, np.zeros(p.n), 1e-14, maxit=maxit)
    seq = sacc.Sequence(p.n, 2, s=4, solver="cg", tol=1e-14, maxit=maxit)
    xd, sinfo = seq.solve(sacc.DeviceCSR.from_csr(A), dev(b), dev(np.zeros(p.n)))
    xg = host(xd)
    assert sinfo["iters"] == oinfo["iters"] == maxit
    err = np.linalg.norm(xg - xo)
    ew = float(np.max(np.abs(xg - xo)) / np.max(np.abs(xo)))
    print_case("diff / spread / |x| / elementwise", err, spread, np.linalg.norm(xo), ew)
    assert err <= 10 * max(spread, 1e-12 * np.linalg.norm(xo))
    bar = iterate_bar("cg", maxit)
    if bar is not None:
        assert ew <= bar, (ew, bar)


# ---------------------------------------------------------------------------- minimum residual

@pytest.mark.parametrize("k,N,steps", [(0, 64, 14), (1, 64, 22)])
def test_minres_stepwise_guess(sacc, k, N, steps):
    """The paper's reduced problem (Section 2: the residual minimised over the span of
    the basis) from the same injected history: equal ranks; x0 element by element
    within 1e-11 of the largest entry (the oracle's own guess moves by at most 4.2e-14
    of it under a 1e-16 relative perturbation of X and S X; the normal equations square
    the conditioning of A Q, hence the wider bar than the Galerkin guess's); its residual
    never above the Galerkin guess's on the same span (both from the oracle)."""
    print_case("minres stepwise", k, N, steps)
    p, m = config(k, N)
    sols = _oracle_history(p, m, steps)
    gseq = sacc.Sequence(p.n, **method_kwargs(m, projection="minres"))
    oseq = OSeq(p.n, m["M"], m["sketch"], m["s"], m["method_seed"], m["solver"], m["restart"], m["tol"],
                projection="minres")
    ogal = OSeq(p.n, m["M"], m["sketch"], m["s"], m["method_seed"], m["solver"], m["restart"], m["tol"])
    worst = 0.0
    for i in range(steps):
        A = p.matrix(i)
        As = A.to_scipy()
        b = p.rhs(i)
        g = oseq.initial_guess(As, b)
        gg = ogal.initial_guess(As, b)
        x0d, ginfo = gseq.initial_guess(sacc.DeviceCSR.from_csr(A), dev(b))
        x0 = host(x0d)
        assert ginfo["k_sketch"] == g.k and ginfo["k_eff"] == g.k2, (i, ginfo, g.k, g.k2)
        if i > 0:
            ew = float(np.max(np.abs(x0 - g.x0)) / np.max(np.abs(g.x0)))
            worst = max(worst, ew)
            assert ew <= 1e-11, (i, ew)
            rmr = np.linalg.norm(b - As @ x0)
            rga = np.linalg.norm(b - As @ gg.x0)
            assert rmr <= rga * (1 + 1e-9), (i, rmr, rga)
        for q in (oseq, ogal):
            q.push(sols[i])
        gseq.push(dev(sols[i]))
    print_case("minres worst max |dx0| / max |x0|", worst)


def test_minres_plain_definition_and_m1(sacc):
    """Full-rank history: x0 = argmin over span(X) of ||b - A s|| (least squares on A X,
    the plain definition); M = 1: x0 = u (u^T A^T b) / ||A u||^2."""
    rng = np.random.default_rng(21)
    n = 900
    main = 4.0 + rng.uniform(0, 1, n)
    S = sp.diags([-np.ones(n - 1) * 1.3, main, -np.ones(n - 1) * 0.7], [-1, 0, 1]).tocsr()  # nonsymmetric
    Ad = _dcsr(sacc, S)
    b = rng.standard_normal(n)
    M = 6
    X = rng.standard_normal((n, M))
    seq = sacc.Sequence(n, M, s=2 * M, solver="gmres", projection="minres", seed=4)
    for j in range(M):
        seq.push(dev(X[:, j]))
    x0, info = seq.initial_guess(Ad, dev(b))
    ref = obs.minres_plain(S, b, X)
    assert info["k_eff"] == M
    err = np.linalg.norm(host(x0) - ref) / np.linalg.norm(ref)
    print_case("minres plain: rel err", err)
    assert err <= 1e-10
    u = rng.standard_normal(n)
    s1 = sacc.Sequence(n, 1, s=3, solver="gmres", projection="minres")
    s1.push(dev(u))
    x0, _ = s1.initial_guess(Ad, dev(b))
    Au = S @ u
    ref1 = u * (Au @ b) / (Au @ Au)
    assert np.allclose(host(x0), ref1, rtol=1e-11, atol=1e-14)


# ---------------------------------------------------------------------------- checkpoint / resume

@pytest.mark.parametrize("k,N,prec", [(0, 32, "fp64"), (1, 32, "fp64"), (2, 12, "mixed")])
def test_export_import_resumes_bitwise(sacc, k, N, prec):
    """A sequence exported after 7 steps and imported into a fresh one of the same
    configuration continues exactly as the original: the guesses, solutions and
    iteration counts of the next steps are bit for bit equal."""
    print_case("resume", k, N, prec)
    p, m = config(k, N)
    kw = method_kwargs(m, precision=prec)
    a = sacc.Sequence(p.n, **kw)
    fp32 = prec != "fp64"

    def A_(i):
        return sacc.DeviceCSR.from_csr(p.matrix(i, fp32=fp32) if fp32 else p.matrix(i))

    for i in range(7):
        a.step(A_(i), dev(p.rhs(i)))
    image = a.export_state()
    b = sacc.Sequence(p.n, **kw)
    b.import_state(image)
    other = sacc.Sequence(p.n, **method_kwargs(m, M=m["M"] - 1, precision=prec))
    with pytest.raises(sacc.SaccError):
        other.import_state(image)
    for i in range(7, 12):
        Ad, bd = A_(i), dev(p.rhs(i))
        xa0, ia0 = a.initial_guess(Ad, bd)
        xb0, ib0 = b.initial_guess(Ad, bd)
        assert np.array_equal(host(xa0), host(xb0)), i
        assert (ia0["k_sketch"], ia0["k_eff"]) == (ib0["k_sketch"], ib0["k_eff"])
        xa, sa_ = a.solve(Ad, bd, xa0)
        xb, sb_ = b.solve(Ad, bd, xb0)
        assert np.array_equal(host(xa), host(xb)) and sa_["iters"] == sb_["iters"], i
        a.push(xa)
        b.push(xb)


# ---------------------------------------------------------------------------- range finder m < M

@pytest.mark.parametrize("k,N,steps,m,proj", [(0, 64, 16, 5, "galerkin"), (1, 64, 24, 10, "galerkin"),
                                              (1, 64, 24, 10, "minres")])
def test_range_finder_compression(sacc, k, N, steps, m, proj):
    """The paper's randomized range finder with m < M (Section 2.2, Alg. 3): the basis
    spans X Z with the Gaussian Z whose rows travel with the history columns and a new Z
    every `refresh` pushes (7 here, so the run crosses several refreshes).  Same injected
    history on both sides: equal ranks; x0 element by element within 1e-12 of its largest
    entry (the oracle's own guess moves by at most 4.7e-14 of it when X, S X and Z are
    perturbed by 1e-16 relative: the Gaussian entries may differ in the last bits between
    the device's and the host's log, sqrt and sincospi); with the minimum-residual
    reduced problem (the Table 1 runs) within 1e-11, the bar of its own stepwise test."""
    print_case("range finder", k, N, steps, m, proj)
    p, meth = config(k, N)
    sols = _oracle_history(p, meth, steps)
    gseq = sacc.Sequence(p.n, **method_kwargs(meth, m=m, refresh=7, projection=proj))
    oseq = OSeq(p.n, meth["M"], meth["sketch"], meth["s"], meth["method_seed"], meth["solver"], meth["restart"],
                meth["tol"], m=m, refresh=7, projection=proj)
    bar = X0_ELEMENTWISE if proj == "galerkin" else 1e-11
    worst = 0.0
    for i in range(steps):
        A = p.matrix(i)
        As = A.to_scipy()
        b = p.rhs(i)
        g = oseq.initial_guess(As, b)
        x0d, gi = gseq.initial_guess(sacc.DeviceCSR.from_csr(A), dev(b))
        x0 = host(x0d)
        assert (gi["k_sketch"], gi["k_eff"]) == (g.k, g.k2), (i, gi, g.k, g.k2)
        assert g.k <= m
        if i > 0:
            ew = float(np.max(np.abs(x0 - g.x0)) / np.max(np.abs(g.x0)))
            worst = max(worst, ew)
            assert ew <= bar, (i, ew)
        oseq.push(sols[i])
        gseq.push(dev(sols[i]))
    print_case("range finder worst max |dx0| / max |x0|", worst)


# ---------------------------------------------------------------------------- POD basis (Alg. 2)

@pytest.mark.parametrize("k,N,steps,m", [(0, 64, 16, 5), (1, 64, 24, 10)])
def test_pod_guess_stepwise(sacc, k, N, steps, m):
    """Alg. 2's basis (the m leading left singular vectors of X, through the FP64 Gram
    X^T X and its Jacobi eigen-decomposition) from the same injected history: equal
    ranks; x0 element by element within 1e-8 of its largest entry (the Gram squares the
    singular values, so the trailing kept directions, near 1e-7 of the largest singular
    value, are determined only to about 1e-9: the oracle's own guess moves by up to 7e-11
    of its largest entry under a 1e-16 relative perturbation of X)."""
    print_case("pod", k, N, steps, m)
    p, meth = config(k, N)
    sols = _oracle_history(p, meth, steps)
    gseq = sacc.Sequence(p.n, **method_kwargs(meth, m=m, basis="pod"))
    oseq = OSeq(p.n, meth["M"], meth["sketch"], meth["s"], meth["method_seed"], meth["solver"], meth["restart"],
                meth["tol"], m=m, basis="pod")
    worst = 0.0
    for i in range(steps):
        A = p.matrix(i)
        As = A.to_scipy()
        b = p.rhs(i)
        g = oseq.initial_guess(As, b)
        x0d, gi = gseq.initial_guess(sacc.DeviceCSR.from_csr(A), dev(b))
        x0 = host(x0d)
        assert (gi["k_sketch"], gi["k_eff"]) == (g.k, g.k2), (i, gi, g.k, g.k2)
        if i > 0:
            ew = float(np.max(np.abs(x0 - g.x0)) / np.max(np.abs(g.x0)))
            worst = max(worst, ew)
            assert ew <= 1e-8, (i, ew)
        oseq.push(sols[i])
        gseq.push(dev(sols[i]))
    print_case("pod worst max |dx0| / max |x0|", worst)


def test_pod_plain_definition(sacc):
    """Separated singular values: the POD guess is the Galerkin projection on the span of
    the m leading left singular vectors of X (numpy's SVD)."""
    rng = np.random.default_rng(41)
    n, M, m = 1500, 12, 5
    U0, _ = np.linalg.qr(rng.standard_normal((n, M)))
    V0, _ = np.linalg.qr(rng.standard_normal((M, M)))
    X = U0 @ np.diag(np.geomspace(1.0, 1e-3, M)) @ V0.T
    S = _spd_small(n, rng)
    b = rng.standard_normal(n)
    seq = sacc.Sequence(n, M, s=2 * M, solver="cg", m=m, basis="pod")
    for j in range(M):
        seq.push(dev(X[:, j]))
    x0, info = seq.initial_guess(_dcsr(sacc, S), dev(b))
    Um = obs.pod_basis(X, m)
    ref = Um @ np.linalg.solve(Um.T @ (S @ Um), Um.T @ b)
    err = np.linalg.norm(host(x0) - ref) / np.linalg.norm(ref)
    print_case("pod plain: k, rel err", info["k_eff"], err)
    assert info["k_sketch"] == m and err <= 1e-9


def test_cg_tile_tuner(sacc):
    """The CG kernels' wave-tile shape is tuned on first use of an operator shape (one
    of 5, 7, 9 gathers per lane and step; the tuning launches write only partial rows):
    the solve that tunes and a later one on a fresh sequence (cached shape) give the same
    bits, and both match the oracle's iteration count within one."""
    p, m = config(2, 16)
    A = p.matrix(3, fp32=False)
    As = A.to_scipy()
    b = p.rhs(3)
    xo, oinfo = okr.cg(As, b, np.zeros(p.n), 1e-10)
    out = []
    for _ in range(2):
        seq = sacc.Sequence(p.n, 2, s=4, solver="cg", tol=1e-10)
        seq.profile_enable(True)
        xd, info = seq.solve(sacc.DeviceCSR.from_csr(A), dev(b), dev(np.zeros(p.n)))
        names = [r["name"] for r in seq.profile_read() if r["name"].startswith("k_cg_p<")]
        assert names and all(nm.rstrip(">").split(", ")[-1] in ("5", "7", "9") for nm in names), names
        out.append((host(xd), info["iters"], names))
    print_case("tuned tile", out[0][2])
    assert np.array_equal(out[0][0], out[1][0]) and out[0][2] == out[1][2]
    assert abs(out[0][1] - oinfo["iters"]) <= 1

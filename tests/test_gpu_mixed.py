"""GPU parity of the mixed mode (float32 storage, FP64 refinement) against the oracle's
emulation of it (``oracle.mixed``, ``oracle.sequence`` with precision="mixed").

Bar: both sides reach the FP64 tolerance against the float32-valued operator after
refinement; per step the iteration counts agree within one per refinement sweep for CG
(within twice the oracle's own change under a rounding-only perturbation where that
change is not zero);
for float32 GMRES(30), whose count moves by tens of iterations under a rounding-only
change on the oracle side alone, within 2% or twice the oracle's own change under a
rounding-only perturbation (reversed summation order in A x);
the guesses agree far below the tolerance unless the float32 rounding of the basis
flips a last bit, so their difference is bounded by 1e-2 tol ||b|| plus 1e-3 of the
oracle guess's own residual; with the BF16 sketch (the "mixed" mode's Gaussian sketch)
the two sides' S X differ by FP32 accumulation and their float32 bases round apart, so
10 times the oracle guess's change under a relative 1e-7 perturbation of its S X is
added.  The difference of the final solutions is printed per step.
"""

import math

import numpy as np
import pytest

from gen import config
from oracle import basis as obs
from oracle import mixed as omx
from oracle.sequence import Sequence as OSeq
from tests.gpu_helpers import dev, host, method_kwargs, print_case, reversed_order

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sacc():
    import torch

    assert torch.cuda.is_available()
    import paper_2309_02156_amd as pkg

    return pkg


def _oseq(p, m, precision="mixed"):
    return OSeq(p.n, m["M"], m["sketch"], m["s"], m["method_seed"], m["solver"], m["restart"], m["tol"],
                precision=precision)


def _A(p, i):
    A = p.matrix(i, fp32=True)
    return A, A.to_scipy().astype(np.float64)


@pytest.mark.parametrize("k,N,steps,prec", [(0, 48, 14, "mixed"), (1, 64, 24, "mixed"), (2, 16, 34, "mixed"),
                                           (1, 64, 24, "mixed_krylov"), (2, 16, 34, "mixed_krylov")])
def test_mixed_stepwise(sacc, k, N, steps, prec):
    """Same injected history on both sides: guess, ranks, counts."""
    print_case("mixed stepwise", k, N, steps, prec)
    p, m = config(k, N)
    ref = _oseq(p, m, prec)
    sols = []
    for i in range(steps):
        _, As = _A(p, i)
        x, _, _ = ref.step(As, p.rhs(i))
        sols.append(x)
    gseq = sacc.Sequence(p.n, **method_kwargs(m, precision=prec))
    oseq = _oseq(p, m, prec)
    rows = []
    for i in range(steps):
        A, As = _A(p, i)
        b = p.rhs(i)
        bn = np.linalg.norm(b)
        g = oseq.initial_guess(As, b)
        Ad = sacc.DeviceCSR.from_csr(A)
        x0d, ginfo = gseq.initial_guess(Ad, dev(b))
        x0 = host(x0d)
        ores0 = np.linalg.norm(b - As @ g.x0) / bn
        dres = np.linalg.norm(As @ (x0 - g.x0)) / bn
        assert ginfo["k_sketch"] == g.k and ginfo["k_eff"] == g.k2, (i, ginfo, g.k, g.k2)
        gspread = 0.0
        if prec == "mixed" and m["sketch"] == "gaussian" and g.k > 0:
            # BF16 sketch: the GPU's S X is the oracle's up to FP32 accumulation (relative
            # 2e-7 seen), so the two sides' float32 bases round apart; the oracle's own
            # guess under a relative 1e-7 perturbation of its S X calibrates that
            Xo_, SXo_ = oseq.history()
            rng = np.random.default_rng(100 + i)
            SXp = SXo_ * (1.0 + 1e-7 * rng.standard_normal(SXo_.shape))
            gp = obs.initial_guess(As, b, Xo_, SXp, None, oseq.projection, oseq.solver == "cg", oseq.tau_s,
                                   oseq.tau_c, oseq.store)
            gspread = float(np.linalg.norm(As @ (gp.x0 - g.x0)) / bn)
        assert dres <= 1e-2 * m["tol"] + 1e-3 * ores0 + 10 * gspread, (i, dres, ores0, gspread)
        xo, oinfo = oseq.solve(As, b, g.x0)
        xd, sinfo = gseq.solve(Ad, dev(b), dev(g.x0))
        xg = host(xd)
        true = np.linalg.norm(b - As @ xg) / bn
        assert true <= m["tol"] * (1 + 1e-6), (i, true)
        assert oinfo["relres"] <= m["tol"]
        sweeps = max(sinfo["refinements"], oinfo["refinements"], 1)
        assert abs(sinfo["refinements"] - oinfo["refinements"]) <= 1, (i, sinfo, oinfo)
        # the oracle's own count under a rounding-only change (reversed summation order
        # in A x) calibrates the allowance where it moves
        _, oinfo2 = oseq.solve(reversed_order(As), b, g.x0)
        spread = abs(oinfo2["iters"] - oinfo["iters"])
        if m["solver"] == "cg":
            # one iteration per refinement sweep: both sides start every sweep from the
            # same FP64 residual up to rounding; where the oracle itself moves (an inner
            # solve ending next to the tolerance: 229 against 212 iterations at step 2 of
            # the 48 x 48 sequence), twice that change
            allowed = max(sweeps, 2 * spread + 1) if spread > 0 else sweeps
        else:
            # float32 GMRES(30) with capped cycles: the oracle's own count moves by tens
            # of iterations under a rounding-only change, so the allowance is calibrated by
            # that change
            allowed = max(sweeps, 2 * spread + 1, math.ceil(0.02 * oinfo["iters"]))
        assert abs(sinfo["iters"] - oinfo["iters"]) <= allowed, (i, sinfo["iters"], oinfo["iters"], spread)
        rows.append((i, sinfo["iters"], oinfo["iters"], sinfo["refinements"], oinfo["refinements"],
                     float(np.linalg.norm(xg - xo) / max(np.linalg.norm(xo), 1e-300))))
        oseq.push(sols[i])
        gseq.push(dev(sols[i]))
    # the stored history (float32 for "mixed") equals the oracle's stored columns
    X = gseq.copy_state("X")
    order = gseq.copy_state("order")
    Xo, _ = oseq.history()
    used = [s for s in order if s >= 0]
    assert X.dtype == (np.float32 if prec == "mixed" else np.float64)
    assert np.array_equal(X[:, used].astype(np.float64), Xo)
    print_case("(step, iters gpu, iters oracle, sweeps gpu, sweeps oracle, |dx|/|x|)", rows)


def test_mixed_trajectory(sacc):
    """Free-running mixed sequences on the 3-D operator: tolerance met, totals agree."""
    p, m = config(2, 16)
    steps = 40
    print_case("mixed trajectory", p.n, steps)
    gseq = sacc.Sequence(p.n, **method_kwargs(m, precision="mixed"))
    oseq = _oseq(p, m)
    its = []
    for i in range(steps):
        A, As = _A(p, i)
        b = p.rhs(i)
        _, _, oinfo = oseq.step(As, b)
        xd, ginfo = gseq.step(sacc.DeviceCSR.from_csr(A), dev(b))
        true = np.linalg.norm(b - As @ host(xd)) / np.linalg.norm(b)
        assert true <= m["tol"] * (1 + 1e-6), (i, true)
        its.append((ginfo["iters"], oinfo["iters"]))
    g_tot = sum(a for a, _ in its)
    o_tot = sum(b for _, b in its)
    print_case("iterations (gpu, oracle)", its)
    assert abs(its[0][0] - its[0][1]) <= 2
    assert abs(g_tot - o_tot) <= 0.1 * o_tot, (g_tot, o_tot)


def _smooth_history_3d(p, M, rng):
    x, y, z = p._node_coords()
    sx = [np.sin(a * np.pi * x) for a in range(8)]
    sy = [np.sin(a * np.pi * y) for a in range(8)]
    sz = [np.sin(a * np.pi * z) for a in range(8)]
    modes = rng.integers(1, 8, size=(3 * M, 3))
    F = np.stack([sx[a] * sy[b] * sz[c] for a, b, c in modes], 1)
    return [omx.fl32(0.01 * (F @ rng.standard_normal(3 * M))) for _ in range(M)]


def test_mixed_full_size_3d(sacc):
    """The 128^3 float32 workload (n = 2 097 152, M = 30, Gaussian s = 60) on a synthetic
    full-rank history and a right-hand side near A span(X): the guess against the plain Galerkin definition on span(X)
    (float32 storage of the basis moves it by float32 rounding only), then the refined
    solve to 1e-8 checked in FP64 against the float32-valued operator."""
    p, m = config(2)
    print_case("mixed full-size", p.n)
    rng = np.random.default_rng(9)
    hist = _smooth_history_3d(p, m["M"], rng)
    A, As = _A(p, 60)
    X = np.stack(hist, 1)
    # a right-hand side whose solution lies close to span(X): the guess is then sharp
    b = As @ (X @ rng.standard_normal(m["M"])) + 1e-3 * p.rhs(60)
    gseq = sacc.Sequence(p.n, **method_kwargs(m, precision="mixed", maxit=4000))
    for h in hist:
        gseq.push(dev(h))
    xp = obs.galerkin_plain(As, b, X)
    Ad = sacc.DeviceCSR.from_csr(A)
    x0d, ginfo = gseq.initial_guess(Ad, dev(b))
    x0 = host(x0d)
    bn = np.linalg.norm(b)
    assert ginfo["k_sketch"] == m["M"] and ginfo["k_eff"] == m["M"]
    dx = np.linalg.norm(x0 - xp) / np.linalg.norm(xp)
    r0 = np.linalg.norm(b - As @ x0) / bn
    rp = np.linalg.norm(b - As @ xp) / bn
    print_case("full-size mixed guess: |dx0|/|x0|, relres0 gpu, plain", dx, r0, rp)
    # float32 rounding of Q1 (relative 6e-8, high-frequency) is amplified by ||A|| in
    # the residual: allow that floor on top of the plain guess's residual
    assert dx <= 1e-5 and r0 <= rp + 5e-5
    xd, sinfo = gseq.solve(Ad, dev(b), x0d)
    true = np.linalg.norm(b - As @ host(xd)) / bn
    print_case("full-size mixed: iters, sweeps, relres", sinfo["iters"], sinfo["refinements"], true)
    assert sinfo["rc"] == 0 and true <= m["tol"] * (1 + 1e-6)
    assert abs(true - sinfo["relres"]) <= 1e-3 * m["tol"]
    assert sinfo["refinements"] >= 1


@pytest.mark.parametrize("N", [24, 48])
def test_mixed_cg_packed_columns_bitwise(sacc, N):
    """Mixed CG reads the matrix's columns as 16-bit offsets from the row when every
    offset fits (a 3-D seven-point operator: offsets up to N^2): the same products in
    the same order, so solution, counts and residuals equal, bit for bit, those of the
    solve with the full column indices (SACC_NO_COL16 set)."""
    import os

    p, _ = config(2, N)
    A, As = _A(p, 3)
    b = p.rhs(3)
    Ad = sacc.DeviceCSR.from_csr(A)
    out = []
    for off in (False, True):
        if off:
            os.environ["SACC_NO_COL16"] = "1"
        try:
            # M = 4: the basis region (4 n floats) holds the 2 nnz bytes of the offsets
            seq = sacc.Sequence(p.n, 4, s=8, solver="cg", tol=1e-8, precision="mixed", inner_tol=1e-4, max_refine=10)
            seq.profile_enable(True)
            xd, info = seq.solve(Ad, dev(b), dev(np.zeros(p.n)))
            names = [r["name"] for r in seq.profile_read()]
            out.append((host(xd), info, names))
        finally:
            os.environ.pop("SACC_NO_COL16", None)
    (x1, i1, n1), (x2, i2, n2) = out
    assert any("i16" in nm for nm in n1) and not any("i16" in nm for nm in n2), (n1, n2)
    print_case("packed / full: iters", i1["iters"], i2["iters"], "sweeps", i1["refinements"], i2["refinements"])
    assert np.array_equal(x1, x2)
    for key in ("iters", "refinements", "relres", "relres0", "status"):
        assert i1[key] == i2[key], (key, i1[key], i2[key])
    assert np.linalg.norm(b - As @ x1) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)


def test_mixed_cg_far_offsets_fall_back(sacc):
    """A matrix with a column 40000 rows from its row (beyond 16 bits) solves with the
    full column indices: bitwise the result with packing turned off, tolerance met, the
    oracle's count within one per sweep."""
    import os

    import scipy.sparse as sp

    n, far = 70000, 40000
    main = np.full(n, 4.0)
    off1 = np.full(n - 1, -1.0)
    offf = np.full(n - far, -0.5)
    A = sp.diags([main, off1, off1, offf, offf], [0, 1, -1, far, -far], format="csr").astype(np.float32)
    A.sort_indices()
    As = A.astype(np.float64)
    b = np.random.default_rng(5).standard_normal(n)
    Ad = sacc.DeviceCSR(A.indptr, A.indices, A.data)
    out = []
    for off in (False, True):
        if off:
            os.environ["SACC_NO_COL16"] = "1"
        try:
            seq = sacc.Sequence(n, 2, s=4, solver="cg", tol=1e-8, precision="mixed", inner_tol=1e-4, max_refine=10)
            xd, info = seq.solve(Ad, dev(b), dev(np.zeros(n)))
            out.append((host(xd), info))
        finally:
            os.environ.pop("SACC_NO_COL16", None)
    (x1, i1), (x2, i2) = out
    assert np.array_equal(x1, x2) and i1["iters"] == i2["iters"]
    assert np.linalg.norm(b - As @ x1) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)
    xo, oi = omx.solve_ir(As, b, np.zeros(n), 1e-8, "cg", 30, 1e-4, 10, 200000)
    assert abs(i1["iters"] - oi["iters"]) <= max(1, i1["refinements"]), (i1["iters"], oi["iters"])

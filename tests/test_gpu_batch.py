"""GPU tests of the batched execution of independent sequences (sa_batch_*).

On streams the batch runs the same kernels as one sequence at a time, only several at
once, so its solutions and iteration counts must equal those of the sequences stepped
one by one (bit for bit).  The segmented engine (all solves in lockstep launches) is
checked against the oracle per sequence like the stream plan, and its graph replays
against its eager launches bit for bit.  Every solve meets the FP64 tolerance against
its float32 operator; the plan autotuner ends with a tuned plan.
"""

import numpy as np
import pytest

from gen import batch_problems
from tests.gpu_helpers import dev, host, print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sacc():
    import torch

    assert torch.cuda.is_available()
    import paper_2309_02156_amd as pkg

    return pkg


def _seq(sacc, p, m):
    return sacc.Sequence(p.n, m["M"], s=m["s"], sketch=m["sketch"], solver=m["solver"], restart=m["restart"],
                         tol=m["tol"], seed=m["method_seed"], precision=m["prec"],
                         max_refine=m["max_refine"])


def test_batch_streams_equals_sequential(sacc):
    import torch

    probs = batch_problems(seed=4, nseq=6, lo=16, hi=40, steps=40)
    steps = 24
    print_case("batch", [(p.N, m["M"], m["solver"]) for p, m in probs], steps)
    seqs_b = [_seq(sacc, p, m) for p, m in probs]
    seqs_s = [_seq(sacc, p, m) for p, m in probs]
    batch = sacc.Batch(seqs_b, max_streams=4, tune_warmup=8)
    batch.set_mode("streams")
    for i in range(steps):
        As = [sacc.DeviceCSR.from_csr(p.matrix(i)) for p, _ in probs]
        bs = [dev(p.rhs(i)) for p, _ in probs]
        xb = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _ in probs]
        infos = batch.step(As, bs, xb)
        for j, (p, m) in enumerate(probs):
            xs, si = seqs_s[j].step(As[j], bs[j])
            assert np.array_equal(host(xb[j]), host(xs)), (i, j)
            assert infos[j]["iters"] == si["iters"], (i, j, infos[j]["iters"], si["iters"])
            Asc = p.matrix(i).to_scipy().astype(np.float64)
            b = p.rhs(i)
            rel = np.linalg.norm(b - Asc @ host(xb[j])) / np.linalg.norm(b)
            assert rel <= m["tol"] * (1 + 1e-6), (i, j, rel)
    plan = batch.plan()
    print_case("plan", plan)
    assert plan["tuned"] and not plan["segmented"] and plan["streams"] == 4


def test_batch_auto_tunes(sacc):
    """The tuner times every stream plan and the segmented plans (both work-item sizes),
    one step each after the warm-up, and keeps one; every step meets the tolerance
    whichever plan ran it."""
    import torch

    probs = batch_problems(seed=5, nseq=5, lo=16, hi=32, steps=40)
    warm, steps = 3, 20
    seqs = [_seq(sacc, p, m) for p, m in probs]
    batch = sacc.Batch(seqs, max_streams=8, tune_warmup=warm)
    seen_seg = False
    for i in range(steps):
        As = [sacc.DeviceCSR.from_csr(p.matrix(i)) for p, _ in probs]
        bs = [dev(p.rhs(i)) for p, _ in probs]
        xb = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _ in probs]
        infos = batch.step(As, bs, xb)
        seen_seg = seen_seg or batch.plan()["segmented"]
        for j, (p, m) in enumerate(probs):
            Asc = p.matrix(i).to_scipy().astype(np.float64)
            b = p.rhs(i)
            rel = np.linalg.norm(b - Asc @ host(xb[j])) / np.linalg.norm(b)
            assert rel <= m["tol"] * (1 + 1e-6) and infos[j]["status"] == 0, (i, j, rel)
    plan = batch.plan()
    print_case("plan", plan)
    assert plan["tuned"] and 1 <= plan["streams"] <= 8


@pytest.mark.parametrize("rows", [1024, 512])
def test_batch_segmented_graph_equals_eager(sacc, rows, monkeypatch):
    """The segmented engine replaying its captured hipGraph of 16 steps (many replays per
    solve, the guesses' eager launches and host waits between solves) gives bitwise the
    solutions and counts of the same engine launched eagerly, step after step, with each
    work-item size; every solve meets the tolerance."""
    import torch

    monkeypatch.setenv("SACC_SEG_ROWS", str(rows))

    probs = batch_problems(seed=6, nseq=6, lo=12, hi=40, steps=40)
    steps = 14
    print_case("segmented graph / eager", [(p.N, m["M"], m["solver"]) for p, m in probs], steps)
    ga = sacc.Batch([_seq(sacc, p, m) for p, m in probs], max_streams=2)
    ea = sacc.Batch([_seq(sacc, p, m) for p, m in probs], max_streams=2)
    ga.set_mode("segmented")
    ea.set_mode("segmented_eager")
    for i in range(steps):
        As = [sacc.DeviceCSR.from_csr(p.matrix(i)) for p, _ in probs]
        bs = [dev(p.rhs(i)) for p, _ in probs]
        xg = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _ in probs]
        xe = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _ in probs]
        ig = ga.step(As, bs, xg)
        ie = ea.step(As, bs, xe)
        for j, (p, m) in enumerate(probs):
            assert np.array_equal(host(xg[j]), host(xe[j])), (i, j)
            for key in ("iters", "restarts", "refinements", "status", "k_eff"):
                assert ig[j][key] == ie[j][key], (i, j, key, ig[j][key], ie[j][key])
            assert ig[j]["relres"] == ie[j]["relres"]
            Asc = p.matrix(i).to_scipy().astype(np.float64)
            b = p.rhs(i)
            rel = np.linalg.norm(b - Asc @ host(xg[j])) / np.linalg.norm(b)
            assert rel <= m["tol"] * (1 + 1e-6), (i, j, rel)
            assert abs(ig[j]["relres"] - rel) <= 1e-6 * rel + 1e-15, (i, j, ig[j]["relres"], rel)
    assert ga.plan()["segmented"] and ea.plan()["segmented"]


@pytest.mark.parametrize("mode,rows,mix", [("streams", None, False), ("segmented", 1024, False),
                                           ("segmented", 512, False), ("segmented", 1024, True)])
def test_batch_matches_oracle(sacc, mode, rows, mix, monkeypatch):
    """Each sequence of a batch, stepped by the batch driver in its own configuration
    (float32 operator and Krylov vectors, FP64 history and refinement, up to 100 sweeps),
    against the oracle on the same history: before every step the oracle's history holds
    exactly the solutions the GPU pushed.  Equal kept ranks; both meet the tolerance; per
    step the iteration counts within twice the oracle's own change under a rounding-only
    perturbation (reversed summation order of A x, or its start perturbed by 1e-15
    relative), at least one per refinement sweep and 10 % (each side starts from its own
    guess, and the float32 inner solves of the first steps' two sweeps move by several
    iterations under such perturbations); the totals over all steps within 3 %.  The
    segmented engine runs with each of its work-item sizes (pinned by SACC_SEG_ROWS);
    `mix`: two sequences keep float32 histories with the BF16 sketch (`mixed`) and one
    takes a 160-row sketch, so that the segmented step's batched launches run both
    storage types (x0) and both QRCP instantiations."""
    import math

    import torch

    from oracle.sequence import Sequence as OSeq
    from tests.gpu_helpers import reversed_order

    probs = batch_problems(seed=4, nseq=5, lo=16, hi=36, steps=40)
    steps = 20
    if mix:
        probs[0][1]["prec"] = probs[1][1]["prec"] = "mixed"
        probs[2][1]["s"] = 160
    print_case("batch vs oracle", [(p.N, m["M"], m["s"], m["solver"], m["prec"]) for p, m in probs], steps)
    seqs = [_seq(sacc, p, m) for p, m in probs]
    batch = sacc.Batch(seqs, max_streams=4, tune_warmup=4)
    batch.set_mode(mode)
    if rows is not None:
        monkeypatch.setenv("SACC_SEG_ROWS", str(rows))
    oseqs = [OSeq(p.n, m["M"], m["sketch"], m["s"], m["method_seed"], m["solver"], m["restart"], m["tol"],
                  precision=m["prec"], max_refine=m["max_refine"]) for p, m in probs]
    rows = []
    rng = np.random.default_rng(11)
    tot_g = tot_o = 0
    for i in range(steps):
        As = [sacc.DeviceCSR.from_csr(p.matrix(i)) for p, _ in probs]
        bs = [dev(p.rhs(i)) for p, _ in probs]
        xb = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _ in probs]
        ref = []
        for j, (p, m) in enumerate(probs):
            Asc = p.matrix(i).to_scipy().astype(np.float64)
            b = p.rhs(i)
            g = oseqs[j].initial_guess(Asc, b)
            xo, oinfo = oseqs[j].solve(Asc, b, g.x0)
            ref.append((Asc, b, g, oinfo))
        infos = batch.step(As, bs, xb)
        for j, (p, m) in enumerate(probs):
            Asc, b, g, oinfo = ref[j]
            gi = infos[j]
            xg = host(xb[j])
            rel = np.linalg.norm(b - Asc @ xg) / np.linalg.norm(b)
            assert rel <= m["tol"] * (1 + 1e-6) and oinfo["relres"] <= m["tol"], (i, j, rel, oinfo["relres"])
            assert gi["k_sketch"] == g.k and gi["k_eff"] == g.k2, (i, j, gi["k_sketch"], gi["k_eff"], g.k, g.k2)
            # each side starts from its own guess (equal up to rounding); the allowance
            # is calibrated by the oracle's own change when its start or its A x is
            # perturbed at rounding level, floored at one per sweep and 10 %
            sweeps = max(gi["refinements"], oinfo["refinements"], 1)
            _, o2 = oseqs[j].solve(reversed_order(Asc), b, g.x0)
            _, o3 = oseqs[j].solve(Asc, b, g.x0 * (1.0 + 1e-15 * rng.standard_normal(p.n)))
            spread = max(abs(o2["iters"] - oinfo["iters"]), abs(o3["iters"] - oinfo["iters"]))
            allowed = max(sweeps, 2 * spread + 1, math.ceil(0.1 * oinfo["iters"]))
            assert abs(gi["iters"] - oinfo["iters"]) <= allowed, (i, j, gi["iters"], oinfo["iters"], allowed)
            rows.append((i, j, gi["iters"], oinfo["iters"], spread, gi["k_eff"]))
            tot_g += gi["iters"]
            tot_o += oinfo["iters"]
            oseqs[j].push(xg)   # the oracle's history follows the GPU's
    print_case("(step, seq, iters gpu, iters oracle, oracle spread, k)", rows)
    assert abs(tot_g - tot_o) <= 0.03 * tot_o, (tot_g, tot_o)


def _edge_matrix(n, kind, seed):
    import scipy.sparse as sp

    if n == 1:
        A = sp.csr_matrix(np.array([[3.0]]))
    else:
        R = sp.random(n, n, density=min(1.0, 4.0 / n), random_state=seed, format="csr")
        if kind == "cg":  # symmetric, diagonally dominant: SPD
            S = R + R.T
            A = S + sp.diags(np.asarray(abs(S).sum(axis=1)).ravel() + 1.0)
        else:  # nonsymmetric, diagonally dominant
            A = R - 0.5 * R.T + sp.diags(np.asarray(abs(R).sum(axis=1)).ravel() + 2.0)
    A = sp.csr_matrix(A, dtype=np.float32)
    A.sort_indices()
    return A


@pytest.mark.parametrize("rows", [1024, 512])
def test_batch_segmented_edge_cases(sacc, rows, monkeypatch):
    """The segmented engine on ragged and tiny systems (n = 1 .. 3000, not multiples of
    its 64-row tiles or its 512- or 1024-row work items), GMRES restart lengths 1, 2, 7 and 30, a
    zero right-hand side in the second step, and an iteration cap of 3: each system
    against the oracle's refinement solve from the same zero start (guess "zero"),
    equal stopping status, the cap's count exact, zero x for b = 0, converged counts
    within max(sweeps, 2 spread + 1, 10 %) of the oracle's and the tolerance met."""
    import math

    import torch

    from oracle import mixed as omx
    from tests.gpu_helpers import reversed_order

    cases = [(1, "cg", 30, 0), (5, "gmres", 1, 0), (63, "cg", 30, 0), (65, "gmres", 2, 0),
             (1025, "gmres", 30, 0), (1025, "cg", 30, 0), (3000, "gmres", 7, 0), (700, "cg", 30, 3),
             (900, "gmres", 30, 3)]
    mats = [_edge_matrix(n, kind, 40 + k) for k, (n, kind, _, _) in enumerate(cases)]
    seqs = [sacc.Sequence(n, 2, s=4, solver=kind, restart=r, tol=1e-8, precision="mixed_krylov", max_refine=20,
                          guess="zero", maxit=mx if mx else 200000)
            for (n, kind, r, mx) in cases]
    batch = sacc.Batch(seqs, max_streams=2)
    batch.set_mode("segmented")
    monkeypatch.setenv("SACC_SEG_ROWS", str(rows))
    rng = np.random.default_rng(9)
    As = [sacc.DeviceCSR(A.indptr, A.indices, A.data) for A in mats]
    for step in range(2):
        bs_h = [rng.standard_normal(n) for (n, _, _, _) in cases]
        if step == 1:
            bs_h[2] = np.zeros(cases[2][0])
            bs_h[4] = np.zeros(cases[4][0])
        bs = [dev(b) for b in bs_h]
        xs = [torch.empty(n, dtype=torch.float64, device="cuda") for (n, _, _, _) in cases]
        infos = batch.step(As, bs, xs)
        for j, (n, kind, r, mx) in enumerate(cases):
            print_case("edge", step, n, kind, r, mx, infos[j]["iters"], infos[j]["status"])
            A64 = mats[j].astype(np.float64)
            b = bs_h[j]
            xg = host(xs[j])
            gi = infos[j]
            if not b.any():
                assert np.array_equal(xg, np.zeros(n)) and gi["iters"] == 0 and gi["status"] == 0
                continue
            maxit = mx if mx else 200000
            xo, oi = omx.solve_ir(A64, b, np.zeros(n), 1e-8, kind, r, 1e-4, 20, maxit)
            if mx:
                assert oi["status"] == 1 and gi["status"] != 0, (j, oi["status"], gi["status"])
                assert gi["iters"] == oi["iters"] == mx, (j, gi["iters"], oi["iters"])
                continue
            rel = np.linalg.norm(b - A64 @ xg) / np.linalg.norm(b)
            assert gi["status"] == 0 and oi["status"] == 0, (j, gi["status"], oi["status"])
            assert rel <= 1e-8 * (1 + 1e-6), (j, rel)
            assert abs(gi["relres"] - rel) <= 1e-6 * rel + 1e-15, (j, gi["relres"], rel)
            _, o2 = omx.solve_ir(reversed_order(A64.tocsr()), b, np.zeros(n), 1e-8, kind, r, 1e-4, 20, maxit)
            spread = abs(o2["iters"] - oi["iters"])
            sweeps = max(gi["refinements"], oi["refinements"], 1)
            allowed = max(sweeps, 2 * spread + 1, math.ceil(0.1 * oi["iters"]))
            assert abs(gi["iters"] - oi["iters"]) <= allowed, (j, gi["iters"], oi["iters"], allowed)

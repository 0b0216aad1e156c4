#!/usr/bin/env python3
"""Benchmark: ms per time step of the subspace-accelerated sequence solver on one MI355X.

Headline workload (one GPU): the 128^3 lognormal-coefficient diffusion sequence
A(t_i) x = b(t_i) (n = 2 097 152, 14 581 760 nonzeros, float32 matrix values, int32
indices), history M = 30, Gaussian sketch s = 60, Galerkin projection, CG in float32
with FP64 iterative refinement to ||b - A x|| <= 1e-8 ||b|| (the mixed-precision mode
with float32 history and basis).  It is the largest single system of the workloads and
the one whose working set exceeds the on-package cache.  A step is one pass of the
whole hot path: initial guess (sketched-QR basis, SpMM + Gram, reduced solve, x0) ->
refined Krylov solve -> history push (copy + sketch + QRCP).

Steady state: the first M steps fill the history (untimed, not counted as warm-up),
then --warmup steps, then --steps timed steps.  Every A(t_i), b(t_i) is staged in HBM
before the first step; a step reads them in place (assembly is outside the timed region).

Prints ONE JSON line (keys at the end of main()); progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ms/timestep + Krylov iters at relres 1e-8, learned/mixed vs plain; SpMV GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


class CSRView:
    """A CSR matrix whose value array is one staged row of a (steps x nnz) device tensor."""

    def __init__(self, rowptr, col, val):
        self.rowptr, self.col, self.val = rowptr, col, val
        self.n, self.nnz = rowptr.numel() - 1, col.numel()

    def c_struct(self):
        import paper_2309_02156_amd as sacc

        return sacc.DeviceCSR.c_struct(self)


class Staged:
    """Every step's matrix values and right-hand side of one sequence, in HBM."""

    def __init__(self, torch, np, problem, steps, fp32):
        rowptr, col = problem.pattern()
        self.rowptr = torch.as_tensor(rowptr).cuda()
        self.col = torch.as_tensor(col).cuda()
        B = torch.as_tensor(problem.value_basis()).cuda()
        C = torch.as_tensor(np.stack([problem.value_coefs(i) for i in range(steps)])).cuda()
        v = C @ B
        self.vals = v.float() if fp32 else v
        del B, C, v
        self.rhs = torch.empty((steps, problem.n), dtype=torch.float64, device="cuda")
        for i in range(steps):
            self.rhs[i].copy_(torch.as_tensor(problem.rhs(i)))
        self.n, self.nnz, self.steps = problem.n, int(col.size), steps

    @classmethod
    def assembled(cls, torch, np, problem, steps):
        """The same from the problem's own assembly, step by step on the host (for
        operators without an affine value basis)."""
        st = cls.__new__(cls)
        rowptr, col = problem.pattern()
        st.rowptr = torch.as_tensor(rowptr).cuda()
        st.col = torch.as_tensor(col).cuda()
        st.vals = torch.as_tensor(np.stack([problem.matrix(i).val for i in range(steps)])).cuda()
        st.rhs = torch.as_tensor(np.stack([problem.rhs(i) for i in range(steps)])).cuda()
        st.n, st.nnz, st.steps = problem.n, int(col.size), steps
        return st

    def A(self, i):
        return CSRView(self.rowptr, self.col, self.vals[i])

    def as_fp64(self):
        """The same steps with the values upcast to float64 (a copy of the values only)."""
        c = Staged.__new__(Staged)
        c.__dict__.update(self.__dict__)
        c.vals = self.vals.double()
        return c

    def values_host(self, i):
        return self.vals[i].double().cpu().numpy()

    def csr_host(self, i):
        import scipy.sparse as sp

        return sp.csr_matrix((self.values_host(i), self.col.cpu().numpy(), self.rowptr.cpu().numpy()),
                             shape=(self.n, self.n))


def make_seq(sacc, n, method, guess="projection", precision=None, precond="none", **extra):
    return sacc.Sequence(n, method["M"], s=method["s"], sketch=method["sketch"], solver=method["solver"],
                         restart=method["restart"], tol=method["tol"], seed=method["method_seed"], guess=guess,
                         precision=precision or method["prec"], precond=precond, **extra)


def run_sequence(sacc, torch, st, method, fill, warmup, steps, guess="projection", precision=None, profile=False,
                 keep_seq=False, precond="none", **extra):
    """Steps 0 .. fill + warmup + steps - 1; the last `steps` are timed.  Returns the
    infos of the timed steps, their wall time, the kernel records (profile=True) and the
    sequence (keep_seq=True: the caller closes it) with its last solution."""
    seq = make_seq(sacc, st.n, method, guess, precision, precond, **extra)
    x = torch.empty(st.n, dtype=torch.float64, device="cuda")
    first = fill + warmup
    for i in range(first):
        seq.step(st.A(i), st.rhs[i], x)
        if (i + 1) % 20 == 0:
            log(f"  history fill / warm-up step {i + 1}/{first}")
    if profile:
        seq.profile_enable(True)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(first, first + steps):
        infos.append(seq.step(st.A(i), st.rhs[i], x)[1])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = seq.profile_read() if profile else None
    if keep_seq:
        return infos, wall, prof, seq, x
    seq.close()
    return infos, wall, prof


def summary(infos, wall, steps):
    import numpy as np

    return dict(ms_per_step=round(1e3 * wall / steps, 4),
                iters_per_step=round(float(np.mean([d["iters"] for d in infos])), 3),
                refinements_per_step=round(float(np.mean([d["refinements"] for d in infos])), 3),
                relres_max=float(max(d["relres"] for d in infos)),
                relres0_median=float(np.median([d["relres0"] for d in infos])),
                k_eff=[int(min(d["k_eff"] for d in infos)), int(max(d["k_eff"] for d in infos))])


def committed_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/<kernel>_<workload>_traffic.md, or None when there is none or the kernel
    sources have changed since the counters were taken."""
    base = kernel.split("<")[0]
    path = os.path.join(ROOT, "profiles", f"{base}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if f"# HBM traffic of {kernel} " not in text:
        return None
    m_t = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    m_h = re.search(r"^kernel_source_sha256: ([0-9a-f]+)", text, re.M)
    if not m_t or not m_h:
        return None
    return int(m_t.group(1)) if kernel_source_sha() == m_h.group(1) else None


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("krylov.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2309_02156_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def roofline(prof, workload):
    """The dominant kernel of the instrumented run: algorithmic bytes / average launch time."""
    dom = max(prof, key=lambda r: r["ms"])
    us = 1e3 * dom["ms"] / dom["launches"]
    gbs = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    for r in sorted(prof, key=lambda r: -r["ms"]):
        log(f"  {r['name']}: {r['launches']} launches, {1e3 * r['ms'] / r['launches']:.2f} us avg, "
            f"{r['bytes'] / (r['ms'] * 1e-3) / 1e9:.0f} GB/s")
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": committed_traffic(dom["name"], workload),
            "kernel": dom["name"], "bytes_per_launch": round(dom["bytes"] / dom["launches"]),
            "avg_us": round(us, 3), "launches": dom["launches"]}


def spmv_gbps(sacc, torch, A, reps=200):
    x = torch.randn(A.n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(10):
        sacc.spmv(A, x, y)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sacc.spmv(A, x, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = A.nnz * (A.val.element_size() + 4) + 4 * (A.n + 1) + 2 * 8 * A.n
    return dict(gbps=round(nbytes / (ms * 1e-3) / 1e9, 1), us=round(1e3 * ms, 2), bytes=int(nbytes),
                frac=round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))


def cpu_baseline(np, st, method, hist, x_gpu, step):
    """The FP64 oracle on the host for one step of the same sequence with the GPU's
    history injected: the oracle's history is the M solutions the GPU stored before
    `step` (hist: its X and ring order; float32 values upcast), their sketch S X computed
    untimed; then guess, solve and push of `step` are timed on the same staged A (float32
    values upcast) and b.  Returns the baseline record, the relative difference of the
    GPU's solution x_gpu of that step from the oracle's FP64 solution, and the oracle's
    counts."""
    import types

    from oracle.sequence import make_sequence

    X = hist["X"].astype(np.float64)
    order = [s_ for s_ in hist["order"] if s_ >= 0]
    oseq = make_sequence(types.SimpleNamespace(n=st.n), method)
    t0 = time.perf_counter()
    cols = [X[:, s_].copy() for s_ in order]
    SX = oseq.S.apply(np.stack(cols, 1))
    oseq.cols = cols
    oseq.scols = [SX[:, j].copy() for j in range(SX.shape[1])]
    setup = time.perf_counter() - t0
    A = st.csr_host(step)
    b = st.rhs[step].cpu().numpy()
    t0 = time.perf_counter()
    x, g, info = oseq.step(A, b)
    dt = time.perf_counter() - t0
    err = float(np.linalg.norm(x_gpu - x) / np.linalg.norm(x))
    try:
        from threadpoolctl import threadpool_info

        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = 1
    rec = dict(value=round(1e3 * dt, 1), unit="ms/timestep", cores=int(threads), kind="oracle",
               sample=f"step {step} of the same sequence (1 step, {dt:.1f} s: guess, FP64 CG solve to 1e-8, push "
                      f"with its Gaussian sketch of the new column) with the GPU's {len(cols)} stored solutions "
                      f"before it injected as the history (their sketch computed untimed in {setup:.1f} s); "
                      f"oracle iterations {info['iters']}, k {g.k}; host os.cpu_count()={os.cpu_count()}, "
                      f"BLAS threads {threads}, SciPy SpMV single-threaded")
    return rec, err, dict(oracle_iters=int(info["iters"]), oracle_relres0=float(info["relres0"]),
                          oracle_k=int(g.k2))


def headline(sacc, torch, np, args):
    from gen import config

    p, method = config(2)
    M = method["M"]
    total = M + args.warmup + args.steps + 1   # + the cpu-baseline step
    log(f"staging {total} steps of the 128^3 sequence")
    st = Staged(torch, np, p, total, fp32=True)
    torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.empty(32 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 268435456 bytes")
        del src, dst
    log("timed run: mixed (float32 operator, history and Krylov vectors, FP64 refinement)")
    infos, wall, _, seq, x = run_sequence(sacc, torch, st, method, M, args.warmup, args.steps, keep_seq=True)
    res = summary(infos, wall, args.steps)
    log(f"ms/step {res['ms_per_step']:.3f}, iters/step {res['iters_per_step']:.2f}")
    log("iters per step:", " ".join(str(d["iters"]) for d in infos))
    # the step after the timed ones: the GPU's solution, and the oracle on the same history
    nxt = M + args.warmup + args.steps
    cpu, err, extra = None, None, {}
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle, the GPU's history injected)")
        hist = {"X": seq.copy_state("X"), "order": seq.copy_state("order")}
        xn = torch.empty(st.n, dtype=torch.float64, device="cuda")
        _, ginfo = seq.step(st.A(nxt), st.rhs[nxt], xn)
        cpu, err, extra = cpu_baseline(np, st, method, hist, xn.cpu().numpy(), nxt)
        extra.update(gpu_iters=int(ginfo["iters"]), gpu_relres0=float(ginfo["relres0"]), gpu_k=int(ginfo["k_eff"]))
    seq.close()
    log("instrumented run (per-kernel HIP events)")
    _, pwall, prof = run_sequence(sacc, torch, st, method, M, args.warmup, args.steps, profile=True)
    roof = roofline(prof, "lognormal3d")
    roof["instrumented_ms_per_step"] = round(1e3 * pwall / args.steps, 4)
    comps = {}
    if not args.no_comparators:
        for name, kw in (("plain_fp64", dict(precision="fp64")), ("mixed_krylov", dict(precision="mixed_krylov")),
                         ("previous", dict(guess="previous")), ("mixed_jacobi", dict(precond="jacobi"))):
            log(f"comparator on the same steps: {name}")
            # the plain FP64 method runs on the same operator (its float32 values upcast)
            stc = st.as_fp64() if name == "plain_fp64" else st
            ci, cw, cprof = run_sequence(sacc, torch, stc, method, M, args.warmup, args.steps,
                                         profile=name == "plain_fp64", **kw)
            comps[name] = summary(ci, cw, args.steps)
            if cprof:
                comps[name]["roofline"] = roofline(cprof, "lognormal3d")
            del stc
        comps["speedup_mixed_vs_plain_fp64"] = round(comps["plain_fp64"]["ms_per_step"] / res["ms_per_step"], 3)
    spmv = spmv_gbps(sacc, torch, CSRView(st.rowptr, st.col, st.vals[M].double()))
    spmv32 = spmv_gbps(sacc, torch, st.A(M))
    del st
    torch.cuda.empty_cache()
    return p, method, res, roof, comps, cpu, err, extra, dict(fp64_values=spmv, fp32_values=spmv32)


def advdiff_cmp(sacc, torch, np, warmup, steps):
    """The 512 x 512 advection-diffusion sequence (n = 262 144, FP64, M = 20, SRHT s = 80,
    GMRES(30)): projection against the paper's Baseline guess x0 = x(t_{i-1}), the
    dominant GMRES kernel's bandwidth (its working set fits the on-package cache)."""
    from gen import config

    p, method = config(1)
    M = method["M"]
    total = M + warmup + steps
    log(f"advdiff512: staging {total} steps")
    st = Staged(torch, np, p, total, fp32=False)
    out = {"workload": "advdiff2d 512x512 (n=262144, nnz=1308672), M=20, SRHT s=80, Galerkin, GMRES(30), "
                       "relres 1e-8, FP64", "steps_timed": f"{M + warmup}..{total - 1}"}
    ci, cw, prof = run_sequence(sacc, torch, st, method, M, warmup, steps, profile=True)
    out["projection"] = summary(ci, cw, steps)
    out["projection"]["roofline"] = roofline(prof, "advdiff512")
    ci, cw, _ = run_sequence(sacc, torch, st, method, M, warmup, steps, guess="previous")
    out["previous"] = summary(ci, cw, steps)
    out["spmv"] = spmv_gbps(sacc, torch, st.A(M))
    del st
    return out


def paper4_cmp(sacc, torch, np):
    """The test case of Section 4 (div(a grad f) = g, 4th-order finite differences,
    100 x 100, t0 = 2.3, 200 steps, GMRES(30) to 1e-7 without the paper's ILU): GMRES
    iterations and time per step of the projection guess against the paper's Baseline
    x0 = x(t_{i-1}), over the steps after the history has filled (the quantities of
    Fig. 1 and Fig. 5), for dt = 1e-5 and 1e-3."""
    from gen.paper4 import paper4_config

    out = {}
    for dt in (1e-5, 1e-3):
        p, m = paper4_config(dt)
        M = m["M"]
        log(f"paper4 dt={dt:g}: assembling {p.steps} steps on the host")
        st = Staged.assembled(torch, np, p, p.steps)
        rec = dict(workload=f"Section 4 test case, 100x100 (n={p.n}, nnz={st.nnz}), t0=2.3, dt={dt:g}, "
                            f"M={M}, Gaussian s={2 * M}, GMRES(30), relres 1e-7, FP64, no preconditioner",
                   steps_timed=f"{M}..{p.steps - 1}")
        for name in ("projection", "previous"):
            ci, cw, _ = run_sequence(sacc, torch, st, m, M, 0, p.steps - M, guess=name)
            rec[name] = summary(ci, cw, p.steps - M)
        # the paper's figures are for a preconditioned GMRES (ILU there); Jacobi here
        for name in ("projection", "previous"):
            ci, cw, _ = run_sequence(sacc, torch, st, m, M, 0, p.steps - M, guess=name, precond="jacobi")
            rec[name + "_jacobi"] = summary(ci, cw, p.steps - M)
        rec["iters_ratio_previous_over_projection"] = round(
            rec["previous"]["iters_per_step"] / max(rec["projection"]["iters_per_step"], 1e-9), 3)
        rec["time_ratio_previous_over_projection"] = round(
            rec["previous"]["ms_per_step"] / rec["projection"]["ms_per_step"], 3)
        if dt >= 1e-3:
            rec["table1"] = table1_sweep(sacc, torch, st, m, p.steps)
        out[f"dt={dt:g}"] = rec
        del st
    return out


# the (M, m) pairs of the paper's Table 1
TABLE1 = ((15, 6), (15, 8), (15, 10), (20, 10), (20, 15), (30, 8), (30, 12), (30, 15))


def table1_sweep(sacc, torch, st, m, steps):
    """Table 1's quantities for its (M, m) pairs on the Section 4 sequence: time and GMRES
    iterations per step of the range-finder guess (Gaussian Z, redrawn every 50 pushes;
    the paper's minimum-residual reduced problem; s = 2M) against the Baseline guess
    x0 = x(t_{i-1}), all over the same steps 30..steps-1."""
    fill = max(M for M, _ in TABLE1)
    n_t = steps - fill
    log(f"table1: {len(TABLE1)} (M, m) pairs on steps {fill}..{steps - 1}")
    bi, bw, _ = run_sequence(sacc, torch, st, m, fill, 0, n_t, guess="previous")
    base = summary(bi, bw, n_t)
    rows = []
    for M, mm in TABLE1:
        meth = dict(m, M=M, s=2 * M)
        ci, cw, _ = run_sequence(sacc, torch, st, meth, fill, 0, n_t, m=mm, projection="minres")
        r = summary(ci, cw, n_t)
        rows.append(dict(M=M, m=mm, ms_per_step=r["ms_per_step"], iters_per_step=r["iters_per_step"],
                         time_speedup=round(base["ms_per_step"] / r["ms_per_step"], 3),
                         iters_speedup=round(base["iters_per_step"] / max(r["iters_per_step"], 1e-9), 3),
                         relres_max=r["relres_max"], k_eff=r["k_eff"]))
    return dict(steps_timed=f"{fill}..{steps - 1}", baseline=dict(ms_per_step=base["ms_per_step"],
                iters_per_step=base["iters_per_step"]), rows=rows)


def learned_cmp(sacc, torch, np, n_train, n_eval, epochs=60, batch=32, n_hist=8):
    """The learned guess on the 512 x 512 sequence: the plain method runs steps
    0 .. n_train - 1 while the targets are recorded, the MLP (162 -> 256 x 3 -> 20, SiLU,
    bf16 weights, Adam) is trained on them with the library's kernels, then steps
    n_train .. n_train + n_eval - 1 run with the learned guess, against the plain method
    on the same steps."""
    from gen import config
    from gen.mlp_init import mlp_init

    p, m = config(3)
    M = m["M"]
    total = n_train + n_eval
    log(f"learned: staging {total} steps")
    st = Staged(torch, np, p, total, fp32=False)
    sizes = [n_hist * M + 2, 256, 256, 256, M]
    mlp = sacc.MLP(sizes, mlp_init(sizes, 9), max_batch=batch, lr=1e-3)
    seq = make_seq(sacc, st.n, m)
    seq.learned_attach(mlp, n_hist)
    plain = make_seq(sacc, st.n, m)
    x = torch.empty(st.n, dtype=torch.float64, device="cuda")
    xp = torch.empty_like(x)

    def step(s, i, xx):
        A, b = st.A(i), st.rhs[i]
        s.set_time(p.t(i))
        _, g = s.initial_guess(A, b, xx)
        _, inf = s.solve(A, b, xx)
        s.push(xx)
        return g, inf

    targets = []
    for i in range(n_train):
        step(seq, i, x)
        targets.append(seq.last_target())
        step(plain, i, xp)
        if (i + 1) % 500 == 0:
            log(f"learned: {i + 1} of {n_train} training steps run")
    F = np.array([np.concatenate(targets[i - n_hist:i] + [np.array([np.sin(p.t(i)), np.cos(p.t(i))])])
                  for i in range(n_hist + M, n_train)])
    T = np.array(targets[n_hist + M:n_train])
    mlp.set_scaling(F.mean(0), F.std(0) + 1e-6, T.mean(0), T.std(0) + 1e-6)
    Fd = torch.as_tensor(F.astype(np.float32)).cuda()
    Td = torch.as_tensor(T.astype(np.float32)).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for e in range(epochs):
        perm = torch.as_tensor(np.random.default_rng([10, e]).permutation(F.shape[0]), device="cuda")
        for s0 in range(0, F.shape[0] - batch + 1, batch):
            idx = perm[s0:s0 + batch]
            mlp.train_step(Fd[idx].contiguous(), Td[idx].contiguous(), loss)
        losses.append(float(loss.item()))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    out = {}
    for name, s, xx in (("learned", seq, x), ("plain", plain, xp)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, used = [], []
        for i in range(n_train, total):
            g, inf = step(s, i, xx)
            its.append(inf["iters"])
            used.append(g.get("used_learned", 0))
        torch.cuda.synchronize()
        out[name] = dict(ms_per_step=round(1e3 * (time.perf_counter() - t0) / n_eval, 4),
                         iters_per_step=float(np.mean(its)), learned_accepted=int(sum(used)))
    out.update(workload=f"advdiff2d 512x512, M={M}, GMRES(30), relres 1e-8, FP64; trained on the targets of "
                        f"steps {n_hist + M}..{n_train - 1}, evaluated on steps {n_train}..{total - 1}",
               mlp="162 -> 256 -> 256 -> 256 -> 20, SiLU, bf16 weights, Adam lr 1e-3",
               train_seconds=round(train_s, 3), loss_first=losses[0], loss_last=losses[-1])
    seq.close()
    plain.close()
    del st
    return out


def batch_cmp(sacc, torch, np, warmup, steps, max_streams=8, seed=4, nseq=64, precision=None, lo=96, hi=768,
              mode="auto", fixed_modes=("streams", "segmented")):
    """The batched workload: 64 independent 2-D sequences (sides U{96..768}, M in
    {8, 16, 24}, half advective with GMRES(30), the rest CG), float32 values with FP64
    refinement to 1e-8, stepped together by the library's batch driver on up to
    max_streams streams; the plan is tuned on the steps after the histories fill.
    Timing starts after the longest history (24) is full and `warmup` more steps."""
    from gen import batch_problems

    probs = batch_problems(seed=seed, nseq=nseq, lo=lo, hi=hi, steps=100)
    fill = max(m["M"] for _, m in probs)
    extra = 2  # steps of each fixed mode after the tuned ones
    total = fill + warmup + steps + 2 * extra
    log(f"batch: staging {total} steps of {nseq} sequences")
    sts, seqs, xs = [], [], []
    nnz_tot, n_tot = 0, 0
    for p, m in probs:
        st = Staged(torch, np, p, total, fp32=True)
        sts.append(st)
        xs.append(torch.zeros(p.n, dtype=torch.float64, device="cuda"))
        seqs.append(sacc.Sequence(p.n, m["M"], s=m["s"], sketch=m["sketch"], solver=m["solver"],
                                  restart=m["restart"], tol=m["tol"], seed=m["method_seed"],
                                  precision=precision or m["prec"], max_refine=m["max_refine"]))
        nnz_tot += st.nnz
        n_tot += p.n
    batch = sacc.Batch(seqs, max_streams=max_streams, tune_warmup=fill)
    if mode != "auto":
        batch.set_mode(mode)

    def run(i):
        return batch.step([s.A(i) for s in sts], [s.rhs[i] for s in sts], xs)

    for i in range(fill + warmup):
        run(i)
        if (i + 1) % 10 == 0:
            log(f"  batch fill / warm-up step {i + 1}/{fill + warmup}, plan {batch.plan()}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, rel, stat = 0, 0.0, []
    by_solver = {"cg": 0, "gmres": 0}
    longest = 0
    per_seq = [0] * len(probs)
    for i in range(fill + warmup, fill + warmup + steps):
        infos = run(i)
        its += sum(d["iters"] for d in infos)
        for j, d in enumerate(infos):
            by_solver[probs[j][1]["solver"]] += d["iters"]
            per_seq[j] += d["iters"]
        longest += max(d["iters"] for d in infos)
        rel = max(rel, max(d["relres"] for d in infos))
        stat += [d["status"] for d in infos]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    top = sorted(range(len(probs)), key=lambda j: -per_seq[j])[:5]
    plan = batch.plan()
    # the next steps in each fixed mode: every solve on its own stream, then all solves
    # in the segmented engine (graph replays)
    fixed = {}
    k = fill + warmup + steps
    for fm in fixed_modes:
        batch.set_mode(fm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        its_m, by, ms = 0, 0.0, 0.0
        for _ in range(extra):
            its_m += sum(d["iters"] for d in run(k))
            b_, m_ = batch.solve_stats()
            by, ms = by + b_, ms + m_
            k += 1
        torch.cuda.synchronize()
        fixed[fm] = dict(ms_per_step=round(1e3 * (time.perf_counter() - t1) / extra, 3),
                         krylov_iters_per_step=its_m / extra, steps=f"{k - extra}..{k - 1}")
        if fm == "segmented" and ms > 0:
            # the engine's solve: algorithmic bytes (CSR once and each Krylov vector
            # read or written once per phase) over its wall time, against the HBM peak
            tbs = by / (ms * 1e-3) / 1e12
            fixed[fm].update(solve_ms_per_step=round(ms / extra, 3), solve_gb_per_step=round(by / extra / 1e9, 2),
                             solve_tb_per_s=round(tbs, 3), solve_frac_of_hbm_peak=round(tbs / 8.0, 3))
    batch.close()
    for s in seqs:
        s.close()
    return dict(workload=f"{nseq} sequences, sides U{{{lo}..{hi}}} (seed {seed}), n total {n_tot}, nnz total {nnz_tot}, "
                         f"M in {{8,16,24}}, half GMRES(30) / half CG, float32 operator and Krylov vectors + FP64 "
                         f"refinement ({precision or probs[0][1]['prec']}, at most "
                         f"{probs[0][1]['max_refine']} sweeps), relres 1e-8",
                steps_timed=f"{fill + warmup}..{fill + warmup + steps - 1}", ms_per_step=round(1e3 * wall / steps, 3),
                krylov_iters_per_step=its / steps, relres_max=rel,
                iters_per_step_by_solver={k: v / steps for k, v in by_solver.items()},
                longest_sequence_iters_per_step=longest / steps,
                heaviest_sequences=[dict(n=probs[j][0].n, solver=probs[j][1]["solver"],
                                         iters_per_step=per_seq[j] / steps) for j in top],
                not_converged=int(sum(1 for s_ in stat if s_ != 0)), plan=plan, fixed_modes=fixed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--only-headline", action="store_true", help="the headline workload only (no other workloads)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run 3 plain 256 MiB device copies first (reference for HBM byte counters)")
    ap.add_argument("--batch-warmup", type=int, default=15,
                    help="batch steps after the histories fill, before timing (the plan tuner times 15 candidates)")
    ap.add_argument("--batch-steps", type=int, default=4)
    ap.add_argument("--batch-mode", choices=["auto", "streams", "segmented"], default="auto",
                    help="plan of the timed batch steps (auto: tuned)")
    ap.add_argument("--batch-max-streams", type=int, default=8)
    ap.add_argument("--batch-which", choices=["both", "large", "small"], default="both")
    ap.add_argument("--batch-no-fixed", action="store_true", help="skip the steps in each fixed mode")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--only-batch", action="store_true", help="run only the batched workload")
    ap.add_argument("--only-advdiff", action="store_true",
                    help="run only the 512 x 512 GMRES comparator (for profiling its kernels)")
    ap.add_argument("--learned-train", type=int, default=200)
    ap.add_argument("--learned-eval", type=int, default=100)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--only-learned", action="store_true",
                    help="run only the learned-predictor comparator (window set by --learned-train / --learned-eval)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent sequences would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("--steps must be >= 1 and --warmup >= 0")

    import numpy as np
    import torch

    import paper_2309_02156_amd as sacc

    if args.only_batch:
        kw = dict(max_streams=args.batch_max_streams, mode=args.batch_mode,
                  fixed_modes=() if args.batch_no_fixed else ("streams", "segmented"))
        out = {}
        if args.batch_which in ("both", "large"):
            out["batch64"] = batch_cmp(sacc, torch, np, args.batch_warmup, args.batch_steps, **kw)
        if args.batch_which in ("both", "small"):
            out["batch64_small"] = batch_cmp(sacc, torch, np, args.batch_warmup, args.batch_steps, lo=32, hi=128, **kw)
        print(json.dumps(out), flush=True)
        return
    if args.only_learned:
        print(json.dumps({"learned": learned_cmp(sacc, torch, np, args.learned_train, args.learned_eval)}), flush=True)
        return
    if args.only_advdiff:
        if args.copy_calibration:
            src = torch.empty(32 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            log("copy calibration: 3 copies of 268435456 bytes")
            del src, dst
        print(json.dumps({"advdiff512": advdiff_cmp(sacc, torch, np, args.warmup, args.steps)}), flush=True)
        return

    p, method, res, roof, comps, cpu, err, extra, spmv = headline(sacc, torch, np, args)
    M = method["M"]
    first = M + args.warmup
    others = {}
    if not args.no_comparators and not args.only_headline:
        others["advdiff512"] = advdiff_cmp(sacc, torch, np, args.warmup, args.steps)
        others["paper4"] = paper4_cmp(sacc, torch, np)
        if not args.no_learned:
            others["learned"] = learned_cmp(sacc, torch, np, args.learned_train, args.learned_eval)
        if not args.no_batch:
            others["batch64"] = batch_cmp(sacc, torch, np, args.batch_warmup, args.batch_steps)
            # many small sequences: per-sequence kernels are launch-latency bound there
            others["batch64_small"] = batch_cmp(sacc, torch, np, args.batch_warmup, args.batch_steps, lo=32, hi=128)
    comps.update(others)
    out = {
        "metric": METRIC,
        "value": res["ms_per_step"],
        "unit": "ms/timestep",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"lognormal3d 128^3 (n={p.n}, nnz=14581760, float32 values, int32 indices packed by the solve to 16-bit row offsets), "
                               f"M={M}, Gaussian s={method['s']}, Galerkin, CG in float32 with FP64 "
                               f"refinement to relres {method['tol']:g}, float32 history",
                   "history_fill_steps": M, "steps_timed": f"{first}..{first + args.steps - 1}"},
        "krylov_iters_per_step": res["iters_per_step"],
        "refinements_per_step": res["refinements_per_step"],
        "relres_max": res["relres_max"],
        "relres0_median": res["relres0_median"],
        "k_eff": res["k_eff"],
        "err_vs_fp64_oracle": err,
        "err_vs_fp64_oracle_step": extra or None,
        "spmv": spmv,
        "comparators": comps,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

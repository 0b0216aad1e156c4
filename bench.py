#!/usr/bin/env python3
"""Benchmark: ms per time step of the subspace-accelerated sequence solver on one MI355X.

Workload (one GPU): the 512 x 512 advection-diffusion sequence A(t_i) x = b(t_i)
(n = 262 144, 1 308 672 nonzeros, FP64), history M = 20, SRHT sketch s = 80,
Galerkin projection, GMRES(30) to ||b - A x|| <= 1e-8 ||b||.  A step is one pass of
the whole hot path: initial guess (sketched QR basis, SpMM + Gram, reduced solve,
x0) -> Krylov solve -> history push (copy + sketch + QRCP).  All A(t_i), b(t_i) of
the run are assembled on the host and copied to HBM before timing.

Prints ONE JSON line (see the keys at the end of main()).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ms/timestep + Krylov iters at relres 1e-8, learned/mixed vs plain; SpMV GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def assemble(problem, steps):
    import numpy as np

    vals, rhs = [], []
    for i in range(steps):
        vals.append(problem.matrix(i).val)
        rhs.append(problem.rhs(i))
    return np.stack(vals), np.stack(rhs)


def run_sequence(sacc, torch, A, vals_d, rhs_d, method, steps, warmup, guess="projection", precision="fp64",
                 profile=False):
    """Run warmup + steps; returns per-step infos of the timed steps, the wall time and
    (profile=True) the kernel timing records of the timed steps."""
    seq = sacc.Sequence(A.n, method["M"], s=method["s"], sketch=method["sketch"], solver=method["solver"],
                        restart=method["restart"], tol=method["tol"], seed=method["method_seed"], guess=guess,
                        precision=precision)
    x = torch.empty(A.n, dtype=torch.float64, device="cuda")
    infos = []

    def step(i):
        A.val.copy_(vals_d[i])
        _, inf = seq.step(A, rhs_d[i], x)
        return inf

    for i in range(warmup):
        step(i)
        if (i + 1) % 25 == 0:
            log(f"  warmup step {i + 1}/{warmup}")
    if profile:
        seq.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, warmup + steps):
        infos.append(step(i))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = seq.profile_read() if profile else None
    seq.close()
    return infos, wall, prof


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
    return nbytes / (ms * 1e-3) / 1e9, ms, nbytes


def mixed_3d(sacc, torch, np, warmup, steps):
    """ms/step of the mixed mode against plain FP64 on the 128^3 float32-valued sequence."""
    from gen import config

    p3, m3 = config(2)
    log(f"mixed_3d: assembling {warmup + steps} steps of the 128^3 sequence")
    vals32, rhs3 = [], []
    for i in range(warmup + steps):
        vals32.append(p3.matrix(i, fp32=True).val)
        rhs3.append(p3.rhs(i))
    vals32 = np.stack(vals32)
    rowptr3, col3 = p3.pattern()
    v32_d = torch.as_tensor(vals32).cuda()
    rhs_d = torch.as_tensor(np.stack(rhs3)).cuda()
    out = {"workload": f"lognormal3d 128^3 (n={p3.n}), M={m3['M']}, Gaussian s={m3['s']}, Galerkin, CG, "
                       f"relres {m3['tol']:g}, float32 operator", "steps_timed": f"{warmup}..{warmup + steps - 1}"}
    for prec in ("fp64", "mixed", "mixed_krylov"):
        log(f"mixed_3d: {prec} run")
        f32 = prec != "fp64"
        vd = v32_d if f32 else v32_d.double()
        A3 = sacc.DeviceCSR(rowptr3, col3, vals32[0] if f32 else vals32[0].astype(np.float64))
        ci, cw, _ = run_sequence(sacc, torch, A3, vd, rhs_d, m3, steps, warmup, precision=prec)
        out[prec] = dict(ms_per_step=round(1e3 * cw / steps, 4),
                         iters_per_step=float(np.mean([d["iters"] for d in ci])),
                         refinements_per_step=float(np.mean([d["refinements"] for d in ci])),
                         relres_max=float(max(d["relres"] for d in ci)))
        del A3, vd
    out["speedup_mixed_vs_fp64"] = round(out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"], 3)
    out["speedup_mixed_krylov_vs_fp64"] = round(out["fp64"]["ms_per_step"] / out["mixed_krylov"]["ms_per_step"], 3)
    return out


def learned_cmp(sacc, torch, np, n_train, n_eval, epochs=60, batch=32, n_hist=8):
    """The learned guess on the 512 x 512 sequence: the plain method runs steps
    0 .. n_train - 1 while the targets are recorded, the MLP (162 -> 256 x 3 -> 20, SiLU,
    bf16 weights, Adam) is trained on them with the library's kernels, then steps
    n_train .. n_train + n_eval - 1 run with the learned guess, against the plain method
    on the same steps."""
    from gen import config
    from gen.mlp_init import mlp_init

    p, m = config(1)
    M = m["M"]
    total = n_train + n_eval
    log(f"learned: assembling {total} steps")
    vals, rhs = assemble(p, total)
    rowptr, col = p.pattern()
    A = sacc.DeviceCSR(rowptr, col, vals[0])
    vals_d = torch.as_tensor(vals).cuda()
    rhs_d = torch.as_tensor(rhs).cuda()
    del vals, rhs
    sizes = [n_hist * M + 2, 256, 256, 256, M]
    mlp = sacc.MLP(sizes, mlp_init(sizes, 9), max_batch=batch, lr=1e-3)
    kw = dict(s=m["s"], sketch=m["sketch"], solver=m["solver"], restart=m["restart"], tol=m["tol"],
              seed=m["method_seed"])
    seq = sacc.Sequence(A.n, M, **kw)
    seq.learned_attach(mlp, n_hist)
    plain = sacc.Sequence(A.n, M, **kw)
    x = torch.empty(A.n, dtype=torch.float64, device="cuda")
    xp = torch.empty_like(x)

    def step(s, i, xx):
        A.val.copy_(vals_d[i])
        b = rhs_d[i]
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
    return out


def batch_cmp(sacc, torch, np, warmup, steps, max_streams=4, seed=4, nseq=64, precision=None):
    """The batched workload: 64 independent 2-D sequences (sides U{96..768}, M in
    {8, 16, 24}, half advective with GMRES(30), the rest CG), float32 values with FP64
    refinement to 1e-8, stepped together by the library's batch driver on up to
    max_streams streams; the plan is tuned on the steps after the histories fill.
    Matrix values of every step come from each sequence's affine value basis and the
    right-hand sides from the generator, staged in HBM before the timed steps."""
    from gen import batch_problems

    probs = batch_problems(seed=seed, nseq=nseq, steps=warmup + steps)
    total = warmup + steps
    log(f"batch: staging {total} steps of {nseq} sequences")
    seqs, pats, vals, rhs, xs = [], [], [], [], []
    nnz_tot, n_tot = 0, 0
    for p, m in probs:
        rowptr, col = p.pattern()
        Bv = torch.as_tensor(p.value_basis()).cuda()
        C = torch.as_tensor(np.stack([p.value_coefs(i) for i in range(total)])).cuda()
        vals.append((C @ Bv).float())          # total x nnz, float32 values
        del Bv, C
        rhs.append(torch.as_tensor(np.stack([p.rhs(i) for i in range(total)])).cuda())
        pats.append((torch.as_tensor(rowptr).cuda(), torch.as_tensor(col).cuda()))
        xs.append(torch.zeros(p.n, dtype=torch.float64, device="cuda"))
        seqs.append(sacc.Sequence(p.n, m["M"], s=m["s"], sketch=m["sketch"], solver=m["solver"],
                                  restart=m["restart"], tol=m["tol"], seed=m["method_seed"],
                                  precision=precision or m["prec"], max_refine=m["max_refine"]))
        nnz_tot += int(col.size)
        n_tot += p.n
    batch = sacc.Batch(seqs, max_streams=max_streams, tune_warmup=max(m["M"] for _, m in probs))

    class View:  # a CSR view on one staged step (no copy)
        def __init__(self, rp, cl, v):
            self.rowptr, self.col, self.val = rp, cl, v
            self.n, self.nnz = rp.numel() - 1, cl.numel()

        def c_struct(self):
            return sacc.DeviceCSR.c_struct(self)

    def run(i):
        As = [View(pats[j][0], pats[j][1], vals[j][i]) for j in range(nseq)]
        bs = [rhs[j][i] for j in range(nseq)]
        return batch.step(As, bs, xs)

    for i in range(warmup):
        run(i)
        if (i + 1) % 10 == 0:
            log(f"  batch warmup step {i + 1}/{warmup}, plan {batch.plan()}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, rel, st = 0, 0.0, []
    for i in range(warmup, total):
        infos = run(i)
        its += sum(d["iters"] for d in infos)
        rel = max(rel, max(d["relres"] for d in infos))
        st += [d["status"] for d in infos]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(workload=f"{nseq} sequences, sides U{{96..768}} (seed {seed}), n total {n_tot}, nnz total {nnz_tot}, "
                         f"M in {{8,16,24}}, half GMRES(30) / half CG, float32 operator and Krylov vectors + FP64 "
                         f"refinement ({precision or probs[0][1]['prec']}, at most "
                         f"{probs[0][1]['max_refine']} sweeps), relres 1e-8",
                steps_timed=f"{warmup}..{total - 1}", ms_per_step=round(1e3 * wall / steps, 3),
                krylov_iters_per_step=its / steps, relres_max=rel,
                not_converged=int(sum(1 for s_ in st if s_ != 0)), plan=batch.plan())


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when
    there is none or the kernel sources have changed since the counters were taken."""
    import hashlib
    import re

    base = kernel.split("<")[0]
    path = os.path.join(ROOT, "profiles", f"{base}_advdiff512_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if f"# HBM traffic of {kernel} " not in text:
        return None
    m_t = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    m_h = re.search(r"^kernel_source_sha256: ([0-9a-f]+)", text, re.M)
    if not m_t or not m_h:
        return None
    h = hashlib.sha256()
    for f in ("krylov.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2309_02156_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m_t.group(1)) if h.hexdigest() == m_h.group(1) else None


def cpu_baseline(problem, method, start, seconds):
    """The oracle on the host: history warm-started from sparse-LU solutions of the M
    steps before `start` (untimed), then steps start, start+1, ... timed until
    `seconds` of CPU work have been spent."""
    import numpy as np
    import scipy.sparse.linalg as spla

    from oracle.sequence import make_sequence

    seq = make_sequence(problem, method)
    for i in range(start - method["M"], start):
        A = problem.matrix(i).to_scipy().tocsc()
        seq.push(spla.splu(A).solve(problem.rhs(i)))
    times, iters = [], []
    i = start
    spent = 0.0
    while spent < seconds and i < problem.steps:
        A = problem.matrix(i).to_scipy()
        b = problem.rhs(i)
        t0 = time.perf_counter()
        _, _, info = seq.step(A, b)
        dt = time.perf_counter() - t0
        times.append(dt)
        iters.append(info["iters"])
        spent += dt
        i += 1
    try:
        from threadpoolctl import threadpool_info

        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = 1
    return dict(value=1e3 * float(np.mean(times)), unit="ms/timestep", cores=int(threads), kind="oracle",
                sample=f"steps {start}..{i - 1} of the same sequence ({len(times)} steps, "
                       f"{spent:.1f} s), history warm-started from sparse-LU solutions of steps "
                       f"{start - method['M']}..{start - 1}; mean oracle iterations {np.mean(iters):.1f}; "
                       f"host os.cpu_count()={os.cpu_count()}, BLAS threads {threads}, SciPy SpMV single-threaded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run 3 plain 256 MiB device copies first (reference for HBM byte counters)")
    ap.add_argument("--batch-warmup", type=int, default=31)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--only-batch", action="store_true", help="run only the batched workload")
    ap.add_argument("--only-mixed", action="store_true",
                    help="run only the 128^3 CG mixed-precision comparator (fp64, mixed, mixed_krylov)")
    ap.add_argument("--learned-train", type=int, default=200)
    ap.add_argument("--learned-eval", type=int, default=100)
    ap.add_argument("--mixed-warmup", type=int, default=32)
    ap.add_argument("--mixed-steps", type=int, default=8)
    ap.add_argument("--mixed-2d", action="store_true",
                    help="also run the float32-operator comparator on the 512 x 512 GMRES sequence")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent sequences would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2309_02156_amd as sacc
    from gen import config

    if args.only_batch:
        print(json.dumps({"batch64": batch_cmp(sacc, torch, np, args.batch_warmup, args.batch_steps)}), flush=True)
        return
    if args.only_mixed:
        print(json.dumps({"mixed_3d": mixed_3d(sacc, torch, np, args.mixed_warmup, args.mixed_steps)}), flush=True)
        return

    p, method = config(1)
    total = args.warmup + args.steps
    if total > p.steps:
        raise SystemExit(f"warmup + steps must be <= {p.steps}")
    log("assembling", total, "steps on the host")
    vals, rhs = assemble(p, total)
    rowptr, col = p.pattern()
    A = sacc.DeviceCSR(rowptr, col, vals[0])
    vals_d = torch.as_tensor(vals).cuda()
    rhs_d = torch.as_tensor(rhs).cuda()
    torch.cuda.synchronize()

    if args.copy_calibration:
        src = torch.empty(32 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 268435456 bytes")
        del src, dst

    log("timed run: projection")
    infos, wall, _ = run_sequence(sacc, torch, A, vals_d, rhs_d, method, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    iters = [d["iters"] for d in infos]
    relres = [d["relres"] for d in infos]
    log(f"ms/step {ms_step:.3f}, iters/step {np.mean(iters):.2f}")
    log("iters per step:", " ".join(str(i) for i in iters))

    # the same steps again with HIP events around each launch of the dominant kernels
    log("instrumented run (per-kernel HIP events)")
    _, pwall, prof = run_sequence(sacc, torch, A, vals_d, rhs_d, method, args.steps, args.warmup, profile=True)
    dom = max(prof, key=lambda r: r["ms"])
    dom_us = 1e3 * dom["ms"] / dom["launches"]
    dom_gbs = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    for r in sorted(prof, key=lambda r: -r["ms"]):
        log(f"  {r['name']}: {r['launches']} launches, {1e3 * r['ms'] / r['launches']:.2f} us avg, "
            f"{r['bytes'] / (r['ms'] * 1e-3) / 1e9:.0f} GB/s")

    comparators = {}
    if not args.no_comparators:
        for kind in ("previous",):
            log("comparator run:", kind)
            ci, cw, _ = run_sequence(sacc, torch, A, vals_d, rhs_d, method, args.steps, args.warmup, guess=kind)
            comparators[kind] = dict(ms_per_step=1e3 * cw / args.steps,
                                     iters_per_step=float(np.mean([d["iters"] for d in ci])))
    # float32 operator / Krylov vectors with FP64 history and refinement on the same
    # 512 x 512 sequence (its float32-valued operator); off by default: float32 GMRES(30)
    # contracts this operator's residual too little per capped sweep to reach 1e-8
    # within the default 10 sweeps
    if not args.no_comparators and args.mixed_2d:
        log("comparator run: mixed_krylov (512 x 512)")
        A32 = sacc.DeviceCSR(rowptr, col, vals[0].astype(np.float32))
        v32 = vals_d.float()
        ci, cw, _ = run_sequence(sacc, torch, A32, v32, rhs_d, method, args.steps, args.warmup,
                                 precision="mixed_krylov")
        comparators["mixed_krylov_2d"] = dict(ms_per_step=round(1e3 * cw / args.steps, 4),
                                              iters_per_step=float(np.mean([d["iters"] for d in ci])),
                                              refinements_per_step=float(np.mean([d["refinements"] for d in ci])),
                                              relres_max=float(max(d["relres"] for d in ci)),
                                              note="float32 operator values; relres against it")
        del A32, v32
    if not args.no_comparators:
        # mixed precision where it is meant to run: the 128^3 float32-valued 3-D sequence
        # (CG, M = 30, Gaussian s = 60), against the plain FP64 method on the same
        # operator (the float32 values upcast), both to relres 1e-8
        comparators["mixed_3d"] = mixed_3d(sacc, torch, np, args.mixed_warmup, args.mixed_steps)
        # learned coefficient predictor on the 512 x 512 sequence
        comparators["learned"] = learned_cmp(sacc, torch, np, args.learned_train, args.learned_eval)
        # 64 independent sequences stepped together
        comparators["batch64"] = batch_cmp(sacc, torch, np, args.batch_warmup, args.batch_steps)


    gbs, spmv_ms, spmv_bytes = spmv_gbps(sacc, torch, A)
    log(f"SpMV {gbs:.0f} GB/s ({spmv_ms * 1e3:.1f} us)")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(p, method, args.warmup, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(ms_step, 4),
        "unit": "ms/timestep",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "advdiff2d 512x512 (n=262144, nnz=1308672), M=20, SRHT s=80, "
                               "Galerkin, GMRES(30), relres 1e-8, FP64",
                   "steps_timed": f"{args.warmup}..{args.warmup + args.steps - 1}"},
        "krylov_iters_per_step": round(float(np.mean(iters)), 3),
        "relres_max": float(max(relres)),
        "spmv_gbps": round(gbs, 1),
        "comparators": comparators,
        "roofline": {"bound": "hbm", "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dom_gbs / HBM_PEAK_GBS, 4), "traffic": committed_traffic(dom["name"]),
                     "kernel": dom["name"], "bytes_per_launch": round(dom["bytes"] / dom["launches"]),
                     "avg_us": round(dom_us, 3), "launches": dom["launches"],
                     "instrumented_ms_per_step": round(1e3 * pwall / args.steps, 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

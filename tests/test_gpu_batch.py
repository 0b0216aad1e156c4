"""GPU tests of the batched execution of independent sequences (sa_batch_*).

The batch runs the same kernels as one sequence at a time, only on several streams at
once, so its solutions and iteration counts must equal those of the sequences stepped
one by one (bit for bit); every solve meets the FP64 tolerance against its float32
operator; the plan autotuner ends with a tuned plan.
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


def test_batch_equals_sequential_and_tunes(sacc):
    import torch

    probs = batch_problems(seed=4, nseq=6, lo=16, hi=40, steps=40)
    steps = 24
    print_case("batch", [(p.N, m["M"], m["solver"]) for p, m in probs], steps)
    seqs_b = [_seq(sacc, p, m) for p, m in probs]
    seqs_s = [_seq(sacc, p, m) for p, m in probs]
    batch = sacc.Batch(seqs_b, max_streams=4, tune_warmup=8)
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
    assert plan["tuned"] and 1 <= plan["streams"] <= 4

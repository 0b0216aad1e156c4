"""GPU parity on the Section 4 test case (gen/paper4.py: 4th-order finite differences of
div(a grad f) = g, 100 x 100, t0 = 2.3, GMRES(30) to 1e-7), against the oracle with the
same injected history: equal ranks, the guess element by element within 1e-11 of its
largest entry (the oracle's own guess moves by at most 9.3e-14 of it under a 1e-16
relative perturbation of X and S X, measured on both time steps), iteration counts within
1 from the same start, and the tolerance met."""

import numpy as np
import pytest

from gen.paper4 import paper4_config
from oracle.sequence import make_sequence
from tests.gpu_helpers import dev, host, method_kwargs, print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sacc():
    import torch

    assert torch.cuda.is_available()
    import paper_2309_02156_amd as pkg

    return pkg


@pytest.mark.parametrize("dt", [1e-5, 1e-3])
def test_paper4_stepwise(sacc, dt):
    p, m = paper4_config(dt)
    steps = m["M"] + 4
    print_case("paper4 stepwise", dt, p.n, steps)
    ref = make_sequence(p, m)
    sols = []
    for i in range(steps):
        x, _, _ = ref.step(p.matrix(i).to_scipy(), p.rhs(i))
        sols.append(x)
    oseq = make_sequence(p, m)
    gseq = sacc.Sequence(p.n, **method_kwargs(m))
    rows = []
    for i in range(steps):
        A = p.matrix(i)
        As = A.to_scipy()
        b = p.rhs(i)
        g = oseq.initial_guess(As, b)
        Ad = sacc.DeviceCSR.from_csr(A)
        x0d, gi = gseq.initial_guess(Ad, dev(b))
        x0 = host(x0d)
        assert (gi["k_sketch"], gi["k_eff"]) == (g.k, g.k2), (i, gi, g.k, g.k2)
        ew = 0.0
        if i > 0:
            ew = float(np.max(np.abs(x0 - g.x0)) / np.max(np.abs(g.x0)))
            assert ew <= 1e-11, (i, ew)
        xo, oi = oseq.solve(As, b, g.x0)
        xd, si = gseq.solve(Ad, dev(b), dev(g.x0))
        assert abs(si["iters"] - oi["iters"]) <= 1, (i, si["iters"], oi["iters"])
        rel = np.linalg.norm(b - As @ host(xd)) / np.linalg.norm(b)
        assert rel <= m["tol"] * (1 + 1e-6) and oi["relres"] <= m["tol"]
        rows.append((i, si["iters"], oi["iters"], gi["k_eff"], ew))
        oseq.push(sols[i])
        gseq.push(dev(sols[i]))
    print_case("(step, iters gpu, iters oracle, k, max |dx0| / max |x0|)", rows)

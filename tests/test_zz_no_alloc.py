"""GPU test of the allocation-free solve (sa_solve_static) against sa_solve.

Both run the same kernels in the same order over the same partial-sum layout, so the
solutions must agree bit for bit and the iteration counts and residuals exactly.  Two
calls in a row share the library's fixed device array; the second, on a smaller
system, must not see anything of the first (the control block is reset per call)."""

import numpy as np
import pytest

from gen import config
from tests.gpu_helpers import dev, host, print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sacc():
    import torch

    assert torch.cuda.is_available()
    import paper_2309_02156_amd as pkg

    return pkg


def _case(k, N, i):
    p, m = config(k, N)
    return p.matrix(i), p.rhs(i), m


@pytest.mark.parametrize("solver,k,sizes", [("cg", 0, (96, 40)), ("gmres", 1, (80, 24))])
def test_static_solve_equals_sa_solve(sacc, solver, k, sizes):
    from paper_2309_02156_amd.sequence import solve_static

    for N in sizes:
        print_case("static solve", solver, N)
        A, b, m = _case(k, N, 5)
        Ad = sacc.DeviceCSR.from_csr(A)
        x0 = np.zeros(A.n)
        tol = 1e-10
        seq = sacc.Sequence(A.n, 1, s=2, solver=solver, restart=30, tol=tol)
        xs, si = seq.solve(Ad, dev(b), dev(x0))
        xz, zi = solve_static(Ad, dev(b), dev(x0), solver=solver, restart=30, tol=tol)
        print_case("iters sa_solve / static", si["iters"], zi["iters"], zi["relres"])
        assert zi["rc"] == si["rc"] == 0
        assert zi["iters"] == si["iters"] and zi["restarts"] == si["restarts"]
        assert zi["relres"] == si["relres"] and zi["relres0"] == si["relres0"]
        assert np.array_equal(host(xz), host(xs))
        As = A.to_scipy()
        assert np.linalg.norm(b - As @ host(xz)) <= tol * np.linalg.norm(b) * (1 + 1e-6)
        seq.close()


def test_static_solve_zero_rhs_and_maxit(sacc):
    from paper_2309_02156_amd.sequence import solve_static

    A, b, _ = _case(0, 32, 3)
    Ad = sacc.DeviceCSR.from_csr(A)
    x, info = solve_static(Ad, dev(np.zeros(A.n)), dev(np.ones(A.n)), tol=1e-10)
    assert info["rc"] == 0 and info["iters"] == 0 and np.all(host(x) == 0)
    x, info = solve_static(Ad, dev(b), dev(np.zeros(A.n)), tol=1e-14, maxit=3)
    assert info["rc"] == 1 and info["iters"] == 3

"""Pins of the seeded problem generators: brute-force assembly and closed forms."""

import math

import numpy as np
import pytest

from gen import batch_problems, config
from gen.problems import SeqProblem


def _dense_bruteforce_2d(p: SeqProblem, t: float) -> np.ndarray:
    """Loop-by-loop assembly straight from the PDE definition (independent of the vectorised code)."""
    N, h = p.N, p.h
    n = N * N
    A = np.zeros((n, n))
    vx, vy = p.velocity(t)
    for iy in range(N):
        for ix in range(N):
            P = ix + N * iy
            x, y = (ix + 1) * h, (iy + 1) * h
            A[P, P] += p.ccoef(t)
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                kf = p.kcoef(x + 0.5 * dx * h, y + 0.5 * dy * h, None, t)
                A[P, P] += kf / h**2
                jx, jy = ix + dx, iy + dy
                if 0 <= jx < N and 0 <= jy < N:
                    A[P, jx + N * jy] -= kf / h**2
            for v, (dxb, dyb) in ((vx, (1, 0)), (vy, (0, 1))):
                # v * d/dx upwind: v >= 0 backward difference, v < 0 forward
                if v == 0.0:
                    continue
                if v >= 0:
                    A[P, P] += v / h
                    jx, jy = ix - dxb, iy - dyb
                    if 0 <= jx < N and 0 <= jy < N:
                        A[P, jx + N * jy] -= v / h
                else:
                    A[P, P] -= v / h
                    jx, jy = ix + dxb, iy + dyb
                    if 0 <= jx < N and 0 <= jy < N:
                        A[P, jx + N * jy] += v / h
    return A


@pytest.mark.parametrize("k,step", [(0, 0), (0, 7), (1, 3), (1, 100)])
def test_dense_reassembly(k, step):
    p, _ = config(k, N=6)
    A = p.matrix(step)
    ref = _dense_bruteforce_2d(p, p.t(step))
    assert np.allclose(A.to_dense(), ref, rtol=1e-14, atol=1e-10)
    # columns ascend within every row
    for i in range(A.n):
        c = A.col[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)


class _ConstK(SeqProblem):
    def kcoef(self, x, y, z, t):
        return np.ones_like(x)

    def ccoef(self, t):
        return 1.7


def test_constant_coefficient_eigenvectors():
    N = 12
    p = _ConstK("const", 2, N, dt=0.1, steps=1, seed=0)
    A = p.matrix(0).to_scipy()
    h = p.h
    g = np.arange(1, N + 1) * h
    X, Y = np.meshgrid(g, g, indexing="xy")
    for (pp, qq) in [(1, 1), (2, 5), (N, N)]:
        v = (np.sin(pp * math.pi * X) * np.sin(qq * math.pi * Y)).reshape(-1)
        lam = 1.7 + 4 / h**2 * (math.sin(pp * math.pi * h / 2) ** 2 + math.sin(qq * math.pi * h / 2) ** 2)
        assert np.allclose(A @ v, lam * v, rtol=1e-12, atol=1e-9 * lam)


def test_sizes_match_workloads():
    p0, _ = config(0)
    p1, _ = config(1)
    assert (p0.n, len(p0.pattern()[1])) == (4096, 20224)
    assert (p1.n, len(p1.pattern()[1])) == (262144, 1308672)
    p2, _ = config(2, N=16)
    assert len(p2.pattern()[1]) == 7 * 16**3 - 6 * 16**2


def test_3d_symmetric_fp32_and_positive():
    p, m = config(2, N=8)
    A = p.matrix(5)
    assert A.val.dtype == np.float32 and m["prec"] == "mixed"
    D = p.matrix(5, fp32=False).to_dense()
    assert np.array_equal(D, D.T)
    assert np.linalg.eigvalsh(D).min() > 0
    assert np.array_equal(A.val, p.matrix(5, fp32=False).val.astype(np.float32))


def test_advective_operator_has_positive_definite_symmetric_part():
    p, _ = config(1, N=10)
    D = p.matrix(17).to_dense()
    assert not np.allclose(D, D.T)
    assert np.linalg.eigvalsh(0.5 * (D + D.T)).min() > 0


def test_rhs_bump_and_seeding():
    p, _ = config(0, N=64)
    b = p.rhs(0)
    # the bump centre starts at (0.75, 0.5): maximum near that node
    i = int(np.argmax(b))
    N, h = p.N, p.h
    assert abs((i % N + 1) * h - 0.75) < 2 * h and abs((i // N + 1) * h - 0.5) < 2 * h
    a, _ = config(1, N=32)
    c, _ = config(1, N=32)
    assert np.array_equal(a.rhs(9), c.rhs(9)) and a.bump_phase == c.bump_phase


def test_batch_workload_shape():
    seqs = batch_problems()
    assert len(seqs) == 64
    sides = np.array([p.N for p, _ in seqs])
    assert sides.min() >= 96 and sides.max() <= 768
    assert sum(m["solver"] == "gmres" for _, m in seqs) == 32
    assert {m["M"] for _, m in seqs} <= {8, 16, 24}
    # deterministic
    again = batch_problems()
    assert [p.N for p, _ in again] == sides.tolist()


def test_affine_value_basis_reproduces_assembly():
    """The 2-D matrices are affine in a few time-dependent scalars; the basis form used
    to stage long runs on the device equals the direct assembly to rounding."""
    from gen import batch_problems

    cases = [config(0, N=20)[0], config(1, N=32)[0], config(2, N=12)[0]] + \
        [p for p, _ in batch_problems(nseq=3, lo=16, hi=40)]
    for p in cases:
        B = p.value_basis()
        for i in (0, 7, 33):
            ref = p.matrix(i, fp32=False).val
            assert np.max(np.abs(p.value_coefs(i) @ B - ref)) <= 1e-14 * np.max(np.abs(ref))

"""The oracle against the paper's analysis (Section 3) and the range-finder bound.

* Theorem 2 on an analytic family where kappa_rho is computable: A(t) = diag(a_j + t)
  with a_j > 1, b constant, so x_j(t) = b_j / (a_j + t) has its poles at t = -a_j.
* Theorem 1 on the same family.
* The history-size trend: on nested windows the minimum-residual guess (and, for SPD
  A, the Galerkin guess in the energy norm) can only improve as M grows.
* eq. (errorrandsvd) averaged over range-finder seeds.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gen import config
from oracle import basis as bs
from oracle import theory as th
from oracle.sketch import Sketch


def _analytic_family(n=40, seed=0, far=False):
    """Poles at -a_j: near the interval (loose bound) or far from it (tight bound)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(8.0, 30.0, n) if far else rng.uniform(1.6, 3.0, n)
    b = rng.uniform(0.5, 1.5, n)
    xfun = lambda t: b / (a + t)
    return a, b, xfun


def _uniform_history(M):
    ts = np.linspace(-1.0, 1.0, M)
    dt = 2.0 / (M - 1)
    return ts, 1.0 + dt


@pytest.mark.parametrize("M", [5, 10, 17, 26, 37])
@pytest.mark.parametrize("projection", ["minres", "galerkin"])
@pytest.mark.parametrize("far", [False, True])
def test_theorem2_bound(M, projection, far):
    a, b, xfun = _analytic_family(far=far)
    ts, t_next = _uniform_history(M)
    X = np.stack([xfun(t) for t in ts], 1)
    A = np.diag(a + t_next)
    # rho just inside the nearest pole's ellipse: (rho + 1/rho)/2 < min(a)
    amin = a.min()
    rho_max = amin + math.sqrt(amin * amin - 1.0)
    rho = 0.97 * rho_max
    kappa = th.bernstein_kappa(xfun, rho)
    S = Sketch("gaussian", len(a), 2 * M, 1)
    g = bs.initial_guess(A, b, X, S.apply(X), projection=projection, spd=True,
                         tau_s=1e-14, tau_c=1e-14)
    res = np.linalg.norm(A @ g.x0 - b)
    Rmax = int(math.floor(0.5 * math.sqrt(M - 1)))
    for R in range(0, Rmax + 1):
        bound = th.thm2_residual_bound(np.linalg.norm(A, 2), kappa, rho, M, R, t_next)
        assert res <= bound, (M, R, res, bound)
    if far and M == 37:
        # here the bound is below ||b||: x0 = 0 (or any guess that ignores X) fails it
        assert th.thm2_residual_bound(np.linalg.norm(A, 2), kappa, rho, M, Rmax, t_next) \
            < np.linalg.norm(b)


def test_theorem1_singular_value_decay():
    a, b, xfun = _analytic_family(60, seed=2)
    for M in (8, 20, 40):
        ts, _ = _uniform_history(M)
        X = np.stack([xfun(t) for t in ts], 1)
        sv = np.linalg.svd(X, compute_uv=False)
        amin = a.min()
        rho = 0.97 * (amin + math.sqrt(amin * amin - 1.0))
        kappa = th.bernstein_kappa(xfun, rho)
        for k, s in enumerate(sv, start=1):
            assert s <= th.thm1_sigma_bound(k, rho, kappa, M) * (1 + 1e-12)


def test_history_trend_nested_windows():
    """Exact solutions of the SPD workload on a small grid; M = 1..10 nested windows."""
    p, _ = config(0, N=16)
    steps = 12
    xs = []
    for i in range(steps):
        A = p.matrix(i).to_scipy().tocsc()
        xs.append(spla.spsolve(A, p.rhs(i)))
    A = p.matrix(steps).to_scipy()
    b = p.rhs(steps)
    xstar = spla.spsolve(A.tocsc(), b)
    prev_res, prev_err = np.inf, np.inf
    res_list = []
    for M in range(1, 11):
        X = np.stack(xs[steps - M:], 1)
        SX = Sketch("gaussian", p.n, 2 * M, 0).apply(X)
        gm = bs.initial_guess(A, b, X, SX, projection="minres", tau_s=1e-15, tau_c=1e-15)
        gg = bs.initial_guess(A, b, X, SX, projection="galerkin", tau_s=1e-15, tau_c=1e-15)
        res = np.linalg.norm(b - A @ gm.x0) / np.linalg.norm(b)
        e = xstar - gg.x0
        err = math.sqrt(e @ (A @ e))
        res_list.append(res)
        # nested spans: non-increasing up to the round-off floor
        floor = 1e-13
        assert res <= prev_res * (1 + 1e-6) + floor
        assert err <= prev_err * (1 + 1e-6) + floor * np.linalg.norm(xstar)
        prev_res, prev_err = res, err
    # and the improvement is substantial, as the analysis predicts
    assert res_list[-1] < 1e-4 * res_list[0]


def test_halko_expected_error_bound():
    rng = np.random.default_rng(3)
    n, M = 500, 20
    U, _ = np.linalg.qr(rng.standard_normal((n, M)))
    V, _ = np.linalg.qr(rng.standard_normal((M, M)))
    sv = 0.6 ** np.arange(M)
    X = (U * sv) @ V.T
    for r, p in [(3, 2), (5, 3), (8, 4)]:
        m = r + p
        errs = []
        for seed in range(50):
            Z = bs.range_finder_z(M, m, seed, 0)
            Q, _ = np.linalg.qr(X @ Z)
            errs.append(np.linalg.norm(X - Q @ (Q.T @ X), "fro"))
        assert np.mean(errs) <= th.halko_bound(sv, r, p)

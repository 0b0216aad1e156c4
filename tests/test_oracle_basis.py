"""Pins of the oracle's basis and reduced problem (Alg. 1 (basis and reduced problem), Algs. 2-3).

Each test checks the oracle against something other than itself: the plain
definitions computed by dense SVD / least squares, closed forms (M = 1, polynomial
histories), optimality invariants of the Galerkin and minimum-residual problems,
eq. (optpod), and the equivalence claimed for the progressive update of Alg. 3.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import basis as bs
from oracle.sketch import Sketch


def _spd(n, rng, cond=1e3):
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (U * np.geomspace(1.0, cond, n)) @ U.T


def _nonsym(n, rng):
    return _spd(n, rng, 1e2) + 0.3 * rng.standard_normal((n, n)) * 10.0 / np.sqrt(n)


def _guess(A, b, X, seed=0, kind="gaussian", s=None, **kw):
    n, M = X.shape
    S = Sketch(kind, n, s or 2 * M, seed)
    return bs.initial_guess(A, b, X, S.apply(X), **kw)


@pytest.mark.parametrize("spd", [True, False])
def test_galerkin_equals_plain_definition(spd):
    rng = np.random.default_rng(0)
    n, M = 300, 8
    A = _spd(n, rng) if spd else _nonsym(n, rng)
    X = rng.standard_normal((n, M))
    b = rng.standard_normal(n)
    g = _guess(A, b, X, spd=spd)
    ref = bs.galerkin_plain(A, b, X)
    assert g.k == M and g.k2 == M
    assert np.linalg.norm(g.x0 - ref) <= 1e-12 * np.linalg.norm(ref)
    # and the history-coordinate form reproduces x0
    assert np.linalg.norm(X @ g.cX - g.x0) <= 1e-12 * np.linalg.norm(ref)


def test_minres_equals_least_squares():
    rng = np.random.default_rng(1)
    n, M = 300, 8
    A = _nonsym(n, rng)
    X = rng.standard_normal((n, M))
    b = rng.standard_normal(n)
    g = _guess(A, b, X, projection="minres", spd=False)
    ref = bs.minres_plain(A, b, X)
    assert np.linalg.norm(g.x0 - ref) <= 1e-11 * np.linalg.norm(ref)


def test_basis_invariance_over_sketch_seeds():
    rng = np.random.default_rng(2)
    n, M = 512, 10
    A = _spd(n, rng)
    X = rng.standard_normal((n, M)) @ np.triu(rng.standard_normal((M, M)) + 3 * np.eye(M))
    b = rng.standard_normal(n)
    x0s = [_guess(A, b, X, seed=s).x0 for s in range(10)]
    x0s += [_guess(A, b, X, seed=s, kind="srht", s=4 * M).x0 for s in range(3)]
    for x in x0s[1:]:
        assert np.linalg.norm(x - x0s[0]) <= 1e-11 * np.linalg.norm(x0s[0])


def _smooth_history(n, M, dt=0.01, t0=0.3):
    """Columns of an analytic curve x(t) sampled at M uniform steps: numerically rank-deficient."""
    rng = np.random.default_rng(5)
    V = rng.standard_normal((n, 6))
    ts = t0 + dt * np.arange(M)
    F = np.stack([np.sin(ts), np.cos(2 * ts), np.exp(-ts), ts**2, 1.0 / (2 + ts), np.sinh(ts)])
    return V @ F


def test_sketched_qr_orthonormal_on_ill_conditioned_history():
    n, M = 2000, 12
    X = _smooth_history(n, M)
    assert np.linalg.cond(X) > 1e10
    S = Sketch("gaussian", n, 2 * M, 3)
    B = bs.sketched_basis(X, S.apply(X))
    Q = B.Q()
    k2 = Q.shape[1]
    assert 1 <= k2 <= 6
    assert np.linalg.norm(Q.T @ Q - np.eye(k2), 2) <= 10 * k2 * np.finfo(float).eps
    # the kept basis captures the history up to the truncation level
    P = X - Q @ (Q.T @ X)
    assert np.linalg.norm(P, 2) <= 1e-8 * np.linalg.norm(X, 2)


def test_galerkin_orthogonality_and_energy_optimality():
    rng = np.random.default_rng(6)
    n, M = 500, 9
    A = _spd(n, rng, 1e4)
    X = rng.standard_normal((n, M))
    xs = np.linalg.solve(A, rng.standard_normal(n))
    b = A @ xs
    g = _guess(A, b, X, seed=1)
    B = bs.sketched_basis(X, Sketch("gaussian", n, 2 * M, 1).apply(X))
    Q = B.Q()
    r = b - A @ g.x0
    assert np.linalg.norm(Q.T @ r) <= 1e-12 * np.linalg.norm(A, 2) * np.linalg.norm(g.x0)
    e0 = xs - g.x0
    en0 = e0 @ A @ e0
    for _ in range(100):
        s_ = Q @ rng.standard_normal(Q.shape[1]) * np.linalg.norm(g.x0)
        e = xs - s_
        assert en0 <= e @ A @ e * (1 + 1e-12)


def test_minres_residual_optimality():
    rng = np.random.default_rng(7)
    n, M = 400, 7
    A = _nonsym(n, rng)
    X = rng.standard_normal((n, M))
    b = rng.standard_normal(n)
    g = _guess(A, b, X, projection="minres", spd=False)
    r0 = np.linalg.norm(b - A @ g.x0)
    W = A @ X
    assert np.linalg.norm(W.T @ (b - A @ g.x0)) <= 1e-10 * np.linalg.norm(W) * np.linalg.norm(b)
    for _ in range(100):
        s_ = X @ rng.standard_normal(M)
        assert r0 <= np.linalg.norm(b - A @ s_) * (1 + 1e-12)


def test_m1_closed_forms():
    rng = np.random.default_rng(8)
    n = 200
    A = _nonsym(n, rng)
    u = rng.standard_normal(n)
    b = rng.standard_normal(n)
    X = u[:, None]
    g = _guess(A, b, X, spd=False)
    assert np.allclose(g.x0, u * (u @ b) / (u @ A @ u), rtol=1e-12, atol=0)
    gm = _guess(A, b, X, projection="minres", spd=False)
    Au = A @ u
    assert np.allclose(gm.x0, u * (Au @ b) / (Au @ Au), rtol=1e-12, atol=0)


def test_polynomial_history_is_exact():
    """Fixed A, b(t) polynomial of degree d < M: x(t) lies in span X, x0 is the solution."""
    rng = np.random.default_rng(9)
    n, M, d = 300, 6, 3
    A = _spd(n, rng, 1e2)
    V = rng.standard_normal((n, d + 1))
    bt = lambda t: V @ (t ** np.arange(d + 1))
    ts = 0.1 * np.arange(M + 1)
    X = np.stack([np.linalg.solve(A, bt(t)) for t in ts[:M]], 1)
    b = bt(ts[M])
    g = _guess(A, b, X)
    assert np.linalg.norm(b - A @ g.x0) <= 1e-12 * np.linalg.norm(b)


def test_rank_deficient_and_empty_histories():
    rng = np.random.default_rng(10)
    n = 100
    A = _spd(n, rng)
    b = rng.standard_normal(n)
    u = rng.standard_normal(n)
    X = np.stack([u, 2 * u, u, -u], 1)
    g = _guess(A, b, X)
    assert g.k == 1 and g.k2 == 1
    assert np.allclose(g.x0, u * (u @ b) / (u @ A @ u), rtol=1e-10)
    g0 = _guess(A, b, np.zeros((n, 3)))
    assert g0.k == 0 and np.all(g0.x0 == 0)
    ge = bs.initial_guess(A, b, np.zeros((n, 0)), np.zeros((4, 0)))
    assert ge.k == 0 and np.all(ge.x0 == 0)


def test_nonfinite_history_falls_back_to_previous():
    rng = np.random.default_rng(11)
    n = 50
    A = _spd(n, rng)
    b = rng.standard_normal(n)
    X = rng.standard_normal((n, 3))
    X[4, 0] = np.nan
    g = bs.initial_guess(A, b, X, np.full((6, 3), np.nan))
    assert g.used_fallback and np.array_equal(g.x0, X[:, -1])
    X[7, -1] = np.inf
    g = bs.initial_guess(A, b, X, np.full((6, 3), np.nan))
    assert g.used_fallback and np.all(g.x0 == 0)


def test_qr_pivoted_properties():
    rng = np.random.default_rng(12)
    Y = rng.standard_normal((30, 12)) * np.geomspace(1, 1e-6, 12)
    Q, R, perm = bs.qr_pivoted(Y)
    assert np.allclose(Y[:, perm], Q @ R, atol=1e-14 * np.abs(Y).max())
    d = np.abs(np.diag(R))
    assert np.all(np.diag(R) >= 0) and np.all(d[:-1] >= d[1:] * (1 - 1e-12))
    assert bs.numerical_rank_qr(R, 0.0) == 12
    assert bs.numerical_rank_qr(np.zeros((3, 3)), 1e-12) == 0


def test_pivoted_cholesky_against_library():
    rng = np.random.default_rng(13)
    F = rng.standard_normal((10, 6))
    G = F @ F.T                                     # rank 6
    R, perm, k = bs.pivoted_cholesky(G, 1e-12)
    assert k == 6
    Gp = G[np.ix_(perm[:k], perm[:k])]
    assert np.allclose(R.T @ R, Gp, rtol=1e-12, atol=1e-12 * np.abs(G).max())
    # full-rank SPD: same factor as LAPACK's Cholesky of the permuted matrix
    G2 = _spd(8, rng, 10.0)
    R2, perm2, k2 = bs.pivoted_cholesky(G2, 1e-12)
    assert k2 == 8
    L = sla.cholesky(G2[np.ix_(perm2, perm2)], lower=False)
    assert np.allclose(R2, L, rtol=1e-12, atol=1e-13)
    # the pivot is the largest remaining diagonal entry
    assert perm2[0] == int(np.argmax(np.diag(G2)))


def test_pod_optimality_identity():
    """eq. (optpod): ||(I - Q Q^T) X||_F^2 equals the tail sum of squared singular values."""
    rng = np.random.default_rng(14)
    X = rng.standard_normal((200, 12)) * np.geomspace(1, 1e-3, 12)
    sv = np.linalg.svd(X, compute_uv=False)
    for m in (1, 4, 8):
        Q = bs.pod_basis(X, m)
        err = np.linalg.norm(X - Q @ (Q.T @ X), "fro") ** 2
        assert np.isclose(err, np.sum(sv[m:] ** 2), rtol=1e-10)
        # and no other orthonormal basis of the same size does better
        Qr, _ = np.linalg.qr(rng.standard_normal((200, m)))
        assert np.linalg.norm(X - Qr @ (Qr.T @ X), "fro") ** 2 >= err


def test_progressive_update_matches_scratch():
    """Alg. 3 (rank-one updates of Omega) keep Omega = X Z exactly in exact arithmetic (Section 2.2)."""
    rng = np.random.default_rng(15)
    n, M, m = 300, 8, 4
    ps = bs.ProgressiveSketch(n, M, m, seed=3, refresh=50)
    path = np.cumsum(rng.standard_normal((60, n)), 0)
    for i, x in enumerate(path):
        ps.push(x)
        if len(ps.cols) == M:
            ref = ps.X() @ ps.Z
            assert np.linalg.norm(ps.Omega - ref) <= 1e-11 * np.linalg.norm(ref)
    # the refresh happened: the epoch advanced beyond the initial fills
    assert ps.epoch > M


def test_range_finder_z_rows_shift_consistently():
    Z = bs.range_finder_z(10, 5, seed=1, epoch=2)
    Z2 = bs.range_finder_z(4, 5, seed=1, epoch=2, row0=6)
    assert np.array_equal(Z[6:], Z2)


def test_sequence_z_matches_alg3_progressive():
    """The sequence's m < M mode uses, at every step, the Z that Alg. 3 carries (the
    progressive sketch's): rows travel with their columns, a new epoch every 50 pushes.
    Its basis therefore spans the progressive Omega's range (Section 2.2: the updates
    equal the from-scratch sketch in exact arithmetic)."""
    from oracle.sequence import Sequence

    rng = np.random.default_rng(16)
    n, M, m = 200, 6, 3
    seq = Sequence(n, M, "gaussian", 12, seed=5, m=m, refresh=7)
    ps = bs.ProgressiveSketch(n, M, m, seed=5, refresh=7)
    path = np.cumsum(rng.standard_normal((30, n)), 0)
    for x in path:
        seq.push(x)
        ps.push(x)
        Zs = bs.range_finder_rows(seq.zrows.rows, m, 5, seq.zrows.epoch)
        assert seq.zrows.epoch == ps.epoch
        assert np.array_equal(Zs, ps.Z)
        X, _ = seq.history()
        assert np.linalg.norm(X @ Zs - ps.Omega) <= 1e-10 * np.linalg.norm(ps.Omega)


def test_pod_from_gram_equals_svd_definition():
    """Alg. 2 through X^T X: the basis X T1 spans the m leading left singular vectors of
    X (the SVD definition) when the singular values are separated, is orthonormal, and
    the guess built on it equals the Galerkin projection on span(U_m)."""
    rng = np.random.default_rng(31)
    n, M, m = 400, 10, 4
    U0, _ = np.linalg.qr(rng.standard_normal((n, M)))
    V0, _ = np.linalg.qr(rng.standard_normal((M, M)))
    sv = np.geomspace(1.0, 1e-4, M)
    X = U0 @ np.diag(sv) @ V0.T
    T1, k = bs.pod_gram_factor(X, m)
    assert k == m
    Q1 = X @ T1
    assert np.linalg.norm(Q1.T @ Q1 - np.eye(m)) <= 1e-10
    Um = bs.pod_basis(X, m)
    # principal angles between the two subspaces
    cosines = np.linalg.svd(Um.T @ Q1, compute_uv=False)
    assert np.all(cosines >= 1 - 1e-10)
    # the guess on this basis is the Galerkin projection on span(U_m)
    main = 4.0 + rng.uniform(0, 1, n)
    A = np.diag(main) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    b = rng.standard_normal(n)
    g = bs.initial_guess(A, b, X, np.zeros((2 * M, M)), pod_m=m, spd=True)
    H = Um.T @ A @ Um
    ref = Um @ np.linalg.solve(H, Um.T @ b)
    assert g.k == m and np.linalg.norm(g.x0 - ref) <= 1e-9 * np.linalg.norm(ref)
    # singular values below 1e-7 of the largest are not resolved through the Gram: dropped
    X2 = U0 @ np.diag(np.r_[1.0, 0.5, 1e-9, 1e-10, np.zeros(M - 4)]) @ V0.T
    _, k2 = bs.pod_gram_factor(X2, m)
    assert k2 == 2

"""Pins of the oracle's coefficient-predictor MLP (forward, backward, Adam, bf16).

Independent checks: central finite differences of the FP64 loss, torch autograd and
torch.optim.Adam on the CPU, and torch's float32 -> bfloat16 conversion.
"""

import numpy as np
import pytest
import torch

from gen.mlp_init import mlp_init
from oracle import mlp as om

SIZES = [12, 16, 16, 5]


def _data(B=7, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, SIZES[0])), rng.standard_normal((B, SIZES[-1]))


def test_bf16_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-6, 6, 2000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3.0 * 2.0 ** -8, -2.5, 0.0, 65504.0, 1e-40]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(om.bf16(x), ref)
    assert om.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0       # tie to even (down)
    assert om.bf16(np.array([1.0 + 3.0 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6  # tie to even (up)


def test_gradients_match_finite_differences():
    X, T = _data()
    model = om.MLP(mlp_init(SIZES, 3), rounding=False)
    loss, grads = model.loss_and_grads(X, T)
    h = 1e-6
    for l in range(len(SIZES) - 1):
        for which in (0, 1):
            P = model.params[l][which]
            G = grads[l][which]
            it = np.nditer(P, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = P[idx]
                P[idx] = old + h
                lp, _ = model.loss_and_grads(X, T)
                P[idx] = old - h
                lm, _ = model.loss_and_grads(X, T)
                P[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - G[idx]) <= 1e-6 * max(1.0, abs(fd)), (l, which, idx, fd, G[idx])


def _torch_model(params):
    ps = [(torch.tensor(W, dtype=torch.float64, requires_grad=True),
           torch.tensor(b, dtype=torch.float64, requires_grad=True)) for W, b in params]

    def fwd(X):
        a = X
        for l, (W, b) in enumerate(ps):
            z = a @ W.T + b
            a = torch.nn.functional.silu(z) if l < len(ps) - 1 else z
        return a
    return ps, fwd


def test_gradients_match_torch_autograd():
    X, T = _data(B=9, seed=2)
    params = mlp_init(SIZES, 4)
    model = om.MLP(params, rounding=False)
    loss, grads = model.loss_and_grads(X, T)
    ps, fwd = _torch_model(params)
    y = fwd(torch.tensor(X))
    tl = torch.mean((y - torch.tensor(T)) ** 2)
    tl.backward()
    assert abs(loss - tl.item()) <= 1e-14 * abs(loss)
    for (gW, gb), (W, b) in zip(grads, ps):
        assert np.allclose(gW, W.grad.numpy(), rtol=1e-12, atol=1e-15)
        assert np.allclose(gb, b.grad.numpy(), rtol=1e-12, atol=1e-15)


def test_adam_matches_torch():
    X, T = _data(B=8, seed=5)
    params = mlp_init(SIZES, 6)
    model = om.MLP(params, rounding=False)
    opt = om.Adam(model.params, lr=1e-2)
    ps, fwd = _torch_model(params)
    topt = torch.optim.Adam([p for pair in ps for p in pair], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(5):
        _, g = model.loss_and_grads(X, T)
        model.params = opt.step(model.params, g)
        topt.zero_grad()
        tl = torch.mean((fwd(torch.tensor(X)) - torch.tensor(T)) ** 2)
        tl.backward()
        topt.step()
    for (W, b), (tW, tb) in zip(model.params, ps):
        assert np.allclose(W, tW.detach().numpy(), rtol=1e-10, atol=1e-13)
        assert np.allclose(b, tb.detach().numpy(), rtol=1e-10, atol=1e-13)


def test_rounded_forward_is_close_and_training_learns():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((256, SIZES[0]))
    A = rng.standard_normal((SIZES[-1], SIZES[0])) * 0.3
    T = np.tanh(X @ A.T)
    params = mlp_init(SIZES, 8)
    exact = om.MLP(params, rounding=False).forward(X)[0]
    rounded = om.MLP(params, rounding=True).forward(X)[0]
    assert np.max(np.abs(rounded - exact)) <= 3e-2 * np.max(np.abs(exact)) + 1e-3
    model = om.MLP(params, rounding=True)
    order = np.stack([np.random.default_rng([9, e]).permutation(256) for e in range(40)])
    losses = om.train(model, X, T, epochs=40, batch=32, lr=3e-3, order=order)
    assert losses[-1] < 0.2 * losses[0]


def test_planted_missing_activation_derivative_is_caught():
    """Dropping silu' from the backward pass fails the finite-difference check."""
    X, T = _data(B=5, seed=10)
    model = om.MLP(mlp_init(SIZES, 11), rounding=False)
    orig = om.silu_grad
    try:
        om.silu_grad = lambda z: np.ones_like(z)
        _, grads = model.loss_and_grads(X, T)
    finally:
        om.silu_grad = orig
    P = model.params[0][0]
    h = 1e-6
    old = P[0, 0]
    P[0, 0] = old + h
    lp, _ = model.loss_and_grads(X, T)
    P[0, 0] = old - h
    lm, _ = model.loss_and_grads(X, T)
    P[0, 0] = old
    assert abs((lp - lm) / (2 * h) - grads[0][0][0, 0]) > 1e-6


def test_sketched_target_is_least_squares_for_full_rank_history():
    """With a numerically full-rank history the sketched least-squares coefficients are
    those of the sketched normal equations (plain definition via lstsq)."""
    from oracle.learned import sketched_ls_target
    from oracle.sketch import Sketch

    rng = np.random.default_rng(12)
    n, M = 300, 6
    X = rng.standard_normal((n, M))
    x = X @ rng.standard_normal(M) + 0.01 * rng.standard_normal(n)
    S = Sketch("gaussian", n, 2 * M, 5)
    c = sketched_ls_target(X, S.apply(X), S.apply(x))
    ref, *_ = np.linalg.lstsq(S.apply(X), S.apply(x), rcond=None)
    assert np.allclose(c, ref, rtol=1e-10, atol=1e-12)
    # an exact member of span(X) is recovered exactly
    w = rng.standard_normal(M)
    assert np.allclose(sketched_ls_target(X, S.apply(X), S.apply(X @ w)), w, rtol=1e-10)


def test_learned_guess_never_worse_than_projection():
    """Safeguard: the learned guess's residual never exceeds the projection's."""
    from gen import config
    from oracle.learned import LearnedSequence

    p, m = config(0, N=12)
    M, H = 4, 2
    seq = LearnedSequence(p.n, M, "gaussian", 8, seed=1, solver="cg", tol=1e-10)
    sizes = [H * M + 2, 8, M]
    seq.attach(om.MLP(mlp_init(sizes, 13)), np.zeros(sizes[0]), np.ones(sizes[0]), np.zeros(M), np.ones(M), H)
    for i in range(12):
        A = p.matrix(i).to_scipy()
        b = p.rhs(i)
        seq.t_now = p.t(i)
        g = seq.initial_guess(A, b)
        plain = super(LearnedSequence, seq).initial_guess(A, b)
        assert np.linalg.norm(b - A @ g.x0) <= np.linalg.norm(b - A @ plain.x0) * (1 + 1e-12)
        x, _ = seq.solve(A, b, g.x0)
        seq.push(x)
    assert len(seq.targets) == 12

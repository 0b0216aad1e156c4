"""Pins of the oracle's random draws and sketches (CPU only).

Philox4x64-10 is checked against numpy's independent implementation of the same
generator; the Hadamard entries against scipy's Sylvester construction; the Gaussian
entries against the normal distribution; the embedding property statistically.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.stats as st

from oracle import philox as px
from oracle import sketch as sk


@pytest.mark.parametrize("key", [(0, 0), (1, 0), (2**63 + 12345, 987654321), (2**64 - 1, 2**64 - 1)])
def test_philox_matches_numpy(key):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=0)
    raw = bg.random_raw(4 * 16)
    # numpy advances the counter before each block: block b uses counter b + 1
    mine = np.stack(px.philox4x64(np.arange(1, 17, dtype=np.uint64), 0, 0, 0, *key), 1).reshape(-1)
    assert np.array_equal(raw, mine)


def test_philox_full_counter_words():
    """All four counter words enter the block: compare against numpy with a set counter."""
    ctr = np.array([2**64 - 2, 7, 2**40 + 3, 11], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([5, 6], dtype=np.uint64), counter=ctr)
    raw = bg.random_raw(4)
    mine = np.array(px.philox4x64(2**64 - 1, 7, 2**40 + 3, 11, 5, 6), dtype=np.uint64)
    assert np.array_equal(raw, mine)


def test_uniforms_open_interval_and_index_range():
    w = np.array([0, 2**64 - 1, 2**63], dtype=np.uint64)
    u = px.to_unit_open(w)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert u[0] == 2.0**-53 and u[1] == 1.0 - 2.0**-53
    idx = px.uniform_index(np.array([0, 2**64 - 1], dtype=np.uint64), 1000)
    assert idx[0] == 0 and idx[1] == 999


def test_gaussian_sketch_distribution():
    S = sk.gaussian_block(20, 0, 5000, seed=3) * np.sqrt(20)
    z = S.reshape(-1)
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.02
    assert st.kstest(z, "norm").pvalue > 1e-3
    # different rows and seeds are not copies of each other
    assert abs(np.corrcoef(S[0], S[1])[0, 1]) < 0.05
    S2 = sk.gaussian_block(20, 0, 5000, seed=4) * np.sqrt(20)
    assert abs(np.corrcoef(S[0], S2[0])[0, 1]) < 0.05


def test_gaussian_sketch_blocks_are_consistent():
    full = sk.gaussian_block(13, 0, 300, seed=9)
    part = sk.gaussian_block(13, 100, 250, seed=9)
    assert np.array_equal(full[:, 100:250], part)


def test_hadamard_matches_sylvester():
    n = 64
    H = sk.hadamard_entries(np.arange(n)[:, None], np.arange(n)[None, :])
    assert np.array_equal(H, sla.hadamard(n).astype(np.float64))
    assert np.array_equal(H.T @ H, n * np.eye(n))


def test_srht_structure():
    n, s = 1024, 40
    S = sk.Sketch("srht", n, s, seed=11)
    D = S.dense()
    ref = sla.hadamard(n)[S.rows] * S.d[None, :] / np.sqrt(s)
    assert np.allclose(D, ref, rtol=0, atol=0)
    assert len(set(S.rows.tolist())) == s and S.rows.min() >= 0 and S.rows.max() < n
    assert set(np.unique(S.d)) <= {-1.0, 1.0} and 0.4 < np.mean(S.d > 0) < 0.6
    x = np.random.default_rng(0).standard_normal(n)
    assert np.allclose(S.apply(x), D @ x, rtol=1e-13, atol=1e-12)


def test_srht_rows_fisher_yates_small():
    # with s = n the partial shuffle is a full permutation
    rows = sk.srht_rows(16, 16, seed=5)
    assert sorted(rows.tolist()) == list(range(16))


@pytest.mark.parametrize("kind", ["gaussian", "srht"])
def test_subspace_embedding(kind):
    """||S v||^2 / ||v||^2 stays near 1 on a k-dim subspace for s = 4k."""
    n, k = 4096, 10
    rng = np.random.default_rng(1)
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    S = sk.Sketch(kind, n, 4 * k, seed=2)
    SU = S.apply(U)
    sv = np.linalg.svd(SU, compute_uv=False)
    assert sv.max() < 2.0 and sv.min() > 0.3


def test_bf16_rounding_bit_patterns():
    """FP32 -> BF16 round to nearest, ties to even, on hand-worked values: 1 + 2^-8 is
    halfway between 1 and 1 + 2^-7 (tie -> even mantissa 1.0), 1 + 3 2^-8 is halfway
    between 1 + 2^-7 and 1 + 2^-6 (tie -> even 1 + 2^-6), 1 + 2^-8 + 2^-20 rounds up,
    and values already in BF16 stay."""
    cases = {1.0 + 2.0 ** -8: 1.0, 1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -8 + 2.0 ** -20: 1.0 + 2.0 ** -7,
             -(1.0 + 2.0 ** -8 + 2.0 ** -20): -(1.0 + 2.0 ** -7), 0.75: 0.75, 0.0: 0.0, 2.0 ** -130: 2.0 ** -130}
    for v, want in cases.items():
        assert sk.to_bf16(np.array([v]))[0] == want, v


def test_bf16_rounding_matches_torch():
    """Against torch's own float32 -> bfloat16 conversion (round to nearest even)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        rng.standard_normal(1000).astype(np.float32).astype(np.float64)])
    f32 = v.astype(np.float32)
    ref = torch.from_numpy(f32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(sk.to_bf16(v), ref)


def test_bf16_gaussian_sketch_is_the_rounded_sketch():
    """The BF16 sketch applies BF16(G) / sqrt(s) to fl32(x): S x within the BF16 rounding
    of G (relative 2^-8 bounds it) plus the FP32 rounding of x of the FP64 sketch; sqrt(s)
    S holds BF16 values; and an FP32 value is exactly the sum of three BF16 terms taken by
    successive rounding (the split the GPU feeds its matrix cores)."""
    n, s = 3000, 24
    rng = np.random.default_rng(2)
    x = rng.standard_normal(n)
    S64 = sk.Sketch("gaussian", n, s, 9)
    Sb = sk.Sketch("gaussian", n, s, 9, bf16=True)
    D = Sb.dense() * np.sqrt(s)
    assert np.allclose(sk.to_bf16(D), D, rtol=1e-15, atol=0)
    G = sk.gaussian_normals(s, 0, n, 9)
    assert np.array_equal(sk.to_bf16(G) / np.sqrt(s), Sb.dense())
    x32 = x.astype(np.float32).astype(np.float64)
    assert np.allclose(Sb.apply(x), (sk.to_bf16(G) @ x32) / np.sqrt(s), rtol=1e-14, atol=1e-14)
    bound = (2.0 ** -8 + 2.0 ** -23) * (np.abs(S64.dense()) @ np.abs(x))
    assert np.all(np.abs(Sb.apply(x) - S64.apply(x)) <= bound)
    v = np.concatenate([x, x * 1e-20, x * 1e20]).astype(np.float32).astype(np.float64)
    hi = sk.to_bf16(v)
    mid = sk.to_bf16(v - hi)
    lo = v - hi - mid
    assert np.array_equal(sk.to_bf16(lo), lo)
    assert np.array_equal(hi + mid + lo, v)
    with pytest.raises(ValueError):
        sk.Sketch("srht", 4096, 16, 1, bf16=True)

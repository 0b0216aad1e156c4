"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case monkeypatches one step of the oracle with a plausible error (a transposed
operand, a wrong sign, a dropped term, a wrong pivot or rank) and runs the pin that
should catch it; the pin has to fail.
"""

import numpy as np
import pytest

import oracle.basis as bs
import oracle.krylov as kr
import oracle.sketch as sk
from tests import test_oracle_basis as tb
from tests import test_oracle_krylov as tk
from tests import test_oracle_rng_sketch as ts


class _NumpyProxy:
    """numpy with selected attributes replaced (for planting a mistake in one module)."""

    def __init__(self, **over):
        self._over = over

    def __getattr__(self, name):
        return self._over.get(name, getattr(np, name))


def _transposed_lu(monkeypatch):
    real = bs.sla.lu_factor
    monkeypatch.setattr(bs.sla, "lu_factor", lambda H: real(np.asarray(H).T))


def _rank_off_by_one(monkeypatch):
    real = bs.numerical_rank_qr
    monkeypatch.setattr(bs, "numerical_rank_qr", lambda R, tau: max(real(R, tau) - 1, 0))


def _cholesky_wrong_pivot(monkeypatch):
    monkeypatch.setattr(bs, "np", _NumpyProxy(argmax=np.argmin))


def _givens_sign(monkeypatch):
    real = kr.givens
    monkeypatch.setattr(kr, "givens", lambda a, b: (lambda c, s, r: (c, -s, r))(*real(a, b)))


def _dot_drops_last_term(monkeypatch):
    monkeypatch.setattr(kr, "np", _NumpyProxy(dot=lambda a, b: np.dot(a[..., :-1], b[..., :-1])))


def _hadamard_or(monkeypatch):
    def wrong(rows, cols):
        v = np.bitwise_or(np.asarray(rows, dtype=np.uint64), np.asarray(cols, dtype=np.uint64))
        return 1.0 - 2.0 * (np.bitwise_count(v) & np.uint8(1)).astype(np.float64)
    monkeypatch.setattr(sk, "hadamard_entries", wrong)


def _philox_no_keybump(monkeypatch):
    monkeypatch.setattr(sk.px, "PHILOX_W0", np.uint64(0))


CASES = [
    (_transposed_lu, lambda: tb.test_galerkin_equals_plain_definition(False)),
    (_rank_off_by_one, lambda: tb.test_galerkin_equals_plain_definition(True)),
    (_cholesky_wrong_pivot, tb.test_pivoted_cholesky_against_library),
    (_givens_sign, tk.test_gmres_full_finite_termination),
    (_dot_drops_last_term, tk.test_cg_few_distinct_eigenvalues),
    (_hadamard_or, ts.test_hadamard_matches_sylvester),
    (_philox_no_keybump, lambda: ts.test_philox_matches_numpy((1, 0))),
]


@pytest.mark.parametrize("plant,pin", CASES, ids=[c[0].__name__.strip("_") for c in CASES])
def test_planted_mistake_is_caught(monkeypatch, plant, pin):
    plant(monkeypatch)
    with pytest.raises((AssertionError, np.linalg.LinAlgError, ValueError)):
        pin()

"""Shared helpers of the GPU parity tests (imports torch and the HIP binding lazily)."""

from __future__ import annotations

import numpy as np


def dev(x, dtype=None):
    import torch

    a = np.ascontiguousarray(x)
    t = torch.as_tensor(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def method_kwargs(method: dict, **over) -> dict:
    kw = dict(M=method["M"], s=method["s"], sketch=method["sketch"], solver=method["solver"],
              restart=method["restart"], tol=method["tol"], seed=method["method_seed"])
    kw.update(over)
    return kw


def relres(A, x, b) -> float:
    return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))


def print_case(*args):
    print("[case]", *args, flush=True)


def reversed_order(A):
    """The same CSR matrix with each row's entries stored (and summed) in reverse
    order: a rounding-only perturbation of every product A x."""
    import scipy.sparse as sp

    A = A.tocsr()
    ip = A.indptr
    idx = np.concatenate([np.arange(ip[i + 1] - 1, ip[i] - 1, -1) for i in range(A.shape[0])]) \
        if A.nnz else np.zeros(0, dtype=np.int64)
    R = sp.csr_matrix((A.data[idx], A.indices[idx], ip), shape=A.shape)
    R.has_canonical_format = False
    return R


def rounding_spread(solve, A, *args, **kw):
    """(x, info, spread): the oracle's result and how far a rounding-only perturbation of
    the same run (reversed summation order in A x) moves its iterate."""
    x1, info = solve(A, *args, **kw)
    x2, _ = solve(reversed_order(A), *args, **kw)
    return x1, info, float(np.linalg.norm(x1 - x2))

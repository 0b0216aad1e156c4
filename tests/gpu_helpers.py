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

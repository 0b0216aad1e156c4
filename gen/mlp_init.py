"""Seeded initial weights of the coefficient-predictor MLP (input generator only).

Layer l maps sizes[l] -> sizes[l + 1]; W_l ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) in
float32, biases zero.  Shared by the oracle and the HIP path as their common input.
"""

from __future__ import annotations

import numpy as np


def mlp_init(sizes, seed: int = 0):
    rng = np.random.default_rng([seed, 11])
    params = []
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        lim = 1.0 / np.sqrt(fin)
        W = rng.uniform(-lim, lim, size=(fout, fin)).astype(np.float32)
        params.append((W, np.zeros(fout, dtype=np.float32)))
    return params

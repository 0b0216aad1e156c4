"""Counter-based random numbers: Philox4x64-10 and Box-Muller normals.

The paper draws Gaussian matrices (Section 2.2, the M x m matrix Z of the randomized
range finder) but fixes no generator.  Both sides of this project implement the same
published counter-based generator, Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), so that every random entry is
a pure function of (key, counter) and can be regenerated anywhere.

Pinned against numpy.random.Philox (the same generator, independent implementation)
in the test suite.  Normals use the Box-Muller transform; they may differ from the
device's in the last bits because log/cos are library calls on each side.
"""

from __future__ import annotations

import numpy as np

U64 = np.uint64
MASK32 = U64(0xFFFFFFFF)

# Multipliers and Weyl key increments of Philox4x64 (Salmon et al., Table 2 / Sec. 4)
PHILOX_M0 = U64(0xD2E7470EE14C6C93)
PHILOX_M1 = U64(0xCA5A826395121157)
PHILOX_W0 = U64(0x9E3779B97F4A7C15)
PHILOX_W1 = U64(0xBB67AE8584CAA73B)

# Stream identifiers (third counter word) separating the method's random draws.
STREAM_GAUSS_SKETCH = 1
STREAM_SRHT_SIGNS = 2
STREAM_SRHT_ROWS = 3
STREAM_RANGE_Z = 4


def _mulhilo(a, b):
    """High and low 64-bit halves of the 128-bit product a * b (arrays of uint64)."""
    a = np.asarray(a, dtype=U64)
    b = np.asarray(b, dtype=U64)
    with np.errstate(over="ignore"):
        lo = a * b
        a_lo, a_hi = a & MASK32, a >> U64(32)
        b_lo, b_hi = b & MASK32, b >> U64(32)
        ll = a_lo * b_lo
        lh = a_lo * b_hi
        hl = a_hi * b_lo
        hh = a_hi * b_hi
        mid = (ll >> U64(32)) + (lh & MASK32) + (hl & MASK32)
        hi = hh + (lh >> U64(32)) + (hl >> U64(32)) + (mid >> U64(32))
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds: int = 10):
    """Philox4x64 block function.  All inputs broadcast; returns four uint64 arrays."""
    x0, x1, x2, x3 = (np.asarray(v, dtype=U64) for v in (c0, c1, c2, c3))
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    x0, x1, x2, x3 = (v.copy() for v in (x0, x1, x2, x3))
    k0 = U64(k0)
    k1 = U64(k1)
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = U64(k0 + PHILOX_W0)
                k1 = U64(k1 + PHILOX_W1)
            hi0, lo0 = _mulhilo(PHILOX_M0, x0)
            hi1, lo1 = _mulhilo(PHILOX_M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def to_unit_open(w):
    """Map 64-bit words to doubles in the open interval (0, 1): ((w >> 12) + 1/2) 2^-52.

    Every value is exact in binary64 (at most 53 significant bits), the smallest is
    2^-53 and the largest 1 - 2^-53, so log(u) is always finite.
    """
    return ((np.asarray(w, dtype=U64) >> U64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def box_muller(u_rad, u_ang):
    """Two standard normals from two uniforms in (0, 1) (Box and Muller, 1958)."""
    rad = np.sqrt(-2.0 * np.log(u_rad))
    ang = 2.0 * np.pi * u_ang
    return rad * np.cos(ang), rad * np.sin(ang)


def normals4(c0, c1, c2, seed):
    """Four normals per counter (c0, c1, c2, 0) under key (seed, 0).

    Words (w0, w1) feed one Box-Muller pair, (w2, w3) the other; the result is stacked
    on a new last axis in the order (cos0, sin0, cos1, sin1).
    """
    w0, w1, w2, w3 = philox4x64(c0, c1, c2, 0, seed, 0)
    g0, g1 = box_muller(to_unit_open(w0), to_unit_open(w1))
    g2, g3 = box_muller(to_unit_open(w2), to_unit_open(w3))
    return np.stack([g0, g1, g2, g3], axis=-1)


def uniform_index(word, bound: int):
    """Integer in [0, bound) from a 64-bit word: (high 32 bits * bound) >> 32."""
    hi = np.asarray(word, dtype=U64) >> U64(32)
    return (hi * U64(bound)) >> U64(32)

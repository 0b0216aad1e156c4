"""Closed-form bounds of Section 3 and Section 2.2, evaluated for test pins.

* ``bernstein_kappa``   - kappa_rho = max over the Bernstein ellipse boundary of ||x(t)||_2
                          (Assumption 1), sampled on a fine grid of the boundary.
* ``thm1_sigma_bound``  - Theorem 1: sigma_k(X) <= 2 rho kappa sqrt(M) rho^-k / (1 - 1/rho).
* ``thm2_residual_bound`` - Theorem 2: residual of s* for S = span X and uniform steps.
* ``halko_bound``       - eq. (errorrandsvd): expected range-finder error, m = r + p.
"""

from __future__ import annotations

import math

import numpy as np


def bernstein_points(rho: float, npts: int = 4096) -> np.ndarray:
    """Points on the boundary of the Bernstein ellipse E_rho (foci +-1, a + b = rho)."""
    th = np.linspace(0.0, 2.0 * np.pi, npts, endpoint=False)
    w = rho * np.exp(1j * th)
    return 0.5 * (w + 1.0 / w)


def bernstein_kappa(xfun, rho: float, npts: int = 4096) -> float:
    """kappa_rho = max_{t on boundary of E_rho} ||x(t)||_2 for a callable x(t) (complex t)."""
    return max(float(np.linalg.norm(xfun(t))) for t in bernstein_points(rho, npts))


def thm1_sigma_bound(k: int, rho: float, kappa: float, M: int) -> float:
    return 2.0 * rho * kappa * math.sqrt(M) / (1.0 - 1.0 / rho) * rho ** (-k)


def thm2_constant(M: int, R: int) -> float:
    """C(M, R) of Theorem 2."""
    return 5.0 * math.sqrt(5.0) * math.sqrt(2 * R + 1) * math.sqrt(M) / math.sqrt(2.0 * (M - 1))


def thm2_residual_bound(normA: float, kappa: float, rho: float, M: int, R: int,
                        t_next: float) -> float:
    """Theorem 2 bound on ||A(t_i) s* - b(t_i)||_2 (needs R <= sqrt(M - 1) / 2, r < 1)."""
    r = (t_next + math.sqrt(t_next * t_next - 1.0)) / rho
    if not r < 1.0:
        return math.inf
    C = thm2_constant(M, R)
    term = 1.0 / (1.0 - r) + C * rho / ((rho - 1.0) * math.sqrt(rho * rho * r * r - 1.0))
    return 2.0 * normA * kappa * term * r ** (R + 1)


def halko_bound(sv: np.ndarray, r: int, p: int) -> float:
    """Right-hand side of eq. (errorrandsvd) for m = r + p (p >= 2)."""
    tail = float(np.sum(np.asarray(sv)[r:] ** 2))
    return math.sqrt(1.0 + r / (p - 1.0)) * math.sqrt(tail)

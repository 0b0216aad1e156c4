"""The test case of Section 4: a variable-coefficient elliptic problem with a known solution.

    div(a(x, t) grad f(x, t)) = g(x, t) on the unit square,
    a = exp(-(x - 1/2)^2 - (y - 1/2)^2) cos(t x) + 2.1,
    f = sin(4 pi y t) sin(15 pi x t) [1 + sin(15 pi x t) cos(3 pi y t) exp((x - 1/2)^2 + (y - 1/2)^2 - 1/16)],

with g chosen so that f solves the equation (here: g = div(a grad f) of that f, formed
symbolically), discretised by centred finite differences of order 4 on a uniform grid
and sampled at t_i = t0 + i dt (t0 = 2.3; dt = 1e-5 or 1e-3; 200 steps; a 100 x 100
grid, n = 10 000).

Discretisation (the paper names only the order; these are documented readings):
* N interior nodes per side, h = 1 / (N + 1), node (ix, iy) at ((ix + 1) h, (iy + 1) h),
  index ix + N iy.
* div(a grad f) = a (f_xx + f_yy) + a_x f_x + a_y f_y with a, a_x, a_y evaluated at the
  node, second derivatives by (-f_{-2} + 16 f_{-1} - 30 f_0 + 16 f_{+1} - f_{+2}) / (12 h^2)
  and first derivatives by (f_{-2} - 8 f_{-1} + 8 f_{+1} - f_{+2}) / (12 h) along each axis:
  a 9-point cross stencil, nonsymmetric (the first-derivative terms).
* Stencil points outside the interior grid (the boundary line and one line beyond it)
  carry the known solution f: their terms move to the right-hand side.  The stated
  boundary condition f = 0 does not hold for this f on x = 1 or y = 1 for general t, so
  the boundary data are taken from f itself.

The systems are A(t_i) f(t_i) = b(t_i) with A the stencil on the interior unknowns and
b = g - (terms of the known outside values).  Parity is against what the construction
fixes: the assembly is exact on polynomials of degree <= 4 (the centred formulas of
order 4 differentiate them exactly) and the discrete solution converges to f at order 4.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .problems import CSR

OFFSETS = (-2, -1, 1, 2)
D2 = {-2: -1.0 / 12.0, -1: 16.0 / 12.0, 0: -30.0 / 12.0, 1: 16.0 / 12.0, 2: -1.0 / 12.0}
D1 = {-2: 1.0 / 12.0, -1: -8.0 / 12.0, 1: 8.0 / 12.0, 2: -1.0 / 12.0}

_FUNCS = None


def _functions():
    """numpy callables (x, y, t) -> a, a_x, a_y, f, g, formed once with sympy."""
    global _FUNCS
    if _FUNCS is None:
        import sympy as sy

        x, y, t = sy.symbols("x y t", real=True)
        r2 = (x - sy.Rational(1, 2)) ** 2 + (y - sy.Rational(1, 2)) ** 2
        a = sy.exp(-r2) * sy.cos(t * x) + sy.Rational(21, 10)
        f = sy.sin(4 * sy.pi * y * t) * sy.sin(15 * sy.pi * x * t) * (
            1 + sy.sin(15 * sy.pi * x * t) * sy.cos(3 * sy.pi * y * t) * sy.exp(r2 - sy.Rational(1, 16)))
        g = sy.diff(a * sy.diff(f, x), x) + sy.diff(a * sy.diff(f, y), y)
        mk = lambda e: sy.lambdify((x, y, t), e, "numpy")  # noqa: E731
        _FUNCS = dict(a=mk(a), ax=mk(sy.diff(a, x)), ay=mk(sy.diff(a, y)), f=mk(f), g=mk(g))
    return _FUNCS


@dataclasses.dataclass
class Paper4Problem:
    """One sequence of the Section 4 test case (``matrix(i)``, ``rhs(i)``, ``exact(i)``)."""

    N: int = 100
    dt: float = 1e-5
    steps: int = 200
    t0: float = 2.3
    name: str = "paper4"

    def __post_init__(self):
        self.h = 1.0 / (self.N + 1)
        self.n = self.N * self.N
        self._pattern = None

    def t(self, i: int) -> float:
        return self.t0 + i * self.dt

    def _grid(self):
        N = self.N
        idx = np.arange(self.n)
        ix, iy = idx % N, idx // N
        return ix, iy, (ix + 1) * self.h, (iy + 1) * self.h

    def _entries(self):
        """(dx, dy) of the 9 stencil entries in ascending column order."""
        return [(0, -2), (0, -1), (-2, 0), (-1, 0), (0, 0), (1, 0), (2, 0), (0, 1), (0, 2)]

    def pattern(self):
        """(rowptr, col) int32 arrays of the interior entries of the stencil."""
        if self._pattern is None:
            N = self.N
            ix, iy, _, _ = self._grid()
            cols, masks = [], []
            for dx, dy in self._entries():
                jx, jy = ix + dx, iy + dy
                masks.append((jx >= 0) & (jx < N) & (jy >= 0) & (jy < N))
                cols.append(jx + N * jy)
            cols = np.stack(cols, 1)
            mask = np.stack(masks, 1)
            rowptr = np.zeros(self.n + 1, dtype=np.int64)
            np.cumsum(mask.sum(1), out=rowptr[1:])
            self._pattern = (rowptr.astype(np.int32), cols[mask].astype(np.int32), mask)
        return self._pattern[0], self._pattern[1]

    def _stencil(self, t):
        """Weights (n x 9) of the stencil at time t, in the order of ``_entries``."""
        F = _functions()
        _, _, x, y = self._grid()
        h = self.h
        a, ax, ay = F["a"](x, y, t), F["ax"](x, y, t), F["ay"](x, y, t)
        W = np.zeros((self.n, 9))
        for e, (dx, dy) in enumerate(self._entries()):
            if dx == 0 and dy == 0:
                W[:, e] = 2.0 * D2[0] * a / (h * h)
            elif dy == 0:
                W[:, e] = D2[dx] * a / (h * h) + D1[dx] * ax / h
            else:
                W[:, e] = D2[dy] * a / (h * h) + D1[dy] * ay / h
        return W

    def matrix(self, i: int) -> CSR:
        rowptr, col = self.pattern()
        W = self._stencil(self.t(i))
        return CSR(self.n, rowptr, col, W[self._pattern[2]])

    def _outside(self, t, fun):
        """Sum over the stencil entries outside the interior of weight * fun(point)."""
        W = self._stencil(t)
        _, _, x, y = self._grid()
        h = self.h
        self.pattern()
        mask = self._pattern[2]
        out = np.zeros(self.n)
        for e, (dx, dy) in enumerate(self._entries()):
            off = ~mask[:, e]
            if np.any(off):
                out[off] += W[off, e] * fun(x[off] + dx * h, y[off] + dy * h)
        return out

    def rhs(self, i: int) -> np.ndarray:
        """b(t_i) = g at the nodes minus the known outside values' terms."""
        t = self.t(i)
        F = _functions()
        _, _, x, y = self._grid()
        self.pattern()
        return F["g"](x, y, t) - self._outside(t, lambda px, py: F["f"](px, py, t))

    def exact(self, i: int) -> np.ndarray:
        """The manufactured solution f(t_i) at the interior nodes."""
        F = _functions()
        _, _, x, y = self._grid()
        return F["f"](x, y, self.t(i))


def paper4_config(dt: float = 1e-5, N: int = 100, steps: int = 200):
    """The Section 4 sequence with the method settings used here: GMRES(30) to 1e-7 (the
    paper's tolerance; its ILU preconditioner is not applied), Gaussian sketch s = 2M,
    M = 20 for dt = 1e-5 (the paper's M) and M = 32 for dt = 1e-3 (the paper uses 35;
    32 is this library's longest history), m = M."""
    p = Paper4Problem(N=N, dt=dt, steps=steps)
    M = 20 if dt <= 1e-5 else 32
    return p, dict(M=M, sketch="gaussian", s=2 * M, solver="gmres", restart=30, tol=1e-7, prec="fp64",
                   method_seed=5)

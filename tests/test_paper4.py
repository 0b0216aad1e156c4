"""Pins of the Section 4 test-case generator (gen/paper4.py), independent of the method.

* The assembly differentiates polynomials of degree <= 4 exactly (the centred
  formulas of order 4 are exact there), boundary and ghost terms included.
* The discrete solution converges to the manufactured f at order 4 (error ratio about
  16 per halving of h).
* The symbolic right-hand side g equals div(a grad f) evaluated by central differences
  of the continuous functions.
* The CSR matrix equals a loop-by-loop dense assembly on a small grid.
"""

import numpy as np
import scipy.sparse.linalg as spla

from gen.paper4 import D1, D2, Paper4Problem, _functions, paper4_config


def test_polynomial_exactness():
    p = Paper4Problem(N=9)
    F = _functions()
    t = p.t(3)

    def poly(x, y):
        return x**4 - 2.0 * x**2 * y**2 + 3.0 * x * y**3 + y**2 - x + 0.5

    def Lpoly(x, y):
        # a (p_xx + p_yy) + a_x p_x + a_y p_y
        pxx = 12.0 * x**2 - 4.0 * y**2
        pyy = -4.0 * x**2 + 18.0 * x * y + 2.0
        px = 4.0 * x**3 - 4.0 * x * y**2 + 3.0 * y**3 - 1.0
        py = -4.0 * x**2 * y + 9.0 * x * y**2 + 2.0 * y
        return F["a"](x, y, t) * (pxx + pyy) + F["ax"](x, y, t) * px + F["ay"](x, y, t) * py

    _, _, x, y = p._grid()
    A = p.matrix(3).to_scipy()
    lhs = A @ poly(x, y) + p._outside(t, poly)
    ref = Lpoly(x, y)
    assert np.max(np.abs(lhs - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_fourth_order_convergence():
    errs = []
    for N in (63, 127):
        p = Paper4Problem(N=N)
        f = spla.spsolve(p.matrix(0).to_scipy().tocsc(), p.rhs(0))
        errs.append(np.max(np.abs(f - p.exact(0))))
    assert errs[0] / errs[1] >= 12.0, errs


def test_rhs_is_the_operator_of_f():
    """Central differences of the continuous flux converge to the symbolic g at second
    order in the step (the solution oscillates fast, so the steps are small)."""
    F = _functions()
    rng = np.random.default_rng(4)
    x, y = rng.uniform(0.1, 0.9, 6), rng.uniform(0.1, 0.9, 6)
    t = 2.3
    g = F["g"](x, y, t)
    errs = []
    for e in (1e-4, 3e-5):
        def flux_x(px, py):
            return F["a"](px, py, t) * (F["f"](px + e, py, t) - F["f"](px - e, py, t)) / (2 * e)

        def flux_y(px, py):
            return F["a"](px, py, t) * (F["f"](px, py + e, t) - F["f"](px, py - e, t)) / (2 * e)

        fd = (flux_x(x + e, y) - flux_x(x - e, y)) / (2 * e) + (flux_y(x, y + e) - flux_y(x, y - e)) / (2 * e)
        errs.append(np.max(np.abs(fd - g)) / np.max(np.abs(g)))
    assert errs[1] <= 5e-5, errs
    assert 8.0 <= errs[0] / errs[1] <= 14.0, errs   # (1e-4 / 3e-5)^2 = 11.1


def test_csr_equals_dense_loop_assembly():
    p = Paper4Problem(N=6)
    F = _functions()
    t = p.t(5)
    N, h, n = p.N, p.h, p.n
    D = np.zeros((n, n))
    for iy in range(N):
        for ix in range(N):
            P = ix + N * iy
            x, y = (ix + 1) * h, (iy + 1) * h
            a, ax, ay = F["a"](x, y, t), F["ax"](x, y, t), F["ay"](x, y, t)
            D[P, P] += 2.0 * D2[0] * a / h**2
            for d in (-2, -1, 1, 2):
                for jx, jy, grad in ((ix + d, iy, ax), (ix, iy + d, ay)):
                    if 0 <= jx < N and 0 <= jy < N:
                        D[P, jx + N * jy] += D2[d] * a / h**2 + D1[d] * grad / h
    A = p.matrix(5).to_dense()
    assert np.max(np.abs(A - D)) <= 1e-12 * np.max(np.abs(D))


def test_config_shapes():
    p, m = paper4_config(1e-5)
    assert p.n == 10000 and p.steps == 200 and m["M"] == 20 and m["tol"] == 1e-7
    p, m = paper4_config(1e-3)
    assert abs(p.t(199) - (2.3 + 0.199)) < 1e-12 and m["M"] == 32

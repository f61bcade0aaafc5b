"""Measured convergence of the oracle's full-grid scheme on a smooth manufactured solution of
the nonlinear SWE (Sections 2.1-2.4; the paper's manufactured-solution experiment of
Section 5): 3rd order for Upwind3, 5th order for Upwind5 and WENO5, with dt proportional to
dx^(5/3) so that the SSP-RK3 error does not mask the spatial order.

The forcing S = dU/dt + dF(U)/dx + dG(U)/dy of the chosen smooth periodic solution is
evaluated with complex-step derivatives (exact to round-off for analytic functions) at the
3 x 3 Gauss-Legendre points of every cell."""
import math

import numpy as np
import pytest

from oracle import fv_grid

G = 9.81
TWO_PI = 2.0 * math.pi


def exact(x, y, t):
    """(h, hu, hv) of the manufactured solution; works for complex arguments."""
    h = 1.0 + 0.1 * np.sin(TWO_PI * (x - t)) * np.cos(TWO_PI * y)
    u = 0.1 * np.cos(TWO_PI * (x + y - t))
    v = 0.05 * np.sin(TWO_PI * (x - 2.0 * y + t))
    return h, h * u, h * v


def fluxes(h, hu, hv):
    F = (hu, hu * hu / h + 0.5 * G * h * h, hu * hv / h)
    Gf = (hv, hu * hv / h, hv * hv / h + 0.5 * G * h * h)
    return F, Gf


def forcing(x, y, t):
    d = 1e-30
    ut = [np.imag(c) / d for c in exact(x, y, t + 1j * d)]
    fx = [np.imag(c) / d for c in fluxes(*exact(x + 1j * d, y, t))[0]]
    gy = [np.imag(c) / d for c in fluxes(*exact(x, y + 1j * d, t))[1]]
    return [a + b + c for a, b, c in zip(ut, fx, gy)]


def cell_avg(fun, n):
    xg, wg = np.polynomial.legendre.leggauss(3)
    xg, wg = 0.5 * xg, 0.5 * wg
    c = (np.arange(n) + 0.5) / n
    out = None
    for a in range(3):
        for b in range(3):
            X = (c + xg[a] / n)[:, None]
            Y = (c + xg[b] / n)[None, :]
            vals = fun(X + 0 * Y, Y + 0 * X)
            acc = [wg[a] * wg[b] * v for v in vals]
            out = acc if out is None else [o + q for o, q in zip(out, acc)]
    return out


def error(scheme, n, T=0.02):
    dx = 1.0 / n
    dt0 = 0.3 * dx ** (5.0 / 3.0)
    steps = max(1, int(math.ceil(T / dt0)))
    dt = T / steps
    src = lambda t: cell_avg(lambda x, y: forcing(x, y, t), n)
    gs = fv_grid.GridSolver(n, scheme, True, True, g=G, source=src)
    U = cell_avg(lambda x, y: exact(x, y, 0.0), n)
    t = 0.0
    for _ in range(steps):
        U = gs.step(U, dt, t)
        t += dt
    Ue = cell_avg(lambda x, y: exact(x, y, T), n)
    return max(np.sqrt(np.mean((a - b) ** 2)) for a, b in zip(U, Ue))


def test_forcing_matches_finite_differences():
    """The complex-step forcing agrees with 4th-order central differences of the same
    functions (an independent evaluation of the derivatives)."""
    rng = np.random.default_rng(0)
    x, y, t = rng.random(20), rng.random(20), 0.3
    S = forcing(x, y, t)
    e = 1e-3

    def cd(fun):
        return [(-a + 8 * b - 8 * c + d) / (12 * e) for a, b, c, d in
                zip(fun(2 * e), fun(e), fun(-e), fun(-2 * e))]

    ut = cd(lambda s: exact(x, y, t + s))
    fx = cd(lambda s: fluxes(*exact(x + s, y, t))[0])
    gy = cd(lambda s: fluxes(*exact(x, y + s, t))[1])
    for k in range(3):
        ref = ut[k] + fx[k] + gy[k]
        assert np.max(np.abs(S[k] - ref)) < 1e-7 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("scheme,order,grids", [
    ("upwind3", 3.0, (16, 32, 64)),
    ("upwind5", 5.0, (16, 32, 64)),
    ("weno5", 5.0, (16, 32, 64)),
])
def test_manufactured_solution_order(scheme, order, grids):
    errs = [error(scheme, n) for n in grids]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print(scheme, errs, rates)
    assert rates[-1] >= order - 0.4, (errs, rates)

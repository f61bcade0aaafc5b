"""Seeded synthetic initial states for the 2-D shallow water workloads.

This module only produces input data.  It holds none of the solver's arithmetic:
it evaluates the initial fields, averages them over the cells with a library-grade
Gauss-Legendre rule (numpy.polynomial.legendre.leggauss), and compresses the
cell-average matrix into two factors with numpy's LAPACK QR/SVD.  Both the CPU
oracle and the GPU library receive the very same factors.

Workloads (all on the unit square, g = 9.81):

  linear_gaussian   linear SWE, one Gaussian bump on eta (amplitude 0.01, width 0.05,
                    centre ~ U[0,1]^2), u = v = 0, periodic.          64 x 64, r 8
  nonlinear_bumps   nonlinear SWE, h = 1 + 4 Gaussian bumps (amplitude U[0.01,0.1],
                    width U[0.03,0.1], centres U[0,1]^2), u, v smooth Fourier
                    fields with |k_x|,|k_y| <= 8 scaled to max |.| = 0.05.  1024^2, r 32
  dam_break         nonlinear SWE, h = 1 + 0.5 tanh((0.3 - r)/0.01), r = distance
                    to a centre ~ U[0.3,0.7]^2, u = v = 0, reflective walls. 2048^2, r 64

The random draws are made in a fixed order from numpy.random.default_rng(seed).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

G_DEFAULT = 9.81


@dataclasses.dataclass
class Factored:
    """A field stored as two factors: field[i, j] = sum_a A[i, a] * B[j, a]."""
    A: np.ndarray  # (n1, r) float64, rows = x cells
    B: np.ndarray  # (n2, r) float64, rows = y cells

    @property
    def rank(self) -> int:
        return self.A.shape[1]

    def full(self) -> np.ndarray:
        return self.A @ self.B.T


@dataclasses.dataclass
class State:
    """Initial state: three conserved variables, each as full cell averages and factors."""
    name: str
    n: int
    nonlinear: bool
    periodic: bool
    g: float
    H0: float
    fields: list          # three (n, n) cell-average arrays, x index first
    tt: list              # three Factored
    dt: float             # CFL 0.4 time step from the initial full fields
    meta: dict


# ---------------------------------------------------------------------------
# quadrature helpers (input preparation only)

def _gl(npts: int):
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * x, 0.5 * w          # nodes on [-1/2, 1/2], weights summing to 1


def cell_avg_1d(fun, n: int, npts: int = 8) -> np.ndarray:
    """Average of fun(x) over each of n equal cells of [0, 1]."""
    xg, wg = _gl(npts)
    h = 1.0 / n
    centres = (np.arange(n) + 0.5) * h
    pts = centres[:, None] + h * xg[None, :]
    return (fun(pts) * wg[None, :]).sum(axis=1)


def cell_avg_2d(fun, n: int, npts: int = 3, block: int = 256) -> np.ndarray:
    """Average of fun(x, y) over each cell of an n x n grid of [0, 1]^2."""
    xg, wg = _gl(npts)
    h = 1.0 / n
    centres = (np.arange(n) + 0.5) * h
    px = centres[:, None] + h * xg[None, :]          # (n, q)
    out = np.zeros((n, n))
    for i0 in range(0, n, block):
        X = px[i0:i0 + block]                          # (b, q)
        acc = np.zeros((X.shape[0], n))
        for a in range(npts):
            for b in range(npts):
                acc += wg[a] * wg[b] * fun(X[:, a][:, None], px[:, b][None, :])
        out[i0:i0 + block] = acc
    return out


def compress(terms_x: np.ndarray, terms_y: np.ndarray, eps: float, rmax: int) -> Factored:
    """Best rank-k factors of terms_x @ terms_y.T, relative Frobenius tolerance eps, k <= rmax."""
    qa, ra = np.linalg.qr(terms_x)
    qb, rb = np.linalg.qr(terms_y)
    u, s, vt = np.linalg.svd(ra @ rb.T)
    return _truncate(qa @ u, s, qb @ vt.T, eps, rmax)


def compress_full(field: np.ndarray, eps: float, rmax: int) -> Factored:
    u, s, vt = np.linalg.svd(field, full_matrices=False)
    return _truncate(u, s, vt.T, eps, rmax)


def _truncate(u, s, v, eps, rmax) -> Factored:
    nrm = math.sqrt(float(np.sum(s * s)))
    if nrm == 0.0:
        n1, n2 = u.shape[0], v.shape[0]
        return Factored(np.zeros((n1, 1)), np.zeros((n2, 1)))
    tail = np.sqrt(np.cumsum((s * s)[::-1])[::-1])      # tail[k] = ||s[k:]||
    k = len(s)
    for kk in range(1, len(s) + 1):
        t = tail[kk] if kk < len(s) else 0.0
        if t <= eps * nrm:
            k = kk
            break
    k = min(k, rmax)
    return Factored(np.ascontiguousarray(u[:, :k] * s[None, :k]), np.ascontiguousarray(v[:, :k]))


def _zero(n: int) -> Factored:
    return Factored(np.zeros((n, 1)), np.zeros((n, 1)))


def cfl_dt(fields, nonlinear: bool, g: float, H0: float, n: int, cfl: float = 0.4) -> float:
    dx = 1.0 / n
    if nonlinear:
        h, hu, hv = fields
        c = np.sqrt(g * h)
        sx = float(np.max(np.abs(hu / h) + c))
        sy = float(np.max(np.abs(hv / h) + c))
    else:
        c = math.sqrt(g * H0)
        sx = float(np.max(np.abs(fields[1]))) + c
        sy = float(np.max(np.abs(fields[2]))) + c
    return cfl / (sx / dx + sy / dx)


# ---------------------------------------------------------------------------
# periodised Gaussians and Fourier modes as 1-D factor functions

def _pgauss(c: float, w: float):
    return lambda t: sum(np.exp(-((t - c - m) ** 2) / (2.0 * w * w)) for m in (-1, 0, 1))


def linear_gaussian(seed: int = 0, n: int = 64, rmax: int = 8, eps: float = 1e-12,
                    g: float = G_DEFAULT, H0: float = 1.0) -> State:
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, size=2)
    gx = cell_avg_1d(_pgauss(c[0], 0.05), n)
    gy = cell_avg_1d(_pgauss(c[1], 0.05), n)
    eta = 0.01 * np.outer(gx, gy)
    tt_eta = compress((0.01 * gx)[:, None], gy[:, None], eps, rmax)
    fields = [eta, np.zeros((n, n)), np.zeros((n, n))]
    dt = cfl_dt(fields, False, g, H0, n)
    return State("linear_gaussian", n, False, True, g, H0, fields,
                 [tt_eta, _zero(n), _zero(n)], dt, {"centre": c.tolist(), "seed": seed})


def _fourier_terms(rng, kmax: int):
    """Half-plane set of modes k with |kx|,|ky| <= kmax; returns list of (kx, ky, a, b)."""
    modes = []
    for kx in range(0, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            if kx == 0 and ky <= 0:
                continue
            modes.append((kx, ky))
    coef = rng.standard_normal(size=(len(modes), 2))
    return [(kx, ky, coef[t, 0], coef[t, 1]) for t, (kx, ky) in enumerate(modes)]


def _fourier_factors(modes, n: int, npts: int = 8):
    """Write sum a cos(2pi k.x) + b sin(2pi k.x) as separable terms; return (X, Y) factor columns."""
    two_pi = 2.0 * math.pi
    colsx, colsy = [], []
    for kx, ky, a, b in modes:
        cx = cell_avg_1d(lambda t, k=kx: np.cos(two_pi * k * t), n, npts)
        sx = cell_avg_1d(lambda t, k=kx: np.sin(two_pi * k * t), n, npts)
        cy = cell_avg_1d(lambda t, k=ky: np.cos(two_pi * k * t), n, npts)
        sy = cell_avg_1d(lambda t, k=ky: np.sin(two_pi * k * t), n, npts)
        # a cos(A+B) + b sin(A+B) = a(cAcB - sAsB) + b(sAcB + cAsB)
        colsx += [a * cx, -a * sx, b * sx, b * cx]
        colsy += [cy, sy, cy, sy]
    return np.stack(colsx, axis=1), np.stack(colsy, axis=1)


def _fourier_pointwise(modes):
    two_pi = 2.0 * math.pi

    def f(x, y):
        out = 0.0
        for kx, ky, a, b in modes:
            ph = two_pi * (kx * x + ky * y)
            out = out + a * np.cos(ph) + b * np.sin(ph)
        return out
    return f


def nonlinear_bumps(seed: int = 0, n: int = 1024, rmax: int = 32, eps: float = 1e-10,
                    g: float = G_DEFAULT, nbumps: int = 4, kmax: int = 8,
                    vel_amp: float = 0.05) -> State:
    rng = np.random.default_rng(seed)
    bumps = []
    for _ in range(nbumps):
        a = rng.uniform(0.01, 0.1)
        w = rng.uniform(0.03, 0.1)
        cx = rng.uniform(0.0, 1.0)
        cy = rng.uniform(0.0, 1.0)
        bumps.append((a, w, cx, cy))
    modes_u = _fourier_terms(rng, kmax)
    modes_v = _fourier_terms(rng, kmax)

    # h as separable terms: 1 + sum_k a_k gx_k(x) gy_k(y)
    hx = [np.ones(n)] + [a * cell_avg_1d(_pgauss(cx, w), n) for a, w, cx, cy in bumps]
    hy = [np.ones(n)] + [cell_avg_1d(_pgauss(cy, w), n) for a, w, cx, cy in bumps]
    hX, hY = np.stack(hx, 1), np.stack(hy, 1)

    # u, v: scale so that the largest |cell average| is vel_amp
    uX, uY = _fourier_factors(modes_u, n)
    vX, vY = _fourier_factors(modes_v, n)
    su = vel_amp / float(np.max(np.abs(uX @ uY.T)))
    sv = vel_amp / float(np.max(np.abs(vX @ vY.T)))

    # hu, hv: cell averages of the pointwise products, term by term (separable)
    def prod_terms(scale, modes):
        two_pi = 2.0 * math.pi
        fx = [lambda t: np.ones_like(t)] + [
            (lambda t, a=a, w=w, cx=cx: a * _pgauss(cx, w)(t)) for a, w, cx, cy in bumps]
        fy = [lambda t: np.ones_like(t)] + [
            (lambda t, w=w, cy=cy: _pgauss(cy, w)(t)) for a, w, cx, cy in bumps]
        colsx, colsy = [], []
        for kx, ky, a, b in modes:
            gxs = [lambda t, k=kx: np.cos(two_pi * k * t), lambda t, k=kx: np.sin(two_pi * k * t)]
            gys = [lambda t, k=ky: np.cos(two_pi * k * t), lambda t, k=ky: np.sin(two_pi * k * t)]
            # a(cAcB - sAsB) + b(sAcB + cAsB)
            combos = [(a, 0, 0), (-a, 1, 1), (b, 1, 0), (b, 0, 1)]
            for coef, ix, iy in combos:
                for fxi, fyi in zip(fx, fy):
                    colsx.append(scale * coef * cell_avg_1d(
                        lambda t, p=fxi, q=gxs[ix]: p(t) * q(t), n))
                    colsy.append(cell_avg_1d(lambda t, p=fyi, q=gys[iy]: p(t) * q(t), n))
        return np.stack(colsx, 1), np.stack(colsy, 1)

    huX, huY = prod_terms(su, modes_u)
    hvX, hvY = prod_terms(sv, modes_v)
    h = hX @ hY.T
    hu = huX @ huY.T
    hv = hvX @ hvY.T
    tt = [compress(hX, hY, eps, rmax), compress(huX, huY, eps, rmax), compress(hvX, hvY, eps, rmax)]
    fields = [h, hu, hv]
    dt = cfl_dt(fields, True, g, 1.0, n)
    meta = {"seed": seed, "bumps": bumps, "su": su, "sv": sv,
            "ranks": [t.rank for t in tt]}
    return State("nonlinear_bumps", n, True, True, g, 1.0, fields, tt, dt, meta)


def dam_break(seed: int = 0, n: int = 2048, rmax: int = 64, eps: float = 1e-8,
              g: float = G_DEFAULT, width: float = 0.01, radius: float = 0.3) -> State:
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, size=2)

    def hfun(x, y):
        r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2)
        return 1.0 + 0.5 * np.tanh((radius - r) / width)
    h = cell_avg_2d(hfun, n, npts=3)
    tt = [compress_full(h, eps, rmax), _zero(n), _zero(n)]
    fields = [h, np.zeros((n, n)), np.zeros((n, n))]
    dt = cfl_dt(fields, True, g, 1.0, n)
    return State("dam_break", n, True, False, g, 1.0, fields, tt, dt,
                 {"seed": seed, "centre": c.tolist(), "ranks": [t.rank for t in tt]})


def random_factored(rng, n1: int, n2: int, r: int, decay: float = 0.5) -> Factored:
    """Random factors with geometrically decaying column scales (for primitive tests)."""
    A = rng.standard_normal((n1, r)) * (decay ** np.arange(r))[None, :]
    B = rng.standard_normal((n2, r))
    return Factored(A, B)


def smooth_factored(rng, n1: int, n2: int, r: int, base: float = 1.0) -> Factored:
    """Smooth positive-ish field: base + small smooth perturbation, as factors."""
    x = (np.arange(n1) + 0.5) / n1
    y = (np.arange(n2) + 0.5) / n2
    A = [base * np.ones(n1)]
    B = [np.ones(n2)]
    for k in range(1, r):
        a = rng.uniform(-0.05, 0.05) / k
        A.append(a * np.cos(2 * math.pi * k * x + rng.uniform(0, 2 * math.pi)))
        B.append(np.cos(2 * math.pi * k * y + rng.uniform(0, 2 * math.pi)))
    return Factored(np.stack(A, 1), np.stack(B, 1))


# ---------------------------------------------------------------------------
# Section 5 analytic cases, in the nondimensional variables of the appendix
#
# Dimensional constants of Section 5: g* = 10 m/s^2, f* = 1e-4 1/s.  Table 2's reference
# scales (L_ref, U_ref, H_ref) give t_ref = L_ref/U_ref, g_ref = U_ref^2/H_ref and
# f_ref = U_ref/L_ref; lengths are divided by L_ref (the domain becomes the unit square),
# eta and h by H_ref, velocities by U_ref.

G_STAR, F_STAR = 10.0, 1e-4
SCALES = {"coastal_kelvin": (5e6, 5e-3, 0.1), "inertia_gravity": (1e7, 1.622e-3, 0.2),
          "barotropic_tide": (25e4, 3.163e-3, 0.2), "manufactured": (1e7, 1e-2, 500.0)}
# Table 1: time-step ratio (dt/dx for Upwind3, dt/dx^(5/3) for Upwind5 and WENO5) and C_eps
TABLE1 = {
    "coastal_kelvin": {"upwind3": (5e-5, 1.0), "upwind5": (2.5e-4, 1.0), "weno5": (2.5e-4, 1000.0)},
    "inertia_gravity": {"upwind3": (1e-4, 1.0), "upwind5": (1e-3, 1.0), "weno5": (1e-3, 500.0)},
    "barotropic_tide": {"upwind3": (2.5e-4, 1.0), "upwind5": (5e-4, 1.0), "weno5": (5e-4, 1.0)},
    "manufactured": {"upwind3": (5e-5, 1e-4), "upwind5": (5e-3, 1.0), "weno5": (5e-3, 1.0)},
}


def nondim(case: str, H_star: float):
    """(g, H, f, t_ref) of a Section 5 case in nondimensional form."""
    L, U, Hr = SCALES[case]
    return G_STAR * Hr / (U * U), H_star / Hr, F_STAR * L / U, L / U


def table1_dt(case: str, scheme: str, n: int) -> float:
    ratio, _ = TABLE1[case][scheme]
    dx = 1.0 / n
    return ratio * (dx if scheme == "upwind3" else dx ** (5.0 / 3.0))


def _sinc(z: float) -> float:
    return math.sin(z) / z if z != 0.0 else 1.0


def plane_factors(n: int, kx: float, ky: float, phase: float, a: float, b: float):
    """Exact cell averages of a cos(th) + b sin(th), th = kx x + ky y - phase, on the n x n grid
    of the unit square, as two factor columns each: field = X @ Y.T.

    cos(th) = cx cy - sx sy and sin(th) = sx cy + cx sy with cx = cos(kx x - phase),
    sx = sin(kx x - phase), cy = cos(ky y), sy = sin(ky y); the average of cos or sin of
    k t + c over a cell of side h is sinc(k h/2) times its value at the centre."""
    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    fx, fy = _sinc(kx * h / 2.0), _sinc(ky * h / 2.0)
    cx, sx = fx * np.cos(kx * xc - phase), fx * np.sin(kx * xc - phase)
    cy, sy = fy * np.cos(ky * xc), fy * np.sin(ky * xc)
    X = np.stack([cx, sx], axis=1)
    Y = np.stack([a * cy + b * sy, b * cy - a * sy], axis=1)
    return X, Y


def inertia_gravity_exact(n: int, t: float, f: float, g: float, H: float,
                          modes=((0.5, 1.0), (1.0, 2.0))):
    """Section 5.2's inertia-gravity wave at nondimensional time t: for every mode
    (amplitude, wavenumber multiple m), k = (2 pi m, 2 pi m) and w = sqrt(g H |k|^2 + f^2),
      eta = a cos(th),
      u = g a / (w^2 - f^2) (w kx cos(th) - f ky sin(th)),
      v = g a / (w^2 - f^2) (w ky cos(th) + f kx sin(th)),   th = kx x + ky y - w t.
    Returns three lists of (X, Y) factor pairs (one per variable) of the exact cell averages."""
    out = [([], []), ([], []), ([], [])]
    for amp, m in modes:
        kx = ky = 2.0 * math.pi * m
        w = math.sqrt(g * H * (kx * kx + ky * ky) + f * f)
        s = g * amp / (w * w - f * f)
        for var, (a, b) in enumerate(((amp, 0.0), (s * w * kx, -s * f * ky),
                                      (s * w * ky, s * f * kx))):
            X, Y = plane_factors(n, kx, ky, w * t, a, b)
            out[var][0].append(X)
            out[var][1].append(Y)
    return [(np.concatenate(X, axis=1), np.concatenate(Y, axis=1)) for X, Y in out]


def inertia_gravity(n: int = 1280, scheme: str = "upwind5", rmax: int = 16,
                    t0: float = 0.0) -> State:
    """Section 5.2: linear SWE, doubly periodic, f != 0; two modes with eta amplitudes 0.1 m and
    0.2 m and wavenumbers (2 pi/L)(1, 1) and (2 pi/L)(2, 2), L = 1e7 m, H = 1000 m, to T = 3 h.
    The time step follows Table 1 for the scheme, meta carries f, C_eps and the final time."""
    g, H, f, t_ref = nondim("inertia_gravity", 1000.0)
    Lr, Ur, Hr = SCALES["inertia_gravity"]
    modes = ((0.1 / Hr, 1.0), (0.2 / Hr, 2.0))
    fac = inertia_gravity_exact(n, t0, f, g, H, modes)
    tt = [compress(X, Y, 1e-15, rmax) for X, Y in fac]
    fields = [X @ Y.T for X, Y in fac]
    meta = {"f": f, "c_eps": TABLE1["inertia_gravity"][scheme][1], "scheme": scheme,
            "T": 3.0 * 3600.0 / t_ref, "t0": t0, "modes": modes, "t_ref": t_ref,
            "ranks": [t.rank for t in tt]}
    return State("inertia_gravity", n, False, True, g, H, fields, tt,
                 table1_dt("inertia_gravity", scheme, n), meta)


# ---------------------------------------------------------------------------
# boundary data and forcing as separable terms with a harmonic time factor


@dataclasses.dataclass
class Term:
    """amp cos(omega t + phase) X (x) Y (y) added to variable `var`.

    where = "forcing": X (n cells along x), Y (n cells along y), added to L.
    where = "x_lo" / "x_hi": ghost cells -3, -2, -1 / n, n+1, n+2 along x (X, 3 values,
    ascending) times Y (n cells along y).  "y_lo" / "y_hi": X (n cells along x) times the
    ghost cells along y (Y, 3 values)."""
    var: int
    where: str
    amp: float
    omega: float
    phase: float
    X: np.ndarray
    Y: np.ndarray


def _cells(n: int, lo: int, hi: int):
    """Left and right edges of cells lo .. hi-1 of an n-cell unit interval."""
    h = 1.0 / n
    i = np.arange(lo, hi)
    return i * h, (i + 1) * h


def _avg_trig(n: int, k: float, lo: int, hi: int):
    """Exact cell averages of (cos(k x), sin(k x)) over cells lo .. hi-1."""
    a, b = _cells(n, lo, hi)
    if k == 0.0:
        return np.ones(hi - lo), np.zeros(hi - lo)
    h = 1.0 / n
    return (np.sin(k * b) - np.sin(k * a)) / (k * h), (np.cos(k * a) - np.cos(k * b)) / (k * h)


def _avg_exp(n: int, R: float, lo: int, hi: int):
    """Exact cell averages of exp(-x / R) over cells lo .. hi-1."""
    a, b = _cells(n, lo, hi)
    return R * (np.exp(-a / R) - np.exp(-b / R)) * n


@dataclasses.dataclass
class Case:
    """A Section 5 case: initial state, boundary kinds per axis, separable ghost/forcing terms
    and the exact cell averages at time t (for the accuracy checks)."""
    state: State
    bc: tuple
    terms: list
    exact: object          # t -> list of three (n, n) arrays
    T: float               # final time (nondimensional)


def _factored_state(name, n, nonlinear, bc, g, H, factors, dt, meta, rmax):
    tt = [compress(X, Y, 1e-15, rmax) if X is not None else _zero(n) for X, Y in factors]
    fields = [X @ Y.T if X is not None else np.zeros((n, n)) for X, Y in factors]
    return State(name, n, nonlinear, bc == ("periodic", "periodic"), g, H, fields, tt, dt, meta)


def coastal_kelvin(n: int = 1280, scheme: str = "upwind5", rmax: int = 16) -> Case:
    """Section 5.1: linear SWE, L = 5e6 m, H = 1000 m, R = c/f; two modes
    eta = -H eta_m sin(k_m (y + c t)) exp(-x/R), u = 0, v = sqrt(g H) eta_m sin(...) exp(-x/R)
    with eta_1 = eta_2/2 = 1e-4 and k_1 = k_2/2 = 2 pi/L (the second mode takes k_2, the paper's
    formula repeats k_1); x boundaries from the exact solution, y periodic; T = 3 hours."""
    g, H, f, t_ref = nondim("coastal_kelvin", 1000.0)
    Lr, Ur, Hr = SCALES["coastal_kelvin"]
    c = math.sqrt(g * H)
    R = c / f
    modes = [(1e-4, 2.0 * math.pi), (2e-4, 4.0 * math.pi)]
    # nondimensional amplitudes of eta and v per mode
    amps = [(-1000.0 * e / Hr, 100.0 * e / Ur, k) for e, k in modes]

    def factors(t, lo=0, hi=None):
        hi = n if hi is None else hi
        ex = _avg_exp(n, R, lo, hi)
        out = {0: ([], []), 2: ([], [])}
        for ae, av, k in amps:
            cy, sy = _avg_trig(n, k, 0, n)
            # sin(k (y + c t)) = sin(k y) cos(k c t) + cos(k y) sin(k c t)
            prof = sy * math.cos(k * c * t) + cy * math.sin(k * c * t)
            for var, a in ((0, ae), (2, av)):
                out[var][0].append(a * ex)
                out[var][1].append(prof)
        return out

    def exact(t):
        fac = factors(t)
        return [np.stack(fac[0][0], 1) @ np.stack(fac[0][1], 1).T, np.zeros((n, n)),
                np.stack(fac[2][0], 1) @ np.stack(fac[2][1], 1).T]

    terms = []
    for side, (lo, hi) in (("x_lo", (-NG_CELLS, 0)), ("x_hi", (n, n + NG_CELLS))):
        ex = _avg_exp(n, R, lo, hi)
        for ae, av, k in amps:
            cy, sy = _avg_trig(n, k, 0, n)
            for var, a in ((0, ae), (2, av)):
                terms.append(Term(var, side, a, k * c, 0.0, ex, sy))              # sin ky cos wt
                terms.append(Term(var, side, a, k * c, -0.5 * math.pi, ex, cy))   # cos ky sin wt
    fac0 = factors(0.0)
    fx = [(np.stack(fac0[0][0], 1), np.stack(fac0[0][1], 1)), (None, None),
          (np.stack(fac0[2][0], 1), np.stack(fac0[2][1], 1))]
    ratio, c_eps = TABLE1["coastal_kelvin"][scheme]
    st = _factored_state("coastal_kelvin", n, False, ("exact", "periodic"), g, H, fx,
                         table1_dt("coastal_kelvin", scheme, n),
                         {"f": f, "c_eps": c_eps, "scheme": scheme, "t_ref": t_ref}, rmax)
    return Case(st, ("exact", "periodic"), terms, exact, 3.0 * 3600.0 / t_ref)


def barotropic_tide(n: int = 1280, scheme: str = "upwind5", rmax: int = 16) -> Case:
    """Section 5.3: linear SWE, L = 25e4 m, H = 200 m; two modes
    eta = eta_m cos(k_m x) cos(w_m t), u = g eta_m w_m k_m / (w_m^2 - f^2) sin(k_m x) sin(w_m t),
    v = g eta_m f k_m / (w_m^2 - f^2) sin(k_m x) cos(w_m t), w_m = sqrt(g H k_m^2 + f^2) (the
    paper's w-hat read as w), eta_1 = eta_2/2 = 0.2 m, k_m = 2 pi / lambda_m with
    lambda_1 = 4L/5, lambda_2 = 4L/9; x boundaries from the exact solution, y periodic;
    T = 30 minutes."""
    g, H, f, t_ref = nondim("barotropic_tide", 200.0)
    Lr, Ur, Hr = SCALES["barotropic_tide"]
    modes = [(0.2 / Hr, 2.0 * math.pi * 5.0 / 4.0), (0.4 / Hr, 2.0 * math.pi * 9.0 / 4.0)]
    ones = np.ones(n)
    spec = []     # (var, amplitude, k, x function "cos"/"sin", omega, phase)
    for a, k in modes:
        w = math.sqrt(g * H * k * k + f * f)
        s = g * a / (w * w - f * f)
        spec.append((0, a, k, 0, w, 0.0))
        spec.append((1, s * w * k, k, 1, w, -0.5 * math.pi))
        spec.append((2, s * f * k, k, 1, w, 0.0))

    def exact(t):
        out = [np.zeros((n, n)) for _ in range(3)]
        for var, a, k, fx, w, ph in spec:
            out[var] += a * math.cos(w * t + ph) * np.outer(_avg_trig(n, k, 0, n)[fx], ones)
        return out

    terms = []
    for side, (lo, hi) in (("x_lo", (-NG_CELLS, 0)), ("x_hi", (n, n + NG_CELLS))):
        for var, a, k, fx, w, ph in spec:
            terms.append(Term(var, side, a, w, ph, _avg_trig(n, k, lo, hi)[fx], ones))
    fac = []
    for var in range(3):
        cols = [(a if ph == 0.0 else 0.0) * _avg_trig(n, k, 0, n)[fx]
                for v, a, k, fx, w, ph in spec if v == var]
        X = np.stack(cols, 1)
        fac.append((X, np.ones((n, X.shape[1]))) if np.any(X) else (None, None))
    ratio, c_eps = TABLE1["barotropic_tide"][scheme]
    st = _factored_state("barotropic_tide", n, False, ("exact", "periodic"), g, H, fac,
                         table1_dt("barotropic_tide", scheme, n),
                         {"f": f, "c_eps": c_eps, "scheme": scheme, "t_ref": t_ref}, rmax)
    return Case(st, ("exact", "periodic"), terms, exact, 30.0 * 60.0 / t_ref)


def _theta_series(fun, mmax: int = 4, samples: int = 32):
    """Fourier coefficients (a_m, b_m), m = 0..mmax, of a trigonometric polynomial of theta:
    fun(th) = sum a_m cos(m th) + b_m sin(m th), from equispaced samples (numpy FFT)."""
    th = 2.0 * math.pi * np.arange(samples) / samples
    F = np.fft.rfft(fun(th)) / samples
    a = [float(F[0].real)] + [float(2.0 * F[m].real) for m in range(1, mmax + 1)]
    b = [0.0] + [float(-2.0 * F[m].imag) for m in range(1, mmax + 1)]
    return a, b


def manufactured(n: int = 1280, scheme: str = "upwind5", rmax: int = 32) -> Case:
    """Section 5.4: nonlinear SWE, periodic, L = 1e7 m; h = H + eta with
    eta = eta_hat sin(th), u = u_hat cos(th), v = 0, th = kx x + ky y - w t, kx = ky = 2 pi/L,
    w = c |k| (c = sqrt(g H), H = 1000 m), eta_hat = 1e-2 m, u_hat = 1e-2 m/s; T = 3 hours.
    The forcing dQ/dt + dF/dx + dG/dy - S (S the Coriolis source) depends on th only; it is a
    trigonometric polynomial of degree 3, expanded by FFT of its complex-step values, and each
    harmonic becomes separable terms with exact cell averages."""
    g, H, f, t_ref = nondim("manufactured", 1000.0)
    Lr, Ur, Hr = SCALES["manufactured"]
    a, b = 1e-2 / Hr, 1e-2 / Ur
    kx = ky = 2.0 * math.pi
    w = math.sqrt(g * H * (kx * kx + ky * ky))

    def Q(th):
        h = H + a * np.sin(th)
        return [h, h * b * np.cos(th), 0.0 * th]

    def FG(th):
        h, hu, hv = Q(th)
        F = [hu, hu * hu / h + 0.5 * g * h * h, hu * hv / h]
        G = [hv, hu * hv / h, hv * hv / h + 0.5 * g * h * h]
        return F, G

    def forcing(var):
        def fun(th):
            d = 1e-30
            z = th + 1j * d
            dq = np.imag(Q(z)[var]) / d
            F, G = FG(z)
            dF, dG = np.imag(F[var]) / d, np.imag(G[var]) / d
            h, hu, hv = Q(th)
            S = [0.0 * th, f * hv, -f * hu][var]
            return -w * dq + kx * dF + ky * dG - S
        return fun

    def plane(m, t, c_cos, c_sin):
        """Separable factors of c_cos cos(m th) + c_sin sin(m th) at time t (cell averages)."""
        X, Y = plane_factors(n, m * kx, m * ky, m * w * t, c_cos, c_sin)
        return X, Y

    terms = []
    for var in range(3):
        ac, bs = _theta_series(forcing(var))
        for m in range(len(ac)):
            if abs(ac[m]) + abs(bs[m]) < 1e-300:
                continue
            if m == 0:
                terms.append(Term(var, "forcing", ac[0], 0.0, 0.0, np.ones(n), np.ones(n)))
                continue
            # cos(m th) = cos(m phi) cos(m w t) + sin(m phi) sin(m w t), phi = kx x + ky y;
            # sin(m th) = sin(m phi) cos(m w t) - cos(m phi) sin(m w t)
            cxs, sxs = _avg_trig(n, m * kx, 0, n)
            cys, sys_ = _avg_trig(n, m * ky, 0, n)
            cosphi = [(cxs, cys, 1.0), (sxs, sys_, -1.0)]      # cos(mphi) = cx cy - sx sy
            sinphi = [(sxs, cys, 1.0), (cxs, sys_, 1.0)]       # sin(mphi) = sx cy + cx sy
            om = m * w
            for (X, Y, sg) in cosphi:
                terms.append(Term(var, "forcing", sg * ac[m], om, 0.0, X, Y))
                terms.append(Term(var, "forcing", -sg * bs[m], om, -0.5 * math.pi, X, Y))
            for (X, Y, sg) in sinphi:
                terms.append(Term(var, "forcing", sg * ac[m], om, -0.5 * math.pi, X, Y))
                terms.append(Term(var, "forcing", sg * bs[m], om, 0.0, X, Y))

    def exact(t):
        Xh, Yh = plane(1, t, 0.0, a)
        Xu, Yu = plane(1, t, 1.0, 0.0)
        hfield = H + Xh @ Yh.T
        # h u = H u_hat cos(th) + a u_hat sin(th) cos(th) = H u_hat cos(th) + a u_hat/2 sin(2 th)
        X1, Y1 = plane(1, t, H * b, 0.0)
        X2, Y2 = plane(2, t, 0.0, 0.5 * a * b)
        return [hfield, X1 @ Y1.T + X2 @ Y2.T, np.zeros((n, n))]

    Xh, Yh = plane(1, 0.0, 0.0, a)
    X1, Y1 = plane(1, 0.0, H * b, 0.0)
    X2, Y2 = plane(2, 0.0, 0.0, 0.5 * a * b)
    fac = [(np.concatenate([np.full((n, 1), H), Xh], 1), np.concatenate([np.ones((n, 1)), Yh], 1)),
           (np.concatenate([X1, X2], 1), np.concatenate([Y1, Y2], 1)), (None, None)]
    ratio, c_eps = TABLE1["manufactured"][scheme]
    st = _factored_state("manufactured", n, True, ("periodic", "periodic"), g, H, fac,
                         table1_dt("manufactured", scheme, n),
                         {"f": f, "c_eps": c_eps, "scheme": scheme, "t_ref": t_ref}, rmax)
    return Case(st, ("periodic", "periodic"), terms, exact, 3.0 * 3600.0 / t_ref)


NG_CELLS = 3

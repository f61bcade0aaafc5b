"""Exact linear reconstruction weights for the finite-volume scheme (Section 2.3).

Oracle (test infrastructure only).

Every weight used by the upwind and WENO reconstructions is the value, at a point x0 of
cell j = [-1/2, 1/2] (cell units), of the polynomial whose averages over a set of cells
equal the given cell averages.  With cells at integer offsets o_l, the weights c solve

    sum_l c_l * avg_{[o_l - 1/2, o_l + 1/2]} (y^p) = x0^p,   p = 0 .. len(o) - 1.

Step 1 of Section 2.3 evaluates at the face x0 = 1/2; Step 2 evaluates at the Gauss-Legendre
points (2 points, x0 = -/+ 1/(2 sqrt 3), for the 3rd-order scheme; 3 points,
x0 = -sqrt(15)/10, 0, +sqrt(15)/10, for the 5th-order schemes), listed in ascending order,
so quadrature point m = 1 is the lower one.

The Gauss-Legendre points are irrational, so all weights live in Q(sqrt D); they are kept
exact as pairs of Fractions (a + b sqrt D) and converted to float64 only at the end.  The
printed rational matrices of Section 2.3 are approximations of these values (they differ
by up to ~2e-6); the tests compare the two.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr


class QSqrt:
    """Number a + b*sqrt(D) with rational a, b (fixed squarefree D >= 1, or b == 0)."""

    __slots__ = ("a", "b", "D")

    def __init__(self, a, b=0, D=1):
        self.a, self.b, self.D = Fr(a), Fr(b), int(D)

    def _co(self, o):
        if isinstance(o, QSqrt):
            if o.b != 0 and self.b != 0 and o.D != self.D:
                raise ValueError("mixed radicands")
            D = self.D if self.b != 0 else o.D
            return o.a, o.b, D
        return Fr(o), Fr(0), self.D

    def __add__(self, o):
        a, b, D = self._co(o)
        return QSqrt(self.a + a, self.b + b, D)

    __radd__ = __add__

    def __neg__(self):
        return QSqrt(-self.a, -self.b, self.D)

    def __sub__(self, o):
        return self + (-o if isinstance(o, QSqrt) else QSqrt(-Fr(o)))

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        a, b, D = self._co(o)
        return QSqrt(self.a * a + self.b * b * D, self.a * b + self.b * a, D)

    __rmul__ = __mul__

    def __truediv__(self, o):
        a, b, D = self._co(o)
        den = a * a - b * b * D
        if den == 0:
            raise ZeroDivisionError
        num = self * QSqrt(a, -b, D)
        return QSqrt(num.a / den, num.b / den, D)

    def __rtruediv__(self, o):
        return QSqrt(o, 0, self.D) / self

    def is_zero(self):
        return self.a == 0 and self.b == 0

    def __float__(self):
        return float(self.a) + float(self.b) * math.sqrt(self.D)

    def __repr__(self):
        return f"({self.a} + {self.b}*sqrt({self.D}))"


def _avg_power(lo: Fr, hi: Fr, p: int) -> Fr:
    """Average of y^p over [lo, hi]."""
    return (hi ** (p + 1) - lo ** (p + 1)) / ((p + 1) * (hi - lo))


def _solve(M, rhs):
    """Gaussian elimination over QSqrt numbers (small dense systems)."""
    n = len(M)
    A = [[M[i][j] for j in range(n)] + [rhs[i]] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if not A[r][c].is_zero())
        A[c], A[piv] = A[piv], A[c]
        for r in range(n):
            if r != c and not A[r][c].is_zero():
                f = A[r][c] / A[c][c]
                A[r] = [A[r][k] - f * A[c][k] for k in range(n + 1)]
    return [A[i][n] / A[i][i] for i in range(n)]


def point_weights(offsets, x0: QSqrt):
    """Weights c_l (QSqrt) so that sum_l c_l * avg_l equals the polynomial value at x0."""
    n = len(offsets)
    # rows: moment p; columns: cell l  (transpose of the cell/moment matrix)
    M = [[QSqrt(_avg_power(Fr(o) - Fr(1, 2), Fr(o) + Fr(1, 2), p)) for o in offsets]
         for p in range(n)]
    rhs = []
    xp = QSqrt(1)
    for p in range(n):
        rhs.append(xp)
        xp = xp * x0
    return _solve(M, rhs)


# Gauss-Legendre points (cell units, ascending) and weights  (R2 reading)
def gauss_points(nq: int):
    if nq == 2:
        return [QSqrt(0, Fr(-1, 6), 3), QSqrt(0, Fr(1, 6), 3)], [Fr(1, 2), Fr(1, 2)]
    if nq == 3:
        return ([QSqrt(0, Fr(-1, 10), 15), QSqrt(0), QSqrt(0, Fr(1, 10), 15)],
                [Fr(5, 18), Fr(8, 18), Fr(5, 18)])
    raise ValueError(nq)


def substencil_offsets(k: int, r: int):
    """Cells of candidate stencil r for order 2k+1: j-r .. j-r+k (Section 2.3, Step 2)."""
    return list(range(-r, -r + k + 1))


def substencil_matrix(k: int, x0: QSqrt):
    """C[r][l]: weight of cell j-r+l in candidate stencil r at point x0."""
    return [point_weights(substencil_offsets(k, r), x0) for r in range(k + 1)]


def full_stencil(k: int, x0: QSqrt):
    """Weights of the (2k+1)-cell polynomial value at x0 on offsets -k..k."""
    return point_weights(list(range(-k, k + 1)), x0)


def linear_weights(k: int, x0: QSqrt):
    """gamma_r with sum_r gamma_r C_r == full (2k+1)-cell stencil (embedded on -k..k)."""
    C = substencil_matrix(k, x0)
    F = full_stencil(k, x0)
    if k == 1:
        # offsets -1..1: stencil 0 covers (0, 1), stencil 1 covers (-1, 0)
        g0 = F[2] / C[0][1]
        g1 = F[0] / C[1][0]
        return [g0, g1]
    # k == 2: offset +2 only in stencil 0 (its last cell), offset -2 only in stencil 2
    g0 = F[4] / C[0][2]
    g2 = F[0] / C[2][0]
    g1 = QSqrt(1) - g0 - g2
    return [g0, g1, g2]


def split_weights(gammas):
    """Positive/negative split of linear weights (treatment of negative weights, Section 2.3).

    gamma^+ = (gamma + theta |gamma|)/2 with theta = 3, gamma^- = gamma^+ - gamma;
    sigma^+- = sum gamma^+-, normalised weights gamma^+- / sigma^+-.
    Returns (gp_normalised, gm_normalised, sigma_p, sigma_m) as floats.
    """
    g = [float(x) for x in gammas]
    gp = [(x + 3.0 * abs(x)) / 2.0 for x in g]
    gm = [p - x for p, x in zip(gp, g)]
    sp, sm = sum(gp), sum(gm)
    return [x / sp for x in gp], [x / sm for x in gm], sp, sm


def split_weights_exact(gammas):
    """Exact rational version of split_weights for rational gammas."""
    g = [x.a for x in gammas]
    assert all(x.b == 0 for x in gammas)
    gp = [(x + 3 * abs(x)) / 2 for x in g]
    gm = [p - x for p, x in zip(gp, g)]
    sp, sm = sum(gp), sum(gm)
    return [x / sp for x in gp], [x / sm for x in gm], sp, sm


def to_float(v):
    if isinstance(v, list):
        return [to_float(x) for x in v]
    return float(v)


def scheme_order(scheme: str) -> int:
    return {"upwind3": 1, "upwind5": 2, "weno5": 2}[scheme]


def tables(scheme: str) -> dict:
    """All float64 constants one scheme needs."""
    k = scheme_order(scheme)
    nq = 2 if k == 1 else 3
    face = QSqrt(Fr(1, 2))
    pts, wts = gauss_points(nq)
    out = {
        "k": k,
        "nq": nq,
        "gl_points": [float(p) for p in pts],
        "gl_weights": [float(w) for w in wts],
        "face_sub": to_float(substencil_matrix(k, face)),        # Step 1 candidate stencils
        "face_full": to_float(full_stencil(k, face)),             # combined face stencil
        "face_gamma": to_float(linear_weights(k, face)),          # ideal weights d_r
        "quad_sub": [to_float(substencil_matrix(k, p)) for p in pts],
        "quad_full": [to_float(full_stencil(k, p)) for p in pts],
        "quad_gamma": [to_float(linear_weights(k, p)) for p in pts],
    }
    return out

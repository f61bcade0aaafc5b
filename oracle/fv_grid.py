"""Plain full-grid high-order finite-volume solver for the 2-D shallow water equations.

Oracle (test infrastructure only).

This is the scheme of Sections 2.1-2.4 written out on N x N arrays of cell averages,
with no tensor-train compression:

  * governing equations, linear (eta, u, v) and nonlinear (h, hu, hv), flat bottom,
    Coriolis parameter f (Section 2.1, equations "linear-SWE" and "nonlinear-SWE");
  * dimension-by-dimension reconstruction (Section 2.3): Step 1 "de-cell averages"
    along the flux direction to the faces, Step 2 along the other direction to the
    Gauss-Legendre points; Upwind3 (2 points), Upwind5 and WENO5 (3 points, negative
    weights at the middle point treated by the positive/negative split);
  * local Lax-Friedrichs flux at every face quadrature point and the Gauss-Legendre
    face sum (Section 2.2, 2.4);
  * flux differences (T - 1)F/dx (Section 4.1) and the SSP-RK3 step (Section 4.4 with
    rounding replaced by the identity).

Boundaries, per axis: periodic; reflective walls; or "exact", where the ghost cells hold
given values (the exact solution's cell averages, Section 5's Kelvin wave and barotropic
tide).  Boundary values and forcing come as separable terms with a harmonic time factor,
amp cos(omega t + phase) X(.) Y(.) (see ghost_values and forcing_values); at most one axis is
"exact".  The field is first extended by NG ghost cells along the exact axis (or along x),
then along the other axis, so corner cells follow the second axis's rule.

Array layout: index [i, j] = (x cell, y cell).  Faces along an axis are numbered by the
cell on their right: face f is the left face of cell f.  Periodic axes have N faces,
other axes N + 1.  Readings where the paper is silent (ghost cells at walls, the
LLF eigenvalue, the quadrature ordering) are those listed in the design notes: reflective
walls mirror three ghost cells with the sign of the normal momentum flipped; the LLF
eigenvalue is max(|u-| + sqrt(g h-), |u+| + sqrt(g h+)) pointwise; quadrature points are
in ascending order along the face.
"""
from __future__ import annotations

import math

import numpy as np

from . import stencils

NG = 3  # ghost cells per side


def pad(v: np.ndarray, axis: int, periodic, sign: float, lo=None, hi=None) -> np.ndarray:
    """Extend v by NG ghost cells on both ends of `axis`: periodic wrap (periodic True or
    "periodic"), mirror times sign (False or "wall"), or the given ghost blocks lo, hi
    ("exact"; NG cells each, ascending cell index, the axis first)."""
    kind = periodic if isinstance(periodic, str) else ("periodic" if periodic else "wall")
    v = np.moveaxis(v, axis, 0)
    if kind == "periodic":
        out = np.concatenate([v[-NG:], v, v[:NG]], axis=0)
    elif kind == "wall":
        left = sign * v[:NG][::-1]
        right = sign * v[-NG:][::-1]
        out = np.concatenate([left, v, right], axis=0)
    elif kind == "exact":
        out = np.concatenate([lo, v, hi], axis=0)
    else:
        raise ValueError(f"unknown boundary kind {kind!r}")
    return np.moveaxis(out, 0, axis)


def time_factor(term, t: float) -> float:
    return term.amp * math.cos(term.omega * t + term.phase)


def ghost_values(terms, var: int, where: str, t: float) -> np.ndarray:
    """Sum of the separable ghost terms of one variable and side at time t, with the
    boundary's normal axis first: (NG, n).  x sides: X holds the NG ghost cells (ascending),
    Y the n cells along y; y sides: Y holds the ghost cells, X the n cells along x."""
    out = None
    for tm in terms:
        if tm.var != var or tm.where != where:
            continue
        if where.startswith("x"):
            blk = time_factor(tm, t) * np.outer(tm.X, tm.Y)
        else:
            blk = time_factor(tm, t) * np.outer(tm.Y, tm.X)
        out = blk if out is None else out + blk
    return out


def forcing_values(terms, var: int, t: float, n: int) -> np.ndarray:
    """Sum of the separable forcing terms of one variable at time t: (n, n)."""
    out = np.zeros((n, n))
    for tm in terms:
        if tm.var == var and tm.where == "forcing":
            out = out + time_factor(tm, t) * np.outer(tm.X, tm.Y)
    return out


# ---------------------------------------------------------------------------
# 1-D reconstructions on a padded line (axis 0 = line, trailing axes = batch)

def _smoothness(vm2, vm1, v0, vp1, vp2):
    """WENO5 smoothness indicators beta_0..beta_2 about cell v0 (Section 2.3)."""
    b0 = 13.0 / 12.0 * (v0 - 2 * vp1 + vp2) ** 2 + 0.25 * (3 * v0 - 4 * vp1 + vp2) ** 2
    b1 = 13.0 / 12.0 * (vm1 - 2 * v0 + vp1) ** 2 + 0.25 * (vm1 - vp1) ** 2
    b2 = 13.0 / 12.0 * (vm2 - 2 * vm1 + v0) ** 2 + 0.25 * (vm2 - 4 * vm1 + 3 * v0) ** 2
    return [b0, b1, b2]


def _nonlinear_weights(gam, beta, eps):
    alpha = [g / (b + eps) ** 2 for g, b in zip(gam, beta)]
    s = alpha[0] + alpha[1] + alpha[2]
    return [a / s for a in alpha]


def _candidates(vals, C, k):
    """v^(r) = sum_l C[r][l] v_{c-r+l}; vals maps offset -> array."""
    return [sum(C[r][l] * vals[-r + l] for l in range(k + 1)) for r in range(k + 1)]


def recon_point(vals, tab, which, scheme, eps):
    """Value at one point of cell c from neighbour averages vals[o] (o = -k..k).

    which = "face" (x0 = +1/2, Step 1) or an integer m (Gauss point index, Step 2).
    """
    k = tab["k"]
    if which == "face":
        C, gam = tab["face_sub"], tab["face_gamma"]
    else:
        C, gam = tab["quad_sub"][which], tab["quad_gamma"][which]
    cand = _candidates(vals, C, k)
    negative = min(gam) < 0.0
    if scheme != "weno5":
        if negative:
            gp, gm, sp, sm = stencils.split_weights(gam)
            up = sum(g * c for g, c in zip(gp, cand))
            um = sum(g * c for g, c in zip(gm, cand))
            return sp * up - sm * um
        return sum(g * c for g, c in zip(gam, cand))
    beta = _smoothness(vals[-2], vals[-1], vals[0], vals[1], vals[2])
    if negative:
        gp, gm, sp, sm = stencils.split_weights(gam)
        wp = _nonlinear_weights(gp, beta, eps)
        wm = _nonlinear_weights(gm, beta, eps)
        up = sum(w * c for w, c in zip(wp, cand))
        um = sum(w * c for w, c in zip(wm, cand))
        return sp * up - sm * um
    w = _nonlinear_weights(gam, beta, eps)
    return sum(wi * c for wi, c in zip(w, cand))


def faces_1d(P: np.ndarray, n_faces: int, tab, scheme, eps):
    """Step 1 along axis 0 of the padded array P: (u_minus, u_plus) at faces 0..n_faces-1.

    u_minus at face f: right-face value of cell f-1; u_plus: left-face value of cell f,
    obtained by applying the same formula to the mirrored neighbour sequence.
    """
    k = tab["k"]

    def sl(start):  # cells start .. start + n_faces - 1 (unpadded index), as padded slice
        return P[NG + start: NG + start + n_faces]

    minus_vals = {o: sl(-1 + o) for o in range(-k, k + 1)}
    plus_vals = {o: sl(0 - o) for o in range(-k, k + 1)}      # mirrored about cell f
    um = recon_point(minus_vals, tab, "face", scheme, eps)
    up = recon_point(plus_vals, tab, "face", scheme, eps)
    return um, up


def quad_1d(P: np.ndarray, n: int, tab, scheme, eps):
    """Step 2 along axis 0 of the padded array P: values at the Gauss points, shape (n, ..., nq)."""
    k = tab["k"]
    vals = {o: P[NG + o: NG + o + n] for o in range(-k, k + 1)}
    out = [recon_point(vals, tab, m, scheme, eps) for m in range(tab["nq"])]
    return np.stack(out, axis=-1)


# ---------------------------------------------------------------------------
# fluxes

def physical_flux(U, nonlinear: bool, g: float, H: float, direction: int):
    """F (direction 0) or G (direction 1) of Section 2.1."""
    if nonlinear:
        h, hu, hv = U
        if direction == 0:
            return [hu, hu * hu / h + 0.5 * g * h * h, hu * hv / h]
        return [hv, hu * hv / h, hv * hv / h + 0.5 * g * h * h]
    eta, u, v = U
    z = np.zeros_like(eta)
    if direction == 0:
        return [H * u, g * eta, z]
    return [H * v, z, g * eta]


def llf_eigenvalue(Um, Up, nonlinear: bool, g: float, H: float, direction: int):
    if not nonlinear:
        return math.sqrt(g * H)
    mom = 1 + direction
    lm = np.abs(Um[mom] / Um[0]) + np.sqrt(g * Um[0])
    lp = np.abs(Up[mom] / Up[0]) + np.sqrt(g * Up[0])
    return np.maximum(lm, lp)


def llf(Um, Up, nonlinear, g, H, direction):
    """Local Lax-Friedrichs flux (Section 2.2, equation LLF, and Section 2.4)."""
    Fm = physical_flux(Um, nonlinear, g, H, direction)
    Fp = physical_flux(Up, nonlinear, g, H, direction)
    lam = llf_eigenvalue(Um, Up, nonlinear, g, H, direction)
    return [0.5 * (fm + fp) - 0.5 * lam * (up - um) for fm, fp, um, up in zip(Fm, Fp, Um, Up)]


# ---------------------------------------------------------------------------

class GridSolver:
    """Full-grid FV right-hand side and SSP-RK3 step."""

    def __init__(self, n: int, scheme: str, nonlinear: bool, periodic: bool = True,
                 g: float = 9.81, H: float = 1.0, f: float = 0.0, length: float = 1.0,
                 source=None, bc=None, terms=()):
        self.n, self.scheme, self.nonlinear = n, scheme, nonlinear
        self.g, self.H, self.f = g, H, f
        self.dx = length / n
        self.tab = stencils.tables(scheme)
        # boundary kind per axis (x, y): "periodic", "wall" or "exact"
        self.bc = tuple(bc) if bc is not None else \
            (("periodic", "periodic") if periodic else ("wall", "wall"))
        if any(b not in ("periodic", "wall", "exact") for b in self.bc) or \
                self.bc.count("exact") > 1:
            raise ValueError(f"bad boundary kinds {self.bc}")
        self.n_faces_axis = [n if b == "periodic" else n + 1 for b in self.bc]
        self.source = source  # optional callable t -> list of 3 arrays (manufactured forcing)
        self.terms = list(terms)  # separable ghost and forcing terms

    # reflection signs (normal momentum flips)
    @staticmethod
    def signs(direction: int):
        return (1.0, -1.0, 1.0) if direction == 0 else (1.0, 1.0, -1.0)

    def padded(self, v, c: int, t: float):
        """Variable c extended by NG ghost cells along both axes, (n + 6) x (n + 6): the exact
        axis first (x when none is exact), then the other; walls negate the momentum normal
        to them."""
        first = 1 if self.bc[1] == "exact" else 0
        P = v
        for axis in (first, 1 - first):
            kind = self.bc[axis]
            lo = hi = None
            if kind == "exact":
                side = "x" if axis == 0 else "y"
                lo = ghost_values(self.terms, c, side + "_lo", t)
                hi = ghost_values(self.terms, c, side + "_hi", t)
                if lo is None or hi is None:
                    lo = np.zeros((NG, self.n)) if lo is None else lo
                    hi = np.zeros((NG, self.n)) if hi is None else hi
            P = pad(P, axis, kind, self.signs(axis)[c], lo, hi)
        return P

    def face_states(self, U, direction: int, t: float = 0.0):
        """(U_minus, U_plus), each a list of 3 arrays of shape (n_faces, n, nq) for x,
        (n, n_faces, nq) for y; the trailing axis is the quadrature point along the face."""
        tab, eps = self.tab, self.dx * self.dx
        nf = self.n_faces_axis[direction]
        Um, Up = [], []
        for c, v in enumerate(U):
            P = self.padded(v, c, t)
            PP = P if direction == 0 else P.T                     # normal axis first
            fm, fp = faces_1d(PP, nf, tab, self.scheme, eps)      # (nf, n + 6)
            qm = quad_1d(fm.T, self.n, tab, self.scheme, eps)
            qp = quad_1d(fp.T, self.n, tab, self.scheme, eps)
            # q*: (n tangent, n_faces, nq) -> (n_faces, n, nq)
            qm, qp = qm.transpose(1, 0, 2), qp.transpose(1, 0, 2)
            if direction == 1:
                qm, qp = qm.transpose(1, 0, 2), qp.transpose(1, 0, 2)
            Um.append(qm)
            Up.append(qp)
        return Um, Up

    def face_flux(self, U, direction: int, t: float = 0.0):
        """Gauss-Legendre sum of the LLF flux over each face: list of 3 arrays."""
        Um, Up = self.face_states(U, direction, t)
        Fp = llf(Um, Up, self.nonlinear, self.g, self.H, direction)
        w = np.asarray(self.tab["gl_weights"])
        return [np.tensordot(F, w, axes=([2], [0])) for F in Fp]

    def diff(self, Fhat, direction: int):
        """(T - 1) F: value at the right face minus value at the left face of each cell."""
        Fn = Fhat if direction == 0 else Fhat.T
        if self.bc[direction] == "periodic":
            d = np.roll(Fn, -1, axis=0) - Fn
        else:
            d = Fn[1:] - Fn[:-1]
        return d if direction == 0 else d.T

    def rhs(self, U, t: float = 0.0):
        Fx = self.face_flux(U, 0, t)
        Fy = self.face_flux(U, 1, t)
        L = [-(self.diff(fx, 0) + self.diff(fy, 1)) / self.dx for fx, fy in zip(Fx, Fy)]
        if self.f != 0.0:
            L[1] = L[1] + self.f * U[2]
            L[2] = L[2] - self.f * U[1]
        if self.source is not None:
            S = self.source(t)
            L = [l + s for l, s in zip(L, S)]
        if any(tm.where == "forcing" for tm in self.terms):
            L = [l + forcing_values(self.terms, c, t, self.n) for c, l in enumerate(L)]
        return L

    def step(self, U, dt: float, t: float = 0.0):
        """SSP-RK3 (Section 4.4 with round = identity)."""
        L0 = self.rhs(U, t)
        U1 = [u + dt * l for u, l in zip(U, L0)]
        L1 = self.rhs(U1, t + dt)
        U2 = [0.75 * u + 0.25 * (u1 + dt * l) for u, u1, l in zip(U, U1, L1)]
        L2 = self.rhs(U2, t + 0.5 * dt)
        return [u / 3.0 + 2.0 / 3.0 * (u2 + dt * l) for u, u2, l in zip(U, U2, L2)]

    def run(self, U, dt: float, nsteps: int, t0: float = 0.0):
        t = t0
        for _ in range(nsteps):
            U = self.step(U, dt, t)
            t += dt
        return U

"""The tensor-train finite-volume step (Section 4), as a fixed sequence of TT operations.

Oracle (test infrastructure only).

State: three 2-core TTs (x index on the first core, y index on the second), the conserved
variables (eta, u, v) of the linear SWE or (h, hu, hv) of the nonlinear SWE.

Boundaries per axis: periodic, reflective walls, or "exact" (ghost cells from given
separable terms amp cos(omega t + phase) X Y, Section 5's exact-solution boundaries).  On an
exact axis the state's cores are extended by zeros and every ghost term becomes extra rank
columns of the reconstructed TTs: its factor along the exact axis is an explicit (n + 6)
column that is zero inside the domain, its other factor is extended by the other axis's rule,
and both pass through the same stencils (the reconstruction is linear).  Forcing terms add
rank-1 TTs to L.  WENO5: on an exact normal boundary the ghost terms are further columns of
Algorithm 2's fibers; on an exact tangent boundary Algorithm 3 needs the Step-1 face values at
the 6 tangent ghost cells, which are evaluated directly (the field there is the ghost terms
alone) and appended to the Step-1 TT as 6 columns with unit tangent factors at those rows.

One evaluation of L(Q) (Sections 4.1-4.3):

  x direction (the y direction is the same sequence applied to the transposed TTs with the
  two momenta swapped, so the normal momentum always comes second):
    reconstruction  Upwind: the face stencils act on the first core (Step 1, faces),
                    the Gauss-point stencils on the second core (Step 2); the minus and plus
                    states share the second core (Section 4.3.1).
                    WENO5: Algorithm 2 (two crosses over the 5 shifted copies in x) and
                    Algorithm 3 (two crosses over 5 shifted copies in y, all Gauss points at
                    once on the merged column index j*nq + m) (Section 4.3.2).
    flux            linear: the LLF flux assembled directly from the states, no rounding
                    (Section 4.2, lambda = sqrt(gH)).
                    nonlinear, for each side s: 1/h by Algorithm 1 (or by a cross of 1/x, the alternative
                    Section 4.2 names), u = round(hu o 1/h),
                    w = round(hv o 1/h), P1 = round(hu o u), P2 = round(h o h),
                    F2 = round(P1 + g/2 P2), F3 = round(hu o w), F1 = hu;
                    lambda by one cross of max(|hu-/h-| + sqrt(g h-), |hu+/h+| + sqrt(g h+));
                    D_c = round(lambda o (q_c+ - q_c-)); Fhat_c = round((F_c- + F_c+)/2 - D_c/2).
                    Or (flux="lf_cross") the whole LLF flux vector by one cross whose column
                    index carries the component (the LF-cross Section 4.2 contrasts with this).
    finish          Gauss-Legendre sum over the quadrature rows of the second core, and the
                    difference (T - 1) on the first core (Section 4.1).
  L_c = -dF_c/dx - dG_c/dy (+ Coriolis source), a concatenation of cores.

SSP-RK3 (Section 4.4): Q1 = F(Qn), Q2 = round(3/4 Qn + 1/4 F(Q1)),
Qn+1 = round(1/3 Qn + 2/3 F(Q2)), with F(q) = round(q + dt L(q)).  One rank cap rmax serves
every rounding.  Tolerances: either one fixed eps for every rounding, or the rule of Section 4.4
(eps_rule="paper"): at the start of each step, eq. eps-tt-formula gives the tolerance of every
rounding inside L and of the crosses, and eq. modified-eps-tt-formula one tolerance per variable
for that variable's forward-Euler and SSP-RK3 combination roundings (see paper_tolerances).
"""
from __future__ import annotations

import math

import numpy as np

from . import stencils
from . import fv_grid
from .tt import TT, add, cross, hadamard, initial_columns, norm, reciprocal, scale, skeleton, \
    tt_round, zero_tt

NG = 3


def paper_tolerances(norms, n: int, order: int, c_eps: float, volume: float = 1.0):
    """Rounding tolerances of one time step (Section 4.4), from the state's Frobenius norms.

    base = C_eps * V^(1/2) * dx^(p - 1/2), with p the order of the scheme and V the volume of
    the domain (the unit square here, dx = 1/n).
      eq. eps-tt-formula:          eps = base / max_q ||q||, for every rounding except the
                                   time-stepping ones;
      eq. modified-eps-tt-formula: eps_q = min(1e-3, base / ||q||), for the forward-Euler
                                   rounding F(q) and the two SSP-RK3 combinations of q.
    ||q|| is read as the L2 norm of the cell-average field on the domain, the Frobenius norm of
    the n x n array times the cell side dx (cells are square); a state whose norms are all zero
    takes eps = 1e-3, the clip of the modified formula (readings in the design notes).

    Returns (eps, [eps_q for the three variables]).
    """
    dx = 1.0 / n
    base = c_eps * math.sqrt(volume) * dx ** (order - 0.5)
    l2 = [dx * float(v) for v in norms]
    top = max(l2)
    eps = base / top if top > 0.0 else 1e-3
    eps_q = [min(1e-3, base / v) if v > 0.0 else 1e-3 for v in l2]
    return eps, eps_q


# reflection signs in "normal-first" variable order (q0, q_normal, q_tangential)
SIGN_NORMAL = (1.0, -1.0, 1.0)
SIGN_TANGENT = (1.0, 1.0, -1.0)


def extend(core: np.ndarray, periodic, sign: float) -> np.ndarray:
    """Ghost-extend a core along its rows by NG rows per side: wrap (periodic True or
    "periodic"), mirror times sign (False or "wall"), or zeros ("exact": the ghost values then
    come from separate boundary terms)."""
    kind = periodic if isinstance(periodic, str) else ("periodic" if periodic else "wall")
    if kind == "periodic":
        return np.concatenate([core[-NG:], core, core[:NG]], axis=0)
    if kind == "wall":
        return np.concatenate([sign * core[:NG][::-1], core, sign * core[-NG:][::-1]], axis=0)
    z = np.zeros((NG,) + core.shape[1:])
    return np.concatenate([z, core, z], axis=0)


def _time_factor(term, t: float) -> float:
    return term.amp * math.cos(term.omega * t + term.phase)


class _Lambda:
    """Entries max(|m-/h-| + sqrt(g h-), |m+/h+| + sqrt(g h+)) from four TTs."""

    def __init__(self, hm, mm, hp, mp, g):
        self.t, self.g = (hm, mm, hp, mp), g

    def _f(self, hm, mm, hp, mp):
        g = self.g
        return np.maximum(np.abs(mm / hm) + np.sqrt(g * hm), np.abs(mp / hp) + np.sqrt(g * hp))

    def cols(self, J):
        return self._f(*[X.A @ X.B[J].T for X in self.t])

    def rows(self, I):
        return self._f(*[X.A[I] @ X.B.T for X in self.t])


def rook_max(fun, n1: int, n2: int, J0, max_alt: int = 8):
    """Largest entry of the matrix fun (entries by .cols(J) and .rows(I)) by rook pivoting from
    several starts: for every starting column j in J0, a walk from the largest entry of that
    column alternates the largest entry of the current row and of the current column until the
    value stops growing (at most max_alt alternations); the best walk wins.  A rook-pivot local
    maximum, hence a lower bound of the true maximum.  Ties go to the smallest index, walks in
    the order of J0.  Returns (value, i, j)."""
    J0 = np.asarray(J0)
    C = fun.cols(J0)
    best = (-np.inf, 0, 0)
    for k, j in enumerate(J0):
        i = int(np.argmax(C[:, k]))
        j = int(j)
        v = float(C[i, k])
        for _ in range(max_alt):
            row = fun.rows(np.array([i]))[0]
            jj = int(np.argmax(row))
            if row[jj] <= v:
                break
            v, j = float(row[jj]), jj
            col = fun.cols(np.array([j]))[:, 0]
            ii = int(np.argmax(col))
            if col[ii] <= v:
                break
            v, i = float(col[ii]), ii
        if v > best[0]:
            best = (v, i, j)
    return best


class _LFFlux:
    """LF-cross entries (the alternative Section 4.2 contrasts with the present approach, from
    the authors' earlier Euler work): the whole LLF flux vector of one direction by a single
    cross, the flux component folded into the column index, column c * n2 + j.  The states are
    in normal-first order (h, m, t): F = (m, m^2/h + g h^2/2, m t/h),
    Fhat = (F(U-) + F(U+))/2 - lambda/2 (U+ - U-), lambda = max(|m-/h-| + sqrt(g h-),
    |m+/h+| + sqrt(g h+))."""

    def __init__(self, qm, qp, g, n2):
        self.t, self.g, self.n2 = list(qm) + list(qp), g, n2

    def _f(self, vals, comps):
        hm, mm, tm, hp, mp, tp = vals
        g = self.g
        lam = np.maximum(np.abs(mm / hm) + np.sqrt(g * hm), np.abs(mp / hp) + np.sqrt(g * hp))
        Fm = (mm, mm * mm / hm + 0.5 * g * hm * hm, mm * tm / hm)
        Fp = (mp, mp * mp / hp + 0.5 * g * hp * hp, mp * tp / hp)
        Um, Up = (hm, mm, tm), (hp, mp, tp)
        out = np.empty_like(hm)
        for c in range(3):
            sel = comps == c
            out[:, sel] = (0.5 * (Fm[c] + Fp[c]) - 0.5 * lam * (Up[c] - Um[c]))[:, sel]
        return out

    def cols(self, J):
        J = np.asarray(J)
        comps, j = J // self.n2, J % self.n2
        return self._f([X.A @ X.B[j].T for X in self.t], comps)

    def rows(self, I):
        I = np.asarray(I)
        comps = np.repeat(np.arange(3), self.n2)
        vals = [np.tile(X.A[I] @ X.B.T, (1, 3)) for X in self.t]
        return self._f(vals, comps)


class _Recip:
    """Entries 1/x of one TT (the cross alternative to Algorithm 1 named in Section 4.2)."""

    def __init__(self, x: TT):
        self.x = x

    def cols(self, J):
        return 1.0 / (self.x.A @ self.x.B[J].T)

    def rows(self, I):
        return 1.0 / (self.x.A[I] @ self.x.B.T)


class _WenoFace:
    """Algorithm 2 entries: WENO5 Step-1 face value of the cells around face f, column j."""

    def __init__(self, q: TT, periodic, sign, side, n_faces, tab, eps, extra=None):
        """extra = (normal-axis columns, n + 6 rows already extended; their factors along
        the columns' index): ghost terms of an exact normal boundary, summed into the field."""
        self.Ae, self.B = extend(q.A, periodic, sign), q.B
        if extra is not None:
            self.Ae = np.concatenate([self.Ae, extra[0]], axis=1)
            self.B = np.concatenate([self.B, extra[1]], axis=1)
        self.side, self.nf, self.tab, self.eps = side, n_faces, tab, eps

    @classmethod
    def from_cores(cls, Ae, B, side, n_faces, tab, eps):
        """Entries of the field Ae B^T with its first core already extended (n + 6 rows)."""
        f = cls.__new__(cls)
        f.Ae, f.B = Ae, B
        f.side, f.nf, f.tab, f.eps = side, n_faces, tab, eps
        return f

    def _vals(self, rows_of):
        if self.side < 0:   # right face of cell f-1
            return {o: rows_of(NG + (-1 + o)) for o in range(-2, 3)}
        return {o: rows_of(NG + (0 - o)) for o in range(-2, 3)}  # left face of cell f, mirrored

    def cols(self, J):
        f = np.arange(self.nf)
        BJ = self.B[J].T
        vals = self._vals(lambda off: self.Ae[f + off] @ BJ)
        return fv_grid.recon_point(vals, self.tab, "face", "weno5", self.eps)

    def rows(self, I):
        I = np.asarray(I)
        vals = self._vals(lambda off: self.Ae[I + off] @ self.B.T)
        return fv_grid.recon_point(vals, self.tab, "face", "weno5", self.eps)


class _WenoQuad:
    """Algorithm 3 entries: WENO5 Step-2 value at Gauss point m of cell j, column j*nq + m."""

    def __init__(self, v: TT, periodic, sign, n, tab, eps, Be=None):
        """Be: v's second core already extended to n + 6 rows (an exact tangent boundary)."""
        self.A, self.Be = v.A, (extend(v.B, periodic, sign) if Be is None else Be)
        self.n, self.tab, self.eps, self.nq = n, tab, eps, tab["nq"]

    def _quad(self, vals):
        return np.stack([fv_grid.recon_point(vals, self.tab, m, "weno5", self.eps)
                         for m in range(self.nq)], axis=-1)

    def cols(self, J):
        J = np.asarray(J)
        j, m = J // self.nq, J % self.nq
        vals = {o: self.A @ self.Be[NG + j + o].T for o in range(-2, 3)}
        allq = self._quad(vals)                              # n_f x |J| x nq
        return allq[:, np.arange(len(J)), m]

    def rows(self, I):
        I = np.asarray(I)
        jj = np.arange(self.n)
        vals = {o: self.A[I] @ self.Be[NG + jj + o].T for o in range(-2, 3)}
        return self._quad(vals).reshape(len(I), -1)          # column j*nq + m


class TTSolver:
    def __init__(self, n: int, scheme: str, nonlinear: bool, periodic: bool = True,
                 g: float = 9.81, H: float = 1.0, f: float = 0.0, eps: float = 1e-10,
                 rmax: int = 32, taylor_terms: int = 8, cross_sweeps: int = 3,
                 cross_kick: int = 4, cross_full: bool = False, recip: str = "taylor",
                 replay=None, cross_drop: float = 1e-13, eps_rule: str = "fixed",
                 c_eps: float = 1.0, bc=None, terms=(), t0: float = 0.0,
                 flux: str = "products", cross_enrich: str = "random"):
        self.n, self.scheme, self.nonlinear = n, scheme, nonlinear
        self.bc = tuple(bc) if bc is not None else \
            (("periodic", "periodic") if periodic else ("wall", "wall"))
        if any(b not in ("periodic", "wall", "exact") for b in self.bc) or \
                self.bc.count("exact") > 1:
            raise ValueError(f"bad boundary kinds {self.bc}")
        self.terms = list(terms)
        self.t = t0                        # time at the start of the next step
        self.g, self.H, self.f = g, H, f
        self.eps, self.rmax, self.K = eps, rmax, taylor_terms
        if eps_rule not in ("fixed", "paper"):
            raise ValueError("eps_rule must be 'fixed' or 'paper'")
        self.eps_rule, self.c_eps = eps_rule, c_eps
        self.order = 3 if scheme == "upwind3" else 5
        self.eps_q = [eps, eps, eps]       # tolerances of the time-stepping roundings
        self.sweeps, self.kick, self.cross_full = cross_sweeps, cross_kick, cross_full
        self.recip = recip
        if flux not in ("products", "lf_cross"):
            raise ValueError("flux must be 'products' or 'lf_cross'")
        self.flux = flux                   # nonlinear LLF: products of Section 4.2 or LF-cross
        self.enrich = cross_enrich         # cross enrichment: seeded kicks or largest residual
        self.cross_drop = cross_drop     # orth drop threshold of the crosses (reading R12)
        self.dx = 1.0 / n
        self.tab = stencils.tables(scheme)
        self.nq = self.tab["nq"]
        self.nf_axis = [n if b == "periodic" else n + 1 for b in self.bc]
        k = self.tab["k"]
        self.face_w = np.asarray(self.tab["face_full"])       # offsets -k..k, at +1/2
        self.quad_w = [np.asarray(w) for w in self.tab["quad_full"]]
        self.k = k
        self.pivots = {}
        # (step, site) -> (J, I) of every cross's last sweep; with `replay` given, each cross
        # takes its (J, I) from there and forms only the skeleton (several pivot sets are
        # equally valid at the rank cap; replaying one set makes two implementations
        # comparable)
        self.cross_log = {}
        self.replay = replay
        self.step_index = 0
        self.stats = {"taylor_terms": [], "taylor_err": [], "ranks": [], "eps": []}

    # -- helpers ---------------------------------------------------------------
    def rnd(self, X: TT) -> TT:
        return tt_round(X, self.eps, self.rmax)

    def face_cores(self, A: np.ndarray, sign: float, axis: int = 0, explicit=None):
        """(Rf- A, Rf+ A): face values of every column of the core along `axis`, n_f x r each;
        `explicit` (n + 6 rows, already extended) is appended as further columns."""
        E = extend(A, self.bc[axis], sign)
        if explicit is not None:
            E = np.concatenate([E, explicit], axis=1)
        f = np.arange(self.nf_axis[axis])
        k = self.k
        m = sum(self.face_w[o + k] * E[NG + f - 1 + o] for o in range(-k, k + 1))
        p = sum(self.face_w[o + k] * E[NG + f - o] for o in range(-k, k + 1))
        return m, p

    def quad_core(self, B: np.ndarray, sign: float, axis: int = 1, explicit=None) -> np.ndarray:
        """Gauss-point values of every column along `axis`, rows j*nq + m, (n*nq) x r;
        `explicit` (n + 6 rows, already extended) is appended as further columns."""
        E = extend(B, self.bc[axis], sign)
        if explicit is not None:
            E = np.concatenate([E, explicit], axis=1)
        j = np.arange(self.n)
        k = self.k
        out = np.stack([sum(w[o + k] * E[NG + j + o] for o in range(-k, k + 1))
                        for w in self.quad_w], axis=1)        # n x nq x r
        return out.reshape(self.n * self.nq, -1)

    def _cross(self, fun, n1, n2, y0: TT, site: int):
        if self.cross_full:
            J0 = np.arange(n2)
            X, J = cross(fun, n1, n2, J0, self.eps, self.rmax, sweeps=1, kick=0)
            return X
        if self.replay is not None:
            J, I = self.replay[(self.step_index, site)]
            self.pivots[site] = np.asarray(J, dtype=np.int64)
            self.cross_log[(self.step_index, site)] = (np.asarray(J), np.asarray(I))
            return skeleton(fun, n1, n2, J, I, self.eps, self.rmax)
        J0 = self.pivots.get(site)
        if J0 is None:
            J0 = initial_columns(y0, self.cross_drop)
        key = (site << 32) | (self.step_index & 0xFFFFFFFF)
        rows = []
        X, J = cross(fun, n1, n2, J0, self.eps, self.rmax, self.sweeps, self.kick, key,
                     rows_out=rows, drop=self.cross_drop, enrich=self.enrich)
        self.pivots[site] = J
        self.cross_log[(self.step_index, site)] = (J.copy(), rows[0])
        return X

    # -- one direction -----------------------------------------------------------
    def ghost_columns(self, var: int, d: int, t: float):
        """The ghost terms of natural variable `var` at time t in direction-d orientation:
        (normal-axis columns, tangent-axis columns), each (n + 6) x J and already extended."""
        n = self.n
        sgn = ((1.0, -1.0, 1.0), (1.0, 1.0, -1.0))    # momentum normal to each axis flips
        cols = ([], [])
        for tm in self.terms:
            if tm.var != var or tm.where == "forcing":
                continue
            ax = 0 if tm.where.startswith("x") else 1
            ghost = np.zeros(n + 2 * NG)
            vals = _time_factor(tm, t) * np.asarray(tm.X if ax == 0 else tm.Y, dtype=float)
            if tm.where.endswith("lo"):
                ghost[:NG] = vals
            else:
                ghost[n + NG:] = vals
            other = np.asarray(tm.Y if ax == 0 else tm.X, dtype=float)[:, None]
            other = extend(other, self.bc[1 - ax], sgn[1 - ax][var])[:, 0]
            by_axis = {ax: ghost, 1 - ax: other}
            cols[0].append(by_axis[d])
            cols[1].append(by_axis[1 - d])
        if not cols[0]:
            return None, None
        return np.stack(cols[0], axis=1), np.stack(cols[1], axis=1)

    def states(self, Q, site_base: int, d: int = 0, t: float = 0.0):
        """Face-quadrature states (minus, plus) of the three variables, direction d."""
        qm, qp = [], []
        if self.scheme != "weno5":
            natural = (0, 1, 2) if d == 0 else (0, 2, 1)
            for c, q in enumerate(Q):
                gn, gt = self.ghost_columns(natural[c], d, t)
                Am, Ap = self.face_cores(q.A, SIGN_NORMAL[c], d, gn)
                Bq = self.quad_core(q.B, SIGN_TANGENT[c], 1 - d, gt)
                qm.append(TT(Am, Bq))
                qp.append(TT(Ap, Bq))
            return qm, qp
        eps_w = self.dx * self.dx
        nn = self.n * self.nq
        natural = (0, 1, 2) if d == 0 else (0, 2, 1)
        n = self.n
        ghost_rows = np.r_[0:NG, n + NG:n + 2 * NG]
        for c, q in enumerate(Q):
            gn, gt = self.ghost_columns(natural[c], d, t)
            extra = None
            if gn is not None and self.bc[d] == "exact":
                extra = (gn, gt[NG:NG + n])
            out = []
            for side_i, side in enumerate((-1, 1)):
                site = site_base + 16 + c * 4 + side_i
                nf = self.nf_axis[d]
                v = self._cross(_WenoFace(q, self.bc[d], SIGN_NORMAL[c], side, nf,
                                          self.tab, eps_w, extra), nf, n, q, site)
                # initial columns for Step 2: v's second core repeated for every Gauss point
                y0 = TT(v.A, np.repeat(v.B, self.nq, axis=0))
                Be = None
                if self.bc[1 - d] == "exact":
                    # Step-1 values at the tangent ghost cells: the ghost terms alone
                    if gn is not None:
                        V = _WenoFace.from_cores(gn, gt, side, nf, self.tab, eps_w) \
                            .cols(ghost_rows)
                    else:
                        V = np.zeros((nf, 2 * NG))
                    E = np.zeros((n + 2 * NG, 2 * NG))
                    E[ghost_rows, np.arange(2 * NG)] = 1.0
                    Bz = np.concatenate([np.zeros((NG, v.rank)), v.B, np.zeros((NG, v.rank))])
                    v = TT(np.concatenate([v.A, V], axis=1), np.concatenate([Bz, E], axis=1))
                    Be = v.B
                w = self._cross(_WenoQuad(v, self.bc[1 - d], SIGN_TANGENT[c], n, self.tab,
                                          eps_w, Be), nf, nn, y0, site + 2)
                out.append(w)
            qm.append(out[0])
            qp.append(out[1])
        return qm, qp

    def face_flux(self, Q, site_base: int, d: int = 0, t: float = 0.0):
        """Fhat for the direction whose normal core is the first core: 3 TTs n_f x (n*nq)."""
        qm, qp = self.states(Q, site_base, d, t)
        nf = self.nf_axis[d]
        if not self.nonlinear:
            g, H = self.g, self.H
            c = math.sqrt(g * H)
            eta_m, u_m, v_m = qm
            eta_p, u_p, v_p = qp
            F0 = add([(0.5 * H, u_m), (0.5 * H, u_p), (-0.5 * c, eta_p), (0.5 * c, eta_m)])
            F1 = add([(0.5 * g, eta_m), (0.5 * g, eta_p), (-0.5 * c, u_p), (0.5 * c, u_m)])
            F2 = add([(-0.5 * c, v_p), (0.5 * c, v_m)])
            return [F0, F1, F2]
        g = self.g
        if self.flux == "lf_cross":
            n2 = self.n * self.nq
            y0 = qm[1] if norm(qm[1]) > 0.0 else qm[0]
            y0 = TT(y0.A, np.concatenate([y0.B] * 3, axis=0))
            Fv = self._cross(_LFFlux(qm, qp, g, n2), nf, 3 * n2, y0, site_base + 4)
            return [TT(Fv.A, Fv.B[c * n2:(c + 1) * n2]) for c in range(3)]
        F = {}
        for si, (s, (h, m, t)) in enumerate((("m", qm), ("p", qp))):
            if self.recip == "cross":
                rh = self._cross(_Recip(h), nf, self.n * self.nq, h, site_base + 8 + si)
            else:
                rh, err, terms = reciprocal(h, self.eps, self.K, self.rmax)
                self.stats["taylor_terms"].append(terms)
                self.stats["taylor_err"].append(err)
            u = self.rnd(hadamard(m, rh))
            w = self.rnd(hadamard(t, rh))
            P1 = self.rnd(hadamard(m, u))
            P2 = self.rnd(hadamard(h, h))
            F2 = self.rnd(add([(1.0, P1), (0.5 * g, P2)]))
            F3 = self.rnd(hadamard(m, w))
            F[s] = [m, F2, F3]
        hm, mm = qm[0], qm[1]
        hp, mp = qp[0], qp[1]
        y0 = mm if norm(mm) > 0.0 else hm
        lam = self._cross(_Lambda(hm, mm, hp, mp, g), nf, self.n * self.nq, y0, site_base)
        out = []
        for c in range(3):
            dq = add([(1.0, qp[c]), (-1.0, qm[c])])
            D = self.rnd(hadamard(lam, dq))
            out.append(self.rnd(add([(0.5, F["m"][c]), (0.5, F["p"][c]), (-0.5, D)])))
        return out

    def finish(self, Fh: TT, d: int = 0) -> TT:
        """Gauss-Legendre sum on the second core, (T - 1) on the first core."""
        w = np.asarray(self.tab["gl_weights"])
        B = np.tensordot(Fh.B.reshape(self.n, self.nq, -1), w, axes=([1], [0]))
        A = Fh.A
        dA = (np.roll(A, -1, axis=0) - A) if self.bc[d] == "periodic" else (A[1:] - A[:-1])
        return TT(dA, B)

    def L(self, Q, stage: int, t: float = 0.0):
        """Right-hand side as three TTs (concatenations, not rounded) at stage time t."""
        Fx = [self.finish(F, 0) for F in self.face_flux(Q, (0 * 3 + stage) << 6, 0, t)]
        Qy = [Q[0].T(), Q[2].T(), Q[1].T()]
        Gy = [self.finish(F, 1) for F in self.face_flux(Qy, (1 * 3 + stage) << 6, 1, t)]
        G = [Gy[0].T(), Gy[2].T(), Gy[1].T()]
        dx = self.dx
        out = []
        for c in range(3):
            terms = [(-1.0 / dx, Fx[c]), (-1.0 / dx, G[c])]
            if self.f != 0.0 and c == 1:
                terms.append((self.f, Q[2]))
            if self.f != 0.0 and c == 2:
                terms.append((-self.f, Q[1]))
            for tm in self.terms:
                if tm.var == c and tm.where == "forcing":
                    terms.append((_time_factor(tm, t),
                                  TT(np.asarray(tm.X, dtype=float)[:, None],
                                     np.asarray(tm.Y, dtype=float)[:, None])))
            out.append(add(terms))
        return out

    def euler(self, Q, dt: float, stage: int, t: float = 0.0):
        """F(q) = round(q + dt L(q)), L at stage time t."""
        Lq = self.L(Q, stage, t)
        return [tt_round(add([(1.0, q), (dt, l)]), e, self.rmax)
                for q, l, e in zip(Q, Lq, self.eps_q)]

    def step(self, Q, dt: float):
        if self.eps_rule == "paper":
            self.eps, self.eps_q = paper_tolerances([norm(q) for q in Q], self.n, self.order,
                                                    self.c_eps)
            self.stats["eps"].append((self.eps, list(self.eps_q)))
        e = self.eps_q
        t = self.t
        # stage times of SSP-RK3: t, t + dt, t + dt/2
        Q1 = self.euler(Q, dt, 0, t)
        F1 = self.euler(Q1, dt, 1, t + dt)
        Q2 = [tt_round(add([(0.75, q), (0.25, f)]), e[c], self.rmax)
              for c, (q, f) in enumerate(zip(Q, F1))]
        F2 = self.euler(Q2, dt, 2, t + 0.5 * dt)
        Qn = [tt_round(add([(1.0 / 3.0, q), (2.0 / 3.0, f)]), e[c], self.rmax)
              for c, (q, f) in enumerate(zip(Q, F2))]
        self.step_index += 1
        self.t = t + dt
        self.stats["ranks"].append([q.rank for q in Qn])
        return Qn

    def max_speed(self, Q, d: int) -> float:
        """Largest wave speed of direction d over the cells, for the explicit step's CFL
        condition: |m/h| + sqrt(g h) with m the momentum along d (nonlinear; by rook pivoting
        on the TTs, started from the maxvol columns of h's second core), sqrt(g H) (linear)."""
        if not self.nonlinear:
            return math.sqrt(self.g * self.H)
        h, m = Q[0], Q[1 + d]
        J0 = initial_columns(h, self.cross_drop)
        return rook_max(_Lambda(h, m, h, m, self.g), self.n, self.n, J0)[0]

    def cfl_dt(self, Q, cfl: float) -> float:
        """dt = cfl / (s_x / dx + s_y / dy) from the two directions' largest speeds."""
        sx, sy = self.max_speed(Q, 0), self.max_speed(Q, 1)
        return cfl / ((sx + sy) / self.dx)

    def run(self, Q, dt: float, nsteps: int):
        for _ in range(nsteps):
            Q = self.step(Q, dt)
        return Q

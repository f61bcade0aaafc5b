"""Plain 2-core tensor-train algebra (Section 3 of the paper).

Oracle (test infrastructure only).

A 2-core TT of an n1 x n2 matrix is X(i1, i2) = G1(i1) G2(i2) (Section 3.1, the 2-D form
of the TT definition).  It is stored here as two factors A = G1 (n1 x r) and B = G2^T
(n2 x r), so X = A @ B.T.

Operations
  round        Section 3.2: orthogonalise the second core (RQ of G2, done as QR of B),
               then truncated SVD of G1 R at relative Frobenius accuracy eps, rank <= rmax.
  add / scale  sums of TTs concatenate the cores (ranks add); when two terms share the
               second core object the first cores are added instead.
  hadamard     elementwise product: row-wise Kronecker (face-splitting) product of cores,
               ranks multiply (used throughout Section 4.2).
  tt_sum, norm sum of all entries and Frobenius norm (used by Algorithm 1).
  reciprocal   Algorithm 1 (Taylor series of 1/x about the mean of x); raises
               SeriesDiverges when the terms grow (the series has no limit).
  maxvol       maximum-volume row selection (Goreinov et al., cited in Section 3.3).
  cross        alternating skeleton (CUR) cross interpolation with maxvol pivots
               (Section 3.3; a plain alternating-maxvol stand-in for AMEn cross).
  splitmix64   counter-based generator (Steele, Lea and Flood 2014) for the index kicks.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class TT:
    A: np.ndarray   # n1 x r  (first core G1)
    B: np.ndarray   # n2 x r  (second core G2, transposed)

    @property
    def rank(self) -> int:
        return self.A.shape[1]

    @property
    def shape(self):
        return (self.A.shape[0], self.B.shape[0])

    def full(self) -> np.ndarray:
        return self.A @ self.B.T

    def T(self) -> "TT":
        return TT(self.B, self.A)


def zero_tt(n1: int, n2: int) -> TT:
    return TT(np.zeros((n1, 1)), np.zeros((n2, 1)))


def ones_tt(n1: int, n2: int) -> TT:
    return TT(np.ones((n1, 1)), np.ones((n2, 1)))


def trunc_rank(s: np.ndarray, eps: float, rmax: int) -> int:
    """Smallest k >= 1 with ||s[k:]|| <= eps ||s||, then capped at rmax."""
    ss = s * s
    total = float(ss.sum())
    tail = np.cumsum(ss[::-1])[::-1]          # tail[k] = sum_{i >= k} s_i^2
    thr = (eps * eps) * total
    k = len(s)
    for kk in range(1, len(s) + 1):
        t = float(tail[kk]) if kk < len(s) else 0.0
        if t <= thr:
            k = kk
            break
    return max(1, min(k, rmax))


def tt_round(X: TT, eps: float, rmax: int) -> TT:
    """TT rounding (Section 3.2): QR of the second core, truncated SVD of G1 R."""
    qb, rb = np.linalg.qr(X.B)              # B = qb rb  <=>  G2 = rb^T qb^T (RQ of G2)
    W = X.A @ rb.T                          # G1 R, n1 x min(n2, r)
    u, s, vt = np.linalg.svd(W, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return zero_tt(*X.shape)
    k = trunc_rank(s, eps, rmax)
    return TT(u[:, :k] * s[None, :k], qb @ vt[:k].T)


def add(terms) -> TT:
    """Sum of (coefficient, TT) pairs; terms sharing the same B array object add their A."""
    groups = []
    for c, X in terms:
        for g in groups:
            if g[1] is X.B:
                g[0] = g[0] + c * X.A
                break
        else:
            groups.append([c * X.A, X.B])
    return TT(np.concatenate([g[0] for g in groups], axis=1),
              np.concatenate([g[1] for g in groups], axis=1))


def scale(X: TT, c: float) -> TT:
    return TT(c * X.A, X.B)


def hadamard(X: TT, Y: TT) -> TT:
    """Elementwise product; column a*ry + b of each core is X_col(a) * Y_col(b)."""
    n1, n2 = X.shape
    A = (X.A[:, :, None] * Y.A[:, None, :]).reshape(n1, -1)
    B = (X.B[:, :, None] * Y.B[:, None, :]).reshape(n2, -1)
    return TT(A, B)


def tt_sum(X: TT) -> float:
    return float(X.A.sum(axis=0) @ X.B.sum(axis=0))


def norm(X: TT) -> float:
    v = float(np.sum((X.A.T @ X.A) * (X.B.T @ X.B)))
    return math.sqrt(max(v, 0.0))


class SeriesDiverges(ArithmeticError):
    """The Taylor series of 1/x about the mean of x does not converge (|1 - x/mean| >= 1
    somewhere), detected as two consecutive increases of the term norm."""


def reciprocal(x: TT, eps: float, max_terms: int, rmax: int):
    """1/x by the truncated Neumann series of Algorithm 1.

    With m the mean of x and z = 1 - x/m (rounded once), 1/x = (1/m) sum_{k>=0} z^k whenever
    |z| < 1 pointwise.  The terms d_k = z^k are built one from the previous,
    d_k = round(d_{k-1} o z), and accumulated into rounded partial sums
    y_k = round(y_{k-1} + d_k), starting from d_0 = y_0 = 1.  Accumulation ends once the
    root-mean-square size of the newest term, ||d_k||_F / sqrt(N), is at most eps, or when
    max_terms terms (counting d_0) are in the sum.  Since |z| < 1 makes ||d_k|| shrink by at
    least max|z| per term, two consecutive increases mean the series diverges
    (SeriesDiverges).  Returns (y_K / m, last term size, number of terms).
    """
    n1, n2 = x.shape
    N = n1 * n2
    mean = tt_sum(x) / N
    z = tt_round(add([(1.0, ones_tt(n1, n2)), (-1.0 / mean, x)]), eps, rmax)
    partial, term = ones_tt(n1, n2), ones_tt(n1, n2)
    sizes = [1.0]
    while sizes[-1] > eps and len(sizes) < max_terms:
        term = tt_round(hadamard(term, z), eps, rmax)
        partial = tt_round(add([(1.0, partial), (1.0, term)]), eps, rmax)
        sizes.append(norm(term) / math.sqrt(N))
        if len(sizes) >= 3 and sizes[-1] > sizes[-2] > sizes[-3]:
            raise SeriesDiverges("Taylor reciprocal: term norms grow (|1 - x/mean| >= 1)")
    return scale(partial, 1.0 / mean), sizes[-1], len(sizes)


# ---------------------------------------------------------------------------
# maxvol and cross

def greedy_rows(Q: np.ndarray) -> np.ndarray:
    """Initial rows for maxvol: repeatedly take the row of largest residual norm and project
    its direction out of all rows (pivoted QR of Q^T).  For an orthonormal basis Q the
    choice does not depend on which orthonormal basis of the column space is used."""
    n, r = Q.shape
    R = Q.copy()
    rows = []
    for _ in range(r):
        nrm = np.einsum("ij,ij->i", R, R)
        i = int(np.argmax(nrm))          # ties -> smallest index
        rows.append(i)
        v = R[i] / math.sqrt(nrm[i])
        R = R - np.outer(R @ v, v)
    return np.array(rows, dtype=np.int64)


def maxvol(Q: np.ndarray, tau: float = 1.05, maxit: int = 100):
    """Rows I of Q (n x r, n >= r) with |Q Q[I]^{-1}| <= tau entrywise (dominant submatrix).

    Swap loop of Goreinov et al.: B = Q Q[I]^{-1}; while max|B_ij| > tau, replace the j-th
    chosen row by row i and update B by a rank-one correction.  Ties in argmax go to the
    smallest row, then the smallest column.
    """
    n, r = Q.shape
    I = greedy_rows(Q)
    B = np.linalg.solve(Q[I].T, Q.T).T          # Q Q[I]^{-1}
    for _ in range(maxit):
        flat = int(np.argmax(np.abs(B)))
        i, j = divmod(flat, r)
        if abs(B[i, j]) <= tau:
            break
        bj = B[:, j].copy()
        bi = B[i, :].copy()
        bi[j] -= 1.0
        B -= np.outer(bj, bi) / bj[i]
        I[j] = i
    return I


def orth(C: np.ndarray, drop: float = 1e-13, k: int = None) -> np.ndarray:
    """Orthonormal basis of range(C): QR, SVD of R, drop directions with s <= drop*s_max
    (or keep exactly the k leading directions when k is given).

    Each kept column is given a fixed sign (its entry of largest magnitude is positive) so
    the basis is unique up to rounding.
    """
    q, r = np.linalg.qr(C)
    u, s, _ = np.linalg.svd(r)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros((C.shape[0], 0))
    if k is None:
        k = int(np.sum(s > drop * s[0]))
    elif k > s.size or s[k - 1] == 0.0:
        raise ValueError(f"orth: the columns have fewer than {k} nonzero directions")
    U = q @ u[:, :k]
    idx = np.argmax(np.abs(U), axis=0)
    sg = np.sign(U[idx, np.arange(k)])
    sg[sg == 0] = 1.0
    return U * sg[None, :]


MASK64 = (1 << 64) - 1


def splitmix64(state: int):
    """One step of SplitMix64; returns (new_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def kick_indices(existing, n: int, count: int, key: int):
    """`count` new indices in [0, n) not in `existing`, drawn with SplitMix64 from `key`."""
    have = set(int(v) for v in existing)
    out = []
    state = key & MASK64
    tries = 0
    while len(out) < count and len(have) < n and tries < 64 * (count + 1):
        state, z = splitmix64(state)
        idx = int(z % n)
        tries += 1
        if idx not in have:
            have.add(idx)
            out.append(idx)
    return out


def skeleton(fun, n1: int, n2: int, J, I, eps: float, rmax: int, Qc=None) -> TT:
    """Skeleton (CUR) approximation of the matrix defined by `fun` from column set J and row
    set I (Section 3.3): with Qc the |I| leading orthonormal directions of the columns
    f(:, J), X ~ Qc Qc[I]^{-1} f(I, :), then rounded to (eps, rmax).  An empty I (the
    columns are zero) gives the zero TT."""
    I = np.asarray(I, dtype=np.int64)
    if len(I) == 0:
        return zero_tt(n1, n2)
    if Qc is None:
        Qc = orth(fun.cols(np.asarray(J, dtype=np.int64)), k=len(I))
    if Qc.shape[1] != len(I):
        raise ValueError(f"skeleton: {len(I)} rows for a column basis of width {Qc.shape[1]}")
    G1 = np.linalg.solve(Qc[I].T, Qc.T).T         # Qc Qc[I]^{-1}
    return tt_round(TT(G1, fun.rows(I).T), eps, rmax)


def residual_columns(fun, Qc, I, R, J, n2: int, count: int, key: int):
    """Residual-based column enrichment (in the spirit of AMEn's enrichment, Section 3.3): 4 x
    count candidate columns outside J drawn by the kick generator, the skeleton interpolant
    Qc Qc[I]^-1 f(I, j) of each, and the count candidates with the largest residual norms
    |f(:, j) - interpolant| (ties to the earlier candidate; residuals below 1e-12 of the largest
    candidate column's norm, round-off, count as ties at zero).  R = f(I, :)."""
    cand = kick_indices(J, n2, min(4 * count, n2 - len(J)), key)
    if not cand:
        return []
    cand = np.asarray(cand, dtype=np.int64)
    Fc = fun.cols(cand)
    X = Qc @ np.linalg.solve(Qc[I], R[:, cand])
    res = np.linalg.norm(Fc - X, axis=0)
    # residuals at round-off (below 1e-12 of the largest candidate column) are ties
    res[res <= 1e-12 * float(np.max(np.linalg.norm(Fc, axis=0)))] = 0.0
    order = sorted(range(len(cand)), key=lambda t: (-res[t], t))[:count]
    return [int(cand[t]) for t in order]


def cross(fun, n1: int, n2: int, J0, eps: float, rmax: int, sweeps: int = 3,
          kick: int = 4, key: int = 0, rows_out: list = None, drop: float = 1e-13,
          enrich: str = "random"):
    """Alternating maxvol skeleton cross of the n1 x n2 matrix defined by `fun`.

    fun.cols(J) -> n1 x |J| array of entries, fun.rows(I) -> |I| x n2 array.
    Each sweep: C = f(:, J); Qc = orth(C); I = maxvol(Qc); R = f(I, :); and, except in the
    last sweep, J = maxvol(orth(R^T)) enlarged by `kick` fresh indices while |J| < rmax: seeded
    ones (enrich="random"), or the candidates with the largest residual (enrich="residual",
    residual_columns).
    Result: the skeleton of the last sweep's (J, I).  Returns (TT, J of the last sweep); the
    last sweep's I is appended to `rows_out` when given.  `drop`: relative singular value
    below which orth discards a direction.
    """
    J = np.array(J0, dtype=np.int64)
    Qc = I = None
    for s in range(sweeps):
        C = fun.cols(J)
        Qc = orth(C, drop)
        if Qc.shape[1] == 0:
            if rows_out is not None:
                rows_out.append(np.zeros(0, dtype=np.int64))
            return zero_tt(n1, n2), J
        I = maxvol(Qc)
        if s == sweeps - 1:
            break
        R = fun.rows(I)
        Qr = orth(R.T, drop)
        if Qr.shape[1] == 0:
            if rows_out is not None:
                rows_out.append(np.zeros(0, dtype=np.int64))
            return zero_tt(n1, n2), J
        J = maxvol(Qr)
        if len(J) < rmax and kick > 0:
            cnt, k2 = min(kick, rmax - len(J)), key + 1000003 * (s + 1)
            if enrich == "residual":
                extra = residual_columns(fun, Qc, I, R, J, n2, cnt, k2)
            else:
                extra = kick_indices(J, n2, cnt, k2)
            J = np.concatenate([J, np.array(extra, dtype=np.int64)])
    if rows_out is not None:
        rows_out.append(I.copy())
    return skeleton(fun, n1, n2, J, I, eps, rmax, Qc=Qc), J


def initial_columns(Y: TT, drop: float = 1e-13) -> np.ndarray:
    """Starting column set for a cross: maxvol rows of an orthonormal basis of Y's second core."""
    Q = orth(Y.B, drop)
    if Q.shape[1] == 0:
        return np.array([0], dtype=np.int64)
    return maxvol(Q)


def from_full(F: np.ndarray, eps: float, rmax: int) -> TT:
    """Truncated SVD of a full matrix (Section 3.2's truncation applied to F itself): the
    smallest rank k <= rmax whose discarded singular values have norm <= eps ||F||_F; first
    core U_k (orthonormal columns), second V_k Sigma_k.  A zero matrix gives the rank-1 zero TT."""
    U, s, Vt = np.linalg.svd(F, full_matrices=False)
    total = float(np.sum(s * s))
    if total == 0.0:
        return TT(np.zeros((F.shape[0], 1)), np.zeros((F.shape[1], 1)))
    tail = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
    k = len(s)
    for kk in range(1, len(s) + 1):
        if tail[kk] <= eps * eps * total:
            k = kk
            break
    k = max(1, min(k, rmax))
    return TT(U[:, :k].copy(), (Vt[:k].T * s[:k]).copy())


# ---------------------------------------------------------------------------
# The library's randomized rounding, written independently for comparison at round-off.
# It is not in the paper: the library rounds Hadamard products whose rank exceeds its sketch
# width by a randomized range finder (Halko, Martinsson and Tropp 2011) with a seeded Gaussian
# test matrix, so the oracle draws the same matrix from the same published generators
# (SplitMix64's output function of Steele, Lea and Flood 2014 on hashed counters, then
# Box-Muller) and takes the same steps with numpy's QR and SVD.

SKETCH_SEED = 0x5EED5EED12345


def gauss_sketch(rows: int, cols: int, seed: int) -> np.ndarray:
    """rows x cols Gaussian matrix: entry (i, c) from counter idx = c rows + i;
    h1 = mix64(seed xor (2 idx + 1) golden), h2 = mix64(h1 + 0x632BE59BD9B4E019) (mix64 is
    SplitMix64's output function; 64-bit wrap-around arithmetic); u1 = (h1 >> 11 + 1) / (2^53 + 1)
    in (0, 1], u2 = (h2 >> 11) / 2^53; value sqrt(-2 log u1) cos(2 pi u2) (Box-Muller)."""
    u64 = np.uint64
    idx = (np.arange(cols, dtype=np.uint64)[None, :] * u64(rows) +
           np.arange(rows, dtype=np.uint64)[:, None])

    def mix(z):
        z = (z ^ (z >> u64(30))) * u64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> u64(27))) * u64(0x94D049BB133111EB)
        return z ^ (z >> u64(31))

    with np.errstate(over="ignore"):
        h1 = mix(u64(seed) ^ ((idx * u64(2) + u64(1)) * u64(0x9E3779B97F4A7C15)))
        h2 = mix(h1 + u64(0x632BE59BD9B4E019))
    u1 = ((h1 >> u64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740993.0)
    u2 = (h2 >> u64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def tt_round_sketched(X: TT, eps: float, rmax: int, width: int = 0, power_iters: int = 1,
                      max_iters: int = 8) -> TT:
    """The library's rounding of a TT whose rank exceeds the sketch width m = width or
    min(96, max(2 rmax, 16)): Y = X Omega (Omega = gauss_sketch of the shape's seed), power_iters
    subspace iterations, then repeatedly Qa = orth(Y), W = X^T Qa = Qw Rb, the SVD of Rb^T and
    the kept rank k (the tolerance rule of tt_round on those singular values s); stop when k
    reaches m, when s beyond m - max(8, m/4) is below 1e-14 s_0, or when the discarded
    directions can leak at most (s_m / s_k)^(2q+1) s_k <= 1e-13 s_0 into the kept ones after q
    iterations, else iterate once more (Y = X orth(W)); after max(power_iters, max_iters)
    iterations without convergence it returns the exact rounding if the rank is at most 96,
    else the sketch's answer as it stands.  Result Qa U_k (W U_k)^T.
    Inputs whose rank fits the width take the exact rounding."""
    n1, n2, R = X.A.shape[0], X.B.shape[0], X.rank
    m = width if width > 0 else min(96, max(2 * rmax, 16))
    mn = min(n1, n2)
    if R <= m and R <= mn or mn <= m:
        return tt_round(X, eps, rmax)
    m = min(m, mn)
    seed = (SKETCH_SEED ^ ((n1 * 0x9E3779B97F4A7C15) & MASK64) ^ ((n2 << 20) & MASK64) ^
            ((R << 40) & MASK64) ^ m) & MASK64
    Om = gauss_sketch(n2, m, seed)
    A, B = X.A, X.B
    Y = A @ (B.T @ Om)
    q = 0
    for q in range(power_iters):
        Qa, _ = np.linalg.qr(Y)
        Qz, _ = np.linalg.qr(B @ (A.T @ Qa))
        Y = A @ (B.T @ Qz)
    q = power_iters
    qlim = max(power_iters, max_iters)
    while True:
        Qa, _ = np.linalg.qr(Y)
        W = B @ (A.T @ Qa)                          # X^T Qa
        _, Rb = np.linalg.qr(W)
        U, s, _ = np.linalg.svd(Rb.T)
        if s[0] == 0.0:
            return TT(np.zeros((n1, 1)), np.zeros((n2, 1)))
        k = trunc_rank(s, eps, rmax)
        if k >= m:
            break
        pover = max(8, m // 4)
        if m - pover > k and s[m - pover] <= 1e-14 * s[0]:
            break
        if (s[m - 1] / s[k - 1]) ** (2 * q + 1) * s[k - 1] <= 1e-13 * s[0]:
            break
        if q >= qlim:
            # unconverged: the exact rounding when the rank fits a factorisation (96 columns),
            # else the sketch's answer as it stands
            if R <= 96 and R <= mn:
                return tt_round(X, eps, rmax)
            break
        Qz, _ = np.linalg.qr(W)
        Y = A @ (B.T @ Qz)
        q += 1
    return TT(Qa @ U[:, :k], W @ U[:, :k])

"""d-dimensional tensor trains (Section 3.1, equation TT_def) and their rounding (Section 3.2
extended to d cores, the TT-SVD of Oseledets 2011).

Oracle (test infrastructure only).

A d-core TT is a list of cores G_k of shape (r_{k-1}, n_k, r_k), r_0 = r_d = 1, with
X(i_1, ..., i_d) = G_1(:, i_1, :) G_2(:, i_2, :) ... G_d(:, i_d, :).

Rounding to relative accuracy eps and ranks <= rmax:
  1. right-to-left orthogonalisation: for k = d .. 2, the right unfolding of G_k
     (r_{k-1} x n_k r_k) = L Q with Q's rows orthonormal (QR of its transpose); G_k <- Q,
     G_{k-1} <- G_{k-1} times L;
  2. left-to-right truncation: for k = 1 .. d-1, the SVD of the left unfolding of G_k
     ((r_{k-1} n_k) x r_k) = U S V^T truncated at the smallest rank whose discarded singular
     values have norm <= eps / sqrt(d - 1) ||X|| (and at rmax); G_k <- U_k,
     G_{k+1} <- S_k V_k^T times G_{k+1}.
With cores 2..d right-orthonormal, ||X|| = ||G_1||, and each truncation removes at most
eps / sqrt(d - 1) ||X||, so ||X - round(X)|| <= eps ||X|| when no rank cap binds.
"""
from __future__ import annotations

import math

import numpy as np


def full(cores) -> np.ndarray:
    """The full tensor of a TT (small cases only)."""
    X = cores[0]                                   # (1, n1, r1)
    for G in cores[1:]:
        X = np.tensordot(X, G, axes=([X.ndim - 1], [0]))
    return X[0, ..., 0]


def norm(cores) -> float:
    """Frobenius norm by contracting the cores pairwise (no full tensor)."""
    M = np.ones((1, 1))
    for G in cores:
        # M (r x r'), G (r, n, s): M' = sum_{a,b,i} M[a, b] G[a, i, s] G[b, i, t]
        M = np.einsum("ab,ais,bit->st", M, G, G)
    return math.sqrt(max(float(M[0, 0]), 0.0))


def tt_round(cores, eps: float, rmax: int):
    """Rounding of a d-core TT (module docstring); returns (cores, singular values kept at each
    of the d - 1 bonds)."""
    G = [np.array(c, dtype=float) for c in cores]
    d = len(G)
    # 1. right-to-left orthogonalisation
    for k in range(d - 1, 0, -1):
        r0, n, r1 = G[k].shape
        Rk = G[k].reshape(r0, n * r1)
        Q, R = np.linalg.qr(Rk.T)                     # Rk^T = Q R, Rk = R^T Q^T
        G[k] = Q.T.reshape(Q.shape[1], n, r1)
        p0, pn, _ = G[k - 1].shape
        G[k - 1] = (G[k - 1].reshape(p0 * pn, r0) @ R.T).reshape(p0, pn, R.shape[0])
    total = float(np.linalg.norm(G[0]))
    sig = []
    if total == 0.0:
        return [np.zeros((1, c.shape[1], 1)) for c in cores], [[0.0]] * (d - 1)
    delta = eps / math.sqrt(d - 1) * total if d > 1 else 0.0
    # 2. left-to-right truncation
    for k in range(d - 1):
        r0, n, r1 = G[k].shape
        U, s, Vt = np.linalg.svd(G[k].reshape(r0 * n, r1), full_matrices=False)
        tail = np.concatenate([np.sqrt(np.cumsum((s * s)[::-1])[::-1]), [0.0]])
        keep = len(s)
        for kk in range(1, len(s) + 1):
            if tail[kk] <= delta:
                keep = kk
                break
        keep = max(1, min(keep, rmax))
        sig.append(s[:keep].copy())
        G[k] = U[:, :keep].reshape(r0, n, keep)
        SV = s[:keep, None] * Vt[:keep]               # keep x r1
        q0, qn, q1 = G[k + 1].shape
        G[k + 1] = (SV @ G[k + 1].reshape(q0, qn * q1)).reshape(keep, qn, q1)
    return G, sig


def random_tt(rng, modes, ranks, decay: float = 0.7):
    """Random cores with geometrically decaying bond weights (test inputs)."""
    r = [1] + list(ranks) + [1]
    out = []
    for k, n in enumerate(modes):
        G = rng.standard_normal((r[k], n, r[k + 1]))
        G *= (decay ** np.arange(r[k + 1]))[None, None, :]
        out.append(G)
    return out


def add(a, b):
    """Sum of two TTs with equal modes: block-diagonal cores (ranks add)."""
    d = len(a)
    out = []
    for k in range(d):
        A, B = a[k], b[k]
        if d == 1:
            out.append(A + B)
        elif k == 0:
            out.append(np.concatenate([A, B], axis=2))
        elif k == d - 1:
            out.append(np.concatenate([A, B], axis=0))
        else:
            r0a, n, r1a = A.shape
            r0b, _, r1b = B.shape
            C = np.zeros((r0a + r0b, n, r1a + r1b))
            C[:r0a, :, :r1a] = A
            C[r0a:, :, r1a:] = B
            out.append(C)
    return out

"""Pins, on the oracle, of the two facts the fixed-shape (graph) mode of the library rests on:
a TT whose cores carry extra zero columns has the same rounding as without them (so buffers can
keep a static rank with zero columns after the rank chosen on the device), and Algorithm 1 run
for all K terms with the terms after its stopping test entering times zero gives the result of
the loop that stops there (up to the re-rounding of an unchanged partial sum)."""
import math

import numpy as np
import pytest

from oracle import tt as ott


def _graded(rng, n1, n2, r, decay):
    return ott.TT(rng.standard_normal((n1, r)) * decay ** np.arange(r),
                  rng.standard_normal((n2, r)))


def _padded(X: ott.TT, extra: int) -> ott.TT:
    return ott.TT(np.hstack([X.A, np.zeros((X.A.shape[0], extra))]),
                  np.hstack([X.B, np.zeros((X.B.shape[0], extra))]))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("r,extra,eps,rmax", [(12, 20, 1e-8, 10), (30, 2, 1e-12, 40),
                                              (5, 59, 1e-14, 64)])
def test_zero_columns_do_not_change_a_rounding(r, extra, eps, rmax):
    rng = np.random.default_rng(r + extra)
    X = _graded(rng, 90, 70, r, 0.6)
    a = ott.tt_round(X, eps, rmax)
    b = ott.tt_round(_padded(X, extra), eps, rmax)
    assert a.rank == b.rank
    assert _rel(b.full(), a.full()) < 1e-13


def test_zero_columns_in_sums_and_products():
    """Sums and Hadamard products of padded TTs carry only more zero columns: their roundings
    equal those of the unpadded operands."""
    rng = np.random.default_rng(5)
    X, Y = _graded(rng, 80, 60, 6, 0.7), _graded(rng, 80, 60, 5, 0.5)
    Xp, Yp = _padded(X, 4), _padded(Y, 7)
    for a, b in ((ott.add([(1.0, X), (-0.5, Y)]), ott.add([(1.0, Xp), (-0.5, Yp)])),
                 (ott.hadamard(X, Y), ott.hadamard(Xp, Yp))):
        ra, rb = ott.tt_round(a, 1e-10, 20), ott.tt_round(b, 1e-10, 20)
        assert ra.rank == rb.rank
        assert _rel(rb.full(), ra.full()) < 1e-13


def _predicated_reciprocal(x: ott.TT, eps: float, K: int, rmax: int):
    """Algorithm 1 with a fixed K: every term is formed; a flag, cleared by the first term of
    size <= eps, multiplies the terms that enter the partial sum after it."""
    n1, n2 = x.shape
    N = n1 * n2
    mean = ott.tt_sum(x) / N
    z = ott.tt_round(ott.add([(1.0, ott.ones_tt(n1, n2)), (-1.0 / mean, x)]), eps, rmax)
    partial, term, active = ott.ones_tt(n1, n2), ott.ones_tt(n1, n2), 1.0
    for _ in range(1, K):
        term = ott.tt_round(ott.hadamard(term, z), eps, rmax)
        partial = ott.tt_round(ott.add([(1.0, partial), (active, term)]), eps, rmax)
        if active and ott.norm(term) / math.sqrt(N) <= eps:
            active = 0.0
    return ott.scale(partial, 1.0 / mean)


@pytest.mark.parametrize("amp,K", [(0.05, 12), (0.3, 8), (0.02, 20)])
def test_predicated_taylor_equals_the_early_exit_loop(amp, K):
    """Smooth positive fields whose series stops early (amp 0.05 and 0.02: the stop comes before
    K) or runs to K (amp 0.3): the predicated form equals the loop that stops."""
    n = 64
    x_ = (np.arange(n) + 0.5) / n
    X = np.stack([np.ones(n), amp * np.sin(2 * np.pi * x_), amp * np.cos(2 * np.pi * x_)], 1)
    Y = np.stack([np.ones(n), np.cos(2 * np.pi * x_), np.sin(4 * np.pi * x_)], 1)
    x = ott.TT(X, Y)
    ref, err, terms = ott.reciprocal(x, 1e-10, K, 16)
    got = _predicated_reciprocal(x, 1e-10, K, 16)
    assert _rel(got.full(), ref.full()) < 1e-13, terms
    if amp < 0.1:
        assert terms < K                      # the case where the predicate matters


def _masked_maxvol(Qpad: np.ndarray, k: int, tau: float = 1.05, maxit: int = 100):
    """maxvol as the fixed-shape kernels run it on a basis whose columns from k on are zero:
    the greedy start over all m columns (steps after the k-th find residuals of zero and pick
    rows without meaning), Q[I] completed by the identity outside its leading k x k block, then
    the swap loop on B = Q Q[I]^-1."""
    n, m = Qpad.shape
    R = Qpad.copy()
    rows = []
    for _ in range(m):
        nrm = np.einsum("ij,ij->i", R, R)
        i = int(np.argmax(nrm))
        rows.append(i)
        if nrm[i] > 0.0:
            v = R[i] / math.sqrt(nrm[i])
            R = R - np.outer(R @ v, v)
    I = np.array(rows, dtype=np.int64)
    QI = Qpad[I].copy()
    QI[k:, :] = 0.0
    QI[:, k:] = 0.0
    QI[np.arange(k, m), np.arange(k, m)] = 1.0
    B = Qpad @ np.linalg.inv(QI)
    for _ in range(maxit):
        flat = int(np.argmax(np.abs(B)))
        i, j = divmod(flat, m)
        if abs(B[i, j]) <= tau:
            break
        bj = B[:, j].copy()
        bi = B[i, :].copy()
        bi[j] -= 1.0
        B -= np.outer(bj, bi) / bj[i]
        I[j] = i
    return I


@pytest.mark.parametrize("n,k,m", [(200, 7, 16), (500, 24, 32), (129, 1, 40)])
def test_masked_maxvol_picks_the_live_columns_rows(n, k, m):
    """Its first k rows are those of maxvol on the k live columns, and the swaps never touch the
    zero columns."""
    rng = np.random.default_rng(n + k)
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    Qpad = np.hstack([Q, np.zeros((n, m - k))])
    I_live = ott.maxvol(Q)
    I_pad = _masked_maxvol(Qpad, k)
    assert I_pad[:k].tolist() == I_live.tolist()
